"""Served path: requests replayed in real time through the continuous-batching
server.  Every result must be the next slice of its stream's serial sequence
(requests on one stream in arrival order), whatever shared its batch, and the
resident states must end advanced by everything served."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KINDS = ["MWC32", "XS256", "KISS"]


@pytest.fixture(scope="module")
def rng():
    import paper_1101_1846_amd as R
    R.rng_init()
    return R


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available()
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lib.hipMemcpy.restype = ctypes.c_int
    return lib


def _read(hip, ptr, n):
    buf = np.empty(n, dtype=np.uint32)
    assert hip.hipMemcpy(buf.ctypes.data, ptr, 4 * n, 2) == 0  # device to host
    return buf


def _expected_per_stream(oracle, n_streams, seed, streams, lengths):
    """Serial uint32 sequence of every stream over the concatenation of its
    requests, and its final state."""
    seq, fin = {}, {}
    for s in range(n_streams):
        k = s % len(KINDS)
        o = oracle.GENERATORS[KINDS[k]]
        st = oracle.seed(o, seed + k, 1, first_stream=s // len(KINDS))
        total = int(lengths[streams == s].sum())
        seq[s] = oracle.generate(o, st, total)[0] if total else np.zeros(0, np.uint32)
        fin[s] = st[:, 0]
    return seq, fin


@pytest.mark.parametrize("idle_spin_us", [0, 2000])
def test_server_results_are_ordered_stream_slices(rng, hip, oracle, idle_spin_us):
    """With the worker sleeping whenever it is idle, and polling for 2 ms first."""
    from paper_1101_1846_amd import workloads as W
    n_streams, seed, n = 30, 8, 1500
    gens = [rng.GENERATORS[k] for k in KINDS]
    h = rng.rng_server_create(n_streams, gens, seed, 1 << 30, 512, 1 << 22, inflight=3, auto_release=False,
                              idle_spin_us=idle_spin_us)
    try:
        r = np.random.default_rng(12)
        t = W.poisson_arrivals(50_000, n, seed=13)
        streams = r.integers(0, n_streams, n)
        lengths = W.log_uniform_lengths(r, n, 4, 13)
        dtypes = r.integers(0, 2, n)
        tickets = rng.rng_server_replay(h, t, streams, lengths, dtypes)
        st = rng.rng_server_stats(h)
        assert st["completed"] == n and st["batches"] >= 1
        assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
        parts = st["mean_queue_us"] + st["mean_submit_us"] + st["mean_device_us"]
        assert min(st["mean_queue_us"], st["mean_submit_us"], st["mean_device_us"]) >= 0
        assert abs(parts - st["mean_us"]) <= 1e-6 * st["mean_us"] + 1e-3
        seq, fin = _expected_per_stream(oracle, n_streams, seed, streams, lengths)
        pos = {s: 0 for s in range(n_streams)}
        for i, tk in enumerate(tickets):
            done, ptr = rng.rng_server_poll(h, int(tk))
            assert done and ptr
            s, L = int(streams[i]), int(lengths[i])
            exp = seq[s][pos[s]:pos[s] + L]
            if dtypes[i]:
                exp = oracle.to_f32(exp).view(np.uint32)
            assert np.array_equal(_read(hip, ptr, L), exp), (i, s)
            pos[s] += L
            rng.rng_server_release(h, int(tk))
        for s in range(n_streams):
            words = rng.rng_state_words(rng.GENERATORS[KINDS[s % 3]])
            assert np.array_equal(np.array(rng.rng_server_read_state(h, s, words), np.uint32), fin[s])
    finally:
        rng.rng_server_destroy(h)


def test_server_admission_under_memory_pressure(rng, oracle):
    """A 320 KiB output pool and a burst of 400 requests of up to 256 KiB: admission
    waits for released memory, every request completes, and the states end as
    the oracle's after the per-stream totals."""
    from paper_1101_1846_amd import workloads as W
    n_streams, seed, n = 24, 3, 400
    gens = [rng.GENERATORS[k] for k in KINDS]
    h = rng.rng_server_create(n_streams, gens, seed, 320 << 10, 64, 1 << 16, inflight=3, auto_release=True)
    try:
        r = np.random.default_rng(5)
        streams = r.integers(0, n_streams, n)
        lengths = W.log_uniform_lengths(r, n, 6, 16)
        rng.rng_server_replay(h, np.zeros(n), streams, lengths, r.integers(0, 2, n))
        st = rng.rng_server_stats(h)
        assert st["completed"] == n
        assert st["admission_waits"] > 0
        _, fin = _expected_per_stream(oracle, n_streams, seed, streams, lengths)
        for s in range(n_streams):
            words = rng.rng_state_words(rng.GENERATORS[KINDS[s % 3]])
            assert np.array_equal(np.array(rng.rng_server_read_state(h, s, words), np.uint32), fin[s])
    finally:
        rng.rng_server_destroy(h)


def test_server_destroy_abandons_unadmittable(rng):
    """Without auto-release, requests beyond the output pool wait for memory
    that the caller never releases; destroying the server then returns (the
    batches in flight complete, the waiting requests are abandoned) instead of
    waiting for ever."""
    import threading
    import time
    gens = [rng.GENERATORS[k] for k in KINDS]
    h = rng.rng_server_create(12, gens, 4, 256 << 10, 8, 1 << 16, inflight=2, auto_release=False)
    tickets = [rng.rng_server_submit(h, s, 1 << 14, rng.RNG_U32) for s in range(12)]  # 64 KiB each, 4 fit
    deadline = time.time() + 20
    while time.time() < deadline and sum(rng.rng_server_poll(h, t)[0] for t in tickets) < 3:
        time.sleep(0.001)
    time.sleep(0.2)  # whatever fits the pool has completed by now
    done_n = sum(rng.rng_server_poll(h, t)[0] for t in tickets)
    assert 3 <= done_n < len(tickets)
    done = threading.Event()

    def destroy():
        rng.rng_server_destroy(h)
        done.set()

    threading.Thread(target=destroy, daemon=True).start()
    assert done.wait(20), "rng_server_destroy did not return"


def test_server_argument_errors(rng):
    gens = [rng.GENERATORS[k] for k in KINDS]
    with pytest.raises(rng.RngError):
        rng.rng_server_create(9, gens, 1, 1 << 20, 16, 1 << 12, inflight=1, idle_spin_us=2_000_000)
    h = rng.rng_server_create(9, gens, 1, 1 << 20, 16, 1 << 12, inflight=1)
    try:
        L = rng.raw()
        t = ctypes.c_uint64()
        assert L.rng_server_submit(h, 9, 10, 0, ctypes.byref(t)) == rng.RNG_ERANGE
        assert L.rng_server_submit(h, 0, 0, 0, ctypes.byref(t)) == rng.RNG_ERANGE
        assert L.rng_server_submit(h, 0, (1 << 12) + 1, 0, ctypes.byref(t)) == rng.RNG_ERANGE
        assert L.rng_server_submit(h, 0, 10, 3, ctypes.byref(t)) == rng.RNG_EINVAL
        d, p = ctypes.c_int(), ctypes.c_void_p()
        assert L.rng_server_poll(h, 12345, ctypes.byref(d), ctypes.byref(p)) == rng.RNG_EINVAL
        tk = rng.rng_server_submit(h, 4, 100, 1)
        rng.rng_server_drain(h)
        assert rng.rng_server_poll(h, tk)[0]
    finally:
        rng.rng_server_destroy(h)


def test_server_at_bench_scale(rng, hip, oracle):
    """The served workload at the size bench.py runs it: 10^6 resident states
    (generator = stream id mod 3 over MWC32/XS256/KISS), a 16 GiB output pool,
    sizes log-uniform in [2^10, 2^24], dtype 50/50, Poisson arrivals at
    20,000 requests/s, three batches in flight.  1200 requests (about 2e9
    samples): every sample of every request against the oracle (requests on
    one stream as consecutive slices in arrival order), the final state of
    every touched stream, and untouched streams unchanged."""
    import concurrent.futures
    import os
    import sys

    from paper_1101_1846_amd import workloads as W
    threads = max(1, min(16, os.cpu_count() or 1))
    n_streams, seed, n = 10 ** 6, 8, 1200
    gens = [rng.GENERATORS[k] for k in KINDS]
    tab = W.served_table(n, seed=7)
    t = W.poisson_arrivals(20000, n, seed=7)
    assert int(tab["length"].sum()) * 4 < (16 << 30)  # every output fits the pool: no release needed
    h = rng.rng_server_create(n_streams, gens, seed, 16 << 30, 4096, 1 << 31, inflight=3, auto_release=False,
                              idle_spin_us=2000)
    try:
        tickets = rng.rng_server_replay(h, t, tab["stream"], tab["length"], tab["dtype"])
        st = rng.rng_server_stats(h)
        assert st["completed"] == n
        print("served at scale: %d requests in %d batches, p50 %.0f us, p99 %.0f us"
              % (n, st["batches"], st["p50_us"], st["p99_us"]), file=sys.stderr, flush=True)
        for k in KINDS:
            oracle.seed(oracle.GENERATORS[k], seed, 1)  # build the oracle's lazy tables first
        by_stream = {}
        for i, s in enumerate(tab["stream"].tolist()):
            by_stream.setdefault(s, []).append(i)
        ptrs = []
        for tk in tickets:
            done, ptr = rng.rng_server_poll(h, int(tk))
            assert done and ptr
            ptrs.append(ptr)

        def check(streams):
            bad = []
            for s in map(int, streams):
                k = s % 3
                o = oracle.GENERATORS[KINDS[k]]
                stt = oracle.seed(o, seed + k, 1, first_stream=s // 3)
                for i in by_stream[s]:
                    L, d = int(tab["length"][i]), int(tab["dtype"][i])
                    ref = oracle.generate(o, stt, L, d)[0].view(np.uint32)
                    got = _read(hip, ptrs[i], L)
                    if not np.array_equal(got, ref):
                        bad.append("request %d (stream %d, %s, length %d) differs at %d"
                                   % (i, s, KINDS[k], L, int(np.argmax(got != ref))))
                words = rng.rng_state_words(gens[k])
                if not np.array_equal(np.array(rng.rng_server_read_state(h, s, words), np.uint32), stt[:, 0]):
                    bad.append("stream %d: final state differs" % s)
            return bad

        keys = sorted(by_stream)
        bad = []
        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            for r in ex.map(check, np.array_split(np.array(keys), threads)):
                bad.extend(r)
        assert not bad, bad[:5]
        # streams no request touched keep their seeded state
        untouched = [s for s in range(0, n_streams, 99991) if s not in by_stream][:8]
        for s in untouched:
            k = s % 3
            words = rng.rng_state_words(gens[k])
            ref = oracle.seed(oracle.GENERATORS[KINDS[k]], seed + k, 1, first_stream=s // 3)[:, 0]
            assert np.array_equal(np.array(rng.rng_server_read_state(h, s, words), np.uint32), ref), s
        for tk in tickets:
            rng.rng_server_release(h, int(tk))
    finally:
        rng.rng_server_destroy(h)
