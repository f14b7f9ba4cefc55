"""Parity at the full workload sizes, in the launch configuration bench.py times.

- MWC32, 4096 streams x 1024 (base 2^32), states from SplitMix64(0): every sample.
- Bulk store mode, 2^20 streams x 256, XS256 / XS32 / KISS / MWC1616, uint32 and
  FP32, states from SplitMix64(1): every sample and every final state.
- Sequence splitting of one 2^30-sample MWC32 and XS256 sequence over 2^20
  threads: 10^6 uniformly drawn positions plus the first and last 2^20 samples
  and the final state, against one serial pass of the oracle.
- Fused consumer over 2^34 KISS samples (2^20 streams x 2^14): the exact count
  and every final state.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def rng():
    import paper_1101_1846_amd as R
    R.rng_init()
    return R


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def _u32(t):
    import torch as T
    T.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def test_mwc32_4096x1024(rng, torch, oracle):
    g, S, N = rng.RNG_MWC32, 4096, 1024
    st = torch.empty((2, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 0, 0, S, st)
    out = torch.empty((S, N), dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, N, rng.RNG_U32, out)
    ref_st = oracle.seed(oracle.MWC32, 0, S)
    ref = oracle.generate(oracle.MWC32, ref_st, N, threads=THREADS)
    assert np.array_equal(_u32(out), ref)
    assert np.array_equal(_u32(st), ref_st)


@pytest.mark.parametrize("name", ["XS256", "XS32", "KISS", "MWC1616"])
@pytest.mark.parametrize("dt", ["u32", "f32"])
def test_bulk_2p20_streams_x256(rng, torch, oracle, name, dt):
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    S, N = 1 << 20, 256
    st = torch.empty((rng.rng_state_words(g), S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 1, 0, S, st)
    out = torch.empty(S * N, dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, N, t, out)
    got = _u32(out).reshape(S, N)
    ref_st = oracle.seed(o, 1, S)
    ref = oracle.generate(o, ref_st, N, t, threads=THREADS)
    assert np.array_equal(got, ref.view(np.uint32))
    assert np.array_equal(_u32(st), ref_st)


@pytest.mark.parametrize("name", ["MWC32", "XS256"])
def test_split_2p30_over_2p20_threads(rng, torch, oracle, name):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    total, T = 1 << 30, 1 << 20
    W = rng.rng_state_words(g)
    s1 = torch.empty(W, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 2, 0, 1, s1)
    fin = torch.empty(W, dtype=torch.int32, device="cuda")
    wsb = rng.rng_split_workspace_bytes(g, T)
    ws = torch.empty(wsb // 4, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, s1, total, T, rng.RNG_U32, out, fin, ws, wsb)
    pos = np.sort(np.random.default_rng(3).integers(0, total, 10 ** 6, dtype=np.int64))
    idx = torch.from_numpy(pos).to("cuda")
    got_pos = _u32(out[idx])
    head = _u32(out[: 1 << 20])
    tail = _u32(out[total - (1 << 20):])
    one = oracle.seed(o, 2, 1)[:, 0].copy()
    ref_pos, ref_head, ref_tail = oracle.serial_sample(o, one, total, pos.astype(np.uint64), 1 << 20, 1 << 20)
    assert np.array_equal(got_pos, ref_pos)
    assert np.array_equal(head, ref_head)
    assert np.array_equal(tail, ref_tail)
    assert np.array_equal(_u32(fin), one)


@pytest.mark.parametrize("name", ["MWC32", "XS256", "KISS"])
def test_leapfrog_2p30_over_2p20_threads(rng, torch, oracle, name):
    """Leapfrogging one 2^30-sample sequence over 2^20 threads: the same positions,
    head, tail and final state as the split test, against one serial pass."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    total, T = 1 << 30, 1 << 20
    W = rng.rng_state_words(g)
    s1 = torch.empty(W, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 2, 0, 1, s1)
    fin = torch.empty(W, dtype=torch.int32, device="cuda")
    wsb = rng.rng_leapfrog_workspace_bytes(g, T)
    ws = torch.empty(wsb // 4, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    rng.rng_generate_leapfrog(g, s1, total, T, rng.RNG_U32, out, fin, ws, wsb)
    pos = np.sort(np.random.default_rng(3).integers(0, total, 10 ** 6, dtype=np.int64))
    idx = torch.from_numpy(pos).to("cuda")
    got_pos = _u32(out[idx])
    head = _u32(out[: 1 << 20])
    tail = _u32(out[total - (1 << 20):])
    one = oracle.seed(o, 2, 1)[:, 0].copy()
    ref_pos, ref_head, ref_tail = oracle.serial_sample(o, one, total, pos.astype(np.uint64), 1 << 20, 1 << 20)
    assert np.array_equal(got_pos, ref_pos)
    assert np.array_equal(head, ref_head)
    assert np.array_equal(tail, ref_tail)
    assert np.array_equal(_u32(fin), one)


def test_fused_pi_2p34_kiss(rng, torch, oracle):
    g = rng.RNG_KISS
    S, N = 1 << 20, 1 << 14
    st = torch.empty((6, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 6, 0, S, st)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    rng.rng_fused_pi(g, st, S, N, cnt)
    ref_st = oracle.seed(oracle.KISS, 6, S)
    ref = oracle.fused_pi(oracle.KISS, ref_st, N, threads=THREADS)
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert c == ref
    assert np.array_equal(_u32(st), ref_st)
    pairs = S * N // 2
    p = np.pi / 4
    assert abs(4 * c / pairs - np.pi) < 6 * 4 * np.sqrt(p * (1 - p) / pairs)


def test_autotune_keeps_values(rng, torch, oracle):
    g, S, N = rng.RNG_XS32, 1 << 16, 256
    st = torch.empty((1, S), dtype=torch.int32, device="cuda")
    out = torch.empty(S * N, dtype=torch.int32, device="cuda")
    old = rng.rng_get_shape(g, rng.RNG_U32)
    wg, un, us = rng.rng_autotune(g, rng.RNG_U32, S, N, st, out, 2)
    assert wg in (64, 128, 256, 512, 1024) and un in (1, 2, 4, 8, 16) and us > 0
    assert rng.rng_get_shape(g, rng.RNG_U32) == (wg, un)
    rng.rng_seed(g, 5, 0, S, st)
    rng.rng_generate(g, st, S, N, rng.RNG_U32, out)
    ref = oracle.generate(oracle.XS32, oracle.seed(oracle.XS32, 5, S), N)
    assert np.array_equal(_u32(out).reshape(S, N), ref)
    rng.rng_set_shape(g, rng.RNG_U32, *old)


def test_autotune_runs_class(rng, torch, oracle):
    """Tuning on rows of 4 KiB (written as runs) keeps its pick for that class
    only; rng_generate then uses it, bit-exact."""
    g, S, N, t = rng.RNG_XS256, 1 << 14, 1024, rng.RNG_U32
    st = torch.empty((8, S), dtype=torch.int32, device="cuda")
    out = torch.empty(S * N, dtype=torch.int32, device="cuda")
    main, runs0 = rng.rng_get_shape(g, t), rng.rng_row_shape(g, t, S, N)
    rng.rng_seed(g, 3, 0, S, st)
    wg, un, us = rng.rng_autotune(g, t, S, N, st, out, 2)
    assert us > 0 and rng.rng_row_shape(g, t, S, N) == (wg, un)
    assert rng.rng_get_shape(g, t) == main
    rng.rng_seed(g, 5, 0, S, st)
    rng.rng_generate(g, st, S, N, t, out)
    ref_st = oracle.seed(oracle.XS256, 5, S)
    ref = oracle.generate(oracle.XS256, ref_st, N, threads=THREADS)
    assert np.array_equal(_u32(out).reshape(S, N), ref)
    assert np.array_equal(_u32(st), ref_st)
    rng.rng_set_row_shape(g, t, S, N, *runs0)


def _check_requests(oracle, tab, names, where, offs, idx, host_out, base_word, host_pools, seed):
    """Every sample and the final state of requests idx against the oracle:
    the output from one serial pass from the stream's seeded state, the final
    state from the oracle's jump-ahead by the request's length."""
    bad = []
    for i in idx:
        g = names[tab["gen"][i]]
        o = oracle.GENERATORS[g]
        n = int(tab["length"][i])
        st0 = oracle.seed(o, seed, 1, first_stream=where[i][2])
        st = st0.copy()
        ref = oracle.generate(o, st, n, int(tab["dtype"][i]))[0].view(np.uint32)
        a = int(offs[i]) - base_word
        if not np.array_equal(host_out[a:a + n], ref):
            k = int(np.argmax(host_out[a:a + n] != ref))
            bad.append("request %d (%s, length %d): sample %d differs" % (i, g, n, k))
            continue
        fin = oracle.skip(o, st0, n)
        if not (np.array_equal(fin, st) and np.array_equal(host_pools[g][:, where[i][2]], fin[:, 0])):
            bad.append("request %d (%s): final state differs" % (i, g))
    return bad


def test_batched_10k_requests(rng, torch, oracle):
    """The batched workload (10^4 requests, MWC32/XS256/KISS, u32/f32 50/50,
    length log-uniform in [2^8, 2^22], 4.3e9 samples) after autotuning the
    shape as bench.py does: every sample of every request, streamed to the host
    in slices of about 2^28 samples, and every request's final state."""
    import concurrent.futures
    import sys

    import bench
    from paper_1101_1846_amd import workloads as W
    tab = W.batch_table(10000, seed=4)
    names = tab["generators"]
    offs, words = W.layout_outputs(tab["length"])
    out = torch.empty(words, dtype=torch.int32, device="cuda")
    total = int(tab["length"].sum())
    h = rng.rng_batch_create(10000, total)
    try:
        pools, where = bench.batch_pools(torch, rng, "cuda", tab)
        reqs = [(rng.GENERATORS[names[g]], int(d), p, s, 0, int(n), out.data_ptr() + 4 * int(o))
                for g, d, (p, s, _), n, o in zip(tab["gen"], tab["dtype"], where, tab["length"], offs)]
        rng.rng_batch_set(h, reqs)
        rng.rng_batch_autotune(h, reps=1)
        pools, where = bench.batch_pools(torch, rng, "cuda", tab)  # fresh states
        reqs = [(rng.GENERATORS[names[g]], int(d), p, s, 0, int(n), out.data_ptr() + 4 * int(o))
                for g, d, (p, s, _), n, o in zip(tab["gen"], tab["dtype"], where, tab["length"], offs)]
        rng.rng_batch_set(h, reqs)
        rng.rng_batch_launch(h)
        torch.cuda.synchronize()
    finally:
        rng.rng_batch_destroy(h)
    host_pools = {g: _u32(p) for g, p in pools.items()}
    for g in names:  # the oracle's lazy tables are built before the threads start
        oracle.seed(oracle.GENERATORS[g], 5, 1)
    bad, i0, n_req = [], 0, len(reqs)
    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        while i0 < n_req:
            i1, acc = i0, 0
            while i1 < n_req and (acc < (1 << 28) or i1 == i0):
                acc += int(tab["length"][i1])
                i1 += 1
            w0 = int(offs[i0])
            w1 = int(offs[i1 - 1]) + int(tab["length"][i1 - 1])
            host = _u32(out[w0:w1])
            parts = np.array_split(np.arange(i0, i1), THREADS)
            for r in ex.map(lambda idx: _check_requests(oracle, tab, names, where, offs, idx, host, w0,
                                                        host_pools, 5), parts):
                bad.extend(r)
            print("batched parity: requests %d..%d checked" % (i0, i1 - 1), file=sys.stderr, flush=True)
            assert not bad, bad[:5]
            i0 = i1
    assert i0 == 10000
