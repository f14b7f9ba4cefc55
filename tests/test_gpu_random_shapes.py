"""Seeded random sweep of the entry points over their size space: generator,
dtype, stream count and row length log-uniform (odd sizes included), launch
shape, misaligned output rows; a second call continues from the written-back
states; random batches with random shapes and chunk lengths.  Every case is
compared with the oracle element by element."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GENS = ["MWC32", "XS256", "XS32", "KISS", "MWC1616"]
SHAPES = [(wg, u) for wg in (64, 128, 256, 512, 1024) for u in (1, 2, 4, 8, 16)]


def _logu(r, hi):
    return max(1, int(np.exp(r.uniform(0.0, np.log(hi)))))


def _gen_cases(n, seed):
    r = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        name, dt = GENS[r.integers(len(GENS))], ("u32", "f32")[r.integers(2)]
        while True:
            S, N = _logu(r, 1 << 17), _logu(r, 1 << 13)
            if S * N <= 1 << 23:
                break
        shape = SHAPES[r.integers(len(SHAPES))] if r.integers(3) else None
        off = int(r.integers(1, 4)) if r.integers(4) == 0 else 0
        cases.append((i, name, dt, S, N, _logu(r, 300), shape, off))
    return cases


GEN_CASES = _gen_cases(160, 20261202)


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


def _host(torch, t):
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a


def _dev_state(torch, rng, g, seed, S):
    st = torch.empty((rng.rng_state_words(g), S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, seed, 0, S, st)
    return st


@pytest.mark.parametrize("case", GEN_CASES, ids=lambda c: "%d-%s-%s-%dx%d" % c[:5])
def test_random_generate(rng, torch, oracle, case):
    i, name, dt, S, N, N2, shape, off = case
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 1000 + i, S)
    ref_st = oracle.seed(o, 1000 + i, S)
    for n in (N, N2):
        buf = torch.empty(S * n + off + 4, dtype=torch.int32, device="cuda")
        view = buf[off:off + S * n]
        if shape is None:
            rng.rng_generate(g, st, S, n, t, view)
        else:
            rng.rng_generate_ex(g, st, S, n, t, view, *shape)
        got = _host(torch, view).reshape(S, n)
        ref = oracle.generate(o, ref_st, n, t, threads=16).view(np.uint32)
        assert np.array_equal(got, ref), (S, n)
        del buf
    assert np.array_equal(_host(torch, st), ref_st)


def _skip_cases(n, seed):
    r = np.random.default_rng(seed)
    return [(i, GENS[r.integers(len(GENS))], _logu(r, 1 << 18), int(r.integers(1, 1 << 48)))
            for i in range(n)]


@pytest.mark.parametrize("case", _skip_cases(48, 7), ids=lambda c: "%d-%s-%d" % c[:3])
def test_random_skip(rng, torch, oracle, case):
    i, name, S, k = case
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    st = _dev_state(torch, rng, g, 2000 + i, S)
    rng.rng_skip(g, st, S, k)
    ref = oracle.skip(o, oracle.seed(o, 2000 + i, S), k)
    assert np.array_equal(_host(torch, st), ref)


def _split_cases(n, seed):
    r = np.random.default_rng(seed)
    out = []
    for i in range(n):
        total = _logu(r, 1 << 22)
        out.append((i, GENS[r.integers(len(GENS))], ("u32", "f32")[r.integers(2)], total,
                    _logu(r, min(total, 1 << 16))))
    return out


@pytest.mark.parametrize("case", _split_cases(48, 11), ids=lambda c: "%d-%s-%s-%d-%d" % c)
def test_random_split(rng, torch, oracle, case):
    i, name, dt, total, threads = case
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st1 = _dev_state(torch, rng, g, 3000 + i, 1)
    wsb = rng.rng_split_workspace_bytes(g, threads)
    ws = torch.empty(wsb // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    fin = torch.empty(rng.rng_state_words(g), dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, st1, total, threads, t, out, fin, ws, wsb)
    ref_st = oracle.seed(o, 3000 + i, 1)
    ref = oracle.generate(o, ref_st, total, t)[0].view(np.uint32)
    assert np.array_equal(_host(torch, out), ref)
    assert np.array_equal(_host(torch, fin), ref_st[:, 0])


def _consumer_cases(n, seed):
    r = np.random.default_rng(seed)
    out = []
    for i in range(n):
        while True:
            S, N = _logu(r, 1 << 15), _logu(r, 1 << 14)
            if S * N <= 1 << 23:
                break
        out.append((i, GENS[r.integers(len(GENS))], ("u32", "f32")[r.integers(2)], S, N))
    return out


@pytest.mark.parametrize("case", _consumer_cases(48, 13), ids=lambda c: "%d-%s-%s-%dx%d" % c)
def test_random_fused_and_fold(rng, torch, oracle, case):
    i, name, dt, S, N = case
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 4000 + i, S)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    rng.rng_fused_pi(g, st, S, N, cnt)
    ref_st = oracle.seed(o, 4000 + i, S)
    assert int(_host(torch, cnt)[0]) == oracle.fused_pi(o, ref_st, N, threads=16)
    assert np.array_equal(_host(torch, st), ref_st)
    fold = torch.zeros(S, dtype=torch.int32, device="cuda")
    rng.rng_generate_fold(g, st, S, N, t, fold)
    ref = oracle.generate(o, ref_st, N, t, threads=16).view(np.uint32)
    assert np.array_equal(_host(torch, fold), np.bitwise_xor.reduce(ref, axis=1))
    assert np.array_equal(_host(torch, st), ref_st)


def _batch_cases(n, seed):
    r = np.random.default_rng(seed)
    chunks = (0xFFFFFFFF, 64, 128, 192, 256, 1024, 4096)  # RNG_BATCH_CHUNK_AUTO first
    shapes = SHAPES  # every (workgroup, unroll) pair the batch kernel is built for
    return [(i, int(r.integers(1, 300)), _logu(r, 1 << 16), shapes[r.integers(len(shapes))],
             chunks[r.integers(len(chunks))]) for i in range(n)]


@pytest.mark.parametrize("case", _batch_cases(16, 17),
                         ids=lambda c: "%d-n%d-len%d-%dx%d-c%d" % (c[:3] + c[3] + c[4:]))
def test_random_batch(rng, torch, oracle, case):
    from test_gpu_batch import Mix
    i, n, max_len, shape, chunk = case
    m = Mix(rng, torch, oracle, n, 5000 + i, max_len)
    h = rng.rng_batch_create(n, max(1, n * max_len))
    try:
        rng.rng_batch_set_shape(h, shape[0], shape[1], chunk)
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)
