"""Bit-exact parity of the HIP path (through the C ABI) with the serial CPU oracle.

Sizes span several 64-lane waves and 32-sample LDS tiles with ragged tails, the
chunked path (few streams, long rows), unaligned outputs, and every launch
shape.  Full-size configurations live in test_gpu_configs.py.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GENS = ["MWC32", "XS256", "XS32", "KISS", "MWC1616"]


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


def _dev_state(torch, rng, g, seed, S, first=0):
    W = rng.rng_state_words(g)
    st = torch.empty((W, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, seed, first, S, st)
    return st


def _host(t):
    import torch as T
    T.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a


def _gen(torch, rng, g, st, S, N, dt, offset_words=0, shape=None):
    out = torch.empty(S * N + offset_words + 4, dtype=torch.int32, device="cuda")
    view = out[offset_words:offset_words + S * N]
    if shape is None:
        rng.rng_generate(g, st, S, N, dt, view)
    else:
        rng.rng_generate_ex(g, st, S, N, dt, view, shape[0], shape[1])
    res = _host(view).reshape(S, N)
    return res.view(np.float32) if dt == rng.RNG_F32 else res


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("S,first", [(1, 0), (63, 0), (64, 5), (1000, 0), (4097, 123456)])
def test_seed_parity(rng, torch, oracle, name, S, first):
    g = rng.GENERATORS[name]
    st = _dev_state(torch, rng, g, 77, S, first)
    ref = oracle.seed(oracle.GENERATORS[name], 77, S, first_stream=first)
    assert np.array_equal(_host(st), ref)


CASES = [(1, 1), (1, 37), (63, 33), (64, 32), (65, 64), (100, 257), (4097, 40), (3, 5000), (1, 70000),
         (200, 1000)]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", CASES)
def test_generate_parity(rng, torch, oracle, name, dt, S, N):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 1, S)
    out = _gen(torch, rng, g, st, S, N, t)
    ref_st = oracle.seed(o, 1, S)
    ref = oracle.generate(o, ref_st, N, t, threads=4)
    assert out.dtype == ref.dtype
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("name", GENS)
def test_unaligned_output_and_odd_rows(rng, torch, oracle, name):
    """4-byte aligned but not 16-byte aligned output, and N not a multiple of 4:
    the dword store path."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    for S, N, off in ((130, 64, 1), (130, 66, 0), (70, 35, 3)):
        st = _dev_state(torch, rng, g, 9, S)
        out = _gen(torch, rng, g, st, S, N, rng.RNG_U32, offset_words=off)
        ref = oracle.generate(o, oracle.seed(o, 9, S), N)
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("name", GENS)
def test_every_launch_shape_same_values(rng, torch, oracle, name):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S, N = 300, 96
    ref = oracle.generate(o, oracle.seed(o, 4, S), N, oracle.F32)
    for wg in (64, 128, 256, 512, 1024):
        for un in (1, 2, 4, 8, 16):
            st = _dev_state(torch, rng, g, 4, S)
            out = _gen(torch, rng, g, st, S, N, rng.RNG_F32, shape=(wg, un))
            assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (wg, un)


@pytest.mark.parametrize("name", GENS)
def test_resume_equals_one_call(rng, torch, oracle, name):
    """State write-back: generate(N1) then generate(N2) == generate(N1 + N2)."""
    g = rng.GENERATORS[name]
    S = 513
    a = _dev_state(torch, rng, g, 8, S)
    b = _dev_state(torch, rng, g, 8, S)
    one = _gen(torch, rng, g, a, S, 300, rng.RNG_U32)
    p1 = _gen(torch, rng, g, b, S, 123, rng.RNG_U32)
    p2 = _gen(torch, rng, g, b, S, 177, rng.RNG_U32)
    assert np.array_equal(one, np.concatenate([p1, p2], axis=1))
    assert np.array_equal(_host(a), _host(b))


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("shape", [(64, 4), (256, 4), (1024, 4)])
def test_chunked_resume_equals_one_call(rng, torch, oracle, name, shape):
    """Few streams with long rows are cut into chunks that each start from the
    stream's state by jump-ahead; the states must come back advanced by exactly
    N, written only after every chunk has read them.  With 1024-lane
    workgroups each workgroup holds all chunks of its streams (2-16 of them)
    and the kernel writes the states back after a barrier; with 64 lanes a
    separate skip launch advances them.  Three calls in a row, then the oracle."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S, N = 64, 32768 if name == "XS256" else 2048
    a = _dev_state(torch, rng, g, 12, S)
    parts = [_gen(torch, rng, g, a, S, N, rng.RNG_U32, shape=shape) for _ in range(3)]
    ref_st = oracle.seed(o, 12, S)
    ref = oracle.generate(o, ref_st, 3 * N, threads=4)
    assert np.array_equal(np.concatenate(parts, axis=1), ref)
    assert np.array_equal(_host(a), ref_st)


FEW = [(1, (1 << 20) + 13), (2, 70001), (5, 1 << 16), (63, 12345)]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", FEW)
def test_few_streams_one_lane_per_chunk(rng, torch, oracle, name, dt, S, N):
    """Fewer streams than a wave has lanes: every lane takes one chunk of one
    stream (ragged last chunks), the output is 4-byte but not 16-byte aligned
    on the second call, and the states come back advanced by N each time."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 17, S)
    ref_st = oracle.seed(o, 17, S)
    for off in (0, 1, 0):
        out = _gen(torch, rng, g, st, S, N, t, offset_words=off)
        ref = oracle.generate(o, ref_st, N, t, threads=4)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), off
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("name", GENS)
def test_run_twice_identical(rng, torch, name):
    g = rng.GENERATORS[name]
    S, N = 4096, 512
    outs = []
    for _ in range(2):
        st = _dev_state(torch, rng, g, 3, S)
        outs.append(_gen(torch, rng, g, st, S, N, rng.RNG_U32))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("k", [1, 2, 1000, 65536 + 17, (1 << 40) + 7, (1 << 64) - 1])
def test_skip_parity(rng, torch, oracle, name, k):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S = 257 if name != "XS256" or k < (1 << 20) else 70
    st = _dev_state(torch, rng, g, 12, S)
    rng.rng_skip(g, st, S, k)
    ref = oracle.skip(o, oracle.seed(o, 12, S), k)
    assert np.array_equal(_host(st), ref)


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("k", [3, 1 << 40, (1 << 64) - 1 - 12345])
def test_skip_many_states(rng, torch, oracle, name, k):
    """More states than one pass of the grid covers, so each workgroup strides
    over several after building its k-step tables once.  Sampled states
    (the first, the last, both sides of every stride boundary, and random
    ones) against the oracle."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S = (1 << 20) + 4099
    st = _dev_state(torch, rng, g, 21, S)
    rng.rng_skip(g, st, S, k)
    got = _host(st)
    edges = [0, 1, 255, 256, S - 1]
    for b in (65536, 131072, 1 << 20):
        edges += [b - 1, b, b + 1]
    idx = sorted(set(edges) | set(int(i) for i in np.random.default_rng(5).integers(0, S, 100)))
    ref = np.concatenate([oracle.seed(o, 21, 1, first_stream=i) for i in idx], axis=1)
    ref = oracle.skip(o, ref, k)
    assert np.array_equal(got[:, idx], ref)


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("total,threads", [(1, 1), (1000, 1), (1000, 7), (4096 * 7 + 3, 64), (100000, 1000),
                                          (65536, 65536), (5, 8), (1024 * 192 + 900, 193),
                                          (1024 * 384, 384), (2048 * 64, 64), (1024, 1),
                                          (1024 * 512 + 600, 513), (2048 * 128 + 2000, 129),
                                          ((1 << 22) + 5, (1 << 21) + 3)])
def test_split_parity(rng, torch, oracle, name, total, threads):
    """Sequence splitting (Sec. II.A.4): the concatenated thread outputs equal the
    serial sequence of the one logical stream, and the final state matches.
    1024 * 192 + 900 over 193 threads: 192 full rows of 1024 (whole 4 KiB
    rows: the rotated tile order, or for XS256 four jumped chunks per row; 128
    rows in a first launch, 64 in a second) and a 900-sample tail; 1024 * 384
    over 384 and 2048 * 64 over 64: whole 4 KiB rows only.  1024 * 512 + 600
    over 513 and 2048 * 128 + 2000 over 129: 512 (128) full rows written as
    16 KiB runs from thread states at a stride of 513 (129), then the tail.
    2^22 + 5 over 2^21 + 3: two samples per thread, a sixth tree level whose
    2^20 XS256 chains stride over a capped grid."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    st1 = _dev_state(torch, rng, g, 2, 1)
    ws_bytes = rng.rng_split_workspace_bytes(g, threads)
    ws = torch.empty(ws_bytes // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    fin = torch.empty(rng.rng_state_words(g), dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, st1, total, threads, rng.RNG_U32, out, fin, ws, ws_bytes)
    ref_st = oracle.seed(o, 2, 1)
    ref = oracle.generate(o, ref_st, total)[0]
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(_host(fin), ref_st[:, 0])


# Thread counts at the edges of the start tree's levels (16^2 and 16^3: the
# one-launch head and the level kernels; 4 * 16^3 - 1: a level whose source
# threads are not all used; 2^18 + 3: a level of 2^16 source threads, on
# 1024-lane workgroups), with power-of-two and odd samples per thread (XS256
# levels then build their jump tables in each workgroup).
TREE_EDGE_T = [255, 256, 257, 4095, 4096, 4097, 16383, 65535, 65537, (1 << 18) + 3]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("T", TREE_EDGE_T)
@pytest.mark.parametrize("C", [4, 3])
def test_split_tree_edges(rng, torch, oracle, name, T, C):
    """Sequence splitting (Sec. II.A.4) with T threads of C samples each (the
    last one ragged): the concatenated output equals the serial sequence."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    total = T * C - (C - 1)
    st1 = _dev_state(torch, rng, g, 5, 1)
    ws_bytes = rng.rng_split_workspace_bytes(g, T)
    ws = torch.empty(ws_bytes // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    fin = torch.empty(rng.rng_state_words(g), dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, st1, total, T, rng.RNG_U32, out, fin, ws, ws_bytes)
    ref_st = oracle.seed(o, 5, 1)
    ref = oracle.generate(o, ref_st, total)[0]
    assert np.array_equal(_host(out), ref), (name, T, C)
    assert np.array_equal(_host(fin), ref_st[:, 0])


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("T", TREE_EDGE_T)
def test_leapfrog_tree_edges(rng, torch, oracle, name, T):
    """Leapfrogging (Sec. II.A.4) over T threads (unit jumps: the tree's
    power-of-two path), 3T + 5 numbers."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    total = 3 * T + 5
    st1 = _dev_state(torch, rng, g, 6, 1)
    ws_bytes = rng.rng_leapfrog_workspace_bytes(g, T)
    ws = torch.empty(ws_bytes // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    fin = torch.empty(rng.rng_state_words(g), dtype=torch.int32, device="cuda")
    rng.rng_generate_leapfrog(g, st1, total, T, rng.RNG_U32, out, fin, ws, ws_bytes)
    ref_st = oracle.seed(o, 6, 1)
    ref = oracle.generate(o, ref_st, total)[0]
    assert np.array_equal(_host(out), ref), (name, T)
    assert np.array_equal(_host(fin), ref_st[:, 0])


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("total,threads", [(1, 1), (1000, 1), (1000, 7), (4096 * 7 + 3, 64), (100000, 1000),
                                          (65536, 65536), (5, 8), (77777, 4096), (3 << 21, (1 << 21) + 5)])
def test_leapfrog_parity(rng, torch, oracle, name, dt, total, threads):
    """Leapfrogging (Sec. II.A.4): thread j's numbers j, j + T, ... interleave into
    the serial sequence of the one logical stream; the final state matches."""
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st1 = _dev_state(torch, rng, g, 2, 1)
    ws_bytes = rng.rng_leapfrog_workspace_bytes(g, min(threads, total))
    ws = torch.empty(ws_bytes // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    fin = torch.empty(rng.rng_state_words(g), dtype=torch.int32, device="cuda")
    rng.rng_generate_leapfrog(g, st1, total, threads, t, out, fin, ws, ws_bytes)
    ref_st = oracle.seed(o, 2, 1)
    ref = oracle.generate(o, ref_st, total, t)[0].view(np.uint32)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(_host(fin), ref_st[:, 0])
    assert np.array_equal(_host(st1).ravel(), oracle.seed(o, 2, 1)[:, 0])  # input state untouched


def test_leapfrog_arguments(rng, torch):
    g = rng.RNG_MWC32
    st1 = _dev_state(torch, rng, g, 2, 1)
    fin = torch.empty(2, dtype=torch.int32, device="cuda")
    out = torch.empty(100, dtype=torch.int32, device="cuda")
    small = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(rng.RngError) as e:
        rng.rng_generate_leapfrog(g, st1, 100, 10, rng.RNG_U32, out, fin, small, 32)
    assert e.value.code == rng.RNG_ENOMEM
    with pytest.raises(rng.RngError) as e:
        rng.rng_generate_leapfrog(g, st1, 100, 0, rng.RNG_U32, out, fin, small, 32)
    assert e.value.code == rng.RNG_EINVAL
    rng.rng_generate_leapfrog(g, st1, 0, 10, rng.RNG_U32, None, fin, None, 0)  # nothing: final = initial
    assert np.array_equal(_host(fin), _host(st1).ravel())


@pytest.mark.parametrize("name", ["KISS", "XS256", "MWC32"])
@pytest.mark.parametrize("S,N", [(1, 2), (1000, 64), (333, 65), (64, 1000), (2, 40000), (1, (1 << 20) + 3)])
def test_fused_pi_parity(rng, torch, oracle, name, S, N):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    st = _dev_state(torch, rng, g, 6, S)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    rng.rng_fused_pi(g, st, S, N, cnt)
    ref_st = oracle.seed(o, 6, S)
    ref = oracle.fused_pi(o, ref_st, N, threads=4)
    torch.cuda.synchronize()
    assert int(cnt.item()) == ref
    assert np.array_equal(_host(st), ref_st)


# Large grids of whole 64-stream groups with one chunk per stream: 4101 groups
# (more than the device holds at once), one tile per stream (N = 64), 32-deep
# tiles (N = 96 with 1024-lane workgroups), and the smallest stream count that
# still takes one chunk per stream (65600 > 2^16).
PERSIST = [(262464, 192, None), (262464, 64, None), (262464, 96, (1024, 4)), (65600, 128, (64, 16))]


# Long rows on the resident schedule: 1025 groups leave most waves fewer
# groups than the register queue holds; 5, 9 and 36 tiles per row.
LONG_ROWS = [(65600, 640, (256, 8)), (65600, 1152, None), (65600, 1152, (128, 4)), (65600, 1152, (512, 4))]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N,shape", LONG_ROWS)
def test_long_rows_parity(rng, torch, oracle, name, dt, S, N, shape):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 13, S)
    out = _gen(torch, rng, g, st, S, N, t, shape=shape)
    ref_st = oracle.seed(o, 13, S)
    ref = oracle.generate(o, ref_st, N, t, threads=16)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(_host(st), ref_st)


# Rows of whole 4 KiB multiples: MWC32 and XS32 start every row of wave w at
# tile (w mod 4) T / 4 by jump-ahead and wrap round (the other generators
# keep the plain order).
ROT_ROWS = [(65600, 1024, None), (65600, 2048, (128, 4)), (65600, 1024, (64, 16)), (65536, 3072, (256, 8))]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N,shape", ROT_ROWS)
def test_rotated_rows_parity(rng, torch, oracle, name, dt, S, N, shape):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 15, S)
    out = _gen(torch, rng, g, st, S, N, t, shape=shape)
    ref_st = oracle.seed(o, 15, S)
    ref = oracle.generate(o, ref_st, N, t, threads=16)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(_host(st), ref_st)


# Rows of 4 and 8 KiB on up to 256 lanes, stream counts a multiple of 256 or
# 128: each lane writes the rows of 4 or 2 adjacent streams as one 16 KiB run
# (other counts take the orders above).
SEG_ROWS = [(16384, 1024, (256, 8)), (16640, 1024, (128, 16)), (8192, 2048, (64, 4)), (256, 1024, (256, 1)),
            (131584, 2048, (256, 2)), (2304, 1024, (64, 16))]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N,shape", SEG_ROWS)
def test_segmented_rows_parity(rng, torch, oracle, name, dt, S, N, shape):
    """Two calls in a row: every sample and the written-back states."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 17, S)
    ref_st = oracle.seed(o, 17, S)
    for _ in range(2):
        out = _gen(torch, rng, g, st, S, N, t, shape=shape)
        ref = oracle.generate(o, ref_st, N, t, threads=16)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
        assert np.array_equal(_host(st), ref_st)
        del out, ref


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("S", [1 << 20, (1 << 20) - 64])
def test_rotated_rows_full_queue(rng, torch, oracle, name, S):
    """2^20 streams x 1024 with a full register queue per wave (runs of four
    rows), and 2^20 - 64 (the rotated order, or for XS256 the plain one),
    twice in a row: the written-back states must continue the rows."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    N = 1024
    st = _dev_state(torch, rng, g, 16, S)
    ref_st = oracle.seed(o, 16, S)
    for _ in range(2):
        out = _gen(torch, rng, g, st, S, N, rng.RNG_U32, shape=(256, 4))
        ref = oracle.generate(o, ref_st, N, threads=16)
        assert np.array_equal(out, ref)
        del out, ref
    assert np.array_equal(_host(st), ref_st)


# Rows that end in a partial tile (whole 64-stream groups, 16-byte rows): N
# mod 128 = 4, 64, 124 and 104, and every launch shape (the 32-sample tiles
# of 512- and 1024-lane workgroups included).
RAGGED_ROWS = [(1024, 132), (4096, 192), (64 * 2048, 252), (1 << 17, 1000)]


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", RAGGED_ROWS)
def test_ragged_rows(rng, torch, oracle, name, dt, S, N):
    """Two calls in a row: every sample and the written-back states."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 23, S)
    ref_st = oracle.seed(o, 23, S)
    for _ in range(2):
        out = _gen(torch, rng, g, st, S, N, t)
        ref = oracle.generate(o, ref_st, N, t, threads=16)
        assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (name, dt, S, N)
        assert np.array_equal(_host(st), ref_st)
        del out, ref


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("shape", [(64, 1), (128, 16), (256, 4), (512, 8), (1024, 2)])
def test_ragged_rows_every_shape(rng, torch, oracle, name, shape):
    """4096 streams x 1000 samples (7 whole tiles and 104 samples) at several
    launch shapes: every sample and the written-back states."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S, N = 4096, 1000
    st = _dev_state(torch, rng, g, 24, S)
    out = _gen(torch, rng, g, st, S, N, rng.RNG_U32, shape=shape)
    ref_st = oracle.seed(o, 24, S)
    ref = oracle.generate(o, ref_st, N, threads=16)
    assert np.array_equal(out, ref)
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("name", ["XS256", "KISS"])
def test_ragged_rows_2p20x1000(rng, torch, oracle, name):
    """2^20 streams x 1000 samples, rows ending in a partial tile (4 GB)."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S, N = 1 << 20, 1000
    st = _dev_state(torch, rng, g, 25, S)
    out = _gen(torch, rng, g, st, S, N, rng.RNG_U32)
    ref_st = oracle.seed(o, 25, S)
    ref = oracle.generate(o, ref_st, N, threads=16)
    assert np.array_equal(out, ref)
    assert np.array_equal(_host(st), ref_st)
    del out, ref


@pytest.mark.parametrize("name", ["MWC32", "XS256", "KISS"])
def test_long_rows_full_queue(rng, torch, oracle, name):
    """2^20 streams: every wave holds as many groups as its register queue
    does, with 12 tiles per row (1536 samples, 6 GiB)."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S, N = 1 << 20, 1536
    st = _dev_state(torch, rng, g, 14, S)
    out = _gen(torch, rng, g, st, S, N, rng.RNG_U32, shape=(256, 8))
    ref_st = oracle.seed(o, 14, S)
    ref = oracle.generate(o, ref_st, N, threads=16)
    assert np.array_equal(out, ref)
    assert np.array_equal(_host(st), ref_st)
    del out, ref


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N,shape", PERSIST)
def test_large_grid_parity(rng, torch, oracle, name, dt, S, N, shape):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    t = rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 9, S)
    out = _gen(torch, rng, g, st, S, N, t, shape=shape)
    ref_st = oracle.seed(o, 9, S)
    ref = oracle.generate(o, ref_st, N, t, threads=16)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", [(1, 1), (1000, 77), (64, 4096), (3, 100000), (70000, 16), (1, (1 << 20) + 3)])
def test_fold_parity(rng, torch, oracle, name, dt, S, N):
    """Without write-back: the per-stream XOR of the n outputs (chunked with jumps
    for few streams) and the final states equal the oracle's."""
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 61, S)
    fold = torch.zeros(S, dtype=torch.int32, device="cuda")
    rng.rng_generate_fold(g, st, S, N, t, fold)
    ref_st = oracle.seed(o, 61, S)
    ref = oracle.generate(o, ref_st, N, t, threads=4).view(np.uint32)
    assert np.array_equal(_host(fold), np.bitwise_xor.reduce(ref, axis=1))
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("N", [1024, 2048, 3072, 4096, 5120, 8192])
@pytest.mark.parametrize("dt", ["u32", "f32"])
def test_xs256_4k_rows_default_shape(rng, torch, oracle, N, dt):
    """rng_generate on XS256 rows of whole 4 KiB multiples: the odd multiples
    take 512-lane workgroups and four jumped chunks, the even ones the tuned
    shape in the plain order; every sample and the written-back states."""
    g, o, t = rng.RNG_XS256, oracle.XS256, rng.DTYPES[dt]
    S = 4160
    st = _dev_state(torch, rng, g, 53, S)
    out = _gen(torch, rng, g, st, S, N, t)
    ref_st = oracle.seed(o, 53, S)
    ref = oracle.generate(o, ref_st, N, t, threads=16)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(_host(st), ref_st)


@pytest.mark.parametrize("N", [1024, 2048, 3072, 4096])
@pytest.mark.parametrize("S", [64, 192, 4096])
@pytest.mark.parametrize("wg", [512, 1024])
@pytest.mark.parametrize("dt", ["u32", "f32"])
def test_xs256_whole_4k_rows_as_chunks(rng, torch, oracle, N, S, wg, dt):
    """XS256 rows of an odd number of 4 KiB (1024, 3072) on 512- and 1024-lane
    workgroups run as four jumped chunks per row (chunk c starts c N / 4
    samples in), rows of an even number (2048, 4096) in the plain order; two
    calls in a row: every sample and the written-back states of both."""
    g, o, t = rng.RNG_XS256, oracle.XS256, rng.DTYPES[dt]
    st = _dev_state(torch, rng, g, 31, S)
    ref_st = oracle.seed(o, 31, S)
    for _ in range(2):
        out = torch.empty((S, N), dtype=torch.int32, device="cuda")
        rng.rng_generate_ex(g, st, S, N, t, out, wg, 4)
        ref = oracle.generate(o, ref_st, N, t, threads=4).view(np.uint32)
        assert np.array_equal(_host(out), ref)
        assert np.array_equal(_host(st), ref_st)
