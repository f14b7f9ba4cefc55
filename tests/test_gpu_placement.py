"""The XorShift placement comparison (Table II): state in LDS behind a runtime
circular index, in LDS unrolled, and in VGPRs.  Every placement must give the
oracle's numbers (sample-major with write-back; per-stream XOR without) and
leave the oracle's final states, for ragged stream counts (partial 256-lane
workgroups) and lengths that are not multiples of the 8-fold unroll."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [(1000, 77), (256, 8), (1, 1), (300, 0), (70000, 24), (64, 1003)]


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


@pytest.mark.parametrize("place", ["lds_indexed", "lds_unrolled", "vgpr"])
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", CASES)
def test_placement_writeback(rng, torch, oracle, place, dt, S, N):
    g, t = rng.RNG_XS256, rng.DTYPES[dt]
    st = torch.empty((8, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 31, 0, S, st)
    out = torch.empty(max(1, N * S), dtype=torch.int32, device="cuda")
    rng.rng_xs256_placement(rng.PLACEMENTS[place], st, S, N, t, d_out=out)
    ref_st = oracle.seed(oracle.XS256, 31, S)
    ref = oracle.generate(oracle.XS256, ref_st, N, t, threads=4).view(np.uint32)
    assert np.array_equal(_u32(out)[:N * S].reshape(N, S), ref.T)
    assert np.array_equal(_u32(st), ref_st)


@pytest.mark.parametrize("place", ["lds_indexed", "lds_unrolled", "vgpr"])
@pytest.mark.parametrize("dt", ["u32", "f32"])
@pytest.mark.parametrize("S,N", CASES)
def test_placement_fold(rng, torch, oracle, place, dt, S, N):
    g, t = rng.RNG_XS256, rng.DTYPES[dt]
    st = torch.empty((8, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 32, 0, S, st)
    fold = torch.empty(S, dtype=torch.int32, device="cuda")
    rng.rng_xs256_placement(rng.PLACEMENTS[place], st, S, N, t, d_fold=fold)
    ref_st = oracle.seed(oracle.XS256, 32, S)
    ref = oracle.generate(oracle.XS256, ref_st, N, t, threads=4).view(np.uint32)
    exp = np.bitwise_xor.reduce(ref, axis=1) if N else np.zeros(S, np.uint32)
    assert np.array_equal(_u32(fold), exp)
    assert np.array_equal(_u32(st), ref_st)


def test_placement_bench_size(rng, torch, oracle):
    """2^20 streams x 256 (the bench size), every placement, u32 write-back:
    2000 sampled streams against the oracle, and all three placements equal."""
    g, S, N = rng.RNG_XS256, 1 << 20, 256
    outs = []
    for place in ("lds_indexed", "lds_unrolled", "vgpr"):
        st = torch.empty((8, S), dtype=torch.int32, device="cuda")
        rng.rng_seed(g, 33, 0, S, st)
        out = torch.empty(N * S, dtype=torch.int32, device="cuda")
        rng.rng_xs256_placement(rng.PLACEMENTS[place], st, S, N, rng.RNG_U32, d_out=out)
        outs.append(out.view(N, S))
    assert torch.equal(outs[0], outs[2]) and torch.equal(outs[1], outs[2])
    pick = np.sort(np.random.default_rng(5).choice(S, 2000, replace=False))
    start = np.concatenate([oracle.seed(oracle.XS256, 33, 1, first_stream=int(s)) for s in pick], axis=1)
    ref = oracle.generate(oracle.XS256, np.ascontiguousarray(start), N, threads=4)  # [2000][N]
    got = _u32(outs[2][:, torch.from_numpy(pick).to(outs[2].device)].t().contiguous())
    assert got.shape == ref.shape
    bad = np.argwhere(got != ref)
    assert bad.size == 0, "stream %d sample %d" % (pick[bad[0][0]], bad[0][1])
