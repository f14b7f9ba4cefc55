"""The store-schedule calibration kernel (rng_calibrate_store): the generation
kernel's schedule with a counter in place of a generator must write
d_state[s] + k + 1 at [s][k] and advance every state by n, on the resident
path (whole 64-stream groups), the ragged path and unaligned rows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("S,N,shape", [(1 << 16, 256, (256, 4)), (1 << 20, 256, (128, 2)), (1000, 100, (256, 8)),
                                       (4096, 1024, (64, 16)), (65600, 132, (512, 1)), (77, 1030, (1024, 4))])
def test_calibrate_store_pattern(rng, torch, S, N, shape):
    st0 = np.random.default_rng(S * 7 + N).integers(0, 1 << 32, S, dtype=np.uint64).astype(np.uint32)
    st = torch.from_numpy(st0.view(np.int32).copy()).cuda()
    out = torch.empty(S * N, dtype=torch.int32, device="cuda")
    rng.rng_calibrate_store(st, S, N, out, *shape)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(S, N)
    ref = (st0[:, None].astype(np.uint64) + np.arange(1, N + 1, dtype=np.uint64)[None, :]) & 0xFFFFFFFF
    assert np.array_equal(got, ref.astype(np.uint32))
    fin = st.cpu().numpy().view(np.uint32)
    assert np.array_equal(fin, ((st0.astype(np.uint64) + N) & 0xFFFFFFFF).astype(np.uint32))


def test_calibrate_valu_rates(rng):
    """Every calibration returns a positive rate below a loose physical bound
    (4 x the 16-lane int32 issue rate of 256 CUs x 4 SIMDs at 2.4 GHz); the
    fused mix (op 3) in lane-samples per second at 15-25 VALU instructions per
    sample stays below that bound divided by 15."""
    bound = 4 * 256 * 4 * 16 * 2.4e9
    for op in (0, 1, 2):
        r = rng.rng_calibrate_valu(op)
        assert 0 < r < bound, (op, r)
    mix = rng.rng_calibrate_valu(3)
    assert 0 < mix < bound / 15
