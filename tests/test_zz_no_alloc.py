"""The allocation-free sequence split (rng_generate_split_noalloc) against
rng_generate_split with a caller workspace, through the C ABI: identical
output and final state, bit for bit, on consecutive calls that share the
library's scratch array (the second call smaller than the first, so stale
thread states from the first call are present), plus serial-oracle checks of
the head, the tail and sampled positions, and the size limit."""
import ctypes

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


def _u32(torch, t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def _both(rng, torch, name, seed, total, n_threads, dt):
    """Run the workspace form and the allocation-free form on the same start
    state; return (out_ws, fin_ws, out_na, fin_na, start) as host arrays."""
    g = rng.GENERATORS[name]
    W = rng.rng_state_words(g)
    s1 = torch.empty(W, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, seed, 0, 1, s1)
    out_ws = torch.full((total + 64,), -1, dtype=torch.int32, device="cuda")
    out_na = torch.full((total + 64,), -2, dtype=torch.int32, device="cuda")
    fin_ws = torch.empty(W, dtype=torch.int32, device="cuda")
    fin_na = torch.empty(W, dtype=torch.int32, device="cuda")
    wsb = rng.rng_split_workspace_bytes(g, n_threads)
    ws = torch.empty(max(wsb, 256) // 4 + 64, dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, s1, total, n_threads, dt, out_ws, fin_ws, ws, wsb)
    rng.rng_generate_split_noalloc(g, s1, total, n_threads, dt, out_na, fin_na)
    return (_u32(torch, out_ws), _u32(torch, fin_ws), _u32(torch, out_na), _u32(torch, fin_na),
            _u32(torch, s1))


def _check_oracle(oracle, name, start, total, out, fin, dt):
    o = oracle.GENERATORS[name]
    rs = np.random.default_rng(total)
    pos = np.sort(rs.integers(0, total, 2000)).astype(np.uint64)
    n_edge = min(4096, total)
    one = start.copy()
    vals, head, tail = oracle.serial_sample(o, one, total, pos, n_edge, n_edge)
    if dt:
        vals, head, tail = (oracle.to_f32(v).view(np.uint32) for v in (vals, head, tail))
    assert np.array_equal(out[:n_edge], head)
    assert np.array_equal(out[total - n_edge:total], tail)
    assert np.array_equal(out[pos.astype(np.int64)], vals)
    assert np.array_equal(fin, one)


@pytest.mark.parametrize("name", ["XS256", "MWC32", "KISS", "XS32", "MWC1616"])
def test_noalloc_split_equals_workspace_split(rng, torch, oracle, name):
    """Two calls in a row on the shared scratch: a large split (2^20 threads,
    ragged last thread), then a smaller one; each equals the workspace form."""
    for seed, total, n_threads, dt in ((2, (1 << 20) * 64 + 777, 1 << 20, 0), (3, 100003, 3000, 1)):
        out_ws, fin_ws, out_na, fin_na, start = _both(rng, torch, name, seed, total, n_threads, dt)
        assert np.array_equal(out_na[:total], out_ws[:total]), (name, total)
        assert np.array_equal(fin_na, fin_ws), (name, total)
        assert (out_na[total:] == np.uint32(0xFFFFFFFE)).all()  # nothing written past the end
        _check_oracle(oracle, name, start, total, out_na, fin_na, dt)


def test_noalloc_split_full_size_and_limit(rng, torch, oracle):
    """The split workload's shape (2^30 samples over 2^20 threads, XS256: the
    whole 32 MiB of scratch), then a split that needs more than the scratch
    holds, which is refused with RNG_ERANGE and changes nothing."""
    name, total, T = "XS256", 1 << 30, 1 << 20
    out_ws, fin_ws, out_na, fin_na, start = _both(rng, torch, name, 2, total, T, 0)
    assert np.array_equal(out_na[:total], out_ws[:total])
    assert np.array_equal(fin_na, fin_ws)
    _check_oracle(oracle, name, start, total, out_na, fin_na, 0)
    del out_ws, out_na
    g = rng.RNG_XS256
    s1 = torch.empty(8, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 4, 0, 1, s1)
    fin = torch.zeros(8, dtype=torch.int32, device="cuda")
    out = torch.empty(1 << 22, dtype=torch.int32, device="cuda")
    L = rng.raw()
    rc = L.rng_generate_split_noalloc(g, s1.data_ptr(), 1 << 22, 1 << 21, 0, out.data_ptr(), fin.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
    assert rc == rng.RNG_ERANGE
    assert b"allocation-free" in L.rng_last_error()
    torch.cuda.synchronize()
    assert int(fin.abs().sum()) == 0


def test_noalloc_split_zero_total_copies_state(rng, torch):
    g = rng.RNG_KISS
    s1 = torch.empty(6, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 9, 0, 1, s1)
    fin = torch.zeros(6, dtype=torch.int32, device="cuda")
    rng.rng_generate_split_noalloc(g, s1, 0, 16, 0, None, fin)
    torch.cuda.synchronize()
    assert torch.equal(fin, s1)
