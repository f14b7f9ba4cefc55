"""The public device header (include/rng_inline.hpp) drawn from inside a user
kernel: tests/inline/onthefly.hip, built on include/ alone, loads each stream,
draws n numbers on the fly and stores the state back.  Per stream the XOR of
the n outputs, the count of FP32 uniforms below one half and the final state
must equal the oracle's, and the library must continue exactly after them
(and the kernel after the library)."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GENS = ["MWC32", "XS256", "XS32", "KISS", "MWC1616"]
LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "inline", "libonthefly.so")


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


@pytest.fixture(scope="module")
def draw():
    assert os.path.exists(LIB), "tests/inline/libonthefly.so is not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    V, U64 = ctypes.c_void_p, ctypes.c_uint64
    lib.onthefly_draw.argtypes = [ctypes.c_int, V, U64, U64, V, V, V]
    lib.onthefly_draw.restype = ctypes.c_int
    return lib.onthefly_draw


def _u32(t):
    import torch as T
    T.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def _expect(samples):
    """XOR of each row and the count of outputs whose FP32 uniform (u >> 8) * 2^-24
    is below one half, i.e. of outputs below 2^31."""
    x = np.bitwise_xor.reduce(samples, axis=1) if samples.shape[1] else np.zeros(samples.shape[0], np.uint32)
    return x.astype(np.uint32), (samples < (1 << 31)).sum(axis=1).astype(np.uint32)


@pytest.mark.parametrize("name", GENS)
@pytest.mark.parametrize("S,n", [(1000, 777), (1, 1), (257, 0), (64, 4096)])
def test_inline_draws_match_oracle_and_library_continues(rng, torch, draw, oracle, name, S, n):
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    st = torch.empty((rng.rng_state_words(g), S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 21, 0, S, st)
    x = torch.empty(S, dtype=torch.int32, device="cuda")
    h = torch.empty(S, dtype=torch.int32, device="cuda")
    assert draw(g, st.data_ptr(), S, n, x.data_ptr(), h.data_ptr(), None) == 0
    ref_st = oracle.seed(o, 21, S)
    ref = oracle.generate(o, ref_st, n, threads=4)
    ex, eh = _expect(ref)
    assert np.array_equal(_u32(x), ex)
    assert np.array_equal(_u32(h), eh)
    assert np.array_equal(_u32(st), ref_st)
    # the library continues where the kernel stopped
    out = torch.empty(S * 100, dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, 100, rng.RNG_U32, out)
    assert np.array_equal(_u32(out).reshape(S, 100), oracle.generate(o, ref_st, 100, threads=4))
    assert np.array_equal(_u32(st), ref_st)


@pytest.mark.parametrize("name", GENS)
def test_inline_continues_library(rng, torch, draw, oracle, name):
    """Library first (a jumped, chunked launch: 3 streams x 5000), then 333 draws inline."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    S = 3
    st = torch.empty((rng.rng_state_words(g), S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 22, 0, S, st)
    out = torch.empty(S * 5000, dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, 5000, rng.RNG_F32, out)
    x = torch.empty(S, dtype=torch.int32, device="cuda")
    h = torch.empty(S, dtype=torch.int32, device="cuda")
    assert draw(g, st.data_ptr(), S, 333, x.data_ptr(), h.data_ptr(), None) == 0
    ref_st = oracle.seed(o, 22, S)
    oracle.generate(o, ref_st, 5000)
    ex, eh = _expect(oracle.generate(o, ref_st, 333))
    assert np.array_equal(_u32(x), ex)
    assert np.array_equal(_u32(h), eh)
    assert np.array_equal(_u32(st), ref_st)


def test_inline_unknown_generator(draw):
    assert draw(9, None, 0, 0, None, None, None) == -2
