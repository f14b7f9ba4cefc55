"""Statistical smoke battery (tests/quality.py, textbook definitions) on the
generators' output: the oracle's streams on the CPU, the HIP path's output on
the GPU (one long stream, the cross-section of many streams at one position,
leapfrogged output).  Planted defects on the CPU pin the battery itself: a
stuck bit, a Weyl sequence and correlated neighbours must each fail."""
import numpy as np
import pytest

import quality as Q

GENS = ["MWC32", "XS256", "XS32", "KISS", "MWC1616"]
ALPHA = 1e-6


@pytest.mark.parametrize("name", GENS)
def test_oracle_stream_passes(oracle, name):
    o = oracle.GENERATORS[name]
    u = oracle.generate(o, oracle.seed(o, 101, 1), 1 << 20)[0]
    p = Q.battery(u)
    assert Q.passes(p, ALPHA), p


@pytest.mark.parametrize("name", GENS)
def test_oracle_cross_section_passes(oracle, name):
    """The first output of 2^16 seeded streams: seeding gives unrelated streams."""
    o = oracle.GENERATORS[name]
    u = oracle.generate(o, oracle.seed(o, 102, 1 << 16), 2)[:, 0]
    p = Q.battery(u)
    assert Q.passes(p, ALPHA), p


def _good(n=1 << 20):
    return np.random.default_rng(7).integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)


def test_battery_accepts_a_good_source():
    assert Q.passes(Q.battery(_good()), ALPHA)


def test_battery_catches_a_stuck_bit():
    p = Q.battery(_good() & np.uint32(~(1 << 7) & 0xFFFFFFFF))
    assert p["monobit"] < ALPHA


def test_battery_catches_a_weyl_sequence():
    """u_i = i * 0x9E3779B9 mod 2^32: equidistributed, but its spacings repeat."""
    u = (np.arange(1 << 20, dtype=np.uint64) * 0x9E3779B9 % (1 << 32)).astype(np.uint32)
    p = Q.battery(u)
    assert p["birthday_spacings"] < ALPHA


def test_battery_catches_correlated_neighbours():
    u = _good()
    u[1::2] = u[0::2] ^ (np.random.default_rng(8).integers(0, 1 << 20, len(u) // 2).astype(np.uint32))
    p = Q.battery(u)
    assert p["chi2_pairs"] < ALPHA and p["serial_correlation"] < ALPHA


def test_battery_catches_repeated_streams(oracle):
    """Every stream seeded alike: the cross-section is one value repeated."""
    o = oracle.XS256
    st = np.repeat(oracle.seed(o, 103, 1), 1 << 16, axis=1)
    u = oracle.generate(o, st, 2)[:, 0]
    assert not Q.passes(Q.battery(u), ALPHA)


@pytest.mark.gpu
@pytest.mark.parametrize("name", GENS)
def test_gpu_output_passes(oracle, name):
    import torch
    import paper_1101_1846_amd as R
    R.rng_init()
    g = R.GENERATORS[name]
    W = R.rng_state_words(g)
    # one long stream (the chunked, jumped path)
    st = torch.empty((W, 1), dtype=torch.int32, device="cuda")
    R.rng_seed(g, 104, 0, 1, st)
    out = torch.empty(1 << 22, dtype=torch.int32, device="cuda")
    R.rng_generate(g, st, 1, 1 << 22, R.RNG_U32, out)
    torch.cuda.synchronize()
    p = Q.battery(out.cpu().numpy().view(np.uint32))
    assert Q.passes(p, ALPHA), ("stream", p)
    # the cross-section of 2^18 streams at positions 0 and 255
    S = 1 << 18
    st = torch.empty((W, S), dtype=torch.int32, device="cuda")
    R.rng_seed(g, 105, 0, S, st)
    out = torch.empty((S, 256), dtype=torch.int32, device="cuda")
    R.rng_generate(g, st, S, 256, R.RNG_U32, out)
    torch.cuda.synchronize()
    h = out.cpu().numpy().view(np.uint32)
    for k in (0, 255):
        p = Q.battery(h[:, k])
        assert Q.passes(p, ALPHA), ("cross-section", k, p)
    # a leapfrogged sequence over 4096 threads
    s1 = torch.empty(W, dtype=torch.int32, device="cuda")
    R.rng_seed(g, 106, 0, 1, s1)
    fin = torch.empty(W, dtype=torch.int32, device="cuda")
    wsb = R.rng_leapfrog_workspace_bytes(g, 4096)
    ws = torch.empty(wsb // 4, dtype=torch.int32, device="cuda")
    out = torch.empty(1 << 22, dtype=torch.int32, device="cuda")
    R.rng_generate_leapfrog(g, s1, 1 << 22, 4096, R.RNG_U32, out, fin, ws, wsb)
    torch.cuda.synchronize()
    p = Q.battery(out.cpu().numpy().view(np.uint32))
    assert Q.passes(p, ALPHA), ("leapfrog", p)
