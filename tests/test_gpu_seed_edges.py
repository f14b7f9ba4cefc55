"""Seeding edge cases on the GPU: the fix-ups that keep every seeded state
off the generators' fixed points (Sec. II.A.1: an MWC state z = c b + x must
avoid 0 and a b - 1; Sec. II.A.2: an all-zero XorShift state stays zero).

SplitMix64 output n of a generator started at `seed` is mix(seed + (n+1) g)
with g = 0x9E3779B97F4A7C15.  mix is a bijection of 64-bit words, so for any
wanted draw value v, seed = mix^-1(v) - (n+1) g mod 2^64 makes draw n equal v.
The tests pick v so that one stream's state words hit a fix-up (a zero word,
or an MWC word equal to its modulus), check with the oracle's serial
SplitMix64 that the crafted seed really yields v, seed on the device, and
compare with the oracle's seeding and with the fixed-up state the seeding
convention prescribes; then generate from those states.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
C1, C2 = 0xBF58476D1CE4E5B9, 0x94D049BB133111EB


def _mix(z):
    z = ((z ^ (z >> 30)) * C1) & M64
    z = ((z ^ (z >> 27)) * C2) & M64
    return z ^ (z >> 31)


def _unxorshift(y, s):
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x


def _unmix(v):
    z = _unxorshift(v, 31)
    z = (z * pow(C2, -1, 1 << 64)) & M64
    z = _unxorshift(z, 27)
    z = (z * pow(C1, -1, 1 << 64)) & M64
    return _unxorshift(z, 30)


def _seed_for(draw_index, value):
    """A seed whose SplitMix64 draw number draw_index is value."""
    return (_unmix(value) - (draw_index + 1) * GAMMA) & M64


def _oracle_draw(oracle, seed, n):
    L = oracle.lib()
    s = ctypes.c_uint64(seed)
    v = None
    for _ in range(n + 1):
        v = L.orc_sm64_next(ctypes.byref(s))
    return v


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


def _seed_and_check(rng, torch, oracle, name, seed, first, S, target_stream):
    """Device seeding of S streams from `first` against the oracle; then 300
    samples from those states; returns the target stream's seeded state."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    W = rng.rng_state_words(g)
    st = torch.empty((W, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, seed, first, S, st)
    ref = oracle.seed(o, seed, S, first_stream=first)
    got = _u32(torch, st)
    assert np.array_equal(got, ref), name
    out = torch.empty((S, 300), dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, 300, rng.RNG_U32, out)
    ref_out = oracle.generate(o, ref, 300)
    assert np.array_equal(_u32(torch, out), ref_out), name
    assert np.array_equal(_u32(torch, st), ref), name
    return got[:, target_stream - first]


@pytest.mark.parametrize("first", [0, 1000])
def test_mwc32_zero_state_fixup(rng, torch, oracle, first):
    """Draw 0 gives (x, c) = (0, 0), z = 0: the state becomes x = 1, c = 0."""
    s = first + 5
    seed = _seed_for(s, 0)
    assert _oracle_draw(oracle, seed, s) == 0
    got = _seed_and_check(rng, torch, oracle, "MWC32", seed, first, 64, s)
    assert got.tolist() == [1, 0]


def test_mwc32_modulus_state_fixup(rng, torch, oracle):
    """Draw (a - 1) 2^32 + 2^32 - 1 gives x = 2^32 - 1, c = a - 1, z = a b - 1 = m:
    the state becomes z = m - 1, i.e. x = 2^32 - 2, c = a - 1."""
    a = oracle.mwc32_multiplier()
    s = 17
    v = ((a - 1) << 32) | 0xFFFFFFFF
    seed = _seed_for(s, v)
    assert _oracle_draw(oracle, seed, s) == v
    got = _seed_and_check(rng, torch, oracle, "MWC32", seed, 0, 64, s)
    assert got.tolist() == [0xFFFFFFFE, a - 1]


def test_xs32_zero_state_fixup(rng, torch, oracle):
    """Draw whose low word is 0: the xorshift32 state becomes 1."""
    s = 40
    seed = _seed_for(s, 0x1234567800000000)
    got = _seed_and_check(rng, torch, oracle, "XS32", seed, 0, 64, s)
    assert got.tolist() == [1]


@pytest.mark.parametrize("name", ["MWC1616", "KISS"])
def test_mwc16_zero_words_fixup(rng, torch, oracle, name):
    """Draw 1 of the stream is 0: both base-2^16 MWC words (z from its low,
    w from its high half) are 0 and become 1."""
    D = {"MWC1616": 2, "KISS": 3}[name]
    s = 9
    seed = _seed_for(D * s + 1, 0)
    got = _seed_and_check(rng, torch, oracle, name, seed, 0, 64, s)
    assert got[0] == 1 and got[1] == 1


def test_kiss_zero_xorshift_fixup(rng, torch, oracle):
    """Draw 2 of a KISS stream has a zero low word: jsr becomes 1 and jcong is
    the high word."""
    s = 33
    v = 0xDEADBEEF00000000
    seed = _seed_for(3 * s + 2, v)
    got = _seed_and_check(rng, torch, oracle, "KISS", seed, 0, 64, s)
    assert got[2] == 1 and got[3] == 0xDEADBEEF


def _pair(table, d):
    i = (d & 0xFFFFFFFF) % 392
    j = (i + 1 + ((d >> 32) % 391)) % 392
    return int(table[i]), int(table[j])


@pytest.mark.parametrize("name", ["MWC1616", "KISS"])
def test_mwc16_modulus_word_fixup(rng, torch, oracle, name):
    """The z word equal to its modulus a1 2^16 - 1: the low half of draw 1 must
    be (a1 - 1) 2^16 + 2^16 - 1 for the multiplier a1 that draw 0 picks, and
    draw 0 depends on the crafted seed; a search over the high half finds a
    consistent seed.  The word becomes m1 - 1."""
    D = {"MWC1616": 2, "KISS": 3}[name]
    table, _ = oracle.mwc16_table()
    s = 6
    found = None
    r = np.random.default_rng(3)
    for hi in r.integers(1, 1 << 32, 64, dtype=np.uint64).tolist():
        for a in table.tolist():
            v = (int(hi) << 32) | ((a - 1) << 16) | 0xFFFF
            seed = _seed_for(D * s + 1, v)
            a1, _ = _pair(table, _mix((seed + (D * s + 1) * GAMMA) & M64))
            if a1 == a:
                found = (seed, a, v)
                break
        if found:
            break
    assert found, "no consistent seed in the search"
    seed, a, v = found
    assert _oracle_draw(oracle, seed, D * s + 1) == v
    got = _seed_and_check(rng, torch, oracle, name, seed, 0, 64, s)
    W = rng.rng_state_words(rng.GENERATORS[name])
    assert got[W - 2] == a  # the stream's first multiplier
    assert got[0] == a * 65536 - 2
