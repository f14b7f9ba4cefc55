"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
itself: values come from the paper's text (tests/golden/paper_constants.txt),
from published vectors (tests/golden/splitmix64.txt), from number theory done
here with different algorithms (tests/_nt.py), or from brute force.
"""
import ctypes
import os

import numpy as np
import pytest

import _nt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_constants():
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, value, _ = line.split(None, 2)
            out[name] = int(value)
    return out


PAPER = _golden_constants()


# ---------------------------------------------------------------- multipliers
def test_mwc16_multiplier_count_matches_paper(oracle):
    """Sec. III.A.1: exactly 392 multipliers a < 2^16 make a*2^16 - 1 a safe prime."""
    table, n = oracle.mwc16_table()
    assert n == PAPER["mwc16_multiplier_count"]
    assert list(table) == sorted(table) and len(set(table.tolist())) == n


@pytest.mark.slow
def test_mwc16_table_is_exactly_the_safe_prime_set(oracle):
    """Sec. II.A.1: a*b - 1 safe prime.  Miller-Rabin over all a < 2^16."""
    table, _ = oracle.mwc16_table()
    expect = [a for a in range(1, 1 << 16)
              if _nt.is_prime(a * (1 << 15) - 1) and _nt.is_prime(a * (1 << 16) - 1)]
    assert table.tolist() == expect


def test_mwc32_multiplier_rule(oracle):
    """b = 2^32: the largest a < 2^16 with a*2^32 - 1 and (a*2^32 - 2)/2 prime."""
    a = oracle.mwc32_multiplier()
    m = a * (1 << 32) - 1
    assert a < (1 << 16)
    assert _nt.is_prime(m) and _nt.is_prime((m - 1) // 2)
    for b in range(a + 1, 1 << 16):
        mb = b * (1 << 32) - 1
        assert not (_nt.is_prime(mb) and _nt.is_prime((mb - 1) // 2))


# ---------------------------------------------------------------- MWC algebra
def test_mwc32_congruence_invariant(oracle):
    """Eq. (2)-(3): with z = c*b + x, z_{n+1} = a*z_n mod (a*b - 1) at every step."""
    L = oracle.lib()
    a = oracle.mwc32_multiplier()
    m = a * (1 << 32) - 1
    st = oracle.seed(oracle.MWC32, 0, 64)
    for s in range(64):
        x = ctypes.c_uint32(int(st[0, s]))
        c = ctypes.c_uint32(int(st[1, s]))
        z = (c.value << 32) | x.value
        assert 1 <= z <= m - 1 and c.value < a
        for _ in range(200):
            out = L.orc_step_mwc32(a, ctypes.byref(x), ctypes.byref(c))
            z_next = (c.value << 32) | x.value
            assert z_next == a * z % m
            assert out == x.value
            z = z_next


def test_mwc16_congruence_invariant(oracle):
    """Eq. (2)-(3) with b = 2^16 for several table multipliers."""
    L = oracle.lib()
    table, _ = oracle.mwc16_table()
    rng = np.random.default_rng(11)
    for a in [int(table[0]), int(table[-1])] + [int(v) for v in rng.choice(table, 6)]:
        m = a * (1 << 16) - 1
        z = ctypes.c_uint32(int(rng.integers(1, m - 1)))
        for _ in range(500):
            prev = z.value
            L.orc_step_mwc16(a, ctypes.byref(z))
            assert z.value == a * prev % m


@pytest.mark.parametrize("a_index", [0, 1, 2])
def test_mwc16_period_brute_force(oracle, a_index):
    """Sec. II.A.1: with ab - 1 a safe prime the period is about (ab - 1)/2;
    brute force gives exactly (ab - 2)/2 for the smallest table multipliers."""
    table, _ = oracle.mwc16_table()
    a = int(table[a_index])
    period = oracle.lib().orc_period_mwc16(a, 12345 % (a * 65536 - 1))
    assert period == (a * (1 << 16) - 2) // 2


def test_small_word_mwc_period(oracle):
    """The same safe-prime rule on an 8-bit word: every a < 2^8 with a*2^8 - 1
    a safe prime gives a brute-forced period (a*2^8 - 2)/2 or a*2^8 - 2."""
    L = oracle.lib()
    seen = 0
    for a in range(2, 256):
        m = a * 256 - 1
        if not (_nt.is_prime(m) and _nt.is_prime((m - 1) // 2)):
            continue
        p = L.orc_period_mwc_small(a, 8, 1, 0)
        assert p in ((m - 1) // 2, m - 1)
        assert p == _order(a, m)
        seen += 1
    assert seen > 3


def _order(a, m):
    q = (m - 1) // 2
    for d in (1, 2, q, m - 1):
        if pow(a, d, m) == 1:
            return d
    raise AssertionError


def test_mwc32_period_via_jump(oracle):
    """The MWC32 period is the order of a modulo the safe prime m = ab - 1,
    which is q = (m - 1)/2 here: a jump by q returns every state, by 1 or 2 does not."""
    a = oracle.mwc32_multiplier()
    m = a * (1 << 32) - 1
    q = (m - 1) // 2
    assert pow(a, q, m) == 1 and pow(a, 2, m) != 1
    st = oracle.seed(oracle.MWC32, 3, 16)
    st2 = oracle.skip(oracle.MWC32, st.copy(), q)
    assert np.array_equal(st, st2)
    assert not np.array_equal(st, oracle.skip(oracle.MWC32, st.copy(), 2))


# ---------------------------------------------------------------- periods
@pytest.mark.slow
def test_xs32_full_period_brute_force(oracle):
    """Eq. (6) / Sec. II.A.2: r = 1, w = 32 has period 2^32 - 1 (brute force)."""
    assert oracle.lib().orc_period_xs32(1) == (1 << PAPER["xs32_log2_period_plus_1"]) - 1


@pytest.mark.slow
def test_lcg_full_period_brute_force(oracle):
    """Eq. (7) with a = 69069, c = 1234567, m = 2^32: full period 2^32 (Hull-Dobell)."""
    assert PAPER["lcg_multiplier"] % 4 == 1 and PAPER["lcg_increment"] % 2 == 1
    assert oracle.lib().orc_period_lcg(0) == 1 << 32


def test_lcg_constants(oracle):
    """Eq. (7): X <- 69069 X + 1234567 mod 2^32, checked on sample values."""
    L = oracle.lib()
    for x0 in (0, 1, 0xFFFFFFFF, 123456789):
        x = ctypes.c_uint32(x0)
        L.orc_step_lcg(ctypes.byref(x))
        assert x.value == (PAPER["lcg_multiplier"] * x0 + PAPER["lcg_increment"]) % (1 << 32)


def _bit_sequence(oracle, gen, n_bits, bit=0, seed=9):
    st = oracle.seed(gen, seed, 1)
    out = oracle.generate(gen, st, n_bits)[0]
    return [int((v >> bit) & 1) for v in out]


@pytest.mark.parametrize("bit", [0, 17, 31])
def test_xs256_linear_complexity_and_primitive(oracle, bit):
    """Eq. (5): r = 8, w = 32, period 2^256 - 1.  Each output bit of a full-period
    GF(2)-linear generator satisfies a linear recurrence whose minimal polynomial
    is the primitive characteristic polynomial of degree r*w = 256."""
    seq = _bit_sequence(oracle, oracle.XS256, 1200, bit)
    L, C = _nt.berlekamp_massey(seq)
    deg = PAPER["xs256_log2_period_plus_1"]
    assert L == deg
    prod = 1
    for p in _nt.FERMAT_FACTORS_256:
        assert _nt.is_prime(p)
        prod *= p
    assert prod == (1 << deg) - 1
    assert _nt.is_primitive(_nt.reciprocal(C, L), _nt.FERMAT_FACTORS_256)


def test_xs32_linear_complexity_and_primitive(oracle):
    seq = _bit_sequence(oracle, oracle.XS32, 200, 5)
    L, C = _nt.berlekamp_massey(seq)
    assert L == 32
    f = [3, 5, 17, 257, 65537]
    assert np.prod(f, dtype=object) == (1 << 32) - 1
    assert _nt.is_primitive(_nt.reciprocal(C, L), f)


@pytest.mark.slow
def test_xs256_period_via_jump(oracle):
    """Eq. (5): the jump by 2^256 - 1 is the identity and the jump by
    (2^256 - 1)/p is not, for every prime p dividing 2^256 - 1."""
    st = oracle.seed(oracle.XS256, 4, 2)
    order = (1 << 256) - 1
    assert np.array_equal(oracle.skip(oracle.XS256, st.copy(), order), st)
    for p in _nt.FERMAT_FACTORS_256:
        assert not np.array_equal(oracle.skip(oracle.XS256, st.copy(), order // p), st)


def test_xs256_matches_eq5_matrix_form(oracle):
    """Eq. (5) read as matrices: build L^k, R^k as 32x32 bit matrices and form
    v_n = sum_j A_j v_{n-j}; compare with the oracle's shift code on random windows."""
    def shift_mat(k, left):
        M = np.zeros((32, 32), dtype=np.uint8)
        for i in range(32):
            j = i + k if left else i - k  # bit i moves to bit j
            if 0 <= j < 32:
                M[j, i] = 1
        return M
    I = np.eye(32, dtype=np.uint8)
    Lm = lambda k: shift_mat(k, True)
    Rm = lambda k: shift_mat(k, False)
    mm = lambda A, B: (A.astype(np.int64) @ B.astype(np.int64) % 2).astype(np.uint8)
    A = {1: mm(I ^ Lm(9), I ^ Lm(13)), 4: I ^ Lm(7), 5: I ^ Rm(3), 7: I ^ Rm(10),
         8: mm(I ^ Lm(24), I ^ Rm(7))}

    def bits(v):
        return np.array([(v >> i) & 1 for i in range(32)], dtype=np.uint8)

    rng = np.random.default_rng(5)
    L = oracle.lib()
    for _ in range(50):
        v = rng.integers(0, 1 << 32, 8, dtype=np.uint64).astype(np.uint32)
        acc = np.zeros(32, dtype=np.uint8)
        for j, Aj in A.items():
            acc ^= mm(Aj, bits(int(v[8 - j])).reshape(32, 1)).ravel()
        expect = int(sum(int(b) << i for i, b in enumerate(acc)))
        w = v.copy()
        got = L.orc_step_xs256(w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        assert got == expect
        assert np.array_equal(w[:7], v[1:]) and w[7] == expect


def test_xs32_matches_eq6_matrix_form(oracle):
    """Eq. (6) read as matrices: A_1 = (I+L^13)(I+R^17)(I+L^5) in Marsaglia's
    row-vector convention (the generator the paper takes from him, Sec.
    II.A.3), so a state y advances as y <- y A_1, the left factor acting first.
    L and R are built as 32x32 bit matrices with y L = y << 1 and y R = y >> 1,
    and y A_1 is compared with the oracle's step on random and edge words.
    The comparison tells the readings apart: the column-vector order (y <- A_1
    y, <<5 first), L and R exchanged, and every triple with one shift changed
    by one all differ from the oracle on these words, so a transposed order or
    a wrong constant in the oracle cannot pass it."""
    def shift_row(k, left):
        # row-vector convention: (y M)_j = sum_i y_i M[i, j]; bit i moves to i +- k
        M = np.zeros((32, 32), dtype=np.uint8)
        for i in range(32):
            j = i + k if left else i - k
            if 0 <= j < 32:
                M[i, j] = 1
        return M
    I = np.eye(32, dtype=np.uint8)
    mm = lambda A, B: (A.astype(np.int64) @ B.astype(np.int64) % 2).astype(np.uint8)

    def a1(a, b, c):
        return mm(mm(I ^ shift_row(a, True), I ^ shift_row(b, False)), I ^ shift_row(c, True))

    def bits(v):
        return np.array([(v >> i) & 1 for i in range(32)], dtype=np.uint8)

    def word(bv):
        return int(sum(int(b) << i for i, b in enumerate(bv)))

    A = a1(13, 17, 5)
    rng = np.random.default_rng(6)
    words = [1, 2, 0x80000000, 0xFFFFFFFF, 0x12345678] + [int(x) for x in rng.integers(1, 1 << 32, 60)]
    L = oracle.lib()
    for y0 in words:
        y = ctypes.c_uint32(y0)
        got = L.orc_step_xs32(ctypes.byref(y))
        expect = word(mm(bits(y0).reshape(1, 32), A).ravel())
        assert got == expect and y.value == expect, hex(y0)
    # the pin discriminates: other orders and neighbouring triples differ
    # from the oracle on these words
    stepped = []
    for y0 in words:
        y = ctypes.c_uint32(y0)
        stepped.append(L.orc_step_xs32(ctypes.byref(y)))
    wrong = [A.T.copy()]  # L and R exchanged (the bit-reversed reading of L)
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        wrong.append(a1(13 + d[0], 17 + d[1], 5 + d[2]))
    wrong.append(a1(5, 17, 13))  # column vectors, y <- A_1 y: <<5 first
    for W in wrong:
        alt = [word(mm(bits(y0).reshape(1, 32), W).ravel()) for y0 in words]
        assert alt != stepped


# ---------------------------------------------------------------- jump-ahead
ALL_GENS =["MWC32", "XS256", "XS32", "KISS", "MWC1616"]


@pytest.mark.parametrize("name", ALL_GENS)
def test_jump_equals_brute_force(oracle, name):
    """Sec. II.A.4 needs the i-th number without the intermediates: jump(k) must
    equal k single steps."""
    g = oracle.GENERATORS[name]
    base = oracle.seed(g, 21, 8)
    for k in (0, 1, 2, 3, 7, 8, 9, 31, 64, 1000, 4097, 77777):
        ref = base.copy()
        if k:
            oracle.generate(g, ref, k)
        assert np.array_equal(oracle.skip(g, base.copy(), k), ref), k


@pytest.mark.parametrize("name", ALL_GENS)
def test_jump_composes(oracle, name):
    g = oracle.GENERATORS[name]
    base = oracle.seed(g, 22, 4)
    k1, k2 = (1 << 40) + 12345, (1 << 33) + 99
    a = oracle.skip(g, oracle.skip(g, base.copy(), k1), k2)
    b = oracle.skip(g, base.copy(), k1 + k2)
    assert np.array_equal(a, b)
    c = oracle.skip(g, base.copy(), k1 + 5)
    d = oracle.skip(g, base.copy(), k1)
    oracle.generate(g, d, 5)
    assert np.array_equal(c, d)


# ---------------------------------------------------------------- KISS, MWC1616
def test_kiss_is_the_papers_combination(oracle):
    """Sec. II.A.3: KISS = (MWC xor LCG) + XorShift, each component stepped once."""
    L = oracle.lib()
    st = oracle.seed(oracle.KISS, 13, 5)
    ref = st.copy()
    out = oracle.generate(oracle.KISS, ref, 300)
    for s in range(5):
        z, w, jsr, jc, a1, a2 = (ctypes.c_uint32(int(v)) for v in st[:, s])
        for k in range(300):
            L.orc_step_mwc16(a1.value, ctypes.byref(z))
            L.orc_step_mwc16(a2.value, ctypes.byref(w))
            mwc = ((z.value << 16) + w.value) & 0xFFFFFFFF
            lcg = L.orc_step_lcg(ctypes.byref(jc))
            xs = L.orc_step_xs32(ctypes.byref(jsr))
            assert out[s, k] == ((mwc ^ lcg) + xs) & 0xFFFFFFFF
        assert [z.value, w.value, jsr.value, jc.value] == ref[:4, s].tolist()


# ---------------------------------------------------------------- seeding
def test_splitmix64_vectors(oracle):
    L = oracle.lib()
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    states = {}
    for s0, idx, hexv in rows:
        st = states.setdefault(int(s0), [ctypes.c_uint64(int(s0)), 0])
        assert int(idx) == st[1]
        assert L.orc_sm64_next(ctypes.byref(st[0])) == int(hexv, 16)
        st[1] += 1


@pytest.mark.parametrize("name", ALL_GENS)
def test_seed_invariants(oracle, name):
    """Seeded states avoid the fixed points: MWC c < a and z not in {0, ab-1};
    XorShift states non-zero; MWC pairs are two distinct table multipliers."""
    g = oracle.GENERATORS[name]
    S = 4096
    st = oracle.seed(g, 1, S)
    table = set(oracle.mwc16_table()[0].tolist())
    if name == "MWC32":
        a = oracle.mwc32_multiplier()
        z = (st[1].astype(np.uint64) << np.uint64(32)) | st[0].astype(np.uint64)
        assert np.all(st[1] < a) and np.all(z >= 1) and np.all(z <= a * (1 << 32) - 2)
    if name == "XS32":
        assert np.all(st[0] != 0)
    if name == "XS256":
        assert np.all(np.any(st != 0, axis=0))
    if name in ("KISS", "MWC1616"):
        ia = 4 if name == "KISS" else 2
        a1, a2 = st[ia].astype(np.int64), st[ia + 1].astype(np.int64)
        assert set(a1.tolist()) <= table and set(a2.tolist()) <= table
        assert np.all(a1 != a2)
        for word, a in ((st[0], a1), (st[1], a2)):
            w = word.astype(np.int64)
            assert np.all(w >= 1) and np.all(w <= a * 65536 - 2) and np.all((w >> 16) < a)
        if name == "KISS":
            assert np.all(st[2] != 0)


@pytest.mark.parametrize("name", ALL_GENS)
def test_seed_first_stream_offset(oracle, name):
    g = oracle.GENERATORS[name]
    full = oracle.seed(g, 7, 300)
    part = oracle.seed(g, 7, 100, first_stream=200)
    assert np.array_equal(full[:, 200:], part)


# ---------------------------------------------------------------- FP32 map
def test_f32_map_exact(oracle):
    """The uniform map keeps the top 24 bits: f * 2^24 == u >> 8 exactly, f in [0, 1)."""
    edge = np.array([0, 1, 255, 256, 257, 0x7FFFFFFF, 0x80000000, 0xFFFFFF00,
                     0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32)
    f = oracle.to_f32(edge)
    assert np.array_equal(f.astype(np.float64) * 2.0 ** 24, (edge >> 8).astype(np.float64))
    assert f.max() < 1.0 and f.max() == np.float32(1 - 2.0 ** -24)
    for name in ALL_GENS:
        g = oracle.GENERATORS[name]
        u = oracle.generate(g, oracle.seed(g, 1, 64), 256, oracle.U32)
        f = oracle.generate(g, oracle.seed(g, 1, 64), 256, oracle.F32)
        assert np.array_equal(f.astype(np.float64) * 2.0 ** 24, (u >> 8).astype(np.float64))
        assert np.all(f >= 0) and np.all(f < 1)


# ---------------------------------------------------------------- fused consumer
def test_fused_pi_counts_pairs(oracle):
    """The fused consumer counts pairs (u_{2k}, u_{2k+1}) with
    (u_{2k}>>8)^2 + (u_{2k+1}>>8)^2 < 2^48, per stream, and leaves the state
    advanced by all n samples (an odd tail sample is drawn but not counted)."""
    g = oracle.KISS
    for n in (64, 65):
        st = oracle.seed(g, 6, 33)
        ref = st.copy()
        u = oracle.generate(g, ref, n).astype(np.uint64)
        i = u[:, 0:n - 1:2] >> np.uint64(8)
        j = u[:, 1:n:2] >> np.uint64(8)
        expect = int(np.sum(i * i + j * j < np.uint64(1 << 48)))
        assert oracle.fused_pi(g, st, n) == expect
        assert np.array_equal(st, ref)


@pytest.mark.slow
def test_fused_pi_estimates_pi(oracle):
    """Statistical sanity: 4 * count / pairs is within 6 sigma of pi."""
    g = oracle.KISS
    st = oracle.seed(g, 6, 1024)
    n = 4096
    c = oracle.fused_pi(g, st, n, threads=8)
    pairs = 1024 * n // 2
    p = np.pi / 4
    sigma = 4 * np.sqrt(p * (1 - p) / pairs)
    assert abs(4 * c / pairs - np.pi) < 6 * sigma


def test_serial_sample_consistent(oracle):
    g = oracle.XS256
    st = oracle.seed(g, 2, 1)
    ref = oracle.generate(g, st.copy(), 5000)[0]
    one = st[:, 0].copy()
    pos = np.array([0, 5, 5, 100, 4999], dtype=np.uint64)
    vals, head, tail = oracle.serial_sample(g, one, 5000, pos, 10, 7)
    assert np.array_equal(vals, ref[pos.astype(np.int64)])
    assert np.array_equal(head, ref[:10]) and np.array_equal(tail, ref[-7:])
