"""Number theory and GF(2) helpers used only by the tests.

They are written independently of the oracle (different algorithms: Miller-
Rabin instead of trial division, polynomial arithmetic and Berlekamp-Massey
instead of bit matrices), so that a test that uses them checks the oracle
against mathematics rather than against itself.
"""

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases: deterministic for
    n < 3.3e24, probabilistic (error < 4^-12) above."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


# Prime factors of the Fermat numbers F0..F7, whose product is 2^256 - 1.
FERMAT_FACTORS_256 = [
    3, 5, 17, 257, 65537,
    641, 6700417,
    274177, 67280421310721,
    59649589127497217, 5704689200685129054721,
]


def berlekamp_massey(bits):
    """Shortest LFSR of a GF(2) sequence.  Returns (L, C) with C the connection
    polynomial as an int (bit i = coefficient of x^i, C(0) = 1)."""
    C, B = 1, 1
    L, m = 0, 1
    for n, s in enumerate(bits):
        d = s
        for i in range(1, L + 1):
            d ^= ((C >> i) & 1) & bits[n - i]
        if d == 0:
            m += 1
        elif 2 * L <= n:
            T = C
            C ^= B << m
            L = n + 1 - L
            B = T
            m = 1
        else:
            C ^= B << m
            m += 1
    return L, C


def reciprocal(poly: int, degree: int) -> int:
    """x^degree * poly(1/x): turns a connection polynomial into the
    characteristic polynomial."""
    r = 0
    for i in range(degree + 1):
        if (poly >> i) & 1:
            r |= 1 << (degree - i)
    return r


def _pmulmod(a: int, b: int, mod: int, deg: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= mod
    return r


def x_pow_mod(e: int, mod: int) -> int:
    """x^e modulo the GF(2) polynomial mod."""
    deg = mod.bit_length() - 1
    result, base = 1, 0b10
    if deg == 1:
        base = 0b10 ^ mod
    while e:
        if e & 1:
            result = _pmulmod(result, base, mod, deg)
        base = _pmulmod(base, base, mod, deg)
        e >>= 1
    return result


def is_primitive(poly: int, factors_of_order) -> bool:
    """poly of degree n is primitive iff x^(2^n - 1) = 1 and
    x^((2^n - 1)/p) != 1 for each prime p dividing 2^n - 1."""
    n = poly.bit_length() - 1
    order = (1 << n) - 1
    if x_pow_mod(order, poly) != 1:
        return False
    return all(x_pow_mod(order // p, poly) != 1 for p in set(factors_of_order))
