"""A statistical smoke battery for 32-bit generator output, written from the
textbook definitions (Knuth, The Art of Computer Programming vol. 2, 3.3.2:
equidistribution, serial and serial-correlation tests; Marsaglia's birthday
spacings).  Each test returns a p-value under the hypothesis of independent
uniform 32-bit words.  It is a smoke check that catches gross defects
(stuck bits, lattice structure, correlated neighbours, repeated streams); it
is not a substitute for the DIEHARD or TestU01 batteries the paper ran.
"""
import numpy as np
from scipy import stats


def _two_sided_normal(z):
    return float(2.0 * stats.norm.sf(abs(z)))


def chi2_top_byte(u):
    """Equidistribution of the top 8 bits over 256 cells."""
    counts = np.bincount((u >> 24).astype(np.int64), minlength=256)
    exp = len(u) / 256.0
    return float(stats.chi2.sf(((counts - exp) ** 2 / exp).sum(), 255))


def chi2_pairs(u):
    """Serial test on non-overlapping pairs: (top 4 bits, top 4 bits) over 256 cells."""
    n = len(u) // 2 * 2
    a = (u[0:n:2] >> 28).astype(np.int64)
    b = (u[1:n:2] >> 28).astype(np.int64)
    counts = np.bincount(a * 16 + b, minlength=256)
    exp = (n // 2) / 256.0
    return float(stats.chi2.sf(((counts - exp) ** 2 / exp).sum(), 255))


def monobit(u):
    """Frequency of ones at every bit position; the smallest p-value over the 32
    positions, Bonferroni-corrected."""
    n = len(u)
    ps = []
    for b in range(32):
        ones = int(((u >> b) & 1).sum())
        ps.append(_two_sided_normal((ones - n / 2.0) / np.sqrt(n / 4.0)))
    return min(1.0, 32 * min(ps))


def serial_correlation(u):
    """Lag-1 correlation of the FP32 uniforms (u >> 8) 2^-24; sqrt(n) r is
    asymptotically standard normal for independent uniforms."""
    x = (u >> 8).astype(np.float64) * 2.0 ** -24
    x = x - x.mean()
    v = float((x * x).sum())
    if v == 0.0:
        return 0.0  # a constant sequence
    r = float((x[:-1] * x[1:]).sum()) / v
    return _two_sided_normal(r * np.sqrt(len(u)))


def birthday_spacings(u, m=512, bits=25):
    """Marsaglia's birthday spacings: m birthdays (top `bits` bits) in a year of
    n = 2^bits days; the number of repeated values among the m - 1 sorted
    spacings is asymptotically Poisson with mean m^3 / (4 n).  Summed over all
    disjoint blocks of m words, compared with the Poisson of the summed mean.
    The limit is accurate only for a small mean: the default (m = 512,
    n = 2^25, mean 1, error of order m^4 / n^2 = 2^-14) keeps the summed
    count unbiased; with m = 1024, n = 2^24 (mean 16) a uniform source
    averages about 15.7, and a sum over thousands of blocks rejects it."""
    k = len(u) // m
    if k == 0:
        return 1.0
    days = np.sort((u[:k * m] >> (32 - bits)).astype(np.int64).reshape(k, m), axis=1)
    sp = np.sort(np.diff(days, axis=1), axis=1)
    dups = int((sp[:, 1:] == sp[:, :-1]).sum())
    lam = k * m ** 3 / (4.0 * 2 ** bits)
    lo, hi = stats.poisson.cdf(dups, lam), stats.poisson.sf(dups - 1, lam)
    return float(min(1.0, 2 * min(lo, hi)))


TESTS = {
    "chi2_top_byte": chi2_top_byte,
    "chi2_pairs": chi2_pairs,
    "monobit": monobit,
    "serial_correlation": serial_correlation,
    "birthday_spacings": birthday_spacings,
}


def battery(u):
    """p-value of every test on the words u (uint32, at least a few 10^4)."""
    u = np.ascontiguousarray(u, dtype=np.uint32).ravel()
    return {name: f(u) for name, f in TESTS.items()}


def passes(pvals, alpha=1e-6):
    """True when every p-value is above alpha (each test is one- or two-sided as
    defined above, so a small p-value is the failure)."""
    return all(p > alpha for p in pvals.values())
