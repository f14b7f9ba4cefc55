"""Seeded synthetic workloads (request tables and arrival processes).

Input generators only: numpy's PCG64 draws the request parameters; nothing
here computes any of the library's generators.  Shared by the tests and
bench.py so that both see the same inputs.
"""
import numpy as np

BATCH_GENERATORS = ("MWC32", "XS256", "KISS")


def log_uniform_lengths(rng, n, lo_log2, hi_log2):
    """floor(2^(lo + (hi - lo) U)), U uniform in [0, 1)."""
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * rng.random(n))).astype(np.int64)


def batch_table(n=10000, seed=4, generators=BATCH_GENERATORS, lo_log2=8, hi_log2=22):
    """The batched workload: generator uniform over `generators`, dtype uint32 or
    FP32 with probability 1/2, length log-uniform in [2^lo, 2^hi].
    Returns dict of numpy arrays: gen (index into generators), dtype (0/1), length."""
    rng = np.random.default_rng(seed)
    gen = rng.integers(0, len(generators), n)
    dtype = rng.integers(0, 2, n)
    length = log_uniform_lengths(rng, n, lo_log2, hi_log2)
    return {"gen": gen, "dtype": dtype, "length": length, "generators": tuple(generators)}


def poisson_arrivals(rate_per_s, n, seed=7):
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def served_table(n, seed=7, n_streams=10 ** 6, lo_log2=10, hi_log2=24):
    """Served workload: target stream uniform among n_streams resident states,
    dtype 50/50, size log-uniform in [2^lo, 2^hi]."""
    rng = np.random.default_rng(seed + 1000)
    stream = rng.integers(0, n_streams, n)
    dtype = rng.integers(0, 2, n)
    length = log_uniform_lengths(rng, n, lo_log2, hi_log2)
    return {"stream": stream, "dtype": dtype, "length": length}


def layout_outputs(lengths, align_words=64):
    """Word offsets of each request's output inside one flat buffer, every start
    rounded up to align_words (64 words = 256 bytes keeps every chunk row on
    whole 128-byte lines); returns (offsets, total_words)."""
    offs = np.zeros(len(lengths), dtype=np.int64)
    pos = 0
    for i, n in enumerate(lengths):
        pos = (pos + align_words - 1) // align_words * align_words
        offs[i] = pos
        pos += int(n)
    return offs, pos + align_words
