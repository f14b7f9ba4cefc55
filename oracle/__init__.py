"""Python access to the serial CPU oracle (``rng_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  The product library never imports this package.

Each wrapper takes and returns numpy arrays in the library's layouts: state as
structure-of-arrays ``[words][n_streams]`` uint32, output stream-major
``[n_streams][n]`` as uint32 or float32.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

MWC32, XS256, XS32, KISS, MWC1616 = 1, 2, 3, 4, 5
U32, F32 = 0, 1
GENERATORS = {"MWC32": MWC32, "XS256": XS256, "XS32": XS32, "KISS": KISS, "MWC1616": MWC1616}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rng_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)
u16p = ctypes.POINTER(ctypes.c_uint16)
c_u64 = ctypes.c_uint64


def build(force=False):
    """Compile the oracle with gcc (plain -O2, as a portable C program)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def build_variant(path, flags):
    """Compile the same source with other optimisation flags into ``path``
    (for timing only: e.g. -O3 -march=native, built on the machine that runs
    it, since -march=native code may not run on another CPU)."""
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + list(flags) + ["-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, path)
    return path


def _bind(L):
    sig = {
        "orc_mwc16_table": (ctypes.c_int, [u16p, ctypes.c_int]),
        "orc_mwc32_multiplier": (ctypes.c_uint32, []),
        "orc_is_prime": (ctypes.c_int, [c_u64]),
        "orc_sm64_next": (c_u64, [u64p]),
        "orc_step_mwc32": (ctypes.c_uint32, [ctypes.c_uint32, u32p, u32p]),
        "orc_step_mwc16": (ctypes.c_uint32, [ctypes.c_uint32, u32p]),
        "orc_step_mwc1616": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p]),
        "orc_step_xs32": (ctypes.c_uint32, [u32p]),
        "orc_step_lcg": (ctypes.c_uint32, [u32p]),
        "orc_step_xs256": (ctypes.c_uint32, [u32p]),
        "orc_step_kiss": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p, u32p]),
        "orc_to_f32": (ctypes.c_float, [ctypes.c_uint32]),
        "orc_state_words": (ctypes.c_int, [ctypes.c_int]),
        "orc_seed": (None, [ctypes.c_int, c_u64, c_u64, c_u64, u32p]),
        "orc_generate_range": (None, [ctypes.c_int, u32p, c_u64, c_u64, c_u64, c_u64, ctypes.c_int, ctypes.c_void_p]),
        "orc_generate": (None, [ctypes.c_int, u32p, c_u64, c_u64, ctypes.c_int, ctypes.c_void_p]),
        "orc_serial_sample": (None, [ctypes.c_int, u32p, c_u64, u64p, c_u64, u32p, c_u64, u32p, c_u64, u32p]),
        "orc_fused_pi_range": (c_u64, [ctypes.c_int, u32p, c_u64, c_u64, c_u64, c_u64]),
        "orc_skip_big": (None, [ctypes.c_int, u32p, c_u64, u32p, ctypes.c_int]),
        "orc_skip": (None, [ctypes.c_int, u32p, c_u64, c_u64]),
        "orc_period_xs32": (c_u64, [ctypes.c_uint32]),
        "orc_period_lcg": (c_u64, [ctypes.c_uint32]),
        "orc_period_mwc16": (c_u64, [ctypes.c_uint32, ctypes.c_uint32]),
        "orc_period_mwc_small": (c_u64, [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def lib(path=None):
    """The oracle library; ``path`` loads a variant built by build_variant()."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _p32(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(u32p)


def state_words(gen):
    return lib().orc_state_words(gen)


def mwc16_table():
    out = np.zeros(400, dtype=np.uint16)
    n = lib().orc_mwc16_table(out.ctypes.data_as(u16p), 400)
    return out[:n].copy(), n


def mwc32_multiplier():
    return int(lib().orc_mwc32_multiplier())


def seed(gen, seed_value, n_streams, first_stream=0):
    st = np.zeros((state_words(gen), n_streams), dtype=np.uint32)
    lib().orc_seed(gen, seed_value, first_stream, n_streams, _p32(st))
    return st


def generate(gen, state, n, dtype=U32, threads=1, library=None):
    """Serial per stream; ``threads`` > 1 splits whole streams over host threads
    (ctypes releases the GIL).  ``state`` is advanced in place.  ``library``:
    a variant from lib(path) (same source, other compiler flags)."""
    S = state.shape[1]
    out = np.empty((S, n), dtype=np.float32 if dtype == F32 else np.uint32)
    if S == 0 or n == 0:
        return out
    L = library or lib()
    if threads <= 1 or S < threads:
        L.orc_generate_range(gen, _p32(state), S, 0, S, n, dtype, out.ctypes.data)
        return out
    bounds = np.linspace(0, S, threads + 1).astype(np.int64)
    ths = [threading.Thread(target=L.orc_generate_range,
                            args=(gen, _p32(state), S, int(b0), int(b1), n, dtype, out.ctypes.data))
           for b0, b1 in zip(bounds[:-1], bounds[1:])]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return out


def fused_pi(gen, state, n, threads=1):
    """Count of sample pairs inside the quarter circle; ``state`` advanced in place."""
    S = state.shape[1]
    L = lib()
    if threads <= 1 or S < threads:
        return int(L.orc_fused_pi_range(gen, _p32(state), S, 0, S, n))
    bounds = np.linspace(0, S, threads + 1).astype(np.int64)
    res = [0] * threads

    def work(i, b0, b1):
        res[i] = int(L.orc_fused_pi_range(gen, _p32(state), S, b0, b1, n))

    ths = [threading.Thread(target=work, args=(i, int(b0), int(b1)))
           for i, (b0, b1) in enumerate(zip(bounds[:-1], bounds[1:]))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return sum(res)


def skip(gen, state, k):
    """Advance every stream by k (any non-negative Python int)."""
    k = int(k)
    assert k >= 0
    words = []
    while True:
        words.append(k & 0xFFFFFFFF)
        k >>= 32
        if k == 0:
            break
    kw = np.array(words, dtype=np.uint32)
    lib().orc_skip_big(gen, _p32(state), state.shape[1], _p32(kw), len(words))
    return state


def serial_sample(gen, state_one, total, positions, n_head, n_tail):
    """Step one stream ``total`` times; return (values at sorted positions, head, tail).
    ``state_one`` has shape [words] and is advanced in place."""
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    assert np.all(pos[1:] >= pos[:-1])
    out = np.zeros(len(pos), dtype=np.uint32)
    head = np.zeros(n_head, dtype=np.uint32)
    tail = np.zeros(n_tail, dtype=np.uint32)
    lib().orc_serial_sample(gen, _p32(state_one), total, pos.ctypes.data_as(u64p), len(pos),
                            _p32(out), n_head, _p32(head), n_tail, _p32(tail))
    return out, head, tail


def to_f32(u):
    u = np.asarray(u, dtype=np.uint32)
    L = lib()
    return np.array([L.orc_to_f32(int(x)) for x in u.ravel()], dtype=np.float32).reshape(u.shape)
