"""Python binding of the MI355X bulk PRNG-stream library (``librng_mi355x.so``).

Argument marshalling only: every function below forwards to the C ABI entry
point of the same name declared in ``include/rng.h``; all generation work runs
in the library's HIP kernels.  Device buffers are passed as torch tensors (or
raw integer device addresses) and HIP streams as ``torch.cuda.Stream`` (or a
raw ``hipStream_t`` integer); ``None`` means torch's current stream.

If the shared library has not been built this module raises on import: there
is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librng_mi355x.so")

RNG_MWC32, RNG_XS256, RNG_XS32, RNG_KISS, RNG_MWC1616 = 1, 2, 3, 4, 5
RNG_U32, RNG_F32 = 0, 1
GENERATORS = {"MWC32": RNG_MWC32, "XS256": RNG_XS256, "XS32": RNG_XS32, "KISS": RNG_KISS,
              "MWC1616": RNG_MWC1616}
DTYPES = {"u32": RNG_U32, "f32": RNG_F32}
RNG_OK, RNG_EINVAL, RNG_ERANGE, RNG_ENOMEM, RNG_EHIP, RNG_ENODEV, RNG_EAGAIN = 0, -1, -2, -3, -4, -5, -6

if not os.path.exists(LIB_PATH):
    raise ImportError("librng_mi355x.so is not built; run `python -m paper_1101_1846_amd.build` "
                      "(hipcc --offload-arch=gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

_u64, _u32, _int, _vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
_pu32 = ctypes.POINTER(ctypes.c_uint32)
_pu16 = ctypes.POINTER(ctypes.c_uint16)
_pu64 = ctypes.POINTER(ctypes.c_uint64)

_SIGS = {
    "rng_strerror": (ctypes.c_char_p, [_int]),
    "rng_last_error": (ctypes.c_char_p, []),
    "rng_init": (_int, []),
    "rng_shutdown": (_int, []),
    "rng_state_words": (_int, [_int, _pu32]),
    "rng_mwc32_multiplier": (_int, [_pu32]),
    "rng_mwc16_multipliers": (_int, [_pu16, _u32, _pu32]),
    "rng_seed": (_int, [_int, _u64, _u64, _u64, _vp, _vp]),
    "rng_generate": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp]),
    "rng_generate_ex": (_int, [_int, _vp, _u64, _u64, _int, _vp, _u32, _u32, _vp]),
    "rng_set_shape": (_int, [_int, _int, _u32, _u32]),
    "rng_get_shape": (_int, [_int, _int, _pu32, _pu32]),
    "rng_autotune": (_int, [_int, _int, _u64, _u64, _vp, _vp, _u32, _pu32, _pu32,
                            ctypes.POINTER(ctypes.c_float), _vp]),
    "rng_skip": (_int, [_int, _vp, _u64, _u64, _vp]),
    "rng_split_workspace_bytes": (_int, [_int, _u64, _pu64]),
    "rng_generate_split": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp, _vp, _u64, _vp]),
    "rng_fused_pi": (_int, [_int, _vp, _u64, _u64, _vp, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class RngError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.rng_last_error().decode(errors="replace")
        super().__init__("%s: %s (%d): %s" % (where, rng_strerror(code), code, msg))
        self.code = code


def _check(rc, where):
    if rc != RNG_OK:
        raise RngError(rc, where)
    return rc


def _ptr(x):
    """Device address of a torch tensor, or an integer address as is."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def rng_strerror(code):
    return _lib.rng_strerror(code).decode()


def rng_last_error():
    return _lib.rng_last_error().decode(errors="replace")


def rng_init():
    return _check(_lib.rng_init(), "rng_init")


def rng_shutdown():
    return _check(_lib.rng_shutdown(), "rng_shutdown")


def rng_state_words(g):
    w = ctypes.c_uint32()
    _check(_lib.rng_state_words(g, ctypes.byref(w)), "rng_state_words")
    return w.value


def rng_mwc32_multiplier():
    a = ctypes.c_uint32()
    _check(_lib.rng_mwc32_multiplier(ctypes.byref(a)), "rng_mwc32_multiplier")
    return a.value


def rng_mwc16_multipliers():
    n = ctypes.c_uint32()
    _check(_lib.rng_mwc16_multipliers(None, 0, ctypes.byref(n)), "rng_mwc16_multipliers")
    buf = (ctypes.c_uint16 * n.value)()
    _check(_lib.rng_mwc16_multipliers(buf, n.value, ctypes.byref(n)), "rng_mwc16_multipliers")
    return list(buf)


def rng_seed(g, seed, first_stream, n_streams, d_state, stream=None):
    return _check(_lib.rng_seed(g, seed, first_stream, n_streams, _ptr(d_state), _stream(stream)), "rng_seed")


def rng_generate(g, d_state, n_streams, n, t, d_out, stream=None):
    return _check(_lib.rng_generate(g, _ptr(d_state), n_streams, n, t, _ptr(d_out), _stream(stream)),
                  "rng_generate")


def rng_generate_ex(g, d_state, n_streams, n, t, d_out, wg, unroll, stream=None):
    return _check(_lib.rng_generate_ex(g, _ptr(d_state), n_streams, n, t, _ptr(d_out), wg, unroll,
                                       _stream(stream)), "rng_generate_ex")


def rng_set_shape(g, t, wg, unroll):
    return _check(_lib.rng_set_shape(g, t, wg, unroll), "rng_set_shape")


def rng_get_shape(g, t):
    wg, un = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_lib.rng_get_shape(g, t, ctypes.byref(wg), ctypes.byref(un)), "rng_get_shape")
    return wg.value, un.value


def rng_autotune(g, t, n_streams, n, d_state_scratch, d_out_scratch, reps=3, stream=None):
    wg, un, us = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_float()
    _check(_lib.rng_autotune(g, t, n_streams, n, _ptr(d_state_scratch), _ptr(d_out_scratch), reps,
                             ctypes.byref(wg), ctypes.byref(un), ctypes.byref(us), _stream(stream)),
           "rng_autotune")
    return wg.value, un.value, us.value


def rng_skip(g, d_state, n_streams, k, stream=None):
    return _check(_lib.rng_skip(g, _ptr(d_state), n_streams, k, _stream(stream)), "rng_skip")


def rng_split_workspace_bytes(g, n_threads):
    b = ctypes.c_uint64()
    _check(_lib.rng_split_workspace_bytes(g, n_threads, ctypes.byref(b)), "rng_split_workspace_bytes")
    return b.value


def rng_generate_split(g, d_state_one, total, n_threads, t, d_out, d_final_state, d_workspace,
                       workspace_bytes, stream=None):
    return _check(_lib.rng_generate_split(g, _ptr(d_state_one), total, n_threads, t, _ptr(d_out),
                                          _ptr(d_final_state), _ptr(d_workspace), workspace_bytes,
                                          _stream(stream)), "rng_generate_split")


def rng_fused_pi(g, d_state, n_streams, n, d_count, stream=None):
    return _check(_lib.rng_fused_pi(g, _ptr(d_state), n_streams, n, _ptr(d_count), _stream(stream)),
                  "rng_fused_pi")


def raw():
    """The loaded ctypes library (for calls that bypass the checks above)."""
    return _lib
