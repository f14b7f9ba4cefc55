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
RNG_BATCH_CHUNK_AUTO = 0xFFFFFFFF
RNG_XS_LDS_INDEXED, RNG_XS_LDS_UNROLLED, RNG_XS_VGPR = 0, 1, 2
PLACEMENTS = {"lds_indexed": RNG_XS_LDS_INDEXED, "lds_unrolled": RNG_XS_LDS_UNROLLED, "vgpr": RNG_XS_VGPR}
RNG_OK, RNG_EINVAL, RNG_ERANGE, RNG_ENOMEM, RNG_EHIP, RNG_ENODEV, RNG_EAGAIN = 0, -1, -2, -3, -4, -5, -6

if not os.path.exists(LIB_PATH):
    raise ImportError("librng_mi355x.so is not built; run `python paper_1101_1846_amd/build.py` "
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
    "rng_set_row_shape": (_int, [_int, _int, _u64, _u64, _u32, _u32]),
    "rng_row_shape": (_int, [_int, _int, _u64, _u64, _pu32, _pu32]),
    "rng_autotune": (_int, [_int, _int, _u64, _u64, _vp, _vp, _u32, _pu32, _pu32,
                            ctypes.POINTER(ctypes.c_float), _vp]),
    "rng_skip": (_int, [_int, _vp, _u64, _u64, _vp]),
    "rng_split_workspace_bytes": (_int, [_int, _u64, _pu64]),
    "rng_generate_split": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp, _vp, _u64, _vp]),
    "rng_generate_split_noalloc": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp, _vp]),
    "rng_fused_pi": (_int, [_int, _vp, _u64, _u64, _vp, _vp]),
    "rng_calibrate_valu": (_int, [_int, ctypes.POINTER(ctypes.c_double), _vp]),
    "rng_calibrate_store": (_int, [_vp, _u64, _u64, _vp, _u32, _u32, _vp]),
    "rng_xs256_placement": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp, _vp]),
    "rng_generate_fold": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp]),
    "rng_leapfrog_workspace_bytes": (_int, [_int, _u64, _pu64]),
    "rng_generate_leapfrog": (_int, [_int, _vp, _u64, _u64, _int, _vp, _vp, _vp, _u64, _vp]),
}


class rng_request_t(ctypes.Structure):
    """One batched request (mirrors rng_request_t of include/rng.h)."""
    _fields_ = [("gen", ctypes.c_int32), ("dtype", ctypes.c_int32), ("d_state", ctypes.c_void_p),
                ("state_stride", ctypes.c_uint64), ("offset", ctypes.c_uint64), ("length", ctypes.c_uint64),
                ("d_out", ctypes.c_void_p)]


_SIGS.update({
    "rng_batch_create": (_int, [_u32, _u64, ctypes.POINTER(_vp)]),
    "rng_batch_set": (_int, [_vp, ctypes.POINTER(rng_request_t), _u32]),
    "rng_batch_launch": (_int, [_vp, _vp]),
    "rng_batch_set_shape": (_int, [_vp, _u32, _u32, _u32]),
    "rng_batch_set_graph": (_int, [_vp, ctypes.c_int]),
    "rng_batch_get_shape": (_int, [_vp, _pu32, _pu32, _pu32]),
    "rng_batch_destroy": (_int, [_vp]),
    "rng_batch_autotune": (_int, [_vp, _u32, _pu32, _pu32, _pu32, ctypes.POINTER(ctypes.c_float), _vp]),
})


class rng_server_config_t(ctypes.Structure):
    """Mirrors rng_server_config_t of include/rng.h."""
    _fields_ = [("n_streams", ctypes.c_uint64), ("gens", ctypes.c_int32 * 5), ("n_gens", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("pool_bytes", ctypes.c_uint64), ("max_batch_requests", ctypes.c_uint32),
                ("max_batch_samples", ctypes.c_uint64), ("inflight", ctypes.c_uint32),
                ("auto_release", ctypes.c_uint32), ("idle_spin_us", ctypes.c_uint32)]


class rng_server_stats_t(ctypes.Structure):
    """Mirrors rng_server_stats_t of include/rng.h."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("samples", ctypes.c_uint64), ("admission_waits", ctypes.c_uint64), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("gsamples_per_s", ctypes.c_double),
                ("mean_batch_requests", ctypes.c_double), ("mean_queue_us", ctypes.c_double),
                ("mean_submit_us", ctypes.c_double), ("mean_device_us", ctypes.c_double)]


_pdbl = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_SIGS.update({
    "rng_server_create": (_int, [ctypes.POINTER(rng_server_config_t), ctypes.POINTER(_vp)]),
    "rng_server_submit": (_int, [_vp, _u64, _u64, _int, _pu64]),
    "rng_server_poll": (_int, [_vp, _u64, ctypes.POINTER(_int), ctypes.POINTER(_vp)]),
    "rng_server_release": (_int, [_vp, _u64]),
    "rng_server_drain": (_int, [_vp]),
    "rng_server_read_state": (_int, [_vp, _u64, _pu32]),
    "rng_server_stats": (_int, [_vp, ctypes.POINTER(rng_server_stats_t)]),
    "rng_server_reset_stats": (_int, [_vp]),
    "rng_server_replay": (_int, [_vp, _pdbl, _pu64, _pu64, _pi32, _u64, _pu64]),
    "rng_server_destroy": (_int, [_vp]),
})
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


def rng_set_row_shape(g, t, n_streams, n, wg, unroll):
    return _check(_lib.rng_set_row_shape(g, t, n_streams, n, wg, unroll), "rng_set_row_shape")


def rng_row_shape(g, t, n_streams, n):
    wg, un = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_lib.rng_row_shape(g, t, n_streams, n, ctypes.byref(wg), ctypes.byref(un)), "rng_row_shape")
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


RNG_SPLIT_NOALLOC_SCRATCH_BYTES = 32 << 20


def rng_generate_split_noalloc(g, d_state_one, total, n_threads, t, d_out, d_final_state, stream=None):
    return _check(_lib.rng_generate_split_noalloc(g, _ptr(d_state_one), total, n_threads, t, _ptr(d_out),
                                                  _ptr(d_final_state), _stream(stream)),
                  "rng_generate_split_noalloc")


def rng_leapfrog_workspace_bytes(g, n_threads):
    b = ctypes.c_uint64()
    _check(_lib.rng_leapfrog_workspace_bytes(g, n_threads, ctypes.byref(b)), "rng_leapfrog_workspace_bytes")
    return b.value


def rng_generate_leapfrog(g, d_state_one, total, n_threads, t, d_out, d_final_state, d_workspace,
                          workspace_bytes, stream=None):
    return _check(_lib.rng_generate_leapfrog(g, _ptr(d_state_one), total, n_threads, t, _ptr(d_out),
                                             _ptr(d_final_state), _ptr(d_workspace), workspace_bytes,
                                             _stream(stream)), "rng_generate_leapfrog")


def rng_fused_pi(g, d_state, n_streams, n, d_count, stream=None):
    return _check(_lib.rng_fused_pi(g, _ptr(d_state), n_streams, n, _ptr(d_count), _stream(stream)),
                  "rng_fused_pi")


def rng_generate_fold(g, d_state, n_streams, n, t, d_fold, stream=None):
    return _check(_lib.rng_generate_fold(g, _ptr(d_state), n_streams, n, t, _ptr(d_fold), _stream(stream)),
                  "rng_generate_fold")


def rng_xs256_placement(placement, d_state, n_streams, n, t, d_out=None, d_fold=None, stream=None):
    return _check(_lib.rng_xs256_placement(placement, _ptr(d_state), n_streams, n, t, _ptr(d_out), _ptr(d_fold),
                                           _stream(stream)), "rng_xs256_placement")


def rng_calibrate_valu(op, stream=None):
    v = ctypes.c_double()
    _check(_lib.rng_calibrate_valu(op, ctypes.byref(v), _stream(stream)), "rng_calibrate_valu")
    return v.value


def rng_calibrate_store(d_state, n_streams, n, d_out, wg, unroll, stream=None):
    return _check(_lib.rng_calibrate_store(_ptr(d_state), n_streams, n, _ptr(d_out), wg, unroll, _stream(stream)),
                  "rng_calibrate_store")


def rng_batch_create(max_requests, max_samples):
    h = ctypes.c_void_p()
    _check(_lib.rng_batch_create(max_requests, max_samples, ctypes.byref(h)), "rng_batch_create")
    return h.value


def make_requests(reqs):
    """Build a ctypes array of rng_request_t from (gen, dtype, d_state, state_stride, offset,
    length, d_out) tuples; device buffers as torch tensors or integer addresses."""
    arr = (rng_request_t * len(reqs))()
    for i, (g, t, st, stride, off, n, out) in enumerate(reqs):
        arr[i] = rng_request_t(g, t, _ptr(st), stride, off, n, _ptr(out))
    return arr


def rng_batch_set(h, reqs, n=None):
    if not isinstance(reqs, ctypes.Array):
        reqs = make_requests(reqs)
    n = len(reqs) if n is None else n
    return _check(_lib.rng_batch_set(h, reqs, n), "rng_batch_set")


def rng_batch_launch(h, stream=None):
    return _check(_lib.rng_batch_launch(h, _stream(stream)), "rng_batch_launch")


def rng_batch_set_shape(h, wg=0, unroll=0, chunk=0):
    return _check(_lib.rng_batch_set_shape(h, wg, unroll, chunk), "rng_batch_set_shape")


def rng_batch_set_graph(h, use_graph):
    return _check(_lib.rng_batch_set_graph(h, 1 if use_graph else 0), "rng_batch_set_graph")


def rng_batch_get_shape(h):
    a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(_lib.rng_batch_get_shape(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "rng_batch_get_shape")
    return a.value, b.value, c.value


def rng_batch_autotune(h, reps=2, stream=None):
    a, b, c, us = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_float()
    _check(_lib.rng_batch_autotune(h, reps, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(us),
                                   _stream(stream)), "rng_batch_autotune")
    return a.value, b.value, c.value, us.value


def rng_batch_destroy(h):
    return _check(_lib.rng_batch_destroy(h), "rng_batch_destroy")


def rng_server_create(n_streams, gens, seed, pool_bytes, max_batch_requests, max_batch_samples,
                      inflight=3, auto_release=False, idle_spin_us=0):
    cfg = rng_server_config_t()
    cfg.n_streams = n_streams
    for i, g in enumerate(gens):
        cfg.gens[i] = g
    cfg.n_gens = len(gens)
    cfg.seed = seed
    cfg.pool_bytes = pool_bytes
    cfg.max_batch_requests = max_batch_requests
    cfg.max_batch_samples = max_batch_samples
    cfg.inflight = inflight
    cfg.auto_release = 1 if auto_release else 0
    cfg.idle_spin_us = idle_spin_us
    h = ctypes.c_void_p()
    _check(_lib.rng_server_create(ctypes.byref(cfg), ctypes.byref(h)), "rng_server_create")
    return h.value


def rng_server_submit(h, stream_id, length, dtype):
    t = ctypes.c_uint64()
    _check(_lib.rng_server_submit(h, stream_id, length, dtype, ctypes.byref(t)), "rng_server_submit")
    return t.value


def rng_server_poll(h, ticket):
    """(done, device address or None)."""
    done, ptr = ctypes.c_int(), ctypes.c_void_p()
    rc = _lib.rng_server_poll(h, ticket, ctypes.byref(done), ctypes.byref(ptr))
    if rc not in (RNG_OK, RNG_EAGAIN):
        _check(rc, "rng_server_poll")
    return bool(done.value), ptr.value


def rng_server_release(h, ticket):
    return _check(_lib.rng_server_release(h, ticket), "rng_server_release")


def rng_server_drain(h):
    return _check(_lib.rng_server_drain(h), "rng_server_drain")


def rng_server_read_state(h, stream_id, words):
    buf = (ctypes.c_uint32 * words)()
    _check(_lib.rng_server_read_state(h, stream_id, buf), "rng_server_read_state")
    return list(buf)


def rng_server_stats(h):
    st = rng_server_stats_t()
    _check(_lib.rng_server_stats(h, ctypes.byref(st)), "rng_server_stats")
    return {f: getattr(st, f) for f, _ in st._fields_}


def rng_server_reset_stats(h):
    return _check(_lib.rng_server_reset_stats(h), "rng_server_reset_stats")


def rng_server_replay(h, t_arrival_s, stream_ids, lengths, dtypes):
    """Real-time replay of an arrival trace (numpy arrays), then drain; returns tickets."""
    import numpy as np
    t = np.ascontiguousarray(t_arrival_s, dtype=np.float64)
    s = np.ascontiguousarray(stream_ids, dtype=np.uint64)
    n = np.ascontiguousarray(lengths, dtype=np.uint64)
    d = np.ascontiguousarray(dtypes, dtype=np.int32)
    tickets = np.zeros(len(t), dtype=np.uint64)
    _check(_lib.rng_server_replay(h, t.ctypes.data_as(_pdbl), s.ctypes.data_as(_pu64), n.ctypes.data_as(_pu64),
                                  d.ctypes.data_as(_pi32), len(t), tickets.ctypes.data_as(_pu64)),
           "rng_server_replay")
    return tickets


def rng_server_destroy(h):
    return _check(_lib.rng_server_destroy(h), "rng_server_destroy")


def raw():
    """The loaded ctypes library (for calls that bypass the checks above)."""
    return _lib
