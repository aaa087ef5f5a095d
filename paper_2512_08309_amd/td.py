"""ctypes binding of libtd.so: the C-ABI of include/td.h under the same names.

Argument marshalling only: every step of sampling, the cache and the decode
run inside the native library.  Torch tensors supply device memory and
streams for the device-side calls.  The library must have been built
(``paper_2512_08309_amd.build``); importing this module without it raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtd.so")

TD_OK, TD_E_INVAL, TD_E_NOMEM, TD_E_DEVICE, TD_E_IO, TD_E_FORMAT, TD_E_STATE = 0, -1, -2, -3, -4, -5, -6
TD_LEVEL_HEIGHT = -1
STATUS_NAMES = {0: "TD_OK", -1: "TD_E_INVAL", -2: "TD_E_NOMEM", -3: "TD_E_DEVICE", -4: "TD_E_IO",
                -5: "TD_E_FORMAT", -6: "TD_E_STATE"}

# Every symbol include/td.h declares.
EXPORTS = ["td_create", "td_destroy", "td_load_weights", "td_set_conditioning", "td_set_judge", "td_sample_region",
           "td_sample_region_async",
           "td_cache_set_budget", "td_cache_clear", "td_cache_stats", "td_cache_peek", "td_set_option",
           "td_get_info", "td_denoise_windows", "td_denoise_steps", "td_noise_region", "td_lap_decode", "td_lap_decode_noalloc", "td_lap_encode", "td_kappa", "td_cone_windows", "td_kernel_stats",
           "td_server_create", "td_server_destroy", "td_server_submit", "td_server_progress", "td_server_poll",
           "td_server_stats", "td_last_error", "td_train_create", "td_train_destroy", "td_train_last_error",
           "td_train_param_count", "td_train_set_precision", "td_train_forward", "td_train_backward", "td_train_mse", "td_train_adamw"]


class td_cache_stats_t(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_uint64), ("misses", ctypes.c_uint64), ("evictions", ctypes.c_uint64),
                ("bytes_used", ctypes.c_uint64), ("bytes_budget", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("queries", ctypes.c_uint64), ("denoiser_evals", ctypes.c_uint64),
                ("windows_evaluated", ctypes.c_uint64 * 64), ("judge_fallbacks", ctypes.c_uint64)]


class td_kernel_stat_t(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class td_request(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("x0", ctypes.c_int64), ("y0", ctypes.c_int64), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32), ("level", ctypes.c_int32), ("dev_out", ctypes.c_void_p),
                ("out_len", ctypes.c_size_t)]


class td_server_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "rounds", "batched_windows",
                                               "in_flight", "queued", "mem_in_flight", "canvas_bytes")]


class TDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtd.so is not built (run __graft_entry__.build() or paper_2512_08309_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "td_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "td_destroy": ([vp], None),
        "td_load_weights": ([vp, ctypes.c_char_p], ctypes.c_int),
        "td_set_conditioning": ([vp, vp], ctypes.c_int),
        "td_set_judge": ([vp, vp, ctypes.c_float], ctypes.c_int),
        "td_sample_region": ([vp, u64, i64, i64, i32, i32, i32, fp, sz], ctypes.c_int),
        "td_sample_region_async": ([vp, u64, i64, i64, i32, i32, i32, vp, sz, vp], ctypes.c_int),
        "td_cache_set_budget": ([vp, sz], ctypes.c_int),
        "td_cache_clear": ([vp], ctypes.c_int),
        "td_cache_stats": ([vp, ctypes.POINTER(td_cache_stats_t)], ctypes.c_int),
        "td_cache_peek": ([vp, u64, i32, i64, i64, fp, sz], ctypes.c_int),
        "td_set_option": ([vp, ctypes.c_char_p, i64], ctypes.c_int),
        "td_get_info": ([vp, ctypes.c_char_p, ctypes.POINTER(i64)], ctypes.c_int),
        "td_denoise_windows": ([vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "td_denoise_steps": ([vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "td_noise_region": ([u64, i64, i64, i32, i32, i32, ctypes.c_uint32, ctypes.c_float, i32, vp, vp],
                            ctypes.c_int),
        "td_lap_decode": ([vp, vp, i64, i64, i32, i32, i64, i64, i32, i32, vp, vp], ctypes.c_int),
        "td_lap_decode_noalloc": ([vp, vp, i64, i64, i32, i32, i64, i64, i32, i32, vp, vp], ctypes.c_int),
        "td_lap_encode": ([vp, vp, i64, i64, i32, i32, vp, sz, ctypes.POINTER(i64), vp], ctypes.c_int),
        "td_kappa": ([i64, i64, i64, i64, i32, i32, i32, ctypes.POINTER(i64)], ctypes.c_int),
        "td_cone_windows": ([i64, i64, i64, i64, i32, i32, i32, i32, i32, ctypes.POINTER(u64)], ctypes.c_int),
        "td_kernel_stats": ([vp, ctypes.POINTER(td_kernel_stat_t), i32, ctypes.POINTER(i32), i32], ctypes.c_int),
        "td_server_create": ([vp, sz, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "td_server_destroy": ([vp], None),
        "td_server_submit": ([vp, ctypes.POINTER(td_request), ctypes.POINTER(u64)], ctypes.c_int),
        "td_server_progress": ([vp, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "td_server_poll": ([vp, u64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "td_server_stats": ([vp, ctypes.POINTER(td_server_stats_t)], ctypes.c_int),
        "td_last_error": ([vp], ctypes.c_char_p),
        "td_train_create": ([ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(vp)], ctypes.c_int),
        "td_train_destroy": ([vp], None),
        "td_train_last_error": ([vp], ctypes.c_char_p),
        "td_train_param_count": ([vp, ctypes.POINTER(sz)], ctypes.c_int),
        "td_train_set_precision": ([vp, i32], ctypes.c_int),
        "td_train_forward": ([vp, vp, vp, i32, ctypes.c_double, vp, vp], ctypes.c_int),
        "td_train_backward": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "td_train_mse": ([vp, vp, vp, sz, ctypes.c_float, vp, ctypes.POINTER(ctypes.c_double), vp], ctypes.c_int),
        "td_train_adamw": ([vp, vp, vp, vp, vp, sz, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, i32, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(ctx, status):
    if status != TD_OK:
        msg = lib.td_last_error(ctx)
        raise TDError(status, msg.decode() if msg else "")


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev(t, name, shape=None, numel=None):
    """Device address of a contiguous float32 torch tensor on a GPU.  The
    checks raise instead of asserting: a host tensor, another dtype or a
    strided view would otherwise reach a kernel as a wrong address."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s: expected a torch tensor on the GPU" % name)
    if t.dtype != torch.float32:
        raise ValueError("%s: expected float32, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s: expected a contiguous tensor" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s: expected shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s: needs at least %d elements, has %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


TD_STREAM_DEFAULT = 1   # the device's default (null) stream


def _stream(stream):
    """None: the call's own default (the context's stream, or the device's
    default stream for calls without a context).  A torch stream object is
    that stream; torch's default stream (handle 0) maps to TD_STREAM_DEFAULT,
    not to NULL, so the work stays ordered with torch's."""
    if stream is None:
        return None
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return ctypes.c_void_p(h if h else TD_STREAM_DEFAULT)


# ---------------------------------------------------------------- raw calls

def td_create(device=0):
    p = ctypes.c_void_p()
    _check(None, lib.td_create(device, ctypes.byref(p)))
    return p


def td_destroy(ctx):
    lib.td_destroy(ctx)


def td_load_weights(ctx, path):
    _check(ctx, lib.td_load_weights(ctx, os.fsencode(path)))


def td_get_info(ctx, key):
    v = ctypes.c_int64()
    _check(ctx, lib.td_get_info(ctx, key.encode(), ctypes.byref(v)))
    return v.value


def td_sample_region(ctx, seed, x0, y0, w, h, level, out=None):
    """Host result: float32 [C][h][w] (latent) or [h][w] (height)."""
    shape = (h, w) if level == TD_LEVEL_HEIGHT else (td_get_info(ctx, "channels"), h, w)
    if out is None:
        out = np.empty(shape, dtype=np.float32)
    if out.dtype != np.float32 or not out.flags.c_contiguous:
        raise ValueError("out: expected a C-contiguous float32 array")
    _check(ctx, lib.td_sample_region(ctx, seed & (2 ** 64 - 1), x0, y0, w, h, level, _fptr(out), out.size))
    return out


def td_sample_region_async(ctx, seed, x0, y0, w, h, level, dev_out, stream=None):
    """dev_out: contiguous float32 torch tensor on the context's device."""
    p = _dev(dev_out, "dev_out")
    _check(ctx, lib.td_sample_region_async(ctx, seed & (2 ** 64 - 1), x0, y0, w, h, level, p, dev_out.numel(),
                                           _stream(stream)))
    return dev_out


def td_cache_set_budget(ctx, nbytes):
    _check(ctx, lib.td_cache_set_budget(ctx, nbytes))


def td_cache_clear(ctx):
    _check(ctx, lib.td_cache_clear(ctx))


def td_cache_stats(ctx):
    s = td_cache_stats_t()
    _check(ctx, lib.td_cache_stats(ctx, ctypes.byref(s)))
    d = {k: getattr(s, k) for k, _ in td_cache_stats_t._fields_ if k != "windows_evaluated"}
    d["windows_evaluated"] = list(s.windows_evaluated)
    return d


def td_cache_peek(ctx, seed, level, ix, iy):
    H = td_get_info(ctx, "window")
    C = td_get_info(ctx, "channels")
    out = np.empty((H, H, C), dtype=np.float32)
    _check(ctx, lib.td_cache_peek(ctx, seed & (2 ** 64 - 1), level, ix, iy, _fptr(out), out.size))
    return out


def td_set_option(ctx, key, value):
    _check(ctx, lib.td_set_option(ctx, key.encode(), value))


def td_set_conditioning(child, parent):
    """Make parent's final latent condition child (parent None unlinks)."""
    _check(child, lib.td_set_conditioning(child, parent))


def _window_shape(ctx, x_dev):
    """[n][H][H][C] of a batch of the context's windows, n from x_dev."""
    H, C = td_get_info(ctx, "window"), td_get_info(ctx, "channels")
    return (int(x_dev.shape[0]) if x_dev.dim() == 4 else -1, H, H, C)


def td_denoise_steps(ctx, x_dev, k0, k1, out_dev):
    """Sampler steps k0..k1-1 on independent windows [n][H][H][C] (device tensors)."""
    win = _window_shape(ctx, x_dev)
    px, po = _dev(x_dev, "x_dev", win), _dev(out_dev, "out_dev", win)
    _check(ctx, lib.td_denoise_steps(ctx, px, win[0], k0, k1, po))
    return out_dev


def td_noise_region(seed, x0, y0, out_dev, step=0, scale=1.0, stream=None, accumulate=False):
    """scale * G(seed, ., ., c, step) into a contiguous device tensor [h][w][C]
    (accumulate=True: added to what the tensor holds)."""
    if out_dev.dim() != 3:
        raise ValueError("out_dev: expected [h][w][C]")
    h, w, C = out_dev.shape
    status = lib.td_noise_region(seed & (2 ** 64 - 1), x0, y0, w, h, C, step, scale, 1 if accumulate else 0,
                                 _dev(out_dev, "out_dev"), _stream(stream))
    if status != TD_OK:
        raise TDError(status, "td_noise_region")
    return out_dev


def td_set_judge(student, teacher, threshold):
    """Teacher fallback for consistency sampling (teacher None turns it off)."""
    _check(student, lib.td_set_judge(student, teacher, threshold))


def td_denoise_windows(ctx, x_dev, k, out_dev, cond_dev=None):
    """x_dev, out_dev: contiguous float32 torch tensors [n][H][H][C] on the
    device; cond_dev: [n][H][H][C_y] for a conditioned model, else None."""
    win = _window_shape(ctx, x_dev)
    px, po = _dev(x_dev, "x_dev", win), _dev(out_dev, "out_dev", win)
    cp = None
    if cond_dev is not None:
        # an unconditioned model given conditioning is refused by the library
        # itself (TD_E_INVAL, nothing launched): only the buffer is checked then
        cc = td_get_info(ctx, "cond_channels")
        cp = _dev(cond_dev, "cond_dev", win[:3] + (cc,) if cc else None)
    _check(ctx, lib.td_denoise_windows(ctx, px, cp, win[0], k, po))
    return out_dev


def td_lap_decode(ctx, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream=None):
    """latent_dev: float32 [lh][lw][C] tensor; out_dev: float32 [H][W] tensor."""
    if latent_dev.dim() != 3:
        raise ValueError("latent_dev: expected [lh][lw][C]")
    lh, lw = latent_dev.shape[0], latent_dev.shape[1]
    pl = _dev(latent_dev, "latent_dev", (lh, lw, td_get_info(ctx, "channels")))
    _check(ctx, lib.td_lap_decode(ctx, pl, lx0, ly0, lw, lh, X0, Y0, W, H, _dev(out_dev, "out_dev", numel=W * H),
                                  _stream(stream)))
    return out_dev


def td_lap_decode_noalloc(ctx, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream=None):
    """td_lap_decode with the GPU's fixed scratch (no device allocation)."""
    if latent_dev.dim() != 3:
        raise ValueError("latent_dev: expected [lh][lw][C]")
    lh, lw = latent_dev.shape[0], latent_dev.shape[1]
    pl = _dev(latent_dev, "latent_dev", (lh, lw, td_get_info(ctx, "channels")))
    _check(ctx, lib.td_lap_decode_noalloc(ctx, pl, lx0, ly0, lw, lh, X0, Y0, W, H,
                                          _dev(out_dev, "out_dev", numel=W * H), _stream(stream)))
    return out_dev


def td_lap_encode(ctx, height_dev, X0, Y0, W, H, out_dev=None, stream=None):
    """Geometry (ox0, oy0, ow, oh) of the latent the encode of the 8-aligned
    region writes; with out_dev (float32 [oh][ow][C] tensor) also the encode
    of height_dev (float32 [H][W] tensor)."""
    geom = (ctypes.c_int64 * 4)()
    if out_dev is None:
        _check(ctx, lib.td_lap_encode(ctx, None, X0, Y0, W, H, None, 0, geom, None))
    else:
        ph = _dev(height_dev, "height_dev", numel=W * H)
        _check(ctx, lib.td_lap_encode(ctx, ph, X0, Y0, W, H, _dev(out_dev, "out_dev"), out_dev.numel(), geom,
                                      _stream(stream)))
    return tuple(int(v) for v in geom)


def td_kappa(x0, y0, w, h, size, stride, offset=0):
    """(ix_min, ix_max, iy_min, iy_max), or None if no window meets the region."""
    out = (ctypes.c_int64 * 4)()
    s = lib.td_kappa(x0, y0, w, h, size, stride, offset, out)
    if s == TD_E_INVAL and w >= 1 and h >= 1 and size >= 1 and stride >= 1:
        return None
    _check(None, s)
    return tuple(out)


def td_cone_windows(x0, y0, w, h, level, steps, size, stride, offset=0):
    n = ctypes.c_uint64()
    _check(None, lib.td_cone_windows(x0, y0, w, h, level, steps, size, stride, offset, ctypes.byref(n)))
    return n.value


def td_kernel_stats(ctx, reset=False):
    """{class name: {"launches", "ms", "flops", "bytes"}} while timing is on."""
    arr = (td_kernel_stat_t * 32)()
    n = ctypes.c_int32()
    _check(ctx, lib.td_kernel_stats(ctx, arr, 32, ctypes.byref(n), 1 if reset else 0))
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms, "flops": arr[i].flops,
                                   "bytes": arr[i].bytes} for i in range(min(n.value, 32))}


def td_server_create(ctx, hbm_budget, max_inflight):
    p = ctypes.c_void_p()
    _check(ctx, lib.td_server_create(ctx, hbm_budget, max_inflight, ctypes.byref(p)))
    return p


def td_server_destroy(srv):
    lib.td_server_destroy(srv)


def td_server_submit(ctx, srv, seed, x0, y0, w, h, level, dev_out):
    """Queue a latent query whose result goes to dev_out (float32 torch tensor [C][h][w])."""
    r = td_request(seed & (2 ** 64 - 1), x0, y0, w, h, level, _dev(dev_out, "dev_out").value, dev_out.numel())
    t = ctypes.c_uint64()
    _check(ctx, lib.td_server_submit(srv, ctypes.byref(r), ctypes.byref(t)))
    return t.value


def td_server_progress(ctx, srv, rounds=1):
    n = ctypes.c_int32()
    _check(ctx, lib.td_server_progress(srv, rounds, ctypes.byref(n)))
    return n.value


def td_server_poll(ctx, srv, ticket):
    """(done, latency_ms); a finished ticket is released."""
    d = ctypes.c_int32()
    lat = ctypes.c_double()
    _check(ctx, lib.td_server_poll(srv, ticket, ctypes.byref(d), ctypes.byref(lat)))
    return bool(d.value), lat.value


def td_server_stats(ctx, srv):
    st = td_server_stats_t()
    _check(ctx, lib.td_server_stats(srv, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in td_server_stats_t._fields_}


def td_last_error(ctx):
    return lib.td_last_error(ctx).decode()


# ---------------------------------------------------------------- convenience

class Context:
    """Owning wrapper: Context(device).load_weights(path).sample_region(...)."""

    def __init__(self, device=0):
        self.ctx = td_create(device)

    def close(self):
        if self.ctx:
            td_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_weights(self, path):
        td_load_weights(self.ctx, path)
        return self

    def set_judge(self, teacher, threshold):
        """teacher: Context whose one-step estimate judges this consistency model (None: off)."""
        td_set_judge(self.ctx, teacher.ctx if teacher is not None else None, threshold)
        self._judge = teacher
        return self

    def set_conditioning(self, parent):
        """parent: the Context whose final latent conditions this one (None unlinks)."""
        td_set_conditioning(self.ctx, parent.ctx if parent is not None else None)
        self._parent = parent      # keep the parent alive while linked
        return self

    def info(self, key):
        return td_get_info(self.ctx, key)

    def sample_region(self, seed, x0, y0, w, h, level):
        return td_sample_region(self.ctx, seed, x0, y0, w, h, level)

    def sample_region_async(self, seed, x0, y0, w, h, level, dev_out, stream=None):
        return td_sample_region_async(self.ctx, seed, x0, y0, w, h, level, dev_out, stream)

    def cache_set_budget(self, nbytes):
        td_cache_set_budget(self.ctx, nbytes)

    def cache_clear(self):
        td_cache_clear(self.ctx)

    def cache_stats(self):
        return td_cache_stats(self.ctx)

    def cache_peek(self, seed, level, ix, iy):
        return td_cache_peek(self.ctx, seed, level, ix, iy)

    def set_option(self, key, value):
        td_set_option(self.ctx, key, value)

    def denoise_windows(self, x_dev, k, out_dev, cond_dev=None):
        return td_denoise_windows(self.ctx, x_dev, k, out_dev, cond_dev)

    def denoise_steps(self, x_dev, k0, k1, out_dev):
        return td_denoise_steps(self.ctx, x_dev, k0, k1, out_dev)

    def kernel_stats(self, reset=False):
        return td_kernel_stats(self.ctx, reset)

    def lap_decode(self, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream=None):
        return td_lap_decode(self.ctx, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream)

    def lap_decode_noalloc(self, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream=None):
        return td_lap_decode_noalloc(self.ctx, latent_dev, lx0, ly0, X0, Y0, W, H, out_dev, stream)

    def lap_encode(self, height_dev, X0, Y0, W, H, out_dev=None, stream=None):
        return td_lap_encode(self.ctx, height_dev, X0, Y0, W, H, out_dev, stream)


class Server:
    """Continuous-batching request loop over a Context (see td_server_* in td.h)."""

    def __init__(self, ctx, hbm_budget, max_inflight):
        self.c = ctx
        self.srv = td_server_create(ctx.ctx, hbm_budget, max_inflight)

    def submit(self, seed, x0, y0, w, h, level, dev_out):
        return td_server_submit(self.c.ctx, self.srv, seed, x0, y0, w, h, level, dev_out)

    def progress(self, rounds=1):
        return td_server_progress(self.c.ctx, self.srv, rounds)

    def poll(self, ticket):
        return td_server_poll(self.c.ctx, self.srv, ticket)

    def stats(self):
        return td_server_stats(self.c.ctx, self.srv)

    def close(self):
        if self.srv:
            td_server_destroy(self.srv)
            self.srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------- training

def read_tdw_data(path):
    """(header bytes up to the data start, float32 data section) of a .tdw file."""
    import numpy as np
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:4] != b"TDW1":
        raise ValueError("not a TDW1 file")
    n = int.from_bytes(raw[4:8], "little")
    start = (8 + n + 63) // 64 * 64
    return raw[:start], np.frombuffer(raw[start:], dtype="<f4").copy()


def write_tdw_data(path, head, data):
    """Write a .tdw file with the header block of another and new data."""
    import numpy as np
    with open(path, "wb") as f:
        f.write(head)
        f.write(np.ascontiguousarray(data, dtype="<f4").tobytes())


def _torch_stream(stream):
    """The given stream, else torch's current stream (the one the tensors are ordered on)."""
    if stream is not None:
        return _stream(stream)
    import torch
    return _stream(torch.cuda.current_stream())


class Trainer:
    """Hand-written forward/backward of a weight file's UNet (td_train_* in td.h).
    Tensors are contiguous float32 torch tensors on the device; calls run on
    torch's current stream unless a stream is given."""

    def __init__(self, path, device=0):
        h = ctypes.c_void_p()
        status = lib.td_train_create(device, path.encode(), ctypes.byref(h))
        if status != TD_OK:
            raise TDError(status, "td_train_create failed for %s" % path)
        self.tr = h
        n = ctypes.c_size_t()
        self._check(lib.td_train_param_count(self.tr, ctypes.byref(n)))
        self.n_params = n.value
        import json
        head, _ = read_tdw_data(path)
        hdr = json.loads(head[8:8 + int.from_bytes(head[4:8], "little")])
        self.H, self.C = int(hdr["window"]["size"]), int(hdr["denoiser"]["in_channels"])
        self._out_shape = None     # [n][H][H][C] of the last forward (its backward's dD)

    def _check(self, status):
        if status != TD_OK:
            msg = lib.td_train_last_error(self.tr)
            raise TDError(status, msg.decode() if msg else "")

    def set_precision(self, precision):
        """0: FP32 convolutions; 1: BF16 operands with FP32 accumulation and FP32 master weights."""
        self._check(lib.td_train_set_precision(self.tr, precision))
        return self

    def load_params(self, path):
        import torch
        _, data = read_tdw_data(path)
        if data.size < self.n_params:
            raise ValueError("%s holds %d parameters, the network needs %d" % (path, data.size, self.n_params))
        return torch.from_numpy(data[:self.n_params].copy()).cuda()

    def forward(self, params, x, sigma, out, stream=None):
        win = (int(x.shape[0]) if x.dim() == 4 else -1, self.H, self.H, self.C)
        pp = _dev(params, "params", numel=self.n_params)
        px, po = _dev(x, "x", win), _dev(out, "out", win)
        self._check(lib.td_train_forward(self.tr, pp, px, win[0], float(sigma), po, _torch_stream(stream)))
        self._out_shape = win
        return out

    def backward(self, params, dD, grads, stream=None):
        if self._out_shape is None:
            raise ValueError("backward needs a forward first")
        pp, pg = _dev(params, "params", numel=self.n_params), _dev(grads, "grads", numel=self.n_params)
        self._check(lib.td_train_backward(self.tr, pp, _dev(dD, "dD", self._out_shape), pg, _torch_stream(stream)))
        return grads

    def mse(self, D, y, dD, weight=1.0, want_loss=True, stream=None):
        loss = ctypes.c_double()
        pD = _dev(D, "D")
        py_, pdD = _dev(y, "y", tuple(D.shape)), _dev(dD, "dD", tuple(D.shape))
        self._check(lib.td_train_mse(self.tr, pD, py_, D.numel(), float(weight), pdD,
                                     ctypes.byref(loss) if want_loss else None, _torch_stream(stream)))
        return loss.value if want_loss else None

    def adamw(self, params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01, stream=None):
        n = params.numel()
        pp, pg = _dev(params, "params"), _dev(grads, "grads", numel=n)
        pm, pv = _dev(m, "m", numel=n), _dev(v, "v", numel=n)
        self._check(lib.td_train_adamw(self.tr, pp, pg, pm, pv, n,
                                       lr, beta1, beta2, eps, weight_decay, step, _torch_stream(stream)))

    def close(self):
        if self.tr:
            lib.td_train_destroy(self.tr)
            self.tr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def student_function():
    """torch.autograd.Function over the trainer's hand-written kernels:
    D = f.apply(params, x, sigma, trainer); gradients flow to params only.
    One forward may be pending per trainer (its backward uses the saved tape)."""
    import torch

    class StudentD(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, x, sigma, trainer):
            out = torch.empty_like(x)
            trainer.forward(params, x.contiguous(), sigma, out)
            ctx.trainer = trainer
            ctx.save_for_backward(params)
            return out

        @staticmethod
        def backward(ctx, dD):
            (params,) = ctx.saved_tensors
            grads = torch.zeros_like(params)
            ctx.trainer.backward(params, dD.contiguous(), grads)
            return grads, None, None, None

    return StudentD
