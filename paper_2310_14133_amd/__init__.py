"""Python binding of the QoZ GPU library (libqoz.so, gfx950).

The functions named qoz_* mirror the C entry points of include/qoz.h one to
one and only marshal arguments: device pointers are plain integers (for
example torch.Tensor.data_ptr() of a contiguous tensor on the context's
device) and streams are raw hipStream_t handles
(torch.cuda.current_stream().cuda_stream).  Every computation runs in the
library's HIP kernels; nothing here computes on the host.  If the library
has not been built, every call raises.

The Codec class at the bottom is a convenience over torch tensors (torch is
used only for device memory and streams).
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqoz.so")

QOZ_OK, QOZ_EINVAL, QOZ_ENOSPACE, QOZ_EFORMAT, QOZ_EDEVICE, QOZ_ENOMEM = range(6)
TARGETS = {"cr": 0, "psnr": 1, "ssim": 2, "ac": 3}
MAX_LEVELS = 16
HEADER_BYTES = 200  # stream header (format version 4)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOSPACE", 3: "EFORMAT",
                4: "EDEVICE", 5: "ENOMEM"}


class Shape(C.Structure):
    _fields_ = [("ndim", C.c_uint32), ("dims", C.c_uint64 * 3)]


class Params(C.Structure):
    _fields_ = [("anchor_stride", C.c_uint32), ("levels", C.c_uint32),
                ("interp", C.c_uint8 * MAX_LEVELS),
                ("order", (C.c_uint8 * 3) * MAX_LEVELS),
                ("alpha", C.c_double), ("beta", C.c_double)]


class TuneConfig(C.Structure):
    _fields_ = [("block", C.c_uint32), ("sample_stride", C.c_uint32),
                ("sample_rate", C.c_double), ("all_orders", C.c_uint32),
                ("ssim_window", C.c_uint32), ("ablation", C.c_uint32)]


MAX_CAND, NPAIRS = 12, 20


class TuneTrace(C.Structure):
    _fields_ = [("Lt", C.c_uint32), ("ncand", C.c_uint32),
                ("nblocks", C.c_uint64), ("block_points", C.c_uint64),
                ("alg1_err", (C.c_double * MAX_CAND) * MAX_LEVELS),
                ("alg1_choice", C.c_uint32 * MAX_LEVELS),
                ("B", C.c_double * NPAIRS), ("M", C.c_double * NPAIRS),
                ("Bp", C.c_double * NPAIRS), ("Mp", C.c_double * NPAIRS),
                ("eprime", C.c_double * NPAIRS),
                ("cmp_case", C.c_int32 * NPAIRS), ("best_pair", C.c_uint32)]


class BatchItem(C.Structure):
    _fields_ = [("d_x", C.c_void_p), ("shape", Shape), ("abs_eb", C.c_double),
                ("params", C.c_void_p), ("d_out", C.c_void_p),
                ("cap", C.c_size_t), ("out_bytes", C.c_size_t),
                ("status", C.c_int), ("ms", C.c_double),
                ("done_ms", C.c_double)]


class BatchDecItem(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("in_bytes", C.c_size_t),
                ("d_y", C.c_void_p), ("y_cap_elems", C.c_size_t),
                ("shape", Shape), ("status", C.c_int), ("ms", C.c_double),
                ("done_ms", C.c_double)]


class LearnedItem(C.Structure):
    _fields_ = [("d_x", C.c_void_p), ("shape", Shape),
                ("abs_eb", C.c_double), ("params", Params),
                ("used_fallback", C.c_int), ("status", C.c_int)]


class QozError(RuntimeError):
    def __init__(self, status, what, message=""):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}"
                         + (f" ({message})" if message else ""))
        self.status = status


_lib = None


def lib():
    """The loaded libqoz.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"QoZ GPU library not built ({LIB_PATH} missing); run "
                "python -c 'import __graft_entry__ as g; g.build()'")
        L = C.CDLL(LIB_PATH)
        vp, sz, u32, u64, dbl = (C.c_void_p, C.c_size_t, C.c_uint32,
                                 C.c_uint64, C.c_double)
        L.qoz_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.qoz_ctx_destroy.argtypes = [vp]
        L.qoz_ctx_destroy.restype = None
        L.qoz_compress_bound.argtypes = [Shape, C.POINTER(sz)]
        L.qoz_tune.argtypes = [vp, vp, Shape, dbl, C.c_int,
                               C.POINTER(TuneConfig), C.POINTER(Params), vp]
        L.qoz_tune_traced.argtypes = [vp, vp, Shape, dbl, C.c_int,
                                      C.POINTER(TuneConfig),
                                      C.POINTER(Params),
                                      C.POINTER(TuneTrace), vp]
        L.qoz_compress.argtypes = [vp, vp, Shape, dbl, C.POINTER(Params),
                                   C.c_int, C.POINTER(TuneConfig), vp, sz,
                                   C.POINTER(sz), vp]
        L.qoz_decompress.argtypes = [vp, vp, sz, vp, sz, C.POINTER(Shape), vp]
        L.qoz_inspect.argtypes = [vp, sz, C.POINTER(Shape),
                                  C.POINTER(dbl), C.POINTER(Params)]
        L.qoz_metrics.argtypes = [vp, vp, vp, Shape, u32, C.POINTER(dbl),
                                  C.POINTER(dbl), C.POINTER(dbl), vp]
        L.qoz_metrics_noalloc.argtypes = [vp, vp, vp, Shape, u32,
                                          C.POINTER(dbl), C.POINTER(dbl),
                                          C.POINTER(dbl), vp]
        L.qoz_error_ac.argtypes = [vp, vp, vp, Shape, C.POINTER(dbl), vp]
        L.qoz_autotune_tiles.argtypes = [vp, Shape, C.POINTER(Params),
                                         C.POINTER(u32),
                                         C.POINTER(C.c_float),
                                         C.POINTER(C.c_float), vp]
        L.qoz_compress_batch.argtypes = [vp, vp, u32, C.c_int,
                                         C.POINTER(TuneConfig), u32, vp]
        L.qoz_decompress_batch.argtypes = [vp, vp, u32, u32, vp]
        L.qoz_decompress_queue.argtypes = [vp, vp, u32, vp]
        L.qoz_compress_queue.argtypes = [vp, vp, u32, C.c_int,
                                         C.POINTER(TuneConfig), vp]
        L.qoz_ctx_set_queue_graphs.argtypes = [vp, C.c_int]
        L.qoz_tune_learned_batch.argtypes = [vp, vp, u32, vp, vp, dbl,
                                             C.c_int, C.POINTER(TuneConfig),
                                             vp]
        L.qoz_learned_features.argtypes = [vp, vp, Shape, dbl,
                                           C.POINTER(TuneConfig), vp, vp,
                                           u64, C.POINTER(u64), vp]
        L.qoz_mlp_forward.argtypes = [vp, vp, vp, u32, vp, vp]
        L.qoz_mlp_grad.argtypes = [vp, vp, vp, vp, vp, u32, u32, vp, vp, vp]
        L.qoz_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, u32,
                                         u32, C.c_float, u32, vp, vp]
        L.qoz_tune_learned.argtypes = [vp, vp, Shape, dbl, vp, dbl, C.c_int,
                                       C.POINTER(TuneConfig),
                                       C.POINTER(Params), C.POINTER(C.c_int),
                                       vp]
        L.qoz_last_error.restype = C.c_char_p
        L.qoz_ctx_set_timing.argtypes = [vp, C.c_int]
        L.qoz_ctx_set_timing_mask.argtypes = [vp, C.c_uint64]
        L.qoz_ctx_reset_timing.argtypes = [vp]
        L.qoz_prof_name.restype = C.c_char_p
        L.qoz_ctx_get_timing.argtypes = [vp, C.c_int, C.POINTER(u64),
                                         C.POINTER(dbl), C.POINTER(dbl)]
        for fn in ("qoz_ctx_create", "qoz_compress_bound", "qoz_tune",
                   "qoz_tune_traced",
                   "qoz_compress", "qoz_decompress", "qoz_inspect",
                   "qoz_metrics", "qoz_metrics_noalloc", "qoz_error_ac",
                   "qoz_autotune_tiles",
                   "qoz_compress_batch",
                   "qoz_decompress_batch", "qoz_decompress_queue",
                   "qoz_compress_queue",
                   "qoz_ctx_set_queue_graphs", "qoz_tune_learned_batch",
                   "qoz_learned_features",
                   "qoz_mlp_forward", "qoz_mlp_grad", "qoz_mlp_train_step",
                   "qoz_tune_learned", "qoz_ctx_set_timing",
                   "qoz_ctx_set_timing_mask",
                   "qoz_ctx_reset_timing", "qoz_ctx_get_timing"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def _check(st, what):
    if st != QOZ_OK:
        msg = lib().qoz_last_error()
        raise QozError(st, what, msg.decode() if msg else "")


def make_shape(dims):
    s = Shape()
    s.ndim = len(dims)
    for i in range(3):
        s.dims[i] = int(dims[i]) if i < len(dims) else 1
    return s


def make_params(ndim, interp="cubic", order=None, alpha=1.0, beta=1.0,
                anchor_stride=0):
    """interp / order: one value for every level or a per-level list."""
    p = Params()
    p.anchor_stride = anchor_stride
    for l in range(MAX_LEVELS):
        it = interp[l] if isinstance(interp, (list, tuple)) else interp
        p.interp[l] = {"linear": 0, "cubic": 1, 0: 0, 1: 1}[it]
        if order is None:
            o = list(range(ndim))
        elif isinstance(order[0], (list, tuple)):
            o = order[l]
        else:
            o = order
        for j in range(3):
            p.order[l][j] = o[j] if j < ndim else 0
    p.alpha, p.beta = alpha, beta
    return p


ABLATE_AB, ABLATE_LEVELWISE = 1, 2


def make_tune_config(block=0, sample_stride=0, sample_rate=0.0, all_orders=0,
                     ssim_window=0, ablation=0):
    c = TuneConfig()
    c.block, c.sample_stride, c.sample_rate = block, sample_stride, sample_rate
    c.all_orders, c.ssim_window, c.ablation = all_orders, ssim_window, ablation
    return c


def sz3_anchor_stride(shape):
    """Anchor stride that leaves the origin as the only anchor: levels up to
    ceil(log2(max dimension)), the level structure without anchor points
    that the ablation of Sec. VII starts from."""
    s = 2
    while s < max(shape):
        s *= 2
    return s


def params_dict(p, ndim):
    L = p.levels
    return {"anchor_stride": p.anchor_stride, "levels": L,
            "interp": [p.interp[l] for l in range(L)],
            "order": [tuple(p.order[l][j] for j in range(ndim))
                      for l in range(L)],
            "alpha": p.alpha, "beta": p.beta}


# ---- C entry points (same names, argument marshalling only) -------------

def qoz_ctx_create(device=0):
    h = C.c_void_p()
    _check(lib().qoz_ctx_create(int(device), C.byref(h)), "qoz_ctx_create")
    return h


def qoz_ctx_destroy(ctx):
    lib().qoz_ctx_destroy(ctx)


def qoz_compress_bound(shape):
    n = C.c_size_t()
    _check(lib().qoz_compress_bound(shape, C.byref(n)), "qoz_compress_bound")
    return n.value


def qoz_tune(ctx, d_x, shape, abs_eb, target, cfg, params, stream):
    """params: in (anchor_stride) / out Params."""
    _check(lib().qoz_tune(ctx, C.c_void_p(d_x), shape, C.c_double(abs_eb),
                          int(target), C.byref(cfg) if cfg else None,
                          C.byref(params), C.c_void_p(stream)), "qoz_tune")
    return params


def qoz_tune_traced(ctx, d_x, shape, abs_eb, target, cfg, params, trace,
                    stream):
    """As qoz_tune; also fills the TuneTrace `trace`."""
    _check(lib().qoz_tune_traced(ctx, C.c_void_p(d_x), shape,
                                 C.c_double(abs_eb), int(target),
                                 C.byref(cfg) if cfg else None,
                                 C.byref(params), C.byref(trace),
                                 C.c_void_p(stream)), "qoz_tune_traced")
    return params, trace


def qoz_compress(ctx, d_x, shape, abs_eb, params, target, cfg, d_out, cap,
                 stream):
    """Returns the stream size; raises QozError (ENOSPACE carries .needed)."""
    nb = C.c_size_t()
    st = lib().qoz_compress(ctx, C.c_void_p(d_x), shape, C.c_double(abs_eb),
                            C.byref(params) if params else None, int(target),
                            C.byref(cfg) if cfg else None, C.c_void_p(d_out),
                            C.c_size_t(cap), C.byref(nb), C.c_void_p(stream))
    if st == QOZ_ENOSPACE:
        e = QozError(st, "qoz_compress")
        e.needed = nb.value
        raise e
    _check(st, "qoz_compress")
    return nb.value


def qoz_decompress(ctx, d_in, in_bytes, d_y, y_cap_elems, stream):
    sh = Shape()
    _check(lib().qoz_decompress(ctx, C.c_void_p(d_in), C.c_size_t(in_bytes),
                                C.c_void_p(d_y), C.c_size_t(y_cap_elems),
                                C.byref(sh), C.c_void_p(stream)),
           "qoz_decompress")
    return sh


def qoz_inspect(h_bytes):
    """h_bytes: bytes / bytearray / numpy uint8 array of (at least) the
    stream header in host memory."""
    import numpy as np
    buf = np.ascontiguousarray(np.frombuffer(bytes(h_bytes), np.uint8)
                               if not isinstance(h_bytes, np.ndarray)
                               else h_bytes, np.uint8)
    sh, e, p = Shape(), C.c_double(), Params()
    _check(lib().qoz_inspect(buf.ctypes.data_as(C.c_void_p),
                             C.c_size_t(buf.size), C.byref(sh), C.byref(e),
                             C.byref(p)), "qoz_inspect")
    return sh, e.value, p


def qoz_metrics(ctx, d_x, d_y, shape, ssim_window, stream, want_ssim=True):
    ps, ss, me = C.c_double(), C.c_double(), C.c_double()
    _check(lib().qoz_metrics(ctx, C.c_void_p(d_x), C.c_void_p(d_y), shape,
                             C.c_uint32(ssim_window), C.byref(ps),
                             C.byref(ss) if want_ssim else None, C.byref(me),
                             C.c_void_p(stream)), "qoz_metrics")
    return ps.value, (ss.value if want_ssim else None), me.value


def qoz_metrics_noalloc(ctx, d_x, d_y, shape, ssim_window, stream,
                        want_ssim=True):
    ps, ss, me = C.c_double(), C.c_double(), C.c_double()
    _check(lib().qoz_metrics_noalloc(ctx, C.c_void_p(d_x), C.c_void_p(d_y),
                                     shape, C.c_uint32(ssim_window),
                                     C.byref(ps),
                                     C.byref(ss) if want_ssim else None,
                                     C.byref(me), C.c_void_p(stream)),
           "qoz_metrics_noalloc")
    return ps.value, (ss.value if want_ssim else None), me.value


def qoz_error_ac(ctx, d_x, d_y, shape, stream):
    ac = C.c_double()
    _check(lib().qoz_error_ac(ctx, C.c_void_p(d_x), C.c_void_p(d_y), shape,
                              C.byref(ac), C.c_void_p(stream)),
           "qoz_error_ac")
    return ac.value


def qoz_autotune_tiles(ctx, shape, params, stream):
    """Times the sweep launch tiles for this shape and parameters; returns
    (sweeps tuned, ms with the default tiles, ms with the chosen ones)."""
    n = C.c_uint32()
    t0, t1 = C.c_float(), C.c_float()
    _check(lib().qoz_autotune_tiles(ctx, shape, C.byref(params), C.byref(n),
                                    C.byref(t0), C.byref(t1),
                                    C.c_void_p(stream)), "qoz_autotune_tiles")
    return n.value, t0.value, t1.value


def qoz_compress_batch(ctx, items, target, cfg, workers, stream):
    """items: a ctypes array of BatchItem; returns the batch status
    without raising (each item carries its own)."""
    return lib().qoz_compress_batch(ctx, C.cast(items, C.c_void_p),
                                    len(items), int(target),
                                    C.byref(cfg) if cfg else None,
                                    int(workers), C.c_void_p(stream))


def qoz_ctx_set_queue_graphs(ctx, enable):
    _check(lib().qoz_ctx_set_queue_graphs(ctx, int(bool(enable))),
           "qoz_ctx_set_queue_graphs")


def qoz_compress_queue(ctx, items, target, cfg, stream):
    """items: a ctypes array of BatchItem; returns the batch status
    without raising (each item carries its own)."""
    return lib().qoz_compress_queue(ctx, C.cast(items, C.c_void_p),
                                    len(items), int(target),
                                    C.byref(cfg) if cfg else None,
                                    C.c_void_p(stream))


def qoz_decompress_queue(ctx, items, stream):
    """items: a ctypes array of BatchDecItem; returns the status without
    raising."""
    return lib().qoz_decompress_queue(ctx, C.cast(items, C.c_void_p),
                                      len(items), C.c_void_p(stream))


def qoz_decompress_batch(ctx, items, workers, stream):
    return lib().qoz_decompress_batch(ctx, C.cast(items, C.c_void_p),
                                      len(items), int(workers),
                                      C.c_void_p(stream))


MLP_NFEAT, MLP_NOUT, MLP_NPARAM = 32, 11, 22219
MLP_HEADS = (2, 5, 4)
ALPHAS = (1.0, 1.25, 1.5, 1.75, 2.0)
BETAS = (1.5, 2.0, 3.0, 4.0)


def qoz_learned_features(ctx, d_x, shape, abs_eb, cfg, d_mean, d_block,
                         block_cap, stream):
    nb = C.c_uint64()
    _check(lib().qoz_learned_features(
        ctx, C.c_void_p(d_x), shape, C.c_double(abs_eb),
        C.byref(cfg) if cfg else None, C.c_void_p(d_mean),
        C.c_void_p(d_block), C.c_uint64(block_cap), C.byref(nb),
        C.c_void_p(stream)), "qoz_learned_features")
    return nb.value


def qoz_mlp_forward(ctx, d_params, d_feat, batch, d_logits, stream):
    _check(lib().qoz_mlp_forward(ctx, C.c_void_p(d_params),
                                 C.c_void_p(d_feat), C.c_uint32(batch),
                                 C.c_void_p(d_logits), C.c_void_p(stream)),
           "qoz_mlp_forward")


def qoz_mlp_grad(ctx, d_params, d_feat, d_labels, d_index, n_rows, batch,
                 d_grad, d_loss, stream):
    _check(lib().qoz_mlp_grad(ctx, C.c_void_p(d_params), C.c_void_p(d_feat),
                              C.c_void_p(d_labels), C.c_void_p(d_index),
                              C.c_uint32(n_rows), C.c_uint32(batch),
                              C.c_void_p(d_grad), C.c_void_p(d_loss),
                              C.c_void_p(stream)), "qoz_mlp_grad")


def qoz_mlp_train_step(ctx, d_params, d_m, d_v, d_feat, d_labels, d_index,
                       n_rows, batch, lr, t, d_loss, stream):
    _check(lib().qoz_mlp_train_step(
        ctx, C.c_void_p(d_params), C.c_void_p(d_m), C.c_void_p(d_v),
        C.c_void_p(d_feat), C.c_void_p(d_labels), C.c_void_p(d_index),
        C.c_uint32(n_rows), C.c_uint32(batch), C.c_float(lr), C.c_uint32(t),
        C.c_void_p(d_loss), C.c_void_p(stream)), "qoz_mlp_train_step")


def qoz_tune_learned(ctx, d_x, shape, abs_eb, d_params, min_confidence,
                     fallback_target, cfg, params, stream):
    """params: in (anchor_stride) / out; returns (params, used_fallback)."""
    fb = C.c_int(0)
    _check(lib().qoz_tune_learned(ctx, C.c_void_p(d_x), shape,
                                  C.c_double(abs_eb), C.c_void_p(d_params),
                                  C.c_double(min_confidence),
                                  int(fallback_target),
                                  C.byref(cfg) if cfg else None,
                                  C.byref(params), C.byref(fb),
                                  C.c_void_p(stream)), "qoz_tune_learned")
    return params, bool(fb.value)


def qoz_tune_learned_batch(ctx, items, d_params, d_params_2d,
                           min_confidence, fallback_target, cfg, stream):
    """items: a ctypes array of LearnedItem; returns the status without
    raising (each item carries its own)."""
    return lib().qoz_tune_learned_batch(ctx, C.cast(items, C.c_void_p),
                                        len(items), C.c_void_p(d_params),
                                        C.c_void_p(d_params_2d),
                                        C.c_double(min_confidence),
                                        int(fallback_target),
                                        C.byref(cfg) if cfg else None,
                                        C.c_void_p(stream))


def qoz_last_error():
    m = lib().qoz_last_error()
    return m.decode() if m else ""


def qoz_ctx_set_timing(ctx, on):
    _check(lib().qoz_ctx_set_timing(ctx, int(bool(on))), "qoz_ctx_set_timing")


def qoz_ctx_set_timing_mask(ctx, mask):
    _check(lib().qoz_ctx_set_timing_mask(ctx, int(mask)),
           "qoz_ctx_set_timing_mask")


def qoz_ctx_reset_timing(ctx):
    _check(lib().qoz_ctx_reset_timing(ctx), "qoz_ctx_reset_timing")


def qoz_prof_kinds():
    return lib().qoz_prof_kinds()


def qoz_prof_name(kind):
    return lib().qoz_prof_name(int(kind)).decode()


def qoz_ctx_get_timing(ctx, kind):
    n, ms, b = C.c_uint64(), C.c_double(), C.c_double()
    _check(lib().qoz_ctx_get_timing(ctx, int(kind), C.byref(n), C.byref(ms),
                                    C.byref(b)), "qoz_ctx_get_timing")
    return n.value, ms.value, b.value


def timing_table(ctx):
    """{kind name: (launches, total ms, algorithmic bytes)}"""
    return {qoz_prof_name(k): qoz_ctx_get_timing(ctx, k)
            for k in range(qoz_prof_kinds())}


# ---- torch convenience ----------------------------------------------------

class Codec:
    """Owns one library context on a HIP device; tensors in and out.

    torch supplies device memory and the current stream; all compression
    work runs in libqoz.so.
    """

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = qoz_ctx_create(device)

    def close(self):
        if self.ctx:
            qoz_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _field(self, t):
        if t.device != self.device or t.dtype != self.torch.float32 \
                or not t.is_contiguous() or t.dim() not in (2, 3):
            raise ValueError("need a contiguous 2D/3D float32 tensor on "
                             f"{self.device}")
        return make_shape(tuple(t.shape))

    def tune(self, x, abs_eb, target="cr", cfg=None, anchor_stride=0):
        sh = self._field(x)
        p = Params()
        p.anchor_stride = anchor_stride
        return qoz_tune(self.ctx, x.data_ptr(), sh, abs_eb, TARGETS[target],
                        cfg, p, self._stream())

    def tune_traced(self, x, abs_eb, target="cr", cfg=None, anchor_stride=0):
        """(params, TuneTrace) of one tuning."""
        sh = self._field(x)
        p = Params()
        p.anchor_stride = anchor_stride
        return qoz_tune_traced(self.ctx, x.data_ptr(), sh, abs_eb,
                               TARGETS[target], cfg, p, TuneTrace(),
                               self._stream())

    def compress(self, x, abs_eb, params=None, target="cr", cfg=None):
        sh = self._field(x)
        cap = qoz_compress_bound(sh)
        out = self.torch.empty(cap, dtype=self.torch.uint8, device=self.device)
        n = qoz_compress(self.ctx, x.data_ptr(), sh, abs_eb, params,
                         TARGETS[target], cfg, out.data_ptr(), cap,
                         self._stream())
        return out[:n]

    def compress_into(self, x, abs_eb, params, out, target="cr", cfg=None):
        sh = self._field(x)
        return qoz_compress(self.ctx, x.data_ptr(), sh, abs_eb, params,
                            TARGETS[target], cfg, out.data_ptr(),
                            out.numel(), self._stream())

    def decompress(self, buf, out=None):
        head = buf[:HEADER_BYTES].cpu().numpy()
        sh, _, _ = qoz_inspect(head.tobytes()) \
            if buf.numel() >= HEADER_BYTES else (None, None, None)
        if sh is None:
            raise QozError(QOZ_EFORMAT, "decompress", "stream too short")
        dims = tuple(int(sh.dims[i]) for i in range(sh.ndim))
        if out is None:
            out = self.torch.empty(dims, dtype=self.torch.float32,
                                   device=self.device)
        qoz_decompress(self.ctx, buf.data_ptr(), buf.numel(), out.data_ptr(),
                       out.numel(), self._stream())
        return out

    def metrics(self, x, y, ssim_window=7, want_ssim=True):
        sh = self._field(x)
        return qoz_metrics(self.ctx, x.data_ptr(), y.data_ptr(), sh,
                           ssim_window, self._stream(), want_ssim)

    def autotune_tiles(self, shape, params):
        """Sweep launch tiles for fields of `shape` compressed with
        `params`, kept in this codec's context."""
        return qoz_autotune_tiles(self.ctx, make_shape(tuple(shape)), params,
                                  self._stream())

    # ---- batches -------------------------------------------------------
    def compress_batch(self, xs, abs_ebs, params=None, target="cr", cfg=None,
                       workers=4, queue=False, caps=None, check=True):
        """Compress a list of fields in one call (queue=True: through the
        device work queues, qoz_compress_queue; else on worker threads,
        qoz_compress_batch).  params: None (tune each) or a list of Params
        (an entry None: tune that field); caps: output capacities in bytes
        (default: qoz_compress_bound).  Returns (streams, items): uint8
        tensors cut to size, and the BatchItem array (status, out_bytes,
        ms, done_ms per field); with check=False a failing field does not
        raise, its stream is empty and its item says why."""
        torch = self.torch
        n = len(xs)
        items = (BatchItem * n)()
        outs = []
        keep = []
        for i, x in enumerate(xs):
            sh = self._field(x)
            cap = qoz_compress_bound(sh) if caps is None else int(caps[i])
            out = torch.empty(max(cap, 1), dtype=torch.uint8,
                              device=self.device)
            outs.append(out)
            it = items[i]
            it.d_x, it.shape, it.abs_eb = x.data_ptr(), sh, float(abs_ebs[i])
            if params is not None and params[i] is not None:
                keep.append(params[i])
                it.params = C.cast(C.pointer(params[i]), C.c_void_p)
            it.d_out, it.cap = out.data_ptr(), cap
        if queue:
            st = qoz_compress_queue(self.ctx, items, TARGETS[target], cfg,
                                    self._stream())
        else:
            st = qoz_compress_batch(self.ctx, items, TARGETS[target], cfg,
                                    workers, self._stream())
        if st != QOZ_OK and check:
            bad = [i for i in range(n) if items[i].status != QOZ_OK]
            what = "qoz_compress_queue" if queue else "qoz_compress_batch"
            raise QozError(st, f"{what} (fields {bad[:8]})",
                           qoz_last_error())
        return [outs[i][:items[i].out_bytes if items[i].status == QOZ_OK
                        else 0] for i in range(n)], items

    def _dec_items(self, zs, out):
        torch = self.torch
        n = len(zs)
        items = (BatchDecItem * n)()
        keep = []
        for i, z in enumerate(zs):
            zc = z.contiguous()
            if out is not None:
                y = out[i]
            else:
                if zc.numel() < HEADER_BYTES:
                    raise QozError(QOZ_EFORMAT, "decompress_batch",
                                   f"stream {i} too short")
                sh, _, _ = qoz_inspect(
                    zc[:HEADER_BYTES].cpu().numpy().tobytes())
                dims = tuple(int(sh.dims[j]) for j in range(sh.ndim))
                y = torch.empty(dims, dtype=torch.float32, device=self.device)
            keep.append((zc, y))
            it = items[i]
            it.d_in, it.in_bytes = zc.data_ptr(), zc.numel()
            it.d_y, it.y_cap_elems = y.data_ptr(), y.numel()
        return items, keep

    def decompress_batch(self, zs, workers=4, out=None):
        """Decompress a list of streams on worker threads; returns (fields,
        items).  out: preallocated float32 fields (else sized from the
        headers)."""
        items, keep = self._dec_items(zs, out)
        st = qoz_decompress_batch(self.ctx, items, workers, self._stream())
        if st != QOZ_OK:
            bad = [i for i in range(len(zs)) if items[i].status != QOZ_OK]
            raise QozError(st, f"qoz_decompress_batch (fields {bad[:8]})",
                           qoz_last_error())
        return [y for _, y in keep], items

    def set_queue_graphs(self, enable):
        """Replay the work-queue decompression's device work as a HIP graph
        when a call repeats the previous call's launch signature."""
        qoz_ctx_set_queue_graphs(self.ctx, enable)

    def decompress_queue(self, zs, out=None, check=True):
        """Decompress a list of streams through the device work queues;
        returns (fields, items).  With check=False a failing stream does
        not raise (its item carries the status)."""
        items, keep = self._dec_items(zs, out)
        st = qoz_decompress_queue(self.ctx, items, self._stream())
        if st != QOZ_OK and check:
            bad = [i for i in range(len(zs)) if items[i].status != QOZ_OK]
            raise QozError(st, f"qoz_decompress_queue (fields {bad[:8]})",
                           qoz_last_error())
        return [y for _, y in keep], items

    # ---- learned tuner -------------------------------------------------
    def learned_features(self, x, abs_eb, cfg=None, per_block=False):
        """Mean block features (32 float32) of a 2D or 3D field; with
        per_block also the (nblocks, 32) rows."""
        torch = self.torch
        sh = self._field(x)
        mean = torch.empty(MLP_NFEAT, dtype=torch.float32, device=self.device)
        blk = None
        cap = 0
        if per_block:
            cap = 1 << 16
            blk = torch.empty((cap, MLP_NFEAT), dtype=torch.float32,
                              device=self.device)
        nb = qoz_learned_features(self.ctx, x.data_ptr(), sh, abs_eb, cfg,
                                  mean.data_ptr(),
                                  blk.data_ptr() if per_block else None,
                                  cap, self._stream())
        return (mean, blk[:nb]) if per_block else mean

    def _dev(self, t, dtype, shape=None):
        torch = self.torch
        if t.device != self.device or t.dtype != dtype or \
                not t.is_contiguous() or (shape and tuple(t.shape) != shape):
            raise ValueError(f"need a contiguous {dtype} tensor on "
                             f"{self.device}" + (f" of shape {shape}"
                                                 if shape else ""))
        return t

    def mlp_forward(self, params, feat):
        torch = self.torch
        self._dev(params, torch.float32, (MLP_NPARAM,))
        feat = self._dev(feat, torch.float32).reshape(-1, MLP_NFEAT)
        out = torch.empty((feat.shape[0], MLP_NOUT), dtype=torch.float32,
                          device=self.device)
        qoz_mlp_forward(self.ctx, params.data_ptr(), feat.data_ptr(),
                        feat.shape[0], out.data_ptr(), self._stream())
        return out

    def mlp_grad(self, params, feat, labels, index=None, batch=None):
        torch = self.torch
        self._dev(params, torch.float32, (MLP_NPARAM,))
        self._dev(feat, torch.float32)
        self._dev(labels, torch.int32, (feat.shape[0], 3))
        if index is not None:
            self._dev(index, torch.int32)
        B = batch or (index.numel() if index is not None else feat.shape[0])
        if B > (index.numel() if index is not None else feat.shape[0]):
            raise ValueError("batch larger than the index / feature rows")
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32,
                           device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        qoz_mlp_grad(self.ctx, params.data_ptr(), feat.data_ptr(),
                     labels.data_ptr(),
                     index.data_ptr() if index is not None else None,
                     feat.shape[0], B, grad.data_ptr(), loss.data_ptr(),
                     self._stream())
        return grad, loss

    def mlp_train_step(self, params, m, v, feat, labels, index, lr, t,
                       loss=None):
        torch = self.torch
        for a in (params, m, v):
            self._dev(a, torch.float32, (MLP_NPARAM,))
        self._dev(feat, torch.float32)
        self._dev(labels, torch.int32, (feat.shape[0], 3))
        if index is not None:
            self._dev(index, torch.int32)
        B = index.numel() if index is not None else feat.shape[0]
        qoz_mlp_train_step(self.ctx, params.data_ptr(), m.data_ptr(),
                           v.data_ptr(), feat.data_ptr(), labels.data_ptr(),
                           index.data_ptr() if index is not None else None,
                           feat.shape[0], B, lr, t,
                           loss.data_ptr() if loss is not None else None,
                           self._stream())

    def tune_learned(self, x, abs_eb, params, min_confidence=0.0,
                     fallback_target="psnr", cfg=None, anchor_stride=0):
        """Learned tuning; returns (Params, used_fallback)."""
        sh = self._field(x)
        self._dev(params, self.torch.float32, (MLP_NPARAM,))
        p = Params()
        p.anchor_stride = anchor_stride
        return qoz_tune_learned(self.ctx, x.data_ptr(), sh, abs_eb,
                                params.data_ptr(), min_confidence,
                                TARGETS[fallback_target], cfg, p,
                                self._stream())

    def tune_learned_batch(self, xs, abs_ebs, params, min_confidence=0.0,
                           fallback_target="psnr", cfg=None,
                           anchor_stride=0, params_2d=None):
        """Learned tuning of a list of fields (params: the network for 3D
        fields, params_2d for 2D fields or None); returns the items
        (.params, .used_fallback, .status)."""
        self._dev(params, self.torch.float32, (MLP_NPARAM,))
        if params_2d is not None:
            self._dev(params_2d, self.torch.float32, (MLP_NPARAM,))
        items = (LearnedItem * len(xs))()
        for i, (x, e) in enumerate(zip(xs, abs_ebs)):
            items[i].d_x = x.data_ptr()
            items[i].shape = self._field(x)
            items[i].abs_eb = float(e)
            items[i].params.anchor_stride = anchor_stride
        st = qoz_tune_learned_batch(self.ctx, items, params.data_ptr(),
                                    params_2d.data_ptr()
                                    if params_2d is not None else None,
                                    min_confidence, TARGETS[fallback_target],
                                    cfg, self._stream())
        if st != QOZ_OK:
            bad = [i for i in range(len(xs)) if items[i].status != QOZ_OK]
            raise QozError(st, f"qoz_tune_learned_batch (fields {bad[:8]})",
                           qoz_last_error())
        return items

    def error_ac(self, x, y):
        """Lag-1 autocorrelation of the errors x - y (Eq. 4)."""
        sh = self._field(x)
        if self._field(y) is not None and tuple(y.shape) != tuple(x.shape):
            raise ValueError("x and y must have the same shape")
        return qoz_error_ac(self.ctx, x.data_ptr(), y.data_ptr(), sh,
                            self._stream())


def rel_to_abs(vmin, vmax, eps):
    """Value-range-relative bound (Sec. VII-A): e = eps * (max - min)."""
    return float(eps) * (float(vmax) - float(vmin))
