"""ctypes wrapper of the CPU oracle (libqoz_ref.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use it to check and time the GPU library; the
product never imports it.  Arrays are numpy, host memory.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QOZ_REF_LIB selects another build of the same sources (the sanitizer
# build of build.py)
LIB_PATH = os.environ.get("QOZ_REF_LIB") or os.path.join(HERE, "libqoz_ref.so")

OK, EINVAL, ENOSPACE, EFORMAT = 0, 1, 2, 3
TARGETS = {"cr": 0, "psnr": 1, "ssim": 2, "ac": 3}
MAX_LEVELS = 16
RADIUS = 32768
CHUNK = 4096
ALPHAS = (1.0, 1.25, 1.5, 1.75, 2.0)
BETAS = (1.5, 2.0, 3.0, 4.0)


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


class TuneTrace(C.Structure):
    _fields_ = [("Lt", C.c_uint32), ("ncand", C.c_uint32),
                ("nblocks", C.c_uint64), ("block_points", C.c_uint64),
                ("alg1_err", (C.c_double * 12) * MAX_LEVELS),
                ("alg1_choice", C.c_uint32 * MAX_LEVELS),
                ("B", C.c_double * 20), ("M", C.c_double * 20),
                ("Bp", C.c_double * 20), ("Mp", C.c_double * 20),
                ("eprime", C.c_double * 20), ("cmp_case", C.c_int32 * 20),
                ("best_pair", C.c_uint32)]


class TrialResult(C.Structure):
    _fields_ = [("payload_bits", C.c_uint64), ("n_unpred", C.c_uint64),
                ("n_points", C.c_uint64), ("n_codes", C.c_uint64),
                ("sse", C.c_double), ("ssim_sum", C.c_double),
                ("n_windows", C.c_uint64), ("B", C.c_double),
                ("ac", C.c_double)]


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.qref_stencil.restype = C.c_float
        _lib.qref_stencil.argtypes = [C.c_int, C.c_float, C.c_float,
                                      C.c_float, C.c_float, C.c_int,
                                      C.c_int, C.c_int]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def shape_of(dims):
    s = Shape()
    s.ndim = len(dims)
    for i in range(3):
        s.dims[i] = int(dims[i]) if i < len(dims) else 1
    return s


def make_params(ndim, interp="cubic", order=None, alpha=1.0, beta=1.0,
                anchor_stride=0, levels=None):
    """interp / order: one value for every level, or a list indexed l-1."""
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
    p.alpha = alpha
    p.beta = beta
    return p


def params_to_dict(p, ndim):
    L = p.levels
    return {"anchor_stride": p.anchor_stride, "levels": L,
            "interp": [p.interp[l] for l in range(L)],
            "order": [tuple(p.order[l][j] for j in range(ndim))
                      for l in range(L)],
            "alpha": p.alpha, "beta": p.beta}


ABLATE_AB, ABLATE_LEVELWISE = 1, 2


def tune_config(block=0, sample_stride=0, sample_rate=0.0, all_orders=0,
                ssim_window=0, ablation=0):
    c = TuneConfig()
    c.block, c.sample_stride, c.sample_rate = block, sample_stride, sample_rate
    c.all_orders, c.ssim_window, c.ablation = all_orders, ssim_window, ablation
    return c


def _chk(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def level_bounds(e, alpha, beta, L):
    el = np.zeros(L, np.float64)
    tw = np.zeros(L, np.float32)
    iv = np.zeros(L, np.float32)
    _chk(lib().qref_level_bounds(C.c_double(e), C.c_double(alpha),
                                 C.c_double(beta), C.c_uint32(L), _ptr(el),
                                 _ptr(tw), _ptr(iv)), "level_bounds")
    return el, tw, iv


def stencil(cubic, a, b, c, d, has_a, has_c, has_d):
    return lib().qref_stencil(int(cubic), a, b, c, d, int(has_a), int(has_c),
                              int(has_d))


def predict_quantize(x, e, params):
    x = np.ascontiguousarray(x, np.float32)
    N = x.size
    codes = np.zeros(N, np.int32)
    recon = np.zeros(N, np.float32)
    unpred = np.zeros(N, np.float32)
    anchors = np.zeros(N, np.float32)
    nc, nu, na = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _chk(lib().qref_predict_quantize(_ptr(x), shape_of(x.shape),
                                     C.c_double(e), C.byref(params),
                                     _ptr(codes), _ptr(recon), _ptr(unpred),
                                     _ptr(anchors), C.byref(nc), C.byref(nu),
                                     C.byref(na)), "predict_quantize")
    return (codes[:nc.value], recon.reshape(x.shape), unpred[:nu.value],
            anchors[:na.value])


def target_trace(x, e, params):
    """(flat index, prediction, bin) of every target, in stream order."""
    x = np.ascontiguousarray(x, np.float32)
    N = x.size
    idx = np.zeros(N, np.uint32)
    pred = np.zeros(N, np.float32)
    codes = np.zeros(N, np.int32)
    n = C.c_uint64()
    _chk(lib().qref_target_trace(_ptr(x), shape_of(x.shape), C.c_double(e),
                                 C.byref(params), _ptr(idx), _ptr(pred),
                                 _ptr(codes), C.byref(n)), "target_trace")
    k = n.value
    return idx[:k], pred[:k], codes[:k]


def reconstruct(codes, unpred, anchors, dims, e, params):
    codes = np.ascontiguousarray(codes, np.int32)
    unpred = np.ascontiguousarray(unpred, np.float32)
    anchors = np.ascontiguousarray(anchors, np.float32)
    y = np.zeros(int(np.prod(dims)), np.float32)
    _chk(lib().qref_reconstruct(_ptr(codes), C.c_uint64(codes.size),
                                _ptr(unpred), C.c_uint64(unpred.size),
                                _ptr(anchors), C.c_uint64(anchors.size),
                                shape_of(dims), C.c_double(e),
                                C.byref(params), _ptr(y)), "reconstruct")
    return y.reshape(dims)


def huffman_lengths(hist):
    hist = np.ascontiguousarray(hist, np.uint64)
    ln = np.zeros(hist.size, np.uint8)
    _chk(lib().qref_huffman_lengths(_ptr(hist), C.c_uint32(hist.size),
                                    _ptr(ln)), "huffman_lengths")
    return ln


def huffman_codes(lengths):
    lengths = np.ascontiguousarray(lengths, np.uint8)
    code = np.zeros(lengths.size, np.uint64)
    _chk(lib().qref_huffman_codes(_ptr(lengths), C.c_uint32(lengths.size),
                                  _ptr(code)), "huffman_codes")
    return code


def compress_bound(dims):
    n = C.c_size_t()
    _chk(lib().qref_compress_bound(shape_of(dims), C.c_uint32(0),
                                   C.byref(n)), "compress_bound")
    return n.value


def compress(x, e, params=None, target="cr", cfg=None):
    x = np.ascontiguousarray(x, np.float32)
    cap = compress_bound(x.shape)
    out = np.zeros(cap, np.uint8)
    nb = C.c_size_t()
    rc = lib().qref_compress(_ptr(x), shape_of(x.shape), C.c_double(e),
                             C.byref(params) if params is not None else None,
                             C.c_int(TARGETS[target]),
                             C.byref(cfg) if cfg is not None else None,
                             _ptr(out), C.c_size_t(cap), C.byref(nb))
    _chk(rc, "compress")
    return out[:nb.value].copy()


def decompress(buf):
    buf = np.ascontiguousarray(buf, np.uint8)
    sh = Shape()
    rc = lib().qref_inspect(_ptr(buf), C.c_size_t(buf.size), C.byref(sh),
                            None, None)
    _chk(rc, "inspect")
    dims = tuple(sh.dims[i] for i in range(sh.ndim))
    y = np.zeros(int(np.prod(dims)), np.float32)
    rc = lib().qref_decompress(_ptr(buf), C.c_size_t(buf.size), _ptr(y),
                               C.c_size_t(y.size), C.byref(sh))
    _chk(rc, "decompress")
    return y.reshape(dims)


def decompress_status(buf):
    """Status code of decompressing `buf` (for malformed-stream tests)."""
    buf = np.ascontiguousarray(buf, np.uint8)
    sh = Shape()
    rc = lib().qref_inspect(_ptr(buf), C.c_size_t(buf.size), C.byref(sh),
                            None, None)
    if rc != OK:
        return rc
    n = int(np.prod([sh.dims[i] for i in range(sh.ndim)]))
    y = np.zeros(n, np.float32)
    return lib().qref_decompress(_ptr(buf), C.c_size_t(buf.size), _ptr(y),
                                 C.c_size_t(n), C.byref(sh))


def inspect(buf):
    buf = np.ascontiguousarray(buf, np.uint8)
    sh, p, e = Shape(), Params(), C.c_double()
    _chk(lib().qref_inspect(_ptr(buf), C.c_size_t(buf.size), C.byref(sh),
                            C.byref(e), C.byref(p)), "inspect")
    dims = tuple(sh.dims[i] for i in range(sh.ndim))
    return dims, e.value, p


def metrics(x, y, ssim_window=7):
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    ps, ss, me = C.c_double(), C.c_double(), C.c_double()
    _chk(lib().qref_metrics(_ptr(x), _ptr(y), shape_of(x.shape),
                            C.c_uint32(ssim_window), C.byref(ps),
                            C.byref(ss), C.byref(me)), "metrics")
    return ps.value, ss.value, me.value


def error_ac(x, y):
    """Lag-1 autocorrelation of the errors x - y along the fastest
    dimension (Eq. 4)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    ac = C.c_double()
    _chk(lib().qref_error_ac(_ptr(x), _ptr(y), shape_of(x.shape),
                             C.byref(ac)), "error_ac")
    return ac.value


def ssim_sums(x, y, w, vrange, direct=False):
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    s, n = C.c_double(), C.c_uint64()
    fn = lib().qref_ssim_direct if direct else lib().qref_ssim_separable
    _chk(fn(_ptr(x), _ptr(y), shape_of(x.shape), C.c_uint32(w),
            C.c_double(vrange), C.byref(s), C.byref(n)), "ssim")
    return s.value, n.value


def sample_plan(dims, anchor_stride=0, cfg=None):
    b, S, Lt, nb = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint64()
    bd = (C.c_uint64 * 3)()
    cap = 1 << 16
    org = np.zeros(cap, np.uint64)
    _chk(lib().qref_sample_plan(shape_of(dims), C.c_uint32(anchor_stride),
                                C.byref(cfg) if cfg is not None else None,
                                C.byref(b), C.byref(S), C.byref(Lt),
                                C.byref(nb), bd, _ptr(org),
                                C.c_uint64(cap)), "sample_plan")
    d = len(dims)
    return {"b": b.value, "S": S.value, "Lt": Lt.value,
            "nblocks": nb.value, "block_dims": tuple(bd[i] for i in range(d)),
            "origins": org[:nb.value * d].reshape(-1, d)}


def trial(x, e_trial, theta, cfg=None, vrange=None, want_ssim=False,
          want_ac=False):
    x = np.ascontiguousarray(x, np.float32)
    if vrange is None:
        vrange = float(x.max()) - float(x.min())
    r = TrialResult()
    _chk(lib().qref_trial(_ptr(x), shape_of(x.shape), C.c_double(e_trial),
                          C.byref(theta),
                          C.byref(cfg) if cfg is not None else None,
                          C.c_double(vrange),
                          C.c_uint32(int(want_ssim) | 2 * int(want_ac)),
                          C.byref(r)), "trial")
    return r


def table1_case(BI, MI, BII, MII):
    return lib().qref_table1_case(C.c_double(BI), C.c_double(MI),
                                  C.c_double(BII), C.c_double(MII))


def table1_line(BI, MI, BII, MII, BIIp, MIIp):
    return lib().qref_table1_line(C.c_double(BI), C.c_double(MI),
                                  C.c_double(BII), C.c_double(MII),
                                  C.c_double(BIIp), C.c_double(MIIp))


def tune(x, e, target="cr", cfg=None, anchor_stride=0, want_trace=True):
    x = np.ascontiguousarray(x, np.float32)
    p = Params()
    p.anchor_stride = anchor_stride
    tr = TuneTrace() if want_trace else None
    _chk(lib().qref_tune(_ptr(x), shape_of(x.shape), C.c_double(e),
                         C.c_int(TARGETS[target]),
                         C.byref(cfg) if cfg is not None else None,
                         C.byref(p), C.byref(tr) if tr is not None else None),
         "tune")
    return p, tr
