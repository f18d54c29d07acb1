"""Python binding of libcptraj — MI355X-native trajectory-preserving
compression of 2D time-varying vector fields (arXiv 2510.25143).

Argument marshalling only: every step runs in the HIP kernels of
``libcptraj.so`` (built in-tree by ``paper_2510_25143_amd.build``).  Fields are
float32 CUDA tensors of shape (2, T, H, W); streams are uint8 CUDA tensors.
There is no CPU fallback: a missing library raises at first use.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcptraj.so")

OK, EINVAL, ENOMEM, ECORRUPT, ECAPACITY, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PRED_LORENZO, PRED_SL, PRED_MIX2, PRED_MIX4, PRED_LEARNED = 0, 1, 2, 3, 4
SELECTOR_PARAMS = 5124


class CptError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libcptraj status %d: %s" % (status, msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("eb_mode", ctypes.c_int32),
                ("predictor", ctypes.c_int32), ("mode_bt", ctypes.c_int32),
                ("dt_dx", ctypes.c_double), ("dt_dy", ctypes.c_double),
                ("selector_w", ctypes.c_void_p), ("backend", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("T", ctypes.c_int32),
                ("k", ctypes.c_int32), ("eb_abs", ctypes.c_double), ("eps", ctypes.c_int64),
                ("predictor", ctypes.c_int32), ("mode_bt", ctypes.c_int32),
                ("K", ctypes.c_int32), ("R", ctypes.c_int32), ("total_len", ctypes.c_uint64),
                ("n_q", ctypes.c_uint64), ("n_raw", ctypes.c_uint64), ("backend", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class TrainOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64)]


class ExecOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("schedule", ctypes.c_int32), ("group", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("field_tile", ctypes.c_int32),
                ("phase_blocks", ctypes.c_int32)]


SCHEDULES = {"auto": 0, "launch": 1, "fused": 2, "persistent": 3}
# (schedule, graph replay, field tile); the last two take the schedule and
# graph setting of the fastest of the first four
TUNE_CANDIDATES = [("launch", False, 0, 2), ("fused", False, 0, 2), ("launch", True, 0, 2), ("fused", True, 0, 2),
                   ("best", None, 1, 2), ("best", None, 2, 2), ("best", None, None, 1)]
FIELD_TILES = [(32, 16), (64, 8), (16, 32)]


class VerifyResult(ctypes.Structure):
    _fields_ = [("fc_t", ctypes.c_uint64), ("fc_s", ctypes.c_uint64),
                ("max_err", ctypes.c_double), ("psnr", ctypes.c_double)]


EXPORTS = ["cpt_compress_bound", "cpt_compress", "cpt_compress_debug", "cpt_stream_info",
           "cpt_decompress", "cpt_extract_trajectories", "cpt_verify", "cpt_field_params",
           "cpt_selector_grad", "cpt_selector_train", "cpt_timing_enable", "cpt_timing_read",
           "cpt_compress_batch", "cpt_autotune_batch", "cpt_decompress_batch", "cpt_verify_noalloc",
           "cpt_tracks", "cpt_last_error"]

_lib = None


def lib():
    """Load libcptraj.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcptraj.so is not built: run paper_2510_25143_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "cpt_compress_bound": [i32, i32, i32, P],
        "cpt_compress": [P, i32, i32, i32, dbl, P, P, sz, P, P],
        "cpt_compress_debug": [P, i32, i32, i32, dbl, P, P, sz, P, P, P, P, P, P, P, P],
        "cpt_stream_info": [P, sz, P],
        "cpt_decompress": [P, sz, P, sz, P],
        "cpt_extract_trajectories": [P, i32, i32, i32, i32, P, sz, P, P],
        "cpt_verify": [P, P, i32, i32, i32, i32, P, P],
        "cpt_verify_noalloc": [P, P, i32, i32, i32, i32, P, P],
        "cpt_tracks": [P, i32, i32, i32, i32, P, P, P],
        "cpt_field_params": [P, i32, i32, i32, i32, dbl, P, P, P, P],
        "cpt_selector_grad": [P, P, P, i32, P, P, P],
        "cpt_selector_train": [P, P, i32, P, P, P, P, P],
        "cpt_timing_enable": [i32],
        "cpt_timing_read": [i32, P, P, P],
        "cpt_compress_batch": [i32, P, P, dbl, P, P, P, P, P, P, P],
        "cpt_autotune_batch": [i32, P, P, dbl, P, P, P, i32, P, P, P],
        "cpt_decompress_batch": [i32, P, P, P, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.cpt_last_error.restype = ctypes.c_char_p
    L.cpt_last_error.argtypes = []
    _lib = L
    return L


def _check(st):
    if st != OK:
        raise CptError(st, lib().cpt_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _field(f):
    if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float32):
        raise TypeError("field must be a float32 CUDA tensor")
    if f.dim() != 4 or f.shape[0] != 2:
        raise ValueError("field must have shape (2, T, H, W)")
    return f.contiguous()


def _options(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend=0):
    o = Options(ctypes.sizeof(Options), eb_mode, predictor, mode_bt, dt_dx, dt_dy, None, backend)
    if selector_w is not None:
        if not (selector_w.is_cuda and selector_w.dtype in (torch.int16, torch.bfloat16, torch.uint16)):
            raise TypeError("selector_w must be a CUDA bf16/int16 tensor of %d values" % SELECTOR_PARAMS)
        if selector_w.numel() != SELECTOR_PARAMS:
            raise ValueError("selector_w must hold %d values" % SELECTOR_PARAMS)
        if not selector_w.is_contiguous() or selector_w.data_ptr() % 16:
            raise ValueError("selector_w must be a contiguous, 16-byte aligned tensor")
        o.selector_w = selector_w.data_ptr()
    return o


def compress_bound(H, W, T):
    n = ctypes.c_size_t()
    _check(lib().cpt_compress_bound(H, W, T, ctypes.byref(n)))
    return n.value


def compress(field, eb, predictor=PRED_MIX2, mode_bt=1, eb_mode=0, dt_dx=1.0, dt_dy=1.0,
             selector_w=None, out=None, backend=0):
    """Compress ``field`` (2,T,H,W float32 CUDA) under bound ``eb``; returns the
    stream as a uint8 CUDA tensor (a view of ``out`` when given).  backend=1
    adds the zero-byte-elision stage after Huffman coding."""
    f = _field(field)
    _, T, H, W = f.shape
    if out is None:
        out = torch.empty(compress_bound(H, W, T), dtype=torch.uint8, device=f.device)
    o = _options(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend)
    n = ctypes.c_size_t()
    _check(lib().cpt_compress(_ptr(f), H, W, T, eb, ctypes.byref(o), _ptr(out), out.numel(),
                              ctypes.byref(n), _stream()))
    return out[:n.value]


def compress_debug(field, eb, predictor=PRED_MIX2, mode_bt=1, eb_mode=0, dt_dx=1.0, dt_dy=1.0,
                   selector_w=None, backend=0):
    """Compress and also return per-vertex bounds, bound codes, residual codes,
    per-block predictor classes and selector features."""
    f = _field(field)
    _, T, H, W = f.shape
    N = T * H * W
    dev = f.device
    out = torch.empty(compress_bound(H, W, T), dtype=torch.uint8, device=dev)
    nbmax = T * ((H + 15) // 16) * ((W + 15) // 16)
    xi = torch.empty(N, dtype=torch.int32, device=dev)
    xcode = torch.empty(N, dtype=torch.uint8, device=dev)
    qcode = torch.empty(N, dtype=torch.int32, device=dev)
    modes = torch.zeros(max(nbmax, 1), dtype=torch.uint8, device=dev)
    feats = torch.zeros((max(nbmax, 1), 10), dtype=torch.float32, device=dev)
    o = _options(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend)
    n, nb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().cpt_compress_debug(_ptr(f), H, W, T, eb, ctypes.byref(o), _ptr(out), out.numel(),
                                    ctypes.byref(n), _ptr(xi), _ptr(xcode), _ptr(qcode), _ptr(modes),
                                    _ptr(feats), ctypes.byref(nb), _stream()))
    return out[:n.value], dict(xi=xi, xcode=xcode, qcode=qcode, modes=modes[:nb.value],
                               feats=feats[:nb.value])


def _batch_args(fields, outs):
    fs = [_field(f) for f in fields]
    n = len(fs)
    if n == 0:
        raise ValueError("empty batch")
    hwt = (ctypes.c_int32 * (3 * n))()
    for i, f in enumerate(fs):
        _, T, H, W = f.shape
        hwt[3 * i], hwt[3 * i + 1], hwt[3 * i + 2] = H, W, T
    if outs is None:
        outs = [torch.empty(compress_bound(f.shape[2], f.shape[3], f.shape[1]), dtype=torch.uint8, device=f.device)
                for f in fs]
    if len(outs) != n:
        raise ValueError("need one output buffer per field")
    fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    caps = (ctypes.c_size_t * n)(*[o.numel() for o in outs])
    return fs, n, hwt, outs, fp, op, caps


def compress_batch(fields, eb, predictor=PRED_MIX2, mode_bt=1, eb_mode=0, dt_dx=1.0, dt_dy=1.0,
                   selector_w=None, schedule="auto", group=0, grid=0, use_graph=False, outs=None,
                   raise_on_error=True, backend=0, field_tile=0, phase_blocks=0):
    """Compress a list of fields (each (2,T,H,W) float32 CUDA) in one device
    pipeline.  Returns (streams, status): streams[i] is a view of outs[i]
    trimmed to its length (None when field i failed), status[i] its
    cpt_status."""
    fs, n, hwt, outs, fp, op, caps = _batch_args(fields, outs)
    o = _options(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend)
    ex = ExecOptions(ctypes.sizeof(ExecOptions), SCHEDULES[schedule], group, grid, int(bool(use_graph)), field_tile,
                     phase_blocks)
    lens = (ctypes.c_size_t * n)()
    st = (ctypes.c_int32 * n)()
    r = lib().cpt_compress_batch(n, fp, hwt, eb, ctypes.byref(o), ctypes.byref(ex), op, caps, lens, st, _stream())
    if r != OK and (raise_on_error or r not in (EINVAL, ECAPACITY)):
        _check(r)
    streams = [outs[i][:lens[i]] if st[i] == OK else None for i in range(n)]
    return streams, [st[i] for i in range(n)]


def autotune_batch(fields, eb, reps=2, predictor=PRED_MIX2, mode_bt=1, eb_mode=0, dt_dx=1.0, dt_dy=1.0,
                   selector_w=None, outs=None, backend=0):
    """Time every candidate execution choice on this batch and remember the
    fastest for schedule="auto".  Returns (best, ms): best = (schedule,
    use_graph, field_tile, phase_blocks), ms the mean time per run of each
    of TUNE_CANDIDATES."""
    fs, n, hwt, outs, fp, op, caps = _batch_args(fields, outs)
    o = _options(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend)
    best = ExecOptions(ctypes.sizeof(ExecOptions), 0, 0, 0, 0, 0, 0)
    ms = (ctypes.c_double * len(TUNE_CANDIDATES))()
    _check(lib().cpt_autotune_batch(n, fp, hwt, eb, ctypes.byref(o), op, caps, reps, ctypes.byref(best), ms,
                                    _stream()))
    name = {v: k for k, v in SCHEDULES.items()}[best.schedule]
    return (name, bool(best.use_graph), best.field_tile, best.phase_blocks), list(ms)


def _out_field(out):
    """An output field must be a contiguous float32 CUDA tensor; its element
    count is passed to the library as the capacity."""
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float32):
        raise TypeError("output field must be a float32 CUDA tensor")
    if not out.is_contiguous():
        raise ValueError("output field must be contiguous")
    return out


def decompress_batch(streams, outs=None, raise_on_error=True):
    """Decompress a list of streams (uint8 CUDA tensors) in one device
    pipeline.  Returns (fields, status); with raise_on_error=False a corrupt
    stream or an undersized output only sets its status."""
    n = len(streams)
    if n == 0:
        raise ValueError("empty batch")
    ss = [s.contiguous() for s in streams]
    for st in ss:
        if not (st.is_cuda and st.dtype == torch.uint8):
            raise TypeError("streams must be uint8 CUDA tensors")
    if outs is None:
        outs = []
        for st in ss:
            info = stream_info(st)
            outs.append(torch.empty((2, info["T"], info["H"], info["W"]), dtype=torch.float32, device=st.device))
    if len(outs) != n:
        raise ValueError("need one output field per stream")
    outs = [_out_field(o) for o in outs]
    sp = (ctypes.c_void_p * n)(*[st.data_ptr() for st in ss])
    lens = (ctypes.c_size_t * n)(*[st.numel() for st in ss])
    fp = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    caps = (ctypes.c_size_t * n)(*[o.numel() for o in outs])
    status = (ctypes.c_int32 * n)()
    r = lib().cpt_decompress_batch(n, sp, lens, fp, caps, status, _stream())
    if r != OK and (raise_on_error or r not in (ECORRUPT, ECAPACITY)):
        _check(r)
    return outs, [status[i] for i in range(n)]


def stream_info(stream_bytes):
    """Header fields of a stream (CUDA or CPU uint8 tensor)."""
    head = stream_bytes[:256].cpu().contiguous()
    info = Info()
    _check(lib().cpt_stream_info(ctypes.c_void_p(head.data_ptr()), stream_bytes.numel(),
                                 ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in Info._fields_}


def decompress(stream_bytes, out=None):
    """Decompress a stream (uint8 CUDA tensor) into a (2,T,H,W) float32 tensor."""
    if not (stream_bytes.is_cuda and stream_bytes.dtype == torch.uint8):
        raise TypeError("stream must be a uint8 CUDA tensor")
    b = stream_bytes.contiguous()
    if out is None:
        info = stream_info(b)
        out = torch.empty((2, info["T"], info["H"], info["W"]), dtype=torch.float32, device=b.device)
    out = _out_field(out)
    _check(lib().cpt_decompress(_ptr(b), b.numel(), _ptr(out), out.numel(), _stream()))
    return out


def extract_trajectories(field, k):
    """Crossed space-time faces (sorted int64 codes ((g*12+type)<<1)|sign) of
    ``field`` on the fixed-point grid 2^k."""
    f = _field(field)
    _, T, H, W = f.shape
    cnt = ctypes.c_size_t()
    st = lib().cpt_extract_trajectories(_ptr(f), H, W, T, k, None, 0, ctypes.byref(cnt), _stream())
    if st not in (OK, ECAPACITY):
        _check(st)
    codes = torch.empty(max(cnt.value, 1), dtype=torch.int64, device=f.device)
    _check(lib().cpt_extract_trajectories(_ptr(f), H, W, T, k, _ptr(codes), codes.numel(),
                                          ctypes.byref(cnt), _stream()))
    return codes[:cnt.value]


def verify(a, b, k):
    """False-case counts per slice / slab, max error and PSNR of b against a."""
    fa, fb = _field(a), _field(b)
    _, T, H, W = fa.shape
    r = VerifyResult()
    _check(lib().cpt_verify(_ptr(fa), _ptr(fb), H, W, T, k, ctypes.byref(r), _stream()))
    return dict(fc_t=r.fc_t, fc_s=r.fc_s, max_err=r.max_err, psnr=r.psnr)


def tracks(field, k):
    """(Lemma-1 violations, trajectories) of ``field`` on the grid 2^k."""
    f = _field(field)
    _, T, H, W = f.shape
    bad, nt = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().cpt_tracks(_ptr(f), H, W, T, k, ctypes.byref(bad), ctypes.byref(nt), _stream()))
    return bad.value, nt.value


VERIFY_NOALLOC_MAX_VERTICES = 16647040


def verify_noalloc(a, b, k):
    """verify() through the allocation-free entry point (fields of at most
    VERIFY_NOALLOC_MAX_VERTICES vertices)."""
    fa, fb = _field(a), _field(b)
    _, T, H, W = fa.shape
    r = VerifyResult()
    _check(lib().cpt_verify_noalloc(_ptr(fa), _ptr(fb), H, W, T, k, ctypes.byref(r), _stream()))
    return dict(fc_t=r.fc_t, fc_s=r.fc_s, max_err=r.max_err, psnr=r.psnr)


def field_params(field, eb, eb_mode=0):
    """(k, eb_abs, eps') the compressor derives for ``field`` and ``eb``."""
    f = _field(field)
    _, T, H, W = f.shape
    k, ea, eps = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().cpt_field_params(_ptr(f), H, W, T, eb_mode, eb, ctypes.byref(k), ctypes.byref(ea),
                                  ctypes.byref(eps), _stream()))
    return k.value, ea.value, eps.value


TIMING_FAMILIES = {"phase": 0, "modes": 1, "reconstruct": 2, "decode": 3, "encode": 4, "extract": 5}


def timing_enable(on=True, period=1):
    """Bracket every `period`-th launch of each main kernel family with HIP
    events (resets counters); on=False disables."""
    _check(lib().cpt_timing_enable(max(int(period), 1) if on else 0))


def timing_read(family):
    """(total ms, launches, units) accumulated for a kernel family."""
    ms, n, u = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().cpt_timing_read(TIMING_FAMILIES[family], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
    return ms.value, n.value, u.value


def selector_init(seed=0, device="cuda"):
    """He-initialised fp32 selector weights (5124 values) on ``device``."""
    g = torch.Generator().manual_seed(seed)
    w = torch.zeros(SELECTOR_PARAMS, dtype=torch.float32)
    w[0:640] = torch.randn(640, generator=g) * (2.0 / 10) ** 0.5 * 0.1
    w[704:4800] = torch.randn(4096, generator=g) * (2.0 / 64) ** 0.5
    w[4864:5120] = torch.randn(256, generator=g) * (1.0 / 64) ** 0.5
    return w.to(device)


def selector_grad(w, feats, labels):
    """(gradient tensor, mean loss) of the selector network on the device."""
    n = labels.numel()
    grad = torch.empty(SELECTOR_PARAMS, dtype=torch.float32, device=w.device)
    loss = ctypes.c_float()
    _check(lib().cpt_selector_grad(_ptr(w.contiguous()), _ptr(feats.contiguous()), _ptr(labels.contiguous()), n,
                                   _ptr(grad), ctypes.byref(loss), _stream()))
    return grad, loss.value


def selector_train(feats, labels, w=None, epochs=20, batch=1024, lr=2e-3, seed=0):
    """Train the selector on the device; returns (fp32 weights, bf16 weights as
    int16 tensor, final mean loss)."""
    if w is None:
        w = selector_init(seed, feats.device)
    w = w.contiguous().clone()
    wbf = torch.empty(SELECTOR_PARAMS, dtype=torch.int16, device=w.device)
    o = TrainOptions(ctypes.sizeof(TrainOptions), epochs, batch, lr, seed)
    loss = ctypes.c_float()
    _check(lib().cpt_selector_train(_ptr(feats.contiguous()), _ptr(labels.to(torch.int32).contiguous()),
                                    labels.numel(), _ptr(w), _ptr(wbf), ctypes.byref(o), ctypes.byref(loss),
                                    _stream()))
    return w, wbf, loss.value
