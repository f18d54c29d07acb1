"""CPU oracle for the trajectory-preserving compressor (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``libcpo.so``, a plain,
single-threaded C implementation written from the paper (arXiv 2510.25143),
which shares no code with the HIP library.  Arrays are numpy, host memory.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcpo.so")
_SRC = os.path.join(_HERE, "cpo.c")

OK, EINVAL, ENOMEM, ECORRUPT, ECAPACITY = 0, -1, -2, -3, -4
QR = 512
XLOSSLESS = 24
NFEAT, HID, NCLS = 10, 64, 4
NW = 64 * 10 + 64 + 64 * 64 + 64 + 4 * 64 + 4


def build(force=True):
    """Compile libcpo.so with gcc (-ffp-contract=off keeps fmaf explicit)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
           "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Options(ctypes.Structure):
    _fields_ = [("predictor", ctypes.c_int32), ("mode_bt", ctypes.c_int32),
                ("eb_mode", ctypes.c_int32), ("backend", ctypes.c_int32),
                ("dt_dx", ctypes.c_double), ("dt_dy", ctypes.c_double),
                ("selector_w", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("T", ctypes.c_int32),
                ("k", ctypes.c_int32), ("eb_abs", ctypes.c_double), ("eps", ctypes.c_int64),
                ("predictor", ctypes.c_int32), ("mode_bt", ctypes.c_int32),
                ("K", ctypes.c_int32), ("R", ctypes.c_int32),
                ("cx", ctypes.c_int64), ("sx", ctypes.c_int64), ("cy", ctypes.c_int64),
                ("sy", ctypes.c_int64), ("total_len", ctypes.c_uint64),
                ("n_q", ctypes.c_uint64), ("n_raw", ctypes.c_uint64),
                ("backend", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, sz, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        sig = {
            "cpo_params": (ctypes.c_int, [P, i32, i32, i32, i32, dbl, P, P, P]),
            "cpo_to_fixed": (None, [P, sz, i32, P]),
            "cpo_sos_edge": (ctypes.c_int, [i32, i32, i32, i32]),
            "cpo_face_masks": (None, [P, P, i32, i32, i32, P]),
            "cpo_extract_fixed": (ctypes.c_int, [P, P, i32, i32, i32, P, sz, P]),
            "cpo_extract": (ctypes.c_int, [P, i32, i32, i32, i32, P, sz, P]),
            "cpo_face_vertices": (None, [i32, P, P, P]),
            "cpo_lossless_flags": (None, [P, i32, i32, i32, P]),
            "cpo_incident_faces": (ctypes.c_int, [i32, i32, i32, i32, i32, i32, P]),
            "cpo_alg2": (i64, [i64, i64, i64, i64, i64, i64]),
            "cpo_sl_predict": (None, [P, P, i32, i32, i32, i32, i64, i64, i64, i64, i32, i32, P, P]),
            "cpo_sl_factor": (None, [dbl, i32, P, P]),
            "cpo_bilinear": (i64, [P, i32, i32, i64, i64]),
            "cpo_quantize": (i32, [i64, i64, i64, P]),
            "cpo_lorenzo3": (i64, [P, P, i32, i32, i32, i32, i32]),
            "cpo_choose": (ctypes.c_int, [P, i32]),
            "cpo_xi_code": (i32, [i64, i64]),
            "cpo_vertex_bound": (i64, [P, P, P, i32, i32, i32, i32, i32, i32, i64]),
            "cpo_block_mode": (ctypes.c_int, [P, P, P, P, P, i32, i32, i32, i32, P, i32, i64, P]),
            "cpo_block_scores": (ctypes.c_int, [P, P, P, P, P, i32, i32, i32, i32, P, i32, i64, P]),
            "cpo_canonical_codes": (None, [P, i32, P]),
            "cpo_tlog": (i64, [i32]),
            "cpo_score": (i64, [P, i32, i32, i32, i32, i32]),
            "cpo_huffman_lengths": (ctypes.c_int, [P, i32, i32, P]),
            "cpo_mlp_forward": (ctypes.c_int, [P, P, P]),
            "cpo_mlp_loss_grad": (dbl, [P, P, P, i32, P]),
            "cpo_mlp_loss_grad_exact": (dbl, [P, P, P, i32, P]),
            "cpo_compress_ex": (ctypes.c_int, [P, i32, i32, i32, dbl, P, P, sz, P, P, P, P, P, P, P]),
            "cpo_compress_bound": (sz, [i32, i32, i32]),
            "cpo_zbe_bound": (sz, [sz]),
            "cpo_zbe_encode": (ctypes.c_int, [P, sz, P, sz, P]),
            "cpo_zbe_decode": (ctypes.c_int, [P, sz, P, sz, P]),
            "cpo_stream_info": (ctypes.c_int, [P, sz, P]),
            "cpo_decompress": (ctypes.c_int, [P, sz, P]),
            "cpo_verify": (ctypes.c_int, [P, P, i32, i32, i32, i32, P, P, P, P]),
            "cpo_tracks": (ctypes.c_int, [P, i32, i32, i32, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(field):
    a = np.ascontiguousarray(field, dtype=np.float32)
    assert a.ndim == 4 and a.shape[0] == 2, "field must be (2,T,H,W)"
    return a


def params(field, eb, eb_mode=0):
    a = _f32(field)
    _, T, H, W = a.shape
    k, ea, eps = ctypes.c_int(), ctypes.c_double(), ctypes.c_int64()
    st = lib().cpo_params(_p(a), H, W, T, eb_mode, eb, ctypes.byref(k), ctypes.byref(ea),
                          ctypes.byref(eps))
    if st:
        raise ValueError("cpo_params failed: %d" % st)
    return k.value, ea.value, eps.value


def to_fixed(x, k):
    a = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(a.shape, dtype=np.int32)
    lib().cpo_to_fixed(_p(a), a.size, k, _p(out))
    return out


def face_masks_fixed(U, V):
    U = np.ascontiguousarray(U, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.int32)
    T, H, W = U.shape
    m = np.empty((T, H, W), dtype=np.uint32)
    lib().cpo_face_masks(_p(U), _p(V), H, W, T, _p(m))
    return m


def extract_fixed(U, V):
    U = np.ascontiguousarray(U, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.int32)
    T, H, W = U.shape
    cnt = ctypes.c_size_t()
    lib().cpo_extract_fixed(_p(U), _p(V), H, W, T, None, 0, ctypes.byref(cnt))
    out = np.empty(max(cnt.value, 1), dtype=np.uint64)
    st = lib().cpo_extract_fixed(_p(U), _p(V), H, W, T, _p(out), out.size, ctypes.byref(cnt))
    assert st == OK
    return out[:cnt.value]


def extract(field, k):
    a = _f32(field)
    _, T, H, W = a.shape
    cnt = ctypes.c_size_t()
    st = lib().cpo_extract(_p(a), H, W, T, k, None, 0, ctypes.byref(cnt))
    if st not in (OK, ECAPACITY):
        raise ValueError("cpo_extract failed: %d" % st)
    out = np.empty(max(cnt.value, 1), dtype=np.uint64)
    st = lib().cpo_extract(_p(a), H, W, T, k, _p(out), out.size, ctypes.byref(cnt))
    assert st == OK
    return out[:cnt.value]


def face_vertices(f):
    dx, dy, dt = (np.zeros(3, dtype=np.int32) for _ in range(3))
    lib().cpo_face_vertices(f, _p(dx), _p(dy), _p(dt))
    return list(zip(dx.tolist(), dy.tolist(), dt.tolist()))


def lossless_flags(masks):
    m = np.ascontiguousarray(masks, dtype=np.uint32)
    T, H, W = m.shape
    fl = np.empty((T, H, W), dtype=np.uint8)
    lib().cpo_lossless_flags(_p(m), H, W, T, _p(fl))
    return fl


def incident_faces(H, W, T, x, y, t):
    nb = np.zeros((36, 2), dtype=np.int32)
    n = lib().cpo_incident_faces(H, W, T, x, y, t, _p(nb))
    return nb[:n]


def alg2(u0, u1, u2, v0, v1, v2):
    return lib().cpo_alg2(int(u0), int(u1), int(u2), int(v0), int(v1), int(v2))


def sl_factor(dt_dx, k):
    c, s = ctypes.c_int64(), ctypes.c_int64()
    lib().cpo_sl_factor(dt_dx, k, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def bilinear(F, px, py):
    F = np.ascontiguousarray(F, dtype=np.int32)
    H, W = F.shape
    return lib().cpo_bilinear(_p(F), H, W, int(px), int(py))


def sl_predict(Up, Vp, x, y, cx, sx, cy, sy, dmax=2, nmax=32):
    Up = np.ascontiguousarray(Up, dtype=np.int32)
    Vp = np.ascontiguousarray(Vp, dtype=np.int32)
    H, W = Up.shape
    pu, pv = ctypes.c_int64(), ctypes.c_int64()
    lib().cpo_sl_predict(_p(Up), _p(Vp), H, W, x, y, cx, sx, cy, sy, dmax, nmax,
                         ctypes.byref(pu), ctypes.byref(pv))
    return pu.value, pv.value


def quantize(x, pred, xt):
    r = ctypes.c_int64()
    code = lib().cpo_quantize(int(x), int(pred), int(xt), ctypes.byref(r))
    return code, r.value


def lorenzo3(cur_t, prev, x, y, x0, y0):
    c = np.ascontiguousarray(cur_t, dtype=np.int32)
    H, W = c.shape
    p = None if prev is None else np.ascontiguousarray(prev, dtype=np.int32)
    return lib().cpo_lorenzo3(_p(c), None if p is None else _p(p), W, x, y, x0, y0)


def choose(R):
    r = np.ascontiguousarray(R, dtype=np.int64)
    return lib().cpo_choose(_p(r), r.size)


def xi_code(eps, xi):
    return lib().cpo_xi_code(int(eps), int(xi))


def vertex_bound(U, V, flags, x, y, t, eps):
    """Alg. 4 bound of vertex (x, y, t) on the current values U, V
    ((T, H, W) int32: reconstructed where already processed, original
    elsewhere) and the lossless flags (T, H, W)."""
    U = np.ascontiguousarray(U, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.int32)
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    T, H, W = U.shape
    assert V.shape == U.shape and fl.shape == U.shape
    assert 0 <= x < W and 0 <= y < H and 0 <= t < T
    return lib().cpo_vertex_bound(_p(U), _p(V), _p(fl), H, W, T, x, y, t, int(eps))


def block_mode(Ut, Vt, Up, Vp, flags_t, bx, by, k, eps, predictor=2, mode_bt=1, dt_dx=1.0,
               dt_dy=1.0, selector_w=None):
    """Predictor class of block (bx, by) at a decision frame, from the
    frame's original planes, the previous frame's reconstructed planes and
    the frame's lossless flags ((H, W) each); returns (class, features)."""
    planes = [np.ascontiguousarray(a, dtype=np.int32) for a in (Ut, Vt, Up, Vp)]
    fl = np.ascontiguousarray(flags_t, dtype=np.uint8)
    H, W = planes[0].shape
    assert all(a.shape == (H, W) for a in planes) and fl.shape == (H, W)
    o, keep = _opts(predictor, mode_bt, 0, dt_dx, dt_dy, selector_w)
    feat = np.zeros(NFEAT, dtype=np.float32)
    r = lib().cpo_block_mode(*[_p(a) for a in planes], _p(fl), H, W, bx, by, ctypes.byref(o), k,
                             int(eps), _p(feat))
    del keep
    if r < 0:
        raise ValueError("cpo_block_mode failed: %d" % r)
    return r, feat


def block_scores(Ut, Vt, Up, Vp, flags_t, bx, by, k, eps, predictor=2, mode_bt=1, dt_dx=1.0,
                 dt_dy=1.0):
    """Trial scores (Q16 bits per sample) of every class of the exhaustive
    choice for block (bx, by), and the class chosen; planes as block_mode."""
    planes = [np.ascontiguousarray(a, dtype=np.int32) for a in (Ut, Vt, Up, Vp)]
    fl = np.ascontiguousarray(flags_t, dtype=np.uint8)
    H, W = planes[0].shape
    assert all(a.shape == (H, W) for a in planes) and fl.shape == (H, W)
    o, keep = _opts(predictor, mode_bt, 0, dt_dx, dt_dy, None)
    K = 2 if predictor == 2 else 4
    R = np.zeros(K, dtype=np.int64)
    r = lib().cpo_block_scores(*[_p(a) for a in planes], _p(fl), H, W, bx, by, ctypes.byref(o), k,
                               int(eps), _p(R))
    del keep
    if r < 0:
        raise ValueError("cpo_block_scores failed: %d" % r)
    return R, r


def canonical_codes(lengths):
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = np.zeros(ln.size, dtype=np.uint32)
    lib().cpo_canonical_codes(_p(ln), ln.size, _p(out))
    return out


def tlog(h):
    return lib().cpo_tlog(int(h))


def score(hist, n, L, K, bt):
    h = np.ascontiguousarray(hist, dtype=np.int32)
    return lib().cpo_score(_p(h), h.size, n, L, K, bt)


def huffman_lengths(counts, maxlen=16):
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    out = np.zeros(c.size, dtype=np.uint8)
    st = lib().cpo_huffman_lengths(_p(c), c.size, maxlen, _p(out))
    if st:
        raise ValueError("huffman failed %d" % st)
    return out


def mlp_forward(w_bf16, x):
    w = np.ascontiguousarray(w_bf16, dtype=np.uint16)
    xs = np.ascontiguousarray(x, dtype=np.float32)
    lg = np.zeros(NCLS, dtype=np.float32)
    c = lib().cpo_mlp_forward(_p(w), _p(xs), _p(lg))
    return c, lg


def mlp_loss_grad(w, x, labels, exact=False):
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    g = np.zeros(NW, dtype=np.float64)
    f = lib().cpo_mlp_loss_grad_exact if exact else lib().cpo_mlp_loss_grad
    loss = f(_p(w), _p(x), _p(lab), lab.size, _p(g))
    return loss, g


def _opts(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend=0):
    o = Options(predictor, mode_bt, eb_mode, backend, dt_dx, dt_dy, None)
    keep = None
    if selector_w is not None:
        keep = np.ascontiguousarray(selector_w, dtype=np.uint16)
        o.selector_w = keep.ctypes.data
    return o, keep


def compress(field, eb, predictor=2, mode_bt=1, eb_mode=0, dt_dx=1.0, dt_dy=1.0,
             selector_w=None, debug=False, backend=0):
    """Returns the stream bytes (numpy uint8); with debug=True also a dict of
    per-vertex bounds, bound codes, residual codes, block modes and features.
    backend=1 adds the zero-byte-elision stage after Huffman coding."""
    a = _f32(field)
    _, T, H, W = a.shape
    N = T * H * W
    o, keep = _opts(predictor, mode_bt, eb_mode, dt_dx, dt_dy, selector_w, backend)
    cap = lib().cpo_compress_bound(H, W, T)
    out = np.empty(cap, dtype=np.uint8)
    ln = ctypes.c_size_t()
    nblk_max = T * ((H + 15) // 16) * ((W + 15) // 16)
    dbg = None
    if debug:
        dbg = dict(xi=np.empty(N, np.int32), xcode=np.empty(N, np.uint8),
                   qcode=np.empty(N, np.uint32), modes=np.zeros(max(nblk_max, 1), np.uint8),
                   feats=np.zeros((max(nblk_max, 1), NFEAT), np.float32))
        nb = ctypes.c_size_t()
        st = lib().cpo_compress_ex(_p(a), H, W, T, eb, ctypes.byref(o), _p(out), cap,
                                   ctypes.byref(ln), _p(dbg["xi"]), _p(dbg["xcode"]),
                                   _p(dbg["qcode"]), _p(dbg["modes"]), _p(dbg["feats"]),
                                   ctypes.byref(nb))
        dbg["modes"] = dbg["modes"][:nb.value]
        dbg["feats"] = dbg["feats"][:nb.value]
    else:
        st = lib().cpo_compress_ex(_p(a), H, W, T, eb, ctypes.byref(o), _p(out), cap,
                                   ctypes.byref(ln), None, None, None, None, None, None)
    del keep
    if st:
        raise ValueError("cpo_compress failed: %d" % st)
    out = out[:ln.value].copy()
    return (out, dbg) if debug else out


def zbe_encode(b):
    """The lossless stage on a Huffman stream: the container bytes."""
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.empty(lib().cpo_zbe_bound(b.size), dtype=np.uint8)
    n = ctypes.c_size_t()
    st = lib().cpo_zbe_encode(_p(b), b.size, _p(out), out.size, ctypes.byref(n))
    if st:
        raise ValueError("cpo_zbe_encode failed: %d" % st)
    return out[:n.value].copy()


def zbe_decode_status(c, cap=None):
    """(status, inner stream or None) of a container, without raising."""
    c = np.ascontiguousarray(c, dtype=np.uint8)
    n = ctypes.c_size_t()
    st = lib().cpo_zbe_decode(_p(c), c.size, None, 0, ctypes.byref(n))
    if st != ECAPACITY:
        return st, None
    out = np.empty(max(n.value, 1), dtype=np.uint8)
    st = lib().cpo_zbe_decode(_p(c), c.size, _p(out), out.size, ctypes.byref(n))
    return st, (out[:n.value] if st == OK else None)


def stream_info(b):
    b = np.ascontiguousarray(b, dtype=np.uint8)
    info = Info()
    st = lib().cpo_stream_info(_p(b), b.size, ctypes.byref(info))
    if st:
        raise ValueError("corrupt stream: %d" % st)
    return {f: getattr(info, f) for f, _ in Info._fields_}


def decompress_status(b):
    """(status, field or None) without raising."""
    b = np.ascontiguousarray(b, dtype=np.uint8)
    info = Info()
    st = lib().cpo_stream_info(_p(b), b.size, ctypes.byref(info))
    if st:
        return st, None
    out = np.empty((2, info.T, info.H, info.W), dtype=np.float32)
    st = lib().cpo_decompress(_p(b), b.size, _p(out))
    return st, (out if st == OK else None)


def decompress(b):
    st, out = decompress_status(b)
    if st:
        raise ValueError("cpo_decompress failed: %d" % st)
    return out


def verify(a, b, k):
    a = _f32(a)
    b = _f32(b)
    _, T, H, W = a.shape
    ft, fs = ctypes.c_uint64(), ctypes.c_uint64()
    me, ps = ctypes.c_double(), ctypes.c_double()
    st = lib().cpo_verify(_p(a), _p(b), H, W, T, k, ctypes.byref(ft), ctypes.byref(fs),
                     ctypes.byref(me), ctypes.byref(ps))
    if st:
        raise ValueError("cpo_verify failed: %d" % st)
    return dict(fc_t=ft.value, fc_s=fs.value, max_err=me.value, psnr=ps.value)


def tracks(field, k):
    a = _f32(field)
    _, T, H, W = a.shape
    bad, nt = ctypes.c_uint64(), ctypes.c_uint64()
    st = lib().cpo_tracks(_p(a), H, W, T, k, ctypes.byref(bad), ctypes.byref(nt))
    assert st == OK
    return bad.value, nt.value
