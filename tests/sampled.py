"""Oracle expectations for one vertex or one block of a compressed field,
for fields too large for the oracle to compress whole.

Processing order (Sec. V, blocked form of Alg. 3): frames in order; in frame
t the three colour phases in order, block (bx, by) having colour
(bx + by) mod 3; inside a block the vertices in raster order.  When vertex v
is processed, every vertex visited before it holds its reconstructed value
and every other vertex its original value.  Given the original fixed-point
field O and the reconstructed one R (both (2, T, H, W) int32), the oracle
therefore recomputes v's bound (Alg. 4 over Alg. 2), bound code, prediction,
residual codes and reconstruction from that state alone.  The bound and the
lossless flag of v only read vertices within one step of v, so both are
evaluated on the 3x3x3 crop around v (the crop keeps the index order of its
vertices, which is all the simulation-of-simplicity tests depend on).  The
predictor class of a block is recomputed from the decision frame's original
values and the previous frame's reconstruction (Sec. VI-B).

Everything here calls the oracle; nothing reads the HIP library.
"""
import numpy as np

import oracle

TILE = 16
DMAX2 = (0, 2)
DMAX4 = (0, 1, 2, 4)


def n_classes(predictor):
    return 2 if predictor == 2 else (4 if predictor >= 3 else 1)


def group_decided(g, bt, T):
    """Mode group g (frames [g bt, (g+1) bt)) is decided at frame max(g bt, 1)
    when that frame lies inside the group and the field."""
    td = max(g * bt, 1)
    return td < min((g + 1) * bt, T)


def decision_frame(g, bt):
    return max(g * bt, 1)


def block_index(t, bx, by, tx, ty, bt, T):
    """Index of block (bx, by) of frame t's mode group in the per-block class
    array, or None when frame t's group is not decided."""
    g = t // bt
    if t == 0 or not group_decided(g, bt, T):
        return None
    nb = sum(1 for i in range(g) if group_decided(i, bt, T))
    return (nb * ty + by) * tx + bx


def block_class(modes, t, bx, by, tx, ty, predictor, bt, T):
    if t == 0:
        return 0
    if predictor == 1:
        return 1
    if n_classes(predictor) == 1:
        return 0
    bi = block_index(t, bx, by, tx, ty, bt, T)
    return 0 if bi is None else int(modes[bi])


def class_dmax(predictor, cls):
    return DMAX4[cls] if n_classes(predictor) == 4 else DMAX2[1 if cls else 0]


def visited_before(xx, yy, tt, x, y, t):
    """Mask of the vertices (xx, yy, tt) processed before vertex (x, y, t)."""
    cn = (xx // TILE + yy // TILE) % 3
    cv = (x // TILE + y // TILE) % 3
    same_t = tt == t
    same_block = (xx // TILE == x // TILE) & (yy // TILE == y // TILE)
    raster = (yy < y) | ((yy == y) & (xx < x))
    return (tt < t) | (same_t & (cn < cv)) | (same_t & same_block & raster)


def _crop(shape, x, y, t, r=1):
    _, T, H, W = shape
    return (slice(max(t - r, 0), min(t + r + 1, T)), slice(max(y - r, 0), min(y + r + 1, H)),
            slice(max(x - r, 0), min(x + r + 1, W)))


def vertex_state(O, R, x, y, t):
    """Current values and lossless flags on the 3x3x3 crop around (x, y, t)
    at the moment the vertex is processed, and its position in the crop."""
    st, sy, sx = _crop(O.shape, x, y, t)
    Oc = O[:, st, sy, sx]
    tt, yy, xx = np.meshgrid(np.arange(st.start, st.stop), np.arange(sy.start, sy.stop),
                             np.arange(sx.start, sx.stop), indexing="ij")
    cur = np.where(visited_before(xx, yy, tt, x, y, t)[None], R[:, st, sy, sx], Oc)
    flags = oracle.lossless_flags(oracle.face_masks_fixed(Oc[0], Oc[1]))
    return cur, flags, (x - sx.start, y - sy.start, t - st.start)


def expect_vertex(O, R, x, y, t, eps, cls, dmax, slc):
    """(xi, bound code, residual codes u | v << 16, reconstruction (u, v)) of
    vertex (x, y, t) in predictor class cls (d_max dmax); slc = (cx, sx, cy,
    sy), the semi-Lagrangian factors."""
    cur, flags, (cx_, cy_, ct_) = vertex_state(O, R, x, y, t)
    xi = oracle.vertex_bound(cur[0], cur[1], flags, cx_, cy_, ct_, eps)
    code = oracle.xi_code(eps, xi)
    ou, ov = int(O[0, t, y, x]), int(O[1, t, y, x])
    if code == oracle.XLOSSLESS:
        return xi, code, 0, (ou, ov)
    xt = eps >> code
    if cls == 0:
        x0, y0 = (x // TILE) * TILE, (y // TILE) * TILE
        pu = oracle.lorenzo3(R[0, t], R[0, t - 1] if t > 0 else None, x, y, x0, y0)
        pv = oracle.lorenzo3(R[1, t], R[1, t - 1] if t > 0 else None, x, y, x0, y0)
    else:
        pu, pv = oracle.sl_predict(R[0, t - 1], R[1, t - 1], x, y, *slc, dmax=dmax)
    qu, ru = oracle.quantize(ou, pu, xt)
    qv, rv = oracle.quantize(ov, pv, xt)
    return xi, code, qu | (qv << 16), (ru, rv)


def face_masks_kept(O, R, x, y, t):
    """Whether every face of the 3x3x3 crop around (x, y, t) has the same SoS
    status in the original and the reconstructed field."""
    st, sy, sx = _crop(O.shape, x, y, t)
    a = oracle.face_masks_fixed(O[0, st, sy, sx], O[1, st, sy, sx])
    b = oracle.face_masks_fixed(R[0, st, sy, sx], R[1, st, sy, sx])
    return np.array_equal(a, b)


def block_flags(O, t, bx, by):
    """Lossless flags of block (bx, by) of frame t in an (H, W) plane (zero
    elsewhere), from the faces of the block and its one-vertex rim."""
    _, T, H, W = O.shape
    x0, y0 = bx * TILE, by * TILE
    x1, y1 = min(x0 + TILE, W), min(y0 + TILE, H)
    st = slice(max(t - 1, 0), min(t + 2, T))
    sy, sx = slice(max(y0 - 1, 0), min(y1 + 1, H)), slice(max(x0 - 1, 0), min(x1 + 1, W))
    fl = oracle.lossless_flags(oracle.face_masks_fixed(O[0, st, sy, sx], O[1, st, sy, sx]))
    plane = np.zeros((H, W), dtype=np.uint8)
    plane[y0:y1, x0:x1] = fl[t - st.start, y0 - sy.start:y1 - sy.start, x0 - sx.start:x1 - sx.start]
    return plane


def expect_block(O, R, t, bx, by, k, eps, predictor, mode_bt, dt_dx, dt_dy, selector_w=None):
    """(class, features) of block (bx, by) at decision frame t."""
    return oracle.block_mode(O[0, t], O[1, t], R[0, t - 1], R[1, t - 1], block_flags(O, t, bx, by), bx, by,
                             k, eps, predictor=predictor, mode_bt=mode_bt, dt_dx=dt_dx, dt_dy=dt_dy,
                             selector_w=selector_w)
