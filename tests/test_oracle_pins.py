"""Pins of oracle functions that the other pin files leave open.

* The semi-Lagrangian displacement factor (Sec. VI-A, fixed-point reading) at
  time steps that are not powers of two, against exact rationals.
* The micro-encoding trial of Sec. VI-B: closed-form scores on fields where
  one predictor is exact, the trial's histogram equal to the one the real
  encoding of the block writes (which pins the stride-2 sampling, the pooling
  of u and v and the write-back of reconstructed values), and independence
  from the lossless flags.
* The selector's block features, hand-computed on a constant block and on a
  block drifting uniformly in time.
* The check of Sec. IV-A / Sec. VII-A: false-case counts against a brute-force
  enumeration of the prism split with a generic symbolic SoS evaluator, and
  PSNR and maximum error by hand.
* Canonical Huffman codewords by hand.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_mesh import brute_faces, generic_crossed


# ------------------------------------------------------------- SL factor
def test_sl_factor_non_power_of_two(ora):
    """c / 2^s is dt/dx 2^(16-k) rounded to the nearest integer multiple of
    2^-s, with c normalised into [2^30, 2^31) unless s hits its cap of 62 (a
    factor that rounds to 0 there is stored as c = s = 0) or the factor
    itself reaches 2^31 - 1 (then c = 2^31 - 1, s = 0)."""
    rng = np.random.default_rng(11)
    vals = list(rng.uniform(1e-4, 50.0, 300)) + list(np.exp(rng.uniform(-40, 25, 300)))
    vals += [0.5 / 29.7, 0.016835, 1.0 / 3.0, 0.1, 7.0, 1e-30, 3e8, 5e-324, 1e-300, 2.0 ** -47]
    ks = rng.integers(-60, 121, len(vals))
    for dt, k in zip(vals, ks):
        dt, k = float(dt), int(k)
        c, s = ora.sl_factor(dt, k)
        f = Fraction(dt) * Fraction(2) ** (16 - k)
        if f >= 2 ** 31 - 1:
            assert (c, s) == (2 ** 31 - 1, 0), (dt, k)
            continue
        assert 0 <= c < 2 ** 31 and 0 <= s <= 62, (dt, k, c, s)
        if c == 0:   # too small for 62 fraction bits: stored as no displacement
            assert s == 0 and f * 2 ** 62 <= Fraction(1, 2), (dt, k)
            continue
        assert abs(c - f * 2 ** s) <= Fraction(1, 2), (dt, k, c, s)
        assert c >= 2 ** 30 or s == 62, (dt, k, c, s)
    assert ora.sl_factor(0.0, 13) == (0, 0)


# -------------------------------------------------------------- the trial
K2_META = 65536 // 512     # log2(2) bits over the 2 x 256 samples of a 16x16x1 block
K4_META = 2 * 65536 // 512


def test_trial_score_time_constant_field_is_metadata_only(ora):
    """A field constant in time makes every Lorenzo residual zero (also at the
    block edges, where both frames are padded alike): one histogram bin, no
    unpredictable sample, so the score is the metadata share alone."""
    rng = np.random.default_rng(3)
    H = W = 40
    U = rng.integers(-5000, 5000, (H, W)).astype(np.int32)
    V = rng.integers(-5000, 5000, (H, W)).astype(np.int32)
    fl = np.zeros((H, W), np.uint8)
    for bx, by in [(0, 0), (1, 1), (2, 2), (2, 0)]:   # full and ragged (8-wide) blocks
        R, _ = ora.block_scores(U, V, U, V, fl, bx, by, k=13, eps=50, predictor=2,
                                dt_dx=0.37, dt_dy=0.21)
        assert R[0] == K2_META, (bx, by, R)
        R4, _ = ora.block_scores(U, V, U, V, fl, bx, by, k=13, eps=50, predictor=3,
                                 dt_dx=0.37, dt_dy=0.21)
        assert R4[0] == K4_META, (bx, by, R4)


def _sl_exact_planes(H, W, w):
    """u = 2^22 everywhere (one cell per step with k = 13 and dt/dx = 2^-9),
    v(x, y, t) = w h(x - t) g(y): a pure translation by one cell in x.  All
    values are multiples of the bin width w = 2 eps' + 1 except u, which is
    constant, so no reconstruction differs from its original."""
    h = lambda s: (s * s * 7) % 23 - 11
    g = lambda y: (y * 5) % 13 - 6
    U = np.full((2, H, W), 1 << 22, np.int32)
    V = np.array([[[w * h(x - t) * g(y) for x in range(W)] for y in range(H)] for t in range(2)],
                 np.int32)
    return U, V


def test_trial_score_uniform_translation_favours_semi_lagrangian(ora):
    """On the one-cell translation every semi-Lagrangian class predicts both
    components exactly (RK2, d_inf = 1 cell <= d_max for d_max 1, 2 and 4),
    so those scores are the metadata share alone, the Lorenzo score is
    larger, and the choice is the lowest semi-Lagrangian class."""
    H, W, eps = 48, 64, 2
    U, V = _sl_exact_planes(H, W, 2 * eps + 1)
    fl = np.zeros((H, W), np.uint8)
    for bx, by in [(1, 0), (2, 1), (3, 2)]:
        R, cls = ora.block_scores(U[1], V[1], U[0], V[0], fl, bx, by, k=13, eps=eps, predictor=2,
                                  dt_dx=2.0 ** -9, dt_dy=0.0)
        assert R[1] == K2_META and R[0] > R[1] and cls == 1, (bx, by, R)
        R4, cls4 = ora.block_scores(U[1], V[1], U[0], V[0], fl, bx, by, k=13, eps=eps, predictor=3,
                                    dt_dx=2.0 ** -9, dt_dy=0.0)
        assert list(R4[1:]) == [K4_META] * 3 and R4[0] > K4_META and cls4 == 1, (bx, by, R4)


def _offset_field(seed, H, W, T):
    """u, v near +1000 with fine-grained noise: all u and all v positive, so
    the same-sign relaxation of Alg. 2 lifts almost every face bound to eps'
    (a face whose three current vectors happen to be collinear still gets 0)."""
    rng = np.random.default_rng(seed)
    base = rng.normal(0, 3.0, (2, 1, H, W))
    f = 1000.0 + base + np.cumsum(rng.normal(0, 0.7, (2, T, H, W)), axis=1)
    return f.astype(np.float32)


@pytest.mark.parametrize("pred,cls", [(0, 0), (1, 1)])
def test_trial_histogram_equals_real_encoding(ora, pred, cls):
    """With the bound equal to eps' at every vertex, the trial of a class is
    the real encoding of that block under that predictor: its score must be
    the score of the histogram of the residual codes compression writes for
    the block, on the points whose offsets in the block are both even, u and
    v pooled, code 0 (unpredictable) counted apart.  A trial that sampled
    odd points, left out v, or predicted Lorenzo from originals instead of
    written-back reconstructions gives another histogram."""
    H, W, T, eb = 40, 56, 3, 1e-3
    f = _offset_field(5, H, W, T)
    dt = 1e-3
    k, _, eps = ora.params(f, eb)
    stream, dbg = ora.compress(f, eb, predictor=pred, dt_dx=dt, dt_dy=dt, debug=True)
    N = T * H * W
    xcode = dbg["xcode"].reshape(T, H, W)
    rec = ora.decompress(stream)
    Fu, Fv = ora.to_fixed(f[0], k), ora.to_fixed(f[1], k)
    Ru, Rv = ora.to_fixed(rec[0], k), ora.to_fixed(rec[1], k)
    q = dbg["qcode"].reshape(T, H, W)
    qu, qv = (q[1] & 0xFFFF).astype(np.int64), (q[1] >> 16).astype(np.int64)
    fl = np.zeros((H, W), np.uint8)
    changed = compared = 0
    for by in range((H + 15) // 16):
        for bx in range((W + 15) // 16):
            x0, y0 = 16 * bx, 16 * by
            if (xcode[1, y0:y0 + 16, x0:x0 + 16] != 0).any():
                continue   # a reduced or lossless bound there: the trial (global eps') differs
            compared += 1
            codes = np.concatenate([qu[y0:y0 + 16:2, x0:x0 + 16:2].ravel(),
                                    qv[y0:y0 + 16:2, x0:x0 + 16:2].ravel()])
            hist = np.bincount(codes[codes != 0], minlength=1024)
            L = int((codes == 0).sum())
            want = ora.score(hist, int(len(codes) - L), L, 2, 1)
            R, _ = ora.block_scores(Fu[1], Fv[1], Ru[0], Rv[0], fl, bx, by, k, eps, predictor=2,
                                    dt_dx=dt, dt_dy=dt)
            assert R[cls] == want, (bx, by, R, want)
            odd = np.concatenate([qu[y0 + 1:y0 + 16:2, x0 + 1:x0 + 16:2].ravel(),
                                  qv[y0 + 1:y0 + 16:2, x0 + 1:x0 + 16:2].ravel()])
            changed += int(sorted(odd.tolist()) != sorted(codes.tolist()))
    assert compared >= 6, compared
    assert changed > 0, "the odd points must differ somewhere for the pin to bite"
    assert N > 0


def test_trial_ignores_lossless_flags(ora):
    rng = np.random.default_rng(9)
    H, W = 32, 48
    f = _offset_field(9, H, W, 2)
    k, _, eps = ora.params(f, 1e-3)
    U, V = ora.to_fixed(f[0], k), ora.to_fixed(f[1], k)
    none = np.zeros((H, W), np.uint8)
    some = (rng.random((H, W)) < 0.3).astype(np.uint8)
    for bx, by in [(0, 0), (1, 1), (2, 0)]:
        a, _ = ora.block_scores(U[1], V[1], U[0], V[0], none, bx, by, k, eps, predictor=3, dt_dx=1e-3,
                                dt_dy=1e-3)
        b, _ = ora.block_scores(U[1], V[1], U[0], V[0], some, bx, by, k, eps, predictor=3, dt_dx=1e-3,
                                dt_dy=1e-3)
        assert list(a) == list(b)


# --------------------------------------------------------- block features
def test_block_features_constant_block(ora):
    """u = 2^22, v = -2^21 in both frames, k = 13, dt/dx = dt/dy = 2^-9:
    displacements of +1 and -1/2 cell, every residual and gradient zero,
    the top quarter of the block flagged."""
    H = W = 32
    U = np.full((H, W), 1 << 22, np.int32)
    V = np.full((H, W), -(1 << 21), np.int32)
    fl = np.zeros((H, W), np.uint8)
    fl[16:20, 16:32] = 1
    _, feat = ora.block_mode(U, V, U, V, fl, 1, 1, k=13, eps=100, predictor=2,
                             dt_dx=2.0 ** -9, dt_dy=2.0 ** -9)
    assert list(feat) == [0.0, 0.0, 0.0, 1.0, 1.0, 0.25, 0.0, 0.0, 1.0, -0.5]


def test_block_features_uniform_drift_block(ora):
    """Frame t = frame t-1 + (37, -23) on an affine field (slopes 3, -2 in
    u and 1, 5 in v), no displacement (dt = 0), eps' = 3, one 16x16 block:
    mean |f_t - f_{t-1}| = 60 / (2 * 3) = 10; the Lorenzo residual on
    originals is zero except the drift at the block corner (60 / (2 * 256 *
    3) -> 10/256 in Q8); gradients 240 (3 + 2 + 1 + 5) / (512 * 3) -> 440/256;
    the semi-Lagrangian residual is the drift at every stride-4 point (10)
    and the stride-4 Lorenzo residual is the corner alone (60 / 96 -> 0.625)."""
    H = W = 16
    y, x = np.mgrid[0:H, 0:W]
    Up = (3 * x - 2 * y + 100).astype(np.int32)
    Vp = (1 * x + 5 * y - 40).astype(np.int32)
    Ut, Vt = Up + 37, Vp - 23
    fl = np.zeros((H, W), np.uint8)
    _, feat = ora.block_mode(Ut, Vt, Up, Vp, fl, 0, 0, k=13, eps=3, predictor=2, dt_dx=0.0, dt_dy=0.0)
    want = [10.0, 10 / 256, 440 / 256, 0.0, 0.0, 0.0, 10.0, 0.625, 0.0, 0.0]
    assert list(feat) == want, list(feat)


# ------------------------------------------------------------------ check
def _brute_false_cases(a, b, H, W, T):
    """FC_t / FC_s by brute force: every face of the prism split, crossed
    status and sign from the generic SoS expansion, on both fields."""
    Ua, Va = a[0].ravel().astype(int), a[1].ravel().astype(int)
    Ub, Vb = b[0].ravel().astype(int), b[1].ravel().astype(int)
    ft = fs = 0
    for tri in brute_faces(H, W, T):
        ca, sa = generic_crossed(Ua, Va, tri)
        cb, sb = generic_crossed(Ub, Vb, tri)
        if ca != cb or (ca and sa != sb):
            if len({g // (H * W) for g in tri}) == 1:
                ft += 1
            else:
                fs += 1
    return ft, fs


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_verify_counts_flipped_faces(ora, seed):
    rng = np.random.default_rng(100 + seed)
    H, W, T = 4, 5, 3
    a = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
    b = a.copy()
    for _ in range(3):   # perturb three vertices, components independently
        t, yy, xx = rng.integers(0, T), rng.integers(0, H), rng.integers(0, W)
        b[:, t, yy, xx] = rng.integers(-3, 4, 2)
    want = _brute_false_cases(a, b, H, W, T)
    got = ora.verify(a, b, 0)
    assert (got["fc_t"], got["fc_s"]) == want
    assert got["max_err"] == float(np.abs(a - b).max())


def test_verify_counts_sign_changes_of_crossed_faces(ora):
    """Swapping u and v mirrors every vector: a crossed face stays crossed
    (the triangle still holds the origin) with the opposite sign, so every
    crossed face is a false case although none changes status."""
    rng = np.random.default_rng(7)
    H, W, T = 4, 5, 3
    a = rng.integers(-1000, 1001, (2, T, H, W)).astype(np.float32)
    b = a[::-1].copy()
    codes = ora.extract(a, 0)
    assert len(codes) > 0
    want = _brute_false_cases(a, b, H, W, T)
    assert sum(want) == len(codes)
    got = ora.verify(a, b, 0)
    assert (got["fc_t"], got["fc_s"]) == want


def test_verify_counts_are_nonzero_somewhere(ora):
    """The brute-force counts above cover both kinds of false case."""
    seen_t = seen_s = False
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        H, W, T = 4, 5, 3
        a = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
        b = a.copy()
        for _ in range(3):
            t, yy, xx = rng.integers(0, T), rng.integers(0, H), rng.integers(0, W)
            b[:, t, yy, xx] = rng.integers(-3, 4, 2)
        ft, fs = _brute_false_cases(a, b, H, W, T)
        seen_t |= ft > 0
        seen_s |= fs > 0
    assert seen_t and seen_s


def test_verify_psnr_and_max_error_by_hand(ora):
    """Range of the first field 2 (values -1..1), four of the 16 values off
    by 1/2 (two of them widen the second field's range to 3): MSE 1/16,
    PSNR = 20 log10 2 - 10 log10 (1/16) = 60 log10 2."""
    a = np.zeros((2, 2, 2, 2), np.float32)
    a[0, 0, 0, 0], a[1, 1, 1, 1] = -1.0, 1.0
    b = a.copy()
    b[0, 0, 0, 0] -= 0.5
    b[1, 1, 1, 1] += 0.5
    b[0, 0, 1, 1] += 0.5
    b[1, 1, 0, 0] -= 0.5
    r = ora.verify(a, b, 4)
    assert r["max_err"] == 0.5
    assert abs(r["psnr"] - 18.061799739838872) < 1e-12
    assert math.isinf(ora.verify(a, a, 4)["psnr"])


def test_verify_rejects_grid_beyond_24_bits(ora):
    a = np.zeros((2, 2, 2, 2), np.float32)
    a[0, 0, 0, 0] = 2.0 ** 20
    with pytest.raises(ValueError):
        ora.verify(a, a, 4)


# ------------------------------------------------------- canonical codes
def test_canonical_codes_by_hand(ora):
    assert list(ora.canonical_codes([1, 2, 3, 3])) == [0b0, 0b10, 0b110, 0b111]
    # symbols ordered by (length, symbol): 1 -> 0, 3 -> 10, 0 -> 110, 2 -> 111
    assert list(ora.canonical_codes([3, 1, 3, 2, 0])) == [0b110, 0b0, 0b111, 0b10, 0]
    # a longer example: lengths 2,2,3,3,3,4,4 -> 00 01 100 101 110 1110 1111
    assert list(ora.canonical_codes([4, 2, 3, 2, 3, 4, 3])) == [0b1110, 0b00, 0b100, 0b01, 0b101,
                                                                  0b1111, 0b110]


# ---------------------------------------------------------- trajectories
def _brute_tracks(a, H, W, T):
    """(Lemma-1 violations, components) by brute force: the prism split's
    tetrahedra, crossed faces from the generic SoS expansion, and a plain
    union-find joining the two crossed faces of each tetrahedron."""
    import itertools
    from test_oracle_mesh import brute_tets
    U, V = a[0].ravel().astype(int), a[1].ravel().astype(int)
    crossed = {}
    for tri in brute_faces(H, W, T):
        c, _ = generic_crossed(U, V, tri)
        if c:
            crossed[tri] = tri
    parent = {f: f for f in crossed}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    bad = 0
    for tet in brute_tets(H, W, T):
        faces = [f for f in itertools.combinations(sorted(tet), 3) if f in crossed]
        if len(faces) not in (0, 2):
            bad += 1
        if len(faces) == 2:
            ra, rb = find(faces[0]), find(faces[1])
            if ra != rb:
                parent[ra] = rb
    return bad, len({find(f) for f in crossed})


@pytest.mark.parametrize("seed", range(5))
def test_tracks_equal_brute_force_components(ora, seed):
    rng = np.random.default_rng(300 + seed)
    H, W, T = 5, 6, 4
    a = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
    assert ora.tracks(a, 0) == _brute_tracks(a, H, W, T)


def test_tracks_of_two_separated_vortices(ora):
    """Two translating swirls far apart: two trajectories, no violation."""
    import synthfields
    params = (np.array([[8.3, 9.1], [27.6, 21.2]]), np.array([[0.21, -0.13], [-0.17, 0.11]]),
              np.array([1.3, -0.9]), np.array([3.5, 4.0]))
    f, _ = synthfields.vortex_field(32, 36, 7, 2, seed=0, noise=0.0, params=params)
    f = f.numpy()
    k, _, _ = ora.params(f, 1e-2)
    assert ora.tracks(f, k) == (0, 2)
