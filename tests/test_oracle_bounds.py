"""Pins of the oracle's error-bound derivation (Alg. 2, Alg. 4), the bound
code and the residual quantizer.

Alg. 2 is checked against what it must guarantee (no face changes status for
any integer perturbation of vertex 2 inside the box |delta| <= bound, checked
with an independent SoS face test) and against maximality of the unrelaxed
branch (bound + 1 lets a sign term reach zero at a box corner).
"""
import itertools

import numpy as np
import pytest

from tests.test_oracle_mesh import generic_det_sign


def face_status(p0, p1, p2, ids):
    """SoS face predicate of the three values with the given global ids."""
    pts = sorted(zip(ids, (p0, p1, p2)))
    (ga, a), (gb, b), (gc, c) = pts
    s1 = generic_det_sign(a[0], a[1], ga, b[0], b[1], gb)
    s2 = generic_det_sign(b[0], b[1], gb, c[0], c[1], gc)
    s3 = generic_det_sign(c[0], c[1], gc, a[0], a[1], ga)
    return s1 == s2 == s3


def test_alg2_hand_example(ora):
    # p0 = (1, 2), p1 = (3, -1), p2 = (-2, 1):
    # M0 = u2 v0 - u0 v2 = -4 - 1 = -5 ; M1 = u1 v2 - u2 v1 = 3 - 2 = 1
    # M2 = u0 v1 - u1 v0 = -1 - 6 = -7 ; M = -11
    # |M|/(|u1-u0| + |v0-v1|) = 11/5 -> floor(10/5) = 2
    # |M1|/(|u1|+|v1|) = 1/4 -> floor(0/4) = 0 ; |M0|/(|u0|+|v0|) = 5/3 -> 1
    assert ora.alg2(1, 3, -2, 2, -1, 1) == 0
    # p0 = (4, 1), p1 = (5, -2), p2 = (-3, 6): same-signed v? no; u? no
    # M0 = -3*1 - 4*6 = -27 ; M1 = 5*6 - (-3)(-2) = 24 ; M2 = 4*-2 - 5*1 = -13
    # M = -16 ; cand(16, 1+3) = 3 ; cand(24, 7) = 3 ; cand(27, 5) = 5 -> 3
    assert ora.alg2(4, 5, -3, 1, -2, 6) == 3
    # all u positive: relaxation to |u2| - 1 = 6 when that is larger
    # p0 = (2, 1), p1 = (3, -1), p2 = (7, 2): M0 = 7-4 = 3, M1 = 6+7 = 13,
    # M2 = -2-3 = -5, M = 11 ; cand(11, 1+2) = 3 ; cand(13, 4) = 3 ;
    # cand(3, 3) = 0 -> 0, relaxed to 6
    assert ora.alg2(2, 3, 7, 1, -1, 2) == 6
    # M == 0 returns 0 before the relaxation (the paper's order)
    assert ora.alg2(2, 2, 5, 1, 1, 3) == 0


@pytest.mark.parametrize("seed", range(4))
def test_alg2_box_never_flips_a_face(ora, seed):
    rng = np.random.default_rng(seed)
    cap = 5
    checked = 0
    for _ in range(600):
        p = rng.integers(-6, 7, (3, 2))
        p0, p1, p2 = (tuple(int(z) for z in q) for q in p)
        e = min(ora.alg2(p0[0], p1[0], p2[0], p0[1], p1[1], p2[1]), cap)
        for ids in itertools.permutations((0, 1, 2)):
            base = face_status(p0, p1, p2, ids)
            for du in range(-e, e + 1):
                for dv in range(-e, e + 1):
                    q2 = (p2[0] + du, p2[1] + dv)
                    assert face_status(p0, p1, q2, ids) == base, (p0, p1, p2, e, du, dv, ids)
                    checked += 1
    assert checked > 1000


def test_alg2_unrelaxed_bound_is_tight(ora):
    """When no relaxation applies and the bound comes from a quotient, moving
    vertex 2 by bound+1 at some box corner zeroes or flips M, M0 or M1."""
    rng = np.random.default_rng(9)
    tested = 0
    for _ in range(3000):
        u0, u1, u2, v0, v1, v2 = (int(z) for z in rng.integers(-50, 51, 6))
        same_u = (u0 > 0 and u1 > 0 and u2 > 0) or (u0 < 0 and u1 < 0 and u2 < 0)
        same_v = (v0 > 0 and v1 > 0 and v2 > 0) or (v0 < 0 and v1 < 0 and v2 < 0)
        if same_u or same_v:
            continue
        e = ora.alg2(u0, u1, u2, v0, v1, v2)
        if e <= 0:
            continue

        def terms(a, b):
            M0 = a * v0 - u0 * b
            M1 = u1 * b - a * v1
            M2 = u0 * v1 - u1 * v0
            return (M0 + M1 + M2, M0, M1)

        base = [np.sign(z) for z in terms(u2, v2)]
        hit = False
        for su, sv in itertools.product((-1, 1), repeat=2):
            t = terms(u2 + su * (e + 1), v2 + sv * (e + 1))
            if any(np.sign(z) != s for z, s in zip(t, base)):
                hit = True
        assert hit, (u0, u1, u2, v0, v1, v2, e)
        tested += 1
    assert tested > 500


def test_vertex_bound_is_min_over_incident_faces(ora):
    """Alg. 4 on an unprocessed field: xi = min(eps', Alg. 2 over the 36
    faces) for unflagged vertices, 0 for flagged ones (first frame only,
    before any neighbour is processed)."""
    import synthfields
    f, _ = synthfields.workload(0)
    f = f.numpy()
    k, _, eps = ora.params(f, 1e-2)
    F = ora.to_fixed(f, k)
    U, V = F[0].ravel().astype(np.int64), F[1].ravel().astype(np.int64)
    T, H, W = F.shape[1:]
    _, dbg = ora.compress(f, 1e-2, predictor=0, debug=True)
    flags = ora.lossless_flags(ora.face_masks_fixed(F[0], F[1])).ravel()
    # the first vertex of each colour-0 tile sees only original values
    for (bx, by) in [(0, 0), (3, 0), (1, 2), (2, 1)]:
        if (bx + by) % 3:
            continue
        x, y, t = bx * 16, by * 16, 0
        v = (t * H + y) * W + x
        want = 0 if flags[v] else min([eps] + [ora.alg2(U[a], U[b], U[v], V[a], V[b], V[v])
                                               for a, b in ora.incident_faces(H, W, T, x, y, t)])
        assert dbg["xi"][v] == want


def test_xi_code_exhaustive(ora):
    for eps in [1, 2, 3, 7, 100, 155541, (1 << 23) - 1]:
        for xi in list(range(0, 70)) + [eps // 3, eps // 2, eps - 1, eps, eps + 5]:
            q = ora.xi_code(eps, xi)
            if xi <= 0:
                assert q == 24
                continue
            assert 0 <= q <= 23
            assert (eps >> q) <= xi and (eps >> q) >= 1
            assert q == 0 or (eps >> (q - 1)) > xi


def test_quantizer_exhaustive(ora):
    R = ora.QR
    for xt in [0, 1, 2, 3, 10]:
        w = 2 * xt + 1
        for r in range(-(R + 2) * w, (R + 2) * w, max(1, w // 3)):
            pred = 1000
            code, rec = ora.quantize(pred + r, pred, xt)
            q = (r + xt) // w
            if abs(q) >= R:
                assert code == 0 and rec == pred + r
            else:
                assert code == q + R
                assert abs(rec - (pred + r)) <= xt
                assert (rec - pred) % w == 0


def test_params_guarantee(ora):
    rng = np.random.default_rng(3)
    for scale in [1e-30, 1e-3, 1.0, 7.5, 1e6, 1e20]:
        f = (rng.standard_normal((2, 2, 5, 6)) * scale).astype(np.float32)
        for eb in [1e-4, 1e-2, 0.5]:
            k, ea, eps = ora.params(f, eb)
            ma = float(np.abs(f.astype(np.float64)).max())
            m, e = np.frexp(ma)
            assert k == min(23 - int(e), 120)
            assert ea == eb * (float(f.max()) - float(f.min()))
            assert eps >= 0
            assert (eps + 0.5) * 2.0 ** (-k) <= ea or eps == 0
            F = ora.to_fixed(f, k)
            assert np.abs(F.astype(np.int64)).max() <= (1 << 23)


def test_to_fixed_is_round_half_even(ora):
    from fractions import Fraction
    vals = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 3.25, 1e-40, -1e-45, 3.4e38, 1.0000001],
                    dtype=np.float32)
    for k in [0, 1, 3, -100, 100, 120]:
        got = ora.to_fixed(vals, k)
        for x, g in zip(vals.tolist(), got.tolist()):
            exact = Fraction(x) * (Fraction(2) ** k)
            fl = exact.numerator // exact.denominator
            rem = exact - fl
            want = fl + (1 if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2) else 0)
            if abs(want) < (1 << 31):
                assert g == want, (x, k)


def test_invalid_parameters(ora):
    f = np.zeros((2, 2, 3, 3), np.float32)
    with pytest.raises(ValueError):
        ora.params(f, 0.0)
    with pytest.raises(ValueError):
        ora.params(f, 0.6)
    g = f.copy()
    g[0, 0, 1, 1] = np.nan
    with pytest.raises(ValueError):
        ora.params(g, 0.1)
    g[0, 0, 1, 1] = np.inf
    with pytest.raises(ValueError):
        ora.params(g, 0.1)
    with pytest.raises(ValueError):
        ora.params(np.zeros((2, 1, 1, 3), np.float32), 0.1)
