"""Pins of the oracle's predictors: 3-D Lorenzo reproduces fields without an
xyt term (Sec. VI), bilinear sampling reproduces affine functions, and the
semi-Lagrangian predictor (Sec. VI-A) is exact on a uniform integer-cell
translation in both of its regimes, clamps at the domain boundary and takes
the RK2 branch when the displacement equals d_max."""
from fractions import Fraction

import numpy as np
import pytest


def test_lorenzo_reproduces_fields_without_xyt_term(ora):
    rng = np.random.default_rng(0)
    H = W = 16
    for _ in range(20):
        a, b, c, d, e, g = (int(z) for z in rng.integers(-50, 50, 6))
        P = lambda x, y: a * x * y + b * x * x + c * y
        Q = lambda x, t: d * x * t + e * t * t
        R = lambda y, t: g * y * t + 3 * y * y
        f = lambda x, y, t: P(x, y) + Q(x, t) + R(y, t)
        for t in (1, 2):
            cur = np.array([[f(x, y, t) for x in range(W)] for y in range(H)], np.int32)
            prev = np.array([[f(x, y, t - 1) for x in range(W)] for y in range(H)], np.int32)
            for y in range(1, H):
                for x in range(1, W):
                    assert ora.lorenzo3(cur, prev, x, y, 0, 0) == f(x, y, t)


def test_lorenzo_tile_local_zero_padding(ora):
    cur = np.arange(1, 1 + 32 * 32, dtype=np.int32).reshape(32, 32)
    prev = cur * 2
    x0, y0 = 16, 16
    # block corner at t = 0 predicts 0; block edge degrades to 2-D Lorenzo
    assert ora.lorenzo3(cur, None, x0, y0, x0, y0) == 0
    assert ora.lorenzo3(cur, prev, x0, y0, x0, y0) == prev[y0, x0]
    x, y = x0, y0 + 3
    assert ora.lorenzo3(cur, prev, x, y, x0, y0) == cur[y - 1, x] + prev[y, x] - prev[y - 1, x]


def test_bilinear_exact_on_affine_functions(ora):
    rng = np.random.default_rng(1)
    H, W = 7, 9
    for _ in range(50):
        a, b, c = (int(z) for z in rng.integers(-1000, 1000, 3))
        F = np.array([[a * x + b * y + c for x in range(W)] for y in range(H)], np.int32)
        px = int(rng.integers(0, (W - 1) << 16))
        py = int(rng.integers(0, (H - 1) << 16))
        exact = a * Fraction(px, 65536) + b * Fraction(py, 65536) + c
        want = (exact + Fraction(1, 2)).__floor__()
        assert ora.bilinear(F, px, py) == want
    # grid points are reproduced exactly, including the last row/column
    F = rng.integers(-1 << 24, 1 << 24, (H, W)).astype(np.int32)
    for y in range(H):
        for x in range(W):
            assert ora.bilinear(F, x << 16, y << 16) == F[y, x]


def test_sl_factor_power_of_two(ora):
    for k in [0, 5, 16, 27, 40, -14]:
        c, s = ora.sl_factor(1.0, k)
        # c / 2^s == 2^(16-k) exactly
        assert Fraction(c, 2 ** s) == Fraction(2) ** (16 - k)
    # factors of 2^31 Q16 cells per unit and above saturate
    assert ora.sl_factor(1.0, -20) == (2147483647, 0)
    c, s = ora.sl_factor(0.0, 10)
    assert c == 0


@pytest.mark.parametrize("dmax", [1, 2, 4])
def test_sl_exact_on_uniform_translation(ora, dmax):
    """Velocity of exactly (2, 1) cells per step plus a small pattern that does
    not change the displacement: the prediction is the previous frame shifted
    by (2, 1) cells, whether RK2 (d_inf <= d_max) or substeps are taken."""
    k = 27
    c, s = ora.sl_factor(1.0, k)
    H, W = 12, 14
    rng = np.random.default_rng(dmax)
    base_u, base_v = 2 << k, 1 << k
    small = 1 << (k - 16)
    Up = (base_u + rng.integers(0, small, (H, W))).astype(np.int64)
    Vp = (base_v + rng.integers(0, small, (H, W))).astype(np.int64)
    assert Up.max() < 2 ** 31
    Up, Vp = Up.astype(np.int32), Vp.astype(np.int32)
    for y in range(1, H):
        for x in range(2, W):
            pu, pv = ora.sl_predict(Up, Vp, x, y, c, s, c, s, dmax=dmax)
            assert pu == Up[y - 1, x - 2] and pv == Vp[y - 1, x - 2]


def test_sl_clamps_at_domain_boundary(ora):
    k = 27
    c, s = ora.sl_factor(1.0, k)
    H, W = 6, 6
    Up = np.full((H, W), 3 << k, np.int32)   # 3 cells/step to +x
    Vp = np.full((H, W), -(2 << k), np.int32)  # 2 cells/step to -y
    for dmax in (1, 2, 4):
        pu, pv = ora.sl_predict(Up, Vp, 1, 4, c, s, c, s, dmax=dmax)
        assert pu == 3 << k and pv == -(2 << k)  # uniform field, clamped sample
    # a ramp in u shows the clamped departure column x = 0
    Up2 = Up.copy()
    Up2[:, 0] = (3 << k) + 5
    pu, _ = ora.sl_predict(Up2, Vp, 1, 2, c, s, c, s, dmax=4)
    assert pu == (3 << k) + 5


def test_sl_regime_switch_at_dmax(ora):
    """Displacement exactly d_max takes RK2 (midpoint velocity); one unit more
    takes two Euler substeps (velocity at the start and at the midpoint)."""
    k = 20
    c, s = ora.sl_factor(1.0, k)
    H, W = 3, 12
    # u grows by 1/8 cell per cell to the left of x = 8
    Up = np.zeros((H, W), np.int32)
    for x in range(W):
        Up[:, x] = (2 << k) + ((8 - x) << (k - 3)) if x < 8 else 2 << k
    Vp = np.zeros((H, W), np.int32)
    x0 = 8
    pu_rk2, _ = ora.sl_predict(Up, Vp, x0, 1, c, s, c, s, dmax=2)
    # RK2: midpoint at x0 - 1, u there = 2 + 1/8 cells -> departure x0 - 2.125
    P = Fraction(x0) - (2 + Fraction(1, 8))
    xl = int(P)
    fx = P - xl
    exp_val = (1 - fx) * int(Up[1, xl]) + fx * int(Up[1, xl + 1])
    assert abs(pu_rk2 - exp_val) <= 1
    pu_sub, _ = ora.sl_predict(Up, Vp, x0, 1, c, s, c, s, dmax=1)
    # two substeps of half the local displacement: x0 -> x0 - 1 -> x0 - 1 - 1.0625
    P2 = Fraction(x0) - 1 - (2 + Fraction(1, 8)) / 2
    xl = int(P2)
    fx = P2 - xl
    exp2 = (1 - fx) * int(Up[1, xl]) + fx * int(Up[1, xl + 1])
    assert abs(pu_sub - exp2) <= 1
    assert pu_sub != pu_rk2
