"""Pins of the oracle's selector network: the double-precision gradient agrees
with central finite differences, and the fp32 forward pass agrees with a
double-precision evaluation of the same bf16 weights."""
import numpy as np
import pytest


def rand_weights(rng, ora, scale=0.3):
    return (rng.standard_normal(ora.NW) * scale).astype(np.float32)


def bf16_bits(w):
    b = w.astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def forward_double(ora, wbits, x):
    w = (wbits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    W1 = w[0:640].reshape(64, 10)
    b1 = w[640:704]
    W2 = w[704:4800].reshape(64, 64)
    b2 = w[4800:4864]
    W3 = w[4864:5120].reshape(4, 64)
    b3 = w[5120:5124]
    h1 = np.maximum(W1 @ x.astype(np.float64) + b1, 0)
    h2 = np.maximum(W2 @ h1 + b2, 0)
    return W3 @ h2 + b3


def test_forward_matches_double(ora):
    rng = np.random.default_rng(0)
    wb = bf16_bits(rand_weights(rng, ora))
    for _ in range(50):
        x = (rng.standard_normal(10) * 3).astype(np.float32)
        c, lg = ora.mlp_forward(wb, x)
        ref = forward_double(ora, wb, x)
        assert np.allclose(lg, ref, rtol=1e-4, atol=1e-4)
        assert c == int(np.argmax(lg))


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_finite_differences(ora, seed):
    rng = np.random.default_rng(seed)
    w = rand_weights(rng, ora)
    n = 16
    x = (rng.standard_normal((n, 10)) * 2).astype(np.float32)
    lab = rng.integers(0, 4, n).astype(np.int32)
    loss, g = ora.mlp_loss_grad(w, x, lab, exact=True)
    assert np.isfinite(loss) and loss > 0
    idx = rng.choice(ora.NW, 80, replace=False)
    for i in idx:
        h = np.float32(2.0 ** -9)
        wp = w.copy()
        wm = w.copy()
        wp[i] = np.float32(w[i] + h)
        wm[i] = np.float32(w[i] - h)
        lp, _ = ora.mlp_loss_grad(wp, x, lab, exact=True)
        lm, _ = ora.mlp_loss_grad(wm, x, lab, exact=True)
        fd = (lp - lm) / (float(wp[i]) - float(wm[i]))
        assert abs(fd - g[i]) <= 2e-3 * max(1.0, abs(g[i])) + 2e-4, (i, fd, g[i])


def test_bf16_rounding_variant(ora):
    """The trainer's gradient is taken at the bf16-rounded weights."""
    rng = np.random.default_rng(4)
    w = rand_weights(rng, ora)
    x = rng.standard_normal((8, 10)).astype(np.float32)
    lab = rng.integers(0, 4, 8).astype(np.int32)
    wr = (bf16_bits(w).astype(np.uint32) << 16).view(np.float32)
    l1, g1 = ora.mlp_loss_grad(w, x, lab)
    l2, g2 = ora.mlp_loss_grad(wr, x, lab, exact=True)
    assert l1 == l2 and np.array_equal(g1, g2)
