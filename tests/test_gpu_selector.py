"""GPU tests of the learned predictor selector: the device gradient against
the oracle's double-precision gradient, bit-exact learned-mode compression
against the oracle, what the trained network keeps of the exhaustive trial
on an unseen field, and the backtrace classes at large displacements (their
timing is measured by the selector benchmark, not here)."""
import numpy as np
import pytest
import torch

import oracle
import synthfields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpt():
    import paper_2510_25143_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("seed", [0, 1])
def test_selector_gradient_matches_oracle(cpt, seed):
    rng = np.random.default_rng(seed)
    w = cpt.selector_init(seed + 3)
    n = 96
    x = rng.uniform(0, 8, (n, 10)).astype(np.float32)
    x[:, 8:] -= 4
    y = rng.integers(0, 4, n).astype(np.int32)
    g, loss = cpt.selector_grad(w, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    lo, go = oracle.mlp_loss_grad(w.cpu().numpy(), x, y)
    g = g.cpu().numpy()
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    scale = np.abs(go).max()
    assert np.abs(g - go).max() <= 1e-4 * scale + 1e-7


def test_learned_mode_compression_matches_oracle(cpt):
    wf = cpt.selector_init(7).cpu().numpy()
    b = wf.view(np.uint32).astype(np.uint64)
    wb = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    f, m = synthfields.workload(0, shape=(48, 64, 9))
    want, dbg = oracle.compress(f.numpy(), 1e-2, predictor=4, mode_bt=4, selector_w=wb, debug=True)
    got, gd = cpt.compress_debug(f.cuda(), 1e-2, predictor=4, mode_bt=4,
                                 selector_w=torch.from_numpy(wb.view(np.int16)).cuda())
    assert np.array_equal(gd["modes"].cpu().numpy(), dbg["modes"])
    assert np.array_equal(got.cpu().numpy(), want)
    g = cpt.decompress(got)
    assert np.array_equal(g.cpu().numpy().view(np.uint32), oracle.decompress(want).view(np.uint32))


def _labels(cpt, f, dt):
    _, d = cpt.compress_debug(f, 1e-3, predictor=3, mode_bt=4, dt_dx=dt, dt_dy=dt)
    return d["feats"], d["modes"].to(torch.int32)


def test_trained_selector_gain(cpt):
    """Train on exhaustive-trial labels of two synthetic flows; on an unseen
    field the learned choice must track the exhaustive one, lose at most 2 %
    of compression ratio and beat Lorenzo alone."""
    fw, mw = synthfields.workload(1, device="cuda", shape=(360, 720, 16))
    ft, mt = synthfields.workload(2, device="cuda", shape=(512, 512, 16))
    X1, Y1 = _labels(cpt, fw, mw["dt_dx"])
    X2, Y2 = _labels(cpt, ft, mt["dt_dx"])
    X, Y = torch.cat([X1, X2]), torch.cat([Y1, Y2])
    w0 = cpt.selector_init(11)
    _, l0 = cpt.selector_grad(w0, X, Y)
    wf, wb, loss = cpt.selector_train(X, Y, w=w0, epochs=30, batch=512, lr=2e-3, seed=5)
    assert loss < 0.6 * l0
    fe, me = synthfields.turbulence_field(512, 512, 24, seed=4000, device="cuda")
    dt = me["dt_dx"]
    res = {}
    for name, kw in [("exhaustive", dict(predictor=3)), ("learned", dict(predictor=4, selector_w=wb)),
                     ("lorenzo", dict(predictor=0))]:
        # separate predictor-choice launches, so that their time can be read
        cpt.compress_batch([fe], 1e-3, mode_bt=4, dt_dx=dt, dt_dy=dt, schedule="launch", **kw)
        cpt.timing_enable(True)
        (s,), _ = cpt.compress_batch([fe], 1e-3, mode_bt=4, dt_dx=dt, dt_dy=dt, schedule="launch", **kw)
        res[name] = dict(CR=fe.numel() * 4 / s.numel(), modes_ms=cpt.timing_read("modes")[0])
        cpt.timing_enable(False)
        k, ea, _ = cpt.field_params(fe, 1e-3)
        v = cpt.verify(fe, cpt.decompress(s), k)
        assert v["fc_t"] == 0 and v["fc_s"] == 0 and v["max_err"] <= ea
    _, de = cpt.compress_debug(fe, 1e-3, predictor=3, mode_bt=4, dt_dx=dt, dt_dy=dt)
    _, dl = cpt.compress_debug(fe, 1e-3, predictor=4, mode_bt=4, dt_dx=dt, dt_dy=dt, selector_w=wb)
    agree = float((de["modes"] == dl["modes"]).float().mean())
    print("selector: train loss %.4f -> %.4f, agreement %.4f, %s" % (l0, loss, agree, res))
    assert agree >= 0.9
    assert res["learned"]["CR"] >= 0.98 * res["exhaustive"]["CR"]
    assert res["learned"]["CR"] > res["lorenzo"]["CR"]


def test_backtrace_classes_at_large_displacement(cpt):
    """At CFL 6 (the fastest point moves 6 cells per step) the exhaustive
    trial uses every class: the d_max = 1, 2, 4 backtraces predict
    differently (Sec. VI-A substeps), and the choices, streams and decoded
    values equal the oracle's."""
    f, m = synthfields.turbulence_field(256, 256, 6, seed=5000, n_vortices=8, cfl=6.0)
    dt = m["dt_dx"]
    want, dbg = oracle.compress(f.numpy(), 1e-3, predictor=3, dt_dx=dt, dt_dy=dt, debug=True)
    got, gd = cpt.compress_debug(f.cuda(), 1e-3, predictor=3, dt_dx=dt, dt_dy=dt)
    modes = gd["modes"].cpu().numpy()
    assert np.array_equal(modes, dbg["modes"])
    assert np.array_equal(got.cpu().numpy(), want)
    # equal scores go to the lowest class, so classes 2 and 3 are only
    # chosen where their backtraces predict differently from class 1
    h = np.bincount(modes, minlength=4)
    assert (h >= 0.05 * modes.size).all(), h
    g = cpt.decompress(got)
    assert np.array_equal(g.cpu().numpy().view(np.uint32), oracle.decompress(want).view(np.uint32))
