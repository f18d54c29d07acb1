"""The one-vertex and one-block expectations used at full size (sampled.py)
reproduce, on small fields, every per-vertex output and every block
decision of the oracle's own whole-field compression: the processing order,
the crop of the bound and the lossless flags, the prediction from the
reconstructed state and the class decision all match Alg. 3/4 and
Sec. VI as the oracle runs them."""
import numpy as np
import pytest

import sampled
import synthfields


def whole_and_sampled(ora, f, eb, predictor, mode_bt, dt):
    b, dbg = ora.compress(f, eb, predictor=predictor, mode_bt=mode_bt, dt_dx=dt, dt_dy=dt, debug=True)
    g = ora.decompress(b)
    k, _, eps = ora.params(f, eb)
    O = ora.to_fixed(f, k)
    R = ora.to_fixed(g, k)
    return dbg, O, R, k, eps


CASES = [  # workload, shape (H, W, T), rel. bound, predictor, mode_bt
    (1, (37, 45, 5), 1e-3, 2, 1),
    (0, (33, 40, 4), 1e-2, 3, 2),
    (2, (20, 50, 4), 1e-3, 1, 1),
    (0, (18, 17, 3), 1e-1, 0, 1),
]


@pytest.mark.parametrize("cfg,shape,eb,predictor,mode_bt", CASES)
def test_every_vertex_matches_whole_field_compression(ora, cfg, shape, eb, predictor, mode_bt):
    f, m = synthfields.workload(cfg, shape=shape)
    f = f.numpy()
    dt = m["dt_dx"]
    dbg, O, R, k, eps = whole_and_sampled(ora, f, eb, predictor, mode_bt, dt)
    _, T, H, W = f.shape
    tx, ty = -(-W // 16), -(-H // 16)
    slc = ora.sl_factor(dt, k) + ora.sl_factor(dt, k)
    xi, xc, qc = (dbg[n].reshape(T, H, W) for n in ("xi", "xcode", "qcode"))
    n_sl = 0
    for t in range(T):
        for y in range(H):
            for x in range(W):
                cls = sampled.block_class(dbg["modes"], t, x // 16, y // 16, tx, ty, predictor, mode_bt, T)
                n_sl += cls != 0
                e = sampled.expect_vertex(O, R, x, y, t, eps, cls, sampled.class_dmax(predictor, cls), slc)
                got = (int(xi[t, y, x]), int(xc[t, y, x]), int(qc[t, y, x]),
                       (int(R[0, t, y, x]), int(R[1, t, y, x])))
                assert e == got, ((x, y, t), e, got)
                assert sampled.face_masks_kept(O, R, x, y, t)
    if predictor != 0:
        assert n_sl > 0


@pytest.mark.parametrize("cfg,shape,eb,predictor,mode_bt", [c for c in CASES if c[3] >= 2])
def test_every_block_decision_matches(ora, cfg, shape, eb, predictor, mode_bt):
    f, m = synthfields.workload(cfg, shape=shape)
    f = f.numpy()
    dt = m["dt_dx"]
    dbg, O, R, k, eps = whole_and_sampled(ora, f, eb, predictor, mode_bt, dt)
    _, T, H, W = f.shape
    tx, ty = -(-W // 16), -(-H // 16)
    seen = set()
    for t in range(1, T):
        for by in range(ty):
            for bx in range(tx):
                bi = sampled.block_index(t, bx, by, tx, ty, mode_bt, T)
                if bi is None or t != sampled.decision_frame(t // mode_bt, mode_bt):
                    continue
                cls, feat = sampled.expect_block(O, R, t, bx, by, k, eps, predictor, mode_bt, dt, dt)
                assert cls == dbg["modes"][bi], ((bx, by, t), cls, dbg["modes"][bi])
                np.testing.assert_array_equal(feat, dbg["feats"][bi])
                seen.add(bi)
    assert len(seen) == len(dbg["modes"])


def test_block_mode_rejects_predictors_without_choice(ora):
    z = np.zeros((20, 20), np.int32)
    with pytest.raises(ValueError):
        ora.block_mode(z, z, z, z, np.zeros((20, 20), np.uint8), 0, 0, 10, 5, predictor=1)
