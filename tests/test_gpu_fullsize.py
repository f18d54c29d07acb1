"""Parity at full size: the 720x1440x64 wind field at rel. bound 1e-3 with
the K = 2 mixture, compressed through the C ABI exactly as the benchmark
times it (one batched call, per-phase launches, eager).  The oracle cannot
compress 66 M vertices within a test, so it checks sampled outputs one by
one (tests/sampled.py, itself checked against whole-field oracle runs):
per-vertex bounds, bound codes, residual codes and reconstructions, and
per-block predictor classes and features, each recomputed from the state
the compressor saw.  Properties that hold at any size are checked on the
whole field: stream identity across execution paths and runs, header and
parameters, the pointwise bound, bit-identical lossless vertices and the
face status kept."""
import numpy as np
import pytest
import torch

import oracle
import sampled
import synthfields

pytestmark = pytest.mark.gpu

CFG = 1  # wind workload, 720 x 1440 x 64


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def cpt():
    import paper_2510_25143_amd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


@pytest.fixture(scope="module")
def full(cpt):
    log("full size: generating the wind field")
    f, meta = synthfields.workload(CFG, device="cuda")
    f = f.contiguous()
    _, T, H, W = f.shape
    assert (T, H, W) == (64, 720, 1440)
    eb, dt = meta["eb"], meta["dt_dx"]
    opts = dict(predictor=meta["predictor"], mode_bt=meta["mode_bt"], dt_dx=dt, dt_dy=dt)
    out = torch.empty(cpt.compress_bound(H, W, T), dtype=torch.uint8, device="cuda")
    log("full size: batched compression, per-phase launches")
    (s,), st = cpt.compress_batch([f], eb, schedule="launch", outs=[out], **opts)
    assert st == [0]
    s_launch = s.cpu().numpy().copy()
    (s,), st = cpt.compress_batch([f], eb, schedule="launch", outs=[out], **opts)
    s_again = s.cpu().numpy().copy()
    log("full size: fused schedule and debug outputs")
    (s,), st = cpt.compress_batch([f], eb, schedule="fused", outs=[out], **opts)
    s_fused = s.cpu().numpy().copy()
    s_dbg, dbg = cpt.compress_debug(f, eb, **opts)
    dbg = {n: v.cpu().numpy() for n, v in dbg.items()}
    log("full size: decompression")
    back = cpt.decompress(torch.from_numpy(s_launch).to("cuda"))
    k, ea, eps = cpt.field_params(f, eb)
    err = float((back - f).abs().max())
    ll = torch.from_numpy(dbg["xcode"] == oracle.XLOSSLESS).to("cuda")
    ll_same = bool(torch.equal(f.reshape(2, -1)[:, ll].view(torch.int32),
                               back.reshape(2, -1)[:, ll].view(torch.int32)))
    ver = cpt.verify(f, back, k)
    f_cpu = f.cpu().numpy()
    back_cpu = back.cpu().numpy()
    del back, out, ll
    torch.cuda.empty_cache()
    log("full size: fixed point on the host")
    O = oracle.to_fixed(f_cpu, k)
    R = oracle.to_fixed(back_cpu, k)
    return dict(f=f_cpu, O=O, R=R, eb=eb, dt=dt, opts=opts, k=k, ea=ea, eps=eps, err=err, ll_same=ll_same,
                ver=ver, s_launch=s_launch, s_again=s_again, s_fused=s_fused, s_dbg=s_dbg.cpu().numpy(), dbg=dbg,
                shape=(T, H, W))


def test_streams_identical_across_paths_and_runs(full):
    a = full["s_launch"]
    for name in ("s_again", "s_fused", "s_dbg"):
        assert np.array_equal(a, full[name]), name


def test_header_and_parameters_match_oracle(full):
    k, ea, eps = oracle.params(full["f"], full["eb"])
    assert (k, eps) == (full["k"], full["eps"])
    assert ea == full["ea"]
    info = oracle.stream_info(full["s_launch"])
    T, H, W = full["shape"]
    assert (info["H"], info["W"], info["T"], info["k"], info["eps"]) == (H, W, T, k, eps)
    assert info["predictor"] == full["opts"]["predictor"] and info["mode_bt"] == full["opts"]["mode_bt"]
    assert info["total_len"] == full["s_launch"].size
    assert 6.0 < full["f"].nbytes / full["s_launch"].size < 14.0


def test_whole_field_properties(full):
    assert full["err"] <= full["ea"]
    assert full["ll_same"]
    assert full["ver"]["fc_t"] == 0 and full["ver"]["fc_s"] == 0
    assert full["ver"]["max_err"] <= full["ea"]


def _vertex_samples(full):
    T, H, W = full["shape"]
    rng = np.random.default_rng(2510)
    xc = full["dbg"]["xcode"].reshape(T, H, W)
    pts = set()
    for _ in range(2500):
        pts.add((int(rng.integers(W)), int(rng.integers(H)), int(rng.integers(T))))
    # domain corners and edges in the first, second and last frames
    for t in (0, 1, T - 1):
        for x in (0, 1, W - 2, W - 1):
            for y in (0, 1, H - 2, H - 1):
                pts.add((x, y, t))
    # corners of blocks (block edges meet other colours there)
    for _ in range(150):
        bx, by, t = int(rng.integers(W // 16)), int(rng.integers(H // 16)), int(rng.integers(T))
        for dx in (0, 15):
            for dy in (0, 15):
                pts.add((16 * bx + dx, 16 * by + dy, t))
    # vertices of blocks in a semi-Lagrangian class
    pred, bt = full["opts"]["predictor"], full["opts"]["mode_bt"]
    modes = full["dbg"]["modes"]
    tx, ty = W // 16, H // 16
    for t in range(1, T):
        b0 = sampled.block_index(t, 0, 0, tx, ty, bt, T)
        if b0 is None:
            continue
        sl = np.flatnonzero(modes[b0:b0 + tx * ty])
        for i in rng.choice(sl, size=min(5, sl.size), replace=False):
            bx, by = int(i) % tx, int(i) // tx
            pts.add((16 * bx + int(rng.integers(16)), 16 * by + int(rng.integers(16)), t))
    # vertices whose bound is below eps' and lossless ones
    for want in (lambda c: (c > 0) & (c < oracle.XLOSSLESS), lambda c: c == oracle.XLOSSLESS):
        idx = np.flatnonzero(want(xc).ravel())
        for i in rng.choice(idx, size=min(600, idx.size), replace=False):
            t, r = divmod(int(i), H * W)
            pts.add((r % W, r // W, t))
    return sorted(pts)


def test_sampled_vertices_match_oracle(full):
    T, H, W = full["shape"]
    O, R, dbg, eps = full["O"], full["R"], full["dbg"], full["eps"]
    pred, bt = full["opts"]["predictor"], full["opts"]["mode_bt"]
    slc = oracle.sl_factor(full["dt"], full["k"]) + oracle.sl_factor(full["dt"], full["k"])
    xi, xc, qc = (dbg[n].reshape(T, H, W) for n in ("xi", "xcode", "qcode"))
    tx, ty = W // 16, H // 16
    pts = _vertex_samples(full)
    log("full size: %d sampled vertices" % len(pts))
    kinds = {"lossless": 0, "reduced": 0, "sl": 0}
    for (x, y, t) in pts:
        cls = sampled.block_class(dbg["modes"], t, x // 16, y // 16, tx, ty, pred, bt, T)
        e = sampled.expect_vertex(O, R, x, y, t, eps, cls, sampled.class_dmax(pred, cls), slc)
        got = (int(xi[t, y, x]), int(xc[t, y, x]), int(qc[t, y, x]), (int(R[0, t, y, x]), int(R[1, t, y, x])))
        if e[1] == oracle.XLOSSLESS:  # no residual codes: the device's code word is not part of the output
            got = got[:2] + (0,) + got[3:]
        assert e == got, ((x, y, t), e, got)
        assert sampled.face_masks_kept(O, R, x, y, t), (x, y, t)
        kinds["lossless"] += e[1] == oracle.XLOSSLESS
        kinds["reduced"] += 0 < e[1] < oracle.XLOSSLESS
        kinds["sl"] += cls != 0 and e[1] != oracle.XLOSSLESS
    log("full size: kinds %s" % kinds)
    assert min(kinds.values()) >= 100, kinds


def test_sampled_block_decisions_match_oracle(full):
    T, H, W = full["shape"]
    O, R, dbg = full["O"], full["R"], full["dbg"]
    pred, bt = full["opts"]["predictor"], full["opts"]["mode_bt"]
    tx, ty = W // 16, H // 16
    rng = np.random.default_rng(143)
    frames = [t for t in range(1, T) if sampled.block_index(t, 0, 0, tx, ty, bt, T) is not None
              and t == sampled.decision_frame(t // bt, bt)]
    blocks = [(int(rng.integers(tx)), int(rng.integers(ty)), int(rng.choice(frames))) for _ in range(40)]
    blocks += [(0, 0, frames[0]), (tx - 1, ty - 1, frames[-1]), (tx - 1, 0, frames[len(frames) // 2]),
               (0, ty - 1, frames[1])]
    # blocks the device put in a semi-Lagrangian class, if any
    for t in rng.choice(frames, size=4, replace=False):
        b0 = sampled.block_index(int(t), 0, 0, tx, ty, bt, T)
        sl = np.flatnonzero(dbg["modes"][b0:b0 + tx * ty])
        for i in rng.choice(sl, size=min(6, sl.size), replace=False):
            blocks.append((int(i) % tx, int(i) // tx, int(t)))
    log("full size: %d sampled blocks" % len(blocks))
    n_sl = 0
    for (bx, by, t) in blocks:
        bi = sampled.block_index(t, bx, by, tx, ty, bt, T)
        cls, feat = sampled.expect_block(O, R, t, bx, by, full["k"], full["eps"], pred, bt, full["dt"], full["dt"])
        assert cls == dbg["modes"][bi], ((bx, by, t), cls, dbg["modes"][bi])
        np.testing.assert_array_equal(feat, dbg["feats"][bi])
        n_sl += cls != 0
    assert n_sl > 0
