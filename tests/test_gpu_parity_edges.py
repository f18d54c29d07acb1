"""GPU parity on the paths the workload recipes do not reach: displacement
factors at many time steps, parameters of extreme fields, the adaptive
substep branch of the semi-Lagrangian predictor (Sec. VI-A) on a field that
moves several cells per step, the check of Sec. IV-A on pairs whose faces
differ, and the decompressor's rejection of undersized outputs and of hostile
stored floats.  Every comparison is against the CPU oracle on the same seeded
inputs, bit for bit."""
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
    assert torch.cuda.is_available()
    return m


def dev(a):
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(a)
    return a.to("cuda").contiguous()


def assert_bytes_equal(a, b):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    if not np.array_equal(a, b):
        i = int(np.flatnonzero(a != b)[0])
        raise AssertionError("first difference at byte %d of %d" % (i, a.size))


def bf16_weights(cpt, seed):
    wf = cpt.selector_init(seed).cpu().numpy()
    b = wf.view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


# --------------------------------------------------- displacement factors
DT_VALUES = [1.0, 0.5 / 29.7, 0.016835, 1.0 / 3.0, 0.1, 7.25, 0.0, 1e-30, 5e-324, 3e8, 2.0 ** -47, 123.456]


def test_displacement_factors_match_oracle(cpt):
    """The header stores c, s of both axes; with the semi-Lagrangian predictor
    every prediction depends on them, so equal bytes pin the derivation."""
    f, _ = synthfields.workload(0, shape=(20, 24, 3))
    for i, dt in enumerate(DT_VALUES):
        dty = DT_VALUES[(i + 5) % len(DT_VALUES)]
        want = oracle.compress(f.numpy(), 1e-2, predictor=1, dt_dx=dt, dt_dy=dty)
        got = cpt.compress(dev(f), 1e-2, predictor=1, dt_dx=dt, dt_dy=dty)
        assert_bytes_equal(got.cpu().numpy(), want)


def test_field_params_extreme_fields(cpt):
    rng = np.random.default_rng(4)
    cases = [np.zeros((2, 2, 5, 6), np.float32),
             (rng.standard_normal((2, 2, 5, 6)) * 1e-40).astype(np.float32),   # subnormal values
             (rng.standard_normal((2, 2, 5, 6)) * 1e-30).astype(np.float32),
             (rng.standard_normal((2, 2, 5, 6)) * 1e29).astype(np.float32),
             np.full((2, 2, 5, 6), 0.75, np.float32)]
    for a in cases:
        for eb, mode in ((1e-2, 0), (0.5, 0), (1e-3, 1), (2.0 ** -30, 1)):
            assert cpt.field_params(dev(a), eb, eb_mode=mode) == oracle.params(a, eb, eb_mode=mode)
    big = np.zeros((2, 1, 4, 4), np.float32)
    big[0, 0, 1, 1] = 2.0 ** 100
    with pytest.raises(cpt.CptError):
        cpt.field_params(dev(big), 1e-2)
    with pytest.raises(ValueError):
        oracle.params(big, 1e-2)


# ------------------------------------------------- adaptive substepping
def drifting_field():
    """Workload 0's four vortices plus a uniform drift of 0.05 in u and -0.03
    in v; with dt/dx = dt/dy = 60 most vertices move 2-4 cells per step."""
    f, m = synthfields.workload(0)
    f = f.clone()
    f[0] += 0.05
    f[1] -= 0.03
    return f, 60.0


def displacement_cells(fn, dt):
    """d_inf of every vertex of frames 0..T-2 in Q16 cells, from the
    fixed-point field and the header's factors (Sec. VI-A reading)."""
    k, _, _ = oracle.params(fn, 1e-2)
    c, s = oracle.sl_factor(dt, k)
    U = oracle.to_fixed(fn[0], k).astype(np.int64)
    V = oracle.to_fixed(fn[1], k).astype(np.int64)
    dx, dy = (U * c) >> s, (V * c) >> s
    return np.maximum(np.abs(dx), np.abs(dy))[:-1]


def test_drifting_field_takes_substeps():
    f, dt = drifting_field()
    d = displacement_cells(f.numpy(), dt)
    share_sub2 = float((d > 2 * 65536).mean())      # N > 1 at d_max = 2
    share_sub1 = float((d > 1 * 65536).mean())      # N > 1 at d_max = 1
    assert share_sub2 > 0.5 and share_sub1 > 0.9, (share_sub2, share_sub1)
    assert float((d > 4 * 65536).mean()) < 0.5      # d_max = 4 keeps RK2 for most


@pytest.mark.parametrize("pred,bt", [(1, 1), (3, 1), (3, 4), (4, 2)])
def test_substep_branch_matches_oracle(cpt, pred, bt):
    f, dt = drifting_field()
    fn = f.numpy()
    kw = dict(predictor=pred, mode_bt=bt, dt_dx=dt, dt_dy=dt)
    gkw = dict(kw)
    if pred == 4:
        wb = bf16_weights(cpt, 13)
        kw["selector_w"] = wb
        gkw["selector_w"] = dev(wb.view(np.int16))
    for eb in (1e-2, 1e-3):
        want, dbg = oracle.compress(fn, eb, debug=True, **kw)
        got, gd = cpt.compress_debug(dev(f), eb, **gkw)
        assert np.array_equal(gd["xi"].cpu().numpy(), dbg["xi"])
        assert np.array_equal(gd["xcode"].cpu().numpy(), dbg["xcode"])
        lossy = dbg["xcode"] != 24
        assert np.array_equal(gd["qcode"].cpu().numpy().view(np.uint32)[lossy], dbg["qcode"][lossy])
        assert np.array_equal(gd["modes"].cpu().numpy(), dbg["modes"])
        assert np.array_equal(gd["feats"].cpu().numpy(), dbg["feats"])
        assert_bytes_equal(got.cpu().numpy(), want)
        if pred == 3:
            # the exhaustive choice picks more than one backtrace step here
            assert len(set(dbg["modes"].tolist()) - {0}) >= 2, np.bincount(dbg["modes"])
        rec = oracle.decompress(want)
        g = cpt.decompress(got).cpu().numpy()
        assert np.array_equal(g.view(np.uint32), rec.view(np.uint32))
        k, ea, _ = oracle.params(fn, eb)
        v = cpt.verify(dev(f), dev(g), k)
        assert v["fc_t"] == 0 and v["fc_s"] == 0 and v["max_err"] <= ea


# ------------------------------------------------------------- the check
def perturbed_pairs():
    rng = np.random.default_rng(21)
    f, _ = synthfields.workload(0, shape=(40, 48, 5))
    a = f.numpy()
    b = a + rng.normal(0, 0.02, a.shape).astype(np.float32)   # flips faces near the vortex cores
    yield a, b
    c = a.copy()
    c[:, 2, 10:20, 10:20] *= -1.0                               # a reversed patch
    yield a, c
    yield a, a[::-1].copy()                                    # u and v swapped: every sign flips
    ia = rng.integers(-2, 3, (2, 4, 9, 11)).astype(np.float32)
    ib = ia.copy()
    ib[:, 1, 3:6, 4:8] = rng.integers(-2, 3, (2, 3, 4))
    yield ia, ib


def test_verify_matches_oracle_on_differing_fields(cpt):
    seen_t = seen_s = 0
    for a, b in perturbed_pairs():
        k = 0 if np.all(a == np.round(a)) else oracle.params(a, 1e-2)[0]
        want = oracle.verify(a, b, k)
        got = cpt.verify(dev(a), dev(b), k)
        assert (got["fc_t"], got["fc_s"]) == (want["fc_t"], want["fc_s"])
        assert got["max_err"] == want["max_err"]
        assert abs(got["psnr"] - want["psnr"]) <= 1e-9 * abs(want["psnr"])
        seen_t += want["fc_t"] > 0
        seen_s += want["fc_s"] > 0
    assert seen_t >= 3 and seen_s >= 3


# ------------------------------------------------------- decompression
def test_decompress_rejects_small_outputs(cpt):
    f, _ = synthfields.workload(0, shape=(16, 20, 3))
    b = cpt.compress(dev(f), 1e-2)
    need = f.numel()
    with pytest.raises(cpt.CptError) as e:
        cpt.decompress(b, out=torch.empty(need - 1, dtype=torch.float32, device="cuda"))
    assert e.value.status == cpt.ECAPACITY
    with pytest.raises(TypeError):
        cpt.decompress(b, out=torch.empty(need, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        cpt.decompress(b, out=torch.empty((need, 2), dtype=torch.float32, device="cuda")[:, 0])
    outs = [torch.empty(need, dtype=torch.float32, device="cuda"),
            torch.empty(need - 8, dtype=torch.float32, device="cuda")]
    _, status = cpt.decompress_batch([b, b], outs=outs, raise_on_error=False)
    assert status == [cpt.OK, cpt.ECAPACITY]
    assert np.array_equal(outs[0].cpu().numpy(), oracle.decompress(b.cpu().numpy()).ravel())


def test_hostile_stored_floats_rejected_by_both(cpt):
    """Stored raw values replaced by floats no valid stream holds (huge,
    infinite, NaN): the oracle and the library both report a corrupt stream."""
    f, _ = synthfields.workload(0, shape=(20, 24, 3))
    b = oracle.compress(f.numpy(), 1e-3)
    info = oracle.stream_info(b)
    assert info["n_raw"] > 0
    raw_off = len(b) - 4 * info["n_raw"]
    for word in (0x7F7FFFFF, 0xFF7FFFFF, 0x7F800000, 0x7FC00001, 0x5F000000):
        for pos in (0, info["n_raw"] // 2, info["n_raw"] - 1):
            c = b.copy()
            c[raw_off + 4 * pos: raw_off + 4 * pos + 4] = np.frombuffer(np.uint32(word).tobytes(), np.uint8)
            st, _ = oracle.decompress_status(c)
            assert st == oracle.ECORRUPT, (hex(word), pos, st)
            with pytest.raises(cpt.CptError) as e:
                cpt.decompress(dev(c))
            assert e.value.status == cpt.ECORRUPT


@pytest.mark.parametrize("pred,backend", [(0, 0), (2, 0), (0, 1)])
def test_long_codewords_match_oracle(cpt, pred, backend):
    """Residual codewords of 13-16 bits, which the decoder finds through the
    canonical ranges of the long lengths rather than its 12-bit table: bytes
    and decoded values equal the oracle's."""
    from test_oracle_entropy import stream_codebook_lengths
    f, _ = synthfields.spiked_field()
    want = oracle.compress(f.numpy(), 1e-3, predictor=pred, backend=backend)
    plain = oracle.compress(f.numpy(), 1e-3, predictor=pred)
    assert stream_codebook_lengths(plain, 4).max() > 12
    got = cpt.compress(dev(f), 1e-3, predictor=pred, backend=backend)
    assert_bytes_equal(got.cpu().numpy(), want)
    g = cpt.decompress(dev(want)).cpu().numpy()
    assert np.array_equal(g.view(np.uint32), oracle.decompress(plain).view(np.uint32))

