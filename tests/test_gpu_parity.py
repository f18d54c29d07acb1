"""GPU parity: the HIP library, called through its C ABI, against the CPU
oracle on the same seeded inputs — bit-exact for face codes, stream bytes,
per-vertex bounds and codes, block modes and decompressed floats."""
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


def dev(f):
    return f.to("cuda").contiguous()


def assert_bytes_equal(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    if not np.array_equal(a, b):
        i = int(np.flatnonzero(a != b)[0])
        raise AssertionError("first difference at byte %d of %d" % (i, a.size))


# ------------------------------------------------------------ extraction
EXTRACT_CASES = [("w0", 0, None), ("ragged", 0, (37, 45, 5)), ("tiny", 0, (2, 3, 2)),
                 ("wind-crop", 1, (48, 80, 4)), ("turb-crop", 2, (40, 56, 3))]


@pytest.mark.parametrize("name,cfg,shape", EXTRACT_CASES)
def test_extract_matches_oracle(cpt, name, cfg, shape):
    f, _ = synthfields.workload(cfg, shape=shape)
    fn = f.numpy()
    k, _, _ = oracle.params(fn, 1e-2)
    want = oracle.extract(fn, k)
    got = cpt.extract_trajectories(dev(f), k).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(4))
def test_extract_degenerate_integer_fields(cpt, seed):
    rng = np.random.default_rng(seed)
    T, H, W = 3, 9, 11
    f = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
    want = oracle.extract(f, 0)
    got = cpt.extract_trajectories(dev(torch.from_numpy(f)), 0).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, want)


def test_field_params_match(cpt):
    for cfg, shape in [(0, None), (1, (32, 48, 3))]:
        f, _ = synthfields.workload(cfg, shape=shape)
        for eb in (1e-1, 1e-3):
            assert cpt.field_params(dev(f), eb) == oracle.params(f.numpy(), eb)


# ------------------------------------------------------------ compression
COMPRESS_CASES = [
    ("w0-mix2-1e-2", 0, None, 1e-2, 2, 1),
    ("w0-mix2-1e-1", 0, None, 1e-1, 2, 1),
    ("w0-mix2-1e-3", 0, None, 1e-3, 2, 1),
    ("w0-lorenzo", 0, None, 1e-2, 0, 1),
    ("w0-sl", 0, None, 1e-2, 1, 1),
    ("w0-mix4-bt4", 0, None, 1e-2, 3, 4),
    ("ragged-mix2", 0, (37, 45, 5), 1e-2, 2, 1),
    ("ragged-mix4", 0, (37, 45, 5), 1e-2, 3, 2),
    ("wind-crop", 1, (48, 80, 4), 1e-3, 2, 1),
    ("turb-crop", 2, (40, 56, 3), 1e-3, 3, 1),
]


@pytest.mark.parametrize("name,cfg,shape,eb,pred,bt", COMPRESS_CASES)
def test_compress_bytes_and_internals_match_oracle(cpt, name, cfg, shape, eb, pred, bt):
    f, m = synthfields.workload(cfg, shape=shape)
    fn = f.numpy()
    dt = m["dt_dx"]
    want, dbg = oracle.compress(fn, eb, predictor=pred, mode_bt=bt, dt_dx=dt, dt_dy=dt, debug=True)
    got, gd = cpt.compress_debug(dev(f), eb, predictor=pred, mode_bt=bt, dt_dx=dt, dt_dy=dt)
    assert np.array_equal(gd["xi"].cpu().numpy(), dbg["xi"])
    assert np.array_equal(gd["xcode"].cpu().numpy(), dbg["xcode"])
    qc = gd["qcode"].cpu().numpy().view(np.uint32)
    lossy = dbg["xcode"] != 24
    assert np.array_equal(qc[lossy], dbg["qcode"][lossy])
    assert np.array_equal(gd["modes"].cpu().numpy(), dbg["modes"])
    assert np.array_equal(gd["feats"].cpu().numpy(), dbg["feats"])
    assert_bytes_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("name,cfg,shape,eb,pred,bt", COMPRESS_CASES)
def test_decompress_matches_oracle(cpt, name, cfg, shape, eb, pred, bt):
    f, m = synthfields.workload(cfg, shape=shape)
    fn = f.numpy()
    dt = m["dt_dx"]
    b = oracle.compress(fn, eb, predictor=pred, mode_bt=bt, dt_dx=dt, dt_dy=dt)
    want = oracle.decompress(b)
    got = cpt.decompress(torch.from_numpy(b).to("cuda")).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    k, ea, _ = oracle.params(fn, eb)
    v = cpt.verify(dev(f), torch.from_numpy(got).to("cuda"), k)
    assert v["fc_t"] == 0 and v["fc_s"] == 0 and v["max_err"] <= ea


@pytest.mark.parametrize("seed", range(4))
def test_tiny_degenerate_roundtrip(cpt, seed):
    rng = np.random.default_rng(seed)
    T, H, W = int(rng.integers(1, 4)), int(rng.integers(2, 10)), int(rng.integers(2, 10))
    f = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
    for pred in (0, 1, 2, 3):
        want = oracle.compress(f, 0.3, predictor=pred)
        got = cpt.compress(torch.from_numpy(f).to("cuda"), 0.3, predictor=pred)
        assert_bytes_equal(got.cpu().numpy(), want)
        g = cpt.decompress(got)
        assert np.array_equal(g.cpu().numpy().view(np.uint32), oracle.decompress(want).view(np.uint32))


@pytest.mark.parametrize("eb,eb_mode", [(1e-12, 1), (0.5, 0), (5e-7, 0)])
def test_extreme_bounds_match_oracle(cpt, eb, eb_mode):
    """An absolute bound below one fixed-point unit (eps' = 0: every vertex
    lossless), the largest relative bound, and a relative bound of a few
    units."""
    f, _ = synthfields.workload(0, shape=(33, 47, 3))
    fn = f.numpy()
    want = oracle.compress(fn, eb, eb_mode=eb_mode)
    got = cpt.compress(dev(f), eb, eb_mode=eb_mode)
    assert_bytes_equal(got.cpu().numpy(), want)
    back = cpt.decompress(got).cpu().numpy()
    assert np.array_equal(back.view(np.uint32), oracle.decompress(want).view(np.uint32))
    k, _, eps = oracle.params(fn, eb, eb_mode)
    if eps == 0:
        assert np.array_equal(back.view(np.uint32), fn.view(np.uint32))


def _spiked_field():
    """The small smooth field with u shifted away from zero and 60 single-
    vertex spikes of +-3: at a relative bound of 1e-4 the spikes and the
    Lorenzo predictions that read them leave residuals past the quantizer's
    range (unpredictable components, stored raw), so runs of 16 vertices
    come with raw words from lossless vertices only, from unpredictable
    components, from both, or with none."""
    f, _ = synthfields.workload(0, shape=(48, 80, 4))
    fn = f.numpy().copy()
    fn[0] += 4.0
    rng = np.random.default_rng(7)
    _, T, H, W = fn.shape
    for _ in range(60):
        t, y, x = rng.integers(T), rng.integers(H), rng.integers(W)
        fn[int(rng.integers(2)), t, y, x] += float(rng.choice([-3.0, 3.0]))
    return fn


@pytest.mark.parametrize("pred", [0, 2])
def test_unpredictable_components_match_oracle(cpt, pred):
    fn = _spiked_field()
    want, dbg = oracle.compress(fn, 1e-4, predictor=pred, debug=True)
    lossy = dbg["xcode"] != oracle.XLOSSLESS
    unp = lossy & (((dbg["qcode"] & 0xFFFF) == 0) | ((dbg["qcode"] >> 16) == 0))
    runs = (~lossy | unp).reshape(-1, 16).sum(1)
    assert unp.sum() >= 100 and (runs == 0).any() and (runs > 0).any()
    got = cpt.compress(torch.from_numpy(fn).to("cuda"), 1e-4, predictor=pred)
    assert_bytes_equal(got.cpu().numpy(), want)
    back = cpt.decompress(got).cpu().numpy()
    assert np.array_equal(back.view(np.uint32), oracle.decompress(want).view(np.uint32))


def test_constant_field(cpt):
    f = torch.full((2, 3, 20, 18), 0.75)
    want = oracle.compress(f.numpy(), 0.1)
    got = cpt.compress(dev(f), 0.1)
    assert_bytes_equal(got.cpu().numpy(), want)
    assert torch.equal(cpt.decompress(got).cpu(), f)


def test_determinism(cpt):
    f, _ = synthfields.workload(0, shape=(40, 52, 6))
    a = cpt.compress(dev(f), 1e-2, predictor=3).cpu()
    for _ in range(3):
        assert torch.equal(cpt.compress(dev(f), 1e-2, predictor=3).cpu(), a)


def test_invalid_arguments(cpt):
    f = torch.zeros((2, 2, 4, 4), device="cuda")
    with pytest.raises(cpt.CptError):
        cpt.compress(f, 0.0)
    with pytest.raises(cpt.CptError):
        cpt.compress(f, 0.7)
    g = f.clone()
    g[0, 0, 1, 1] = float("nan")
    with pytest.raises(cpt.CptError):
        cpt.compress(g, 0.1)
    with pytest.raises(cpt.CptError):
        cpt.compress(torch.zeros((2, 1, 1, 4), device="cuda"), 0.1)
    with pytest.raises(cpt.CptError):
        cpt.compress(f, 0.1, out=torch.empty(64, dtype=torch.uint8, device="cuda"))


def test_corrupted_streams_rejected(cpt):
    f, _ = synthfields.vortex_field(20, 24, 3, 2, seed=5)
    b = oracle.compress(f.numpy(), 1e-2)
    rng = np.random.default_rng(1)
    seen = set()
    for i in range(60):
        c = b.copy()
        if i % 3 == 0:
            c = c[:max(256, int(rng.integers(0, len(b))) & ~3)]
        else:
            for _ in range(int(rng.integers(1, 4))):
                p = int(rng.integers(256, len(c)))
                c[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            cpt.decompress(torch.from_numpy(c).to("cuda"))
            seen.add(0)
        except cpt.CptError as e:
            assert e.status == cpt.ECORRUPT, e
            seen.add(e.status)
    assert cpt.ECORRUPT in seen
