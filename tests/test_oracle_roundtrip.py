"""End-to-end guarantees of the oracle (Sec. IV-A): after compression and
decompression the pointwise bound holds, every space-time face keeps its
status and sign (FC_t = FC_s = 0), lossless vertices are bit-identical, and
corrupted streams are rejected without crashing."""
import numpy as np
import pytest

import synthfields


def roundtrip(ora, f, eb, **kw):
    b, dbg = ora.compress(f, eb, debug=True, **kw)
    g = ora.decompress(b)
    k, ea, eps = ora.params(f, eb, kw.get("eb_mode", 0))
    v = ora.verify(f, g, k)
    return b, dbg, g, v, (k, ea, eps)


def check_guarantees(ora, f, eb, **kw):
    b, dbg, g, v, (k, ea, eps) = roundtrip(ora, f, eb, **kw)
    assert v["fc_t"] == 0 and v["fc_s"] == 0
    assert v["max_err"] <= ea
    ll = dbg["xcode"] == 24
    N = f[0].size
    assert np.array_equal(f.reshape(2, N)[:, ll].view(np.uint32), g.reshape(2, N)[:, ll].view(np.uint32))
    # the stored bound never exceeds the derived one
    lossy = ~ll
    xt = eps >> dbg["xcode"][lossy].astype(np.int64)
    assert (xt <= dbg["xi"][lossy]).all()
    # quantized vertices stay within their own bound in fixed point
    F = ora.to_fixed(f, k).reshape(2, N).astype(np.int64)
    G = ora.to_fixed(g, k).reshape(2, N).astype(np.int64)
    assert (np.abs(F[:, lossy] - G[:, lossy]) <= xt).all()
    return b, dbg


@pytest.mark.parametrize("eb", [1e-1, 1e-2, 1e-3])
@pytest.mark.parametrize("predictor", [0, 1, 2, 3])
def test_workload0_guarantees(ora, eb, predictor):
    f, m = synthfields.workload(0)
    b, _ = check_guarantees(ora, f.numpy(), eb, predictor=predictor, dt_dx=m["dt_dx"], dt_dy=m["dt_dx"])
    assert len(b) < f.numpy().nbytes


@pytest.mark.parametrize("mode_bt", [2, 4])
def test_mode_blocks_over_frames(ora, mode_bt):
    f, _ = synthfields.workload(0)
    _, dbg = check_guarantees(ora, f.numpy(), 1e-2, predictor=3, mode_bt=mode_bt)
    T = f.shape[1]
    G = -(-T // mode_bt)
    assert len(dbg["modes"]) == G * 4 * 4


@pytest.mark.parametrize("seed", range(8))
def test_tiny_degenerate_fields(ora, seed):
    """Integer-valued fields in {-2..2} with many exact zeros and ties."""
    rng = np.random.default_rng(seed)
    T, H, W = int(rng.integers(1, 4)), int(rng.integers(2, 10)), int(rng.integers(2, 10))
    f = rng.integers(-2, 3, (2, T, H, W)).astype(np.float32)
    for pred in (0, 1, 2):
        check_guarantees(ora, f, 0.3, predictor=pred)


def test_ragged_tiles_and_many_frames(ora):
    f, _ = synthfields.vortex_field(37, 45, 5, 3, seed=77)
    for pred in (0, 2, 3):
        check_guarantees(ora, f.numpy(), 1e-2, predictor=pred)


def test_constant_and_zero_fields(ora):
    for val in (0.0, 1.5):
        f = np.full((2, 3, 5, 6), val, np.float32)
        b, dbg = check_guarantees(ora, f, 0.1)
        assert (dbg["xcode"] == 24).all()  # zero range: every vertex lossless


def test_absolute_bound(ora):
    f, _ = synthfields.workload(0)
    f = f.numpy()
    check_guarantees(ora, f, 2e-3, eb_mode=1)


def test_stream_header(ora):
    f, _ = synthfields.workload(0)
    b = ora.compress(f.numpy(), 1e-2)
    info = ora.stream_info(b)
    assert (info["H"], info["W"], info["T"]) == (64, 64, 8)
    assert info["total_len"] == len(b)
    assert info["K"] == 2 and info["R"] == 512


def test_corrupted_streams_are_rejected(ora):
    f, _ = synthfields.vortex_field(20, 24, 3, 2, seed=5)
    b = ora.compress(f.numpy(), 1e-2)
    rng = np.random.default_rng(0)
    outcomes = set()
    for i in range(300):
        c = b.copy()
        if i % 3 == 0:
            c = c[:int(rng.integers(0, len(b)))]
        else:
            for _ in range(int(rng.integers(1, 4))):
                p = int(rng.integers(0, len(c)))
                c[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, out = ora.decompress_status(c)
        outcomes.add(st)
        assert st in (0, ora.ECORRUPT)
    assert ora.ECORRUPT in outcomes


def test_trajectory_count_preserved(ora):
    f, _ = synthfields.workload(0)
    f = f.numpy()
    k, _, _ = ora.params(f, 1e-2)
    g = ora.decompress(ora.compress(f, 1e-2))
    assert ora.tracks(f, k) == ora.tracks(g, k)
    assert ora.tracks(f, k)[0] == 0
