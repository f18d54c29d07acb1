"""GPU parity of the trajectory graph (Sec. IV-B): Lemma-1 violations and the
number of trajectories equal the CPU oracle's on synthetic, degenerate,
single-vortex and decompressed fields."""
from fractions import Fraction

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


@pytest.mark.parametrize("cfg,shape", [(0, None), (0, (37, 45, 5)), (0, (2, 3, 2)), (1, (64, 96, 6)),
                                       (2, (96, 112, 5)), (0, (40, 40, 1))])
def test_tracks_match_oracle(cpt, cfg, shape):
    f, _ = synthfields.workload(cfg, shape=shape)
    fn = f.numpy()
    k, _, _ = oracle.params(fn, 1e-2)
    want = oracle.tracks(fn, k)
    assert cpt.tracks(dev(f), k) == want
    assert want[0] == 0


@pytest.mark.parametrize("seed", range(4))
def test_tracks_on_degenerate_integer_fields(cpt, seed):
    rng = np.random.default_rng(500 + seed)
    a = rng.integers(-2, 3, (2, 4, 11, 13)).astype(np.float32)
    assert cpt.tracks(dev(a), 0) == oracle.tracks(a, 0)


def test_tracks_of_known_vortex_fields(cpt):
    one = (np.array([[12.3, 11.1]]), np.array([[0.19, -0.11]]), np.array([1.4]), np.array([4.0]))
    two = (np.array([[8.3, 9.1], [27.6, 21.2]]), np.array([[0.21, -0.13], [-0.17, 0.11]]),
           np.array([1.3, -0.9]), np.array([3.5, 4.0]))
    for params, n in ((one, 1), (two, 2)):
        f, _ = synthfields.vortex_field(32, 36, 7, len(params[2]), seed=0, noise=0.0, params=params)
        k, _, _ = oracle.params(f.numpy(), 1e-2)
        assert cpt.tracks(dev(f), k) == (0, n) == oracle.tracks(f.numpy(), k)


def test_tracks_kept_by_compression(cpt):
    f, m = synthfields.workload(2, shape=(128, 144, 6))
    dt = m["dt_dx"]
    fd = dev(f)
    for eb in (1e-3, 1e-2, 1e-1):
        k, _, _ = cpt.field_params(fd, eb)
        s = cpt.compress(fd, eb, dt_dx=dt, dt_dy=dt, backend=1)
        g = cpt.decompress(s)
        before, after = cpt.tracks(fd, k), cpt.tracks(g, k)
        assert before == after == oracle.tracks(f.numpy(), k)


def test_tracks_rejects_a_grid_beyond_24_bits(cpt):
    a = torch.zeros((2, 2, 4, 4), dtype=torch.float32, device="cuda")
    a[0, 0, 1, 1] = 2.0 ** 20
    with pytest.raises(cpt.CptError):
        cpt.tracks(a, 4)
