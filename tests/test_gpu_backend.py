"""GPU parity of the lossless stage after Huffman coding (zero-byte elision,
Sec. V): containers bit-identical to the oracle's for single fields and
batches, decompression of the oracle's containers bit for bit, capacity
errors, and corrupted containers rejected wherever the oracle rejects them."""
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


CASES = [("w0-1e-1", 0, None, 1e-1, 2), ("w0-1e-2", 0, None, 1e-2, 2), ("w0-1e-3", 0, None, 1e-3, 0),
         ("ragged", 0, (37, 45, 5), 1e-2, 3), ("tiny", 0, (2, 3, 2), 1e-2, 2),
         ("wind-crop", 1, (48, 80, 4), 1e-3, 2), ("turb-crop", 2, (96, 112, 4), 1e-2, 2)]


@pytest.mark.parametrize("name,cfg,shape,eb,pred", CASES)
def test_container_matches_oracle(cpt, name, cfg, shape, eb, pred):
    f, m = synthfields.workload(cfg, shape=shape)
    dt = m["dt_dx"]
    kw = dict(predictor=pred, dt_dx=dt, dt_dy=dt)
    want = oracle.compress(f.numpy(), eb, backend=1, **kw)
    got = cpt.compress(dev(f), eb, backend=1, **kw)
    assert_bytes_equal(got.cpu().numpy(), want)
    plain = oracle.compress(f.numpy(), eb, **kw)
    assert cpt.stream_info(got)["total_len"] == len(plain)
    g = cpt.decompress(dev(want)).cpu().numpy()
    assert np.array_equal(g.view(np.uint32), oracle.decompress(plain).view(np.uint32))


def test_batch_of_containers_and_mixed_decompression(cpt):
    shapes = [(17, 23, 3), (48, 64, 5), (2, 2, 1), (64, 31, 2), (40, 40, 6)]
    fields = [synthfields.vortex_field(h, w, t, 3, seed=40 + i)[0] for i, (h, w, t) in enumerate(shapes)]
    want = [oracle.compress(f.numpy(), 1e-2, backend=1) for f in fields]
    for sched in ("launch", "fused"):
        got, st = cpt.compress_batch([dev(f) for f in fields], 1e-2, backend=1, schedule=sched)
        assert st == [0] * len(fields)
        for g, w in zip(got, want):
            assert_bytes_equal(g.cpu().numpy(), w)
    # containers and plain streams in one decompression batch
    streams = [dev(w) if i % 2 == 0 else dev(oracle.compress(fields[i].numpy(), 1e-2))
               for i, w in enumerate(want)]
    dec, st = cpt.decompress_batch(streams)
    assert st == [0] * len(fields)
    for d, w in zip(dec, want):
        assert np.array_equal(d.cpu().numpy().view(np.uint32), oracle.decompress(w).view(np.uint32))


def test_container_capacity(cpt):
    f, _ = synthfields.workload(0)
    want = oracle.compress(f.numpy(), 1e-2, backend=1)
    with pytest.raises(cpt.CptError) as e:
        cpt.compress(dev(f), 1e-2, backend=1, out=torch.empty(len(want) - 4, dtype=torch.uint8, device="cuda"))
    assert e.value.status == cpt.ECAPACITY and str(len(want)) in str(e.value)
    got = cpt.compress(dev(f), 1e-2, backend=1, out=torch.empty(len(want), dtype=torch.uint8, device="cuda"))
    assert_bytes_equal(got.cpu().numpy(), want)


def test_corrupted_containers(cpt):
    f, _ = synthfields.workload(0, shape=(40, 48, 4))
    c = oracle.compress(f.numpy(), 1e-2, backend=1)
    rng = np.random.default_rng(9)
    rejected = 0
    for i in range(80):
        x = c.copy()
        if i % 4 == 0:
            p = 256 + int(rng.integers(0, 4 * ((oracle.stream_info(c)["total_len"] - 256 + 4095) // 4096)))
        else:
            p = int(rng.integers(256, len(x)))
        x[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        zst, _ = oracle.zbe_decode_status(x)
        ost, ref = oracle.decompress_status(x)
        try:
            g = cpt.decompress(dev(x)).cpu().numpy()
            gst = 0
        except cpt.CptError as e:
            assert e.status == cpt.ECORRUPT, e
            gst = cpt.ECORRUPT
        if zst != 0:   # the container itself is malformed: both reject it
            assert gst == cpt.ECORRUPT, (i, p)
            rejected += 1
        elif ost == 0 and gst == 0:
            assert np.array_equal(g.view(np.uint32), ref.view(np.uint32))
    assert rejected > 0
