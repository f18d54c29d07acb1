"""Pins of the oracle's lossless stage after Huffman coding (zero-byte
elision of the stream body in independent 4096-byte blocks): hand-worked
containers, the elision boundary, rejection of every form the encoder cannot
write, round trips, and full compress / decompress with the stage."""
import numpy as np
import pytest

import synthfields

TAG = 0x315A4245


def inner_stream(body, seed=0):
    """A 256-byte header of arbitrary bytes but for slot 30 (the stream's
    length) and slot 31 (zero), followed by body."""
    rng = np.random.default_rng(seed)
    h = rng.integers(0, 256, 256).astype(np.uint8)
    body = np.asarray(body, dtype=np.uint8)
    h[240:248] = np.frombuffer(int(256 + body.size).to_bytes(8, "little"), np.uint8)
    h[248:256] = 0
    return np.concatenate([h, body])


def le32(v):
    return list(int(v).to_bytes(4, "little"))


def test_hand_worked_container(ora):
    s = inner_stream([0, 0, 5, 0, 0, 0, 0, 7])
    c = ora.zbe_encode(s)
    # header with slot 31 = tag, one table entry (4 bytes, elided), then the
    # mask 0b10000100 (bytes 2 and 7 nonzero), the bytes 5 and 7, one pad byte
    want = list(s[:248]) + le32(TAG) + [0, 0, 0, 0] + le32(4 | 0x80000000) + [0x84, 5, 7, 0]
    assert list(c) == want
    st, back = ora.zbe_decode_status(c)
    assert st == 0 and np.array_equal(back, s)


def test_block_without_zeros_is_stored(ora):
    body = [1, 2, 3, 4, 5, 6, 7, 8]
    c = ora.zbe_encode(inner_stream(body))
    assert list(c[256:]) == le32(8) + body


def test_elision_boundary(ora):
    """Eight bytes: mask 1 byte + k nonzero bytes, padded to 4.  k = 3 gives 4
    < 8 (elided); k = 4 gives 8, not shorter (stored)."""
    for k, elided in [(0, True), (3, True), (4, False), (7, False)]:
        body = [9] * k + [0] * (8 - k)
        c = ora.zbe_encode(inner_stream(body))
        entry = int.from_bytes(bytes(c[256:260]), "little")
        assert bool(entry >> 31) == elided, k
        assert (entry & 0x7FFFFFFF) == (4 if elided else 8)


def test_blocks_split_at_4096(ora):
    rng = np.random.default_rng(2)
    body = (rng.random(4096 + 12) < 0.2) * rng.integers(1, 256, 4096 + 12)
    s = inner_stream(body.astype(np.uint8))
    c = ora.zbe_encode(s)
    e0 = int.from_bytes(bytes(c[256:260]), "little")
    e1 = int.from_bytes(bytes(c[260:264]), "little")
    nnz0 = int(np.count_nonzero(body[:4096]))
    assert e0 == (((512 + nnz0) + 3) & ~3) | 0x80000000
    # the 12-byte tail block: mask of 2 bytes
    nnz1 = int(np.count_nonzero(body[4096:]))
    tail = ((2 + nnz1 + 3) & ~3)
    assert (e1 & 0x7FFFFFFF) == (tail if tail < 12 else 12)
    assert len(c) == 256 + 8 + (e0 & 0x7FFFFFFF) + (e1 & 0x7FFFFFFF)
    st, back = ora.zbe_decode_status(c)
    assert st == 0 and np.array_equal(back, s)


@pytest.mark.parametrize("density", [0.0, 0.01, 0.3, 0.7, 1.0])
def test_round_trip_random_bodies(ora, density):
    rng = np.random.default_rng(int(density * 100))
    for n in (4, 4092, 4096, 4100, 3 * 4096 + 8):
        body = ((rng.random(n) < density) * rng.integers(1, 256, n)).astype(np.uint8)
        s = inner_stream(body, seed=n)
        c = ora.zbe_encode(s)
        assert len(c) <= ora.lib().cpo_zbe_bound(len(s))
        st, back = ora.zbe_decode_status(c)
        assert st == 0 and np.array_equal(back, s)


def test_encoder_needs_a_consistent_header(ora):
    s = inner_stream([1, 2, 3, 4])
    s[240] ^= 4   # slot 30 no longer the length
    with pytest.raises(ValueError):
        ora.zbe_encode(s)


def test_decoder_rejects_forms_the_encoder_cannot_write(ora):
    s = inner_stream([0, 0, 5, 0, 0, 0, 0, 7])
    c = ora.zbe_encode(s)
    bad = []
    x = c.copy(); x[248] ^= 1; bad.append(x)                        # wrong tag
    x = c.copy(); x[256:260] = le32(8); bad.append(x)               # stored flag, wrong length
    x = c.copy(); x[260] = 0x85; bad.append(x)                      # mask count != stored bytes
    x = c.copy(); x[262] = 0; x[260] = 0x84; bad.append(x)          # a stored byte of zero
    x = c.copy(); x[263] = 1; bad.append(x)                         # nonzero padding
    bad.append(c[:-4].copy())                                       # truncated
    bad.append(np.concatenate([c, np.zeros(4, np.uint8)]))          # trailing bytes
    for i, x in enumerate(bad):
        st, _ = ora.zbe_decode_status(x)
        assert st == ora.ECORRUPT, i
    # an elided form that is not shorter than the block (k = 4 of 8 bytes)
    t = inner_stream([9, 9, 9, 9, 0, 0, 0, 0])
    c2 = np.concatenate([ora.zbe_encode(t)[:256], np.array(le32(8 | 0x80000000), np.uint8),
                         np.array([0x0F, 9, 9, 9, 9, 0, 0, 0], np.uint8)])
    st, _ = ora.zbe_decode_status(c2)
    assert st == ora.ECORRUPT
    # four zero bytes are stored (mask plus padding would be 4, not shorter)
    assert list(ora.zbe_encode(inner_stream([0, 0, 0, 0]))[256:]) == le32(4) + [0, 0, 0, 0]
    # a mask bit beyond the end of a 12-byte block (mask of 2 bytes, 16 bits)
    t = inner_stream([0] * 12)
    c3 = ora.zbe_encode(t)
    assert list(c3[256:]) == le32(4 | 0x80000000) + [0, 0, 0, 0]
    c3[261] = 0x10
    st, _ = ora.zbe_decode_status(c3)
    assert st == ora.ECORRUPT


@pytest.mark.parametrize("pred", [0, 2, 3])
def test_compress_with_stage_round_trips_and_keeps_guarantees(ora, pred):
    f, _ = synthfields.workload(0, shape=(40, 56, 5))
    fn = f.numpy()
    for eb in (1e-1, 1e-2, 1e-3):
        b = ora.compress(fn, eb, predictor=pred)
        c = ora.compress(fn, eb, predictor=pred, backend=1)
        assert np.array_equal(ora.zbe_encode(b), c)
        assert len(c) < len(b)
        info = ora.stream_info(c)
        assert info["backend"] == 1 and info["total_len"] == len(b)
        g = ora.decompress(c)
        assert np.array_equal(g.view(np.uint32), ora.decompress(b).view(np.uint32))
        k, ea, _ = ora.params(fn, eb)
        v = ora.verify(fn, g, k)
        assert v["fc_t"] == 0 and v["fc_s"] == 0 and v["max_err"] <= ea


def test_corrupted_containers_never_crash(ora):
    f, _ = synthfields.workload(0, shape=(24, 32, 3))
    c = ora.compress(f.numpy(), 1e-2, backend=1)
    rng = np.random.default_rng(5)
    for _ in range(200):
        x = c.copy()
        p = int(rng.integers(256, len(x)))
        x[p] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, _ = ora.decompress_status(x)
        assert st in (ora.OK, ora.ECORRUPT)
