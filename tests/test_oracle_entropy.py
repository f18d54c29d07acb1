"""Pins of the oracle's rate score (Sec. VI-B, eq. entropy) and of its
length-limited canonical Huffman code."""
import heapq
import itertools
import math

import numpy as np
import pytest


def test_tlog_hand_values(ora):
    assert ora.tlog(0) == 0 and ora.tlog(1) == 0
    assert ora.tlog(2) == 2 * 65536
    assert ora.tlog(4) == 8 * 65536
    assert ora.tlog(8) == 24 * 65536
    assert ora.tlog(128) == 896 * 65536
    assert ora.tlog(3) == math.floor(3 * math.log2(3) * 65536)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 128])
def test_zero_order_entropy_hand_cases(ora, n):
    meta = 65536 // 512  # K = 2, one frame per mode block
    h = np.zeros(1024, np.int32)
    h[512] = n
    assert ora.score(h, n, 0, 2, 1) == 0 + meta  # one symbol: 0 bits
    h[:] = 0
    h[511] = h[513] = n // 2
    assert ora.score(h, n, 0, 2, 1) == 65536 + meta  # two equal halves: 1 bit
    h[:] = 0
    h[:n] = 1
    assert ora.score(h, n, 0, 2, 1) == int(math.log2(n)) * 65536 + meta  # log2 n bits


def test_overflow_penalty_and_meta(ora):
    h = np.zeros(1024, np.int32)
    h[512] = 6
    # lambda = 16 bits times L / (n + L) = 16 * 2/8 = 4 bits
    assert ora.score(h, 6, 2, 2, 1) == 4 * 65536 + 65536 // 512
    # K = 4: two bits per block; four frames per block
    assert ora.score(h, 6, 0, 4, 4) == (2 * 65536) // (512 * 4)
    assert ora.score(np.zeros(1024, np.int32), 0, 0, 2, 1) == 65536 // 512


def test_switch_rule_threshold(ora):
    # SL is taken only when it improves the Lorenzo score by more than 0.3 %
    assert ora.choose([100000, 99699]) == 1
    assert ora.choose([100000, 99700]) == 0
    assert ora.choose([100000, 99701]) == 0
    assert ora.choose([100000, 100000]) == 0
    assert ora.choose([100000, 99999, 50000, 50000]) == 2  # ties to the lower class
    assert ora.choose([1000, 998, 1001, 999]) == 0


def huffman_cost(counts):
    h = [c for c in counts if c > 0]
    if len(h) <= 1:
        return sum(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def huffman_maxlen(counts):
    h = [(c, 0) for c in counts if c > 0]
    heapq.heapify(h)
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        heapq.heappush(h, (a[0] + b[0], max(a[1], b[1]) + 1))
    return h[0][1]


@pytest.mark.parametrize("seed", range(10))
def test_huffman_kraft_bound_and_optimality(ora, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 1025))
    counts = np.zeros(1024, np.uint64)
    idx = rng.choice(1024, n, replace=False)
    counts[idx] = rng.geometric(0.05, n).astype(np.uint64) * rng.integers(1, 100, n).astype(np.uint64)
    L = ora.huffman_lengths(counts, 12)
    used = counts > 0
    assert (L[~used] == 0).all() and (L[used] >= 1).all() and L.max() <= 12
    kraft = sum(2.0 ** -int(l) for l in L[used])
    assert abs(kraft - 1.0) < 1e-12  # complete code
    cost = int((L.astype(np.uint64) * counts).sum())
    opt = huffman_cost(counts.tolist())
    assert cost >= opt
    if huffman_maxlen(counts.tolist()) <= 12:
        assert cost == opt


def test_huffman_length_limit_is_optimal_brute_force(ora):
    """For tiny alphabets, package-merge reaches the minimum cost over every
    length vector with lengths <= maxlen and Kraft sum <= 1."""
    rng = np.random.default_rng(3)
    for _ in range(60):
        n = int(rng.integers(2, 7))
        maxlen = int(rng.integers(max(1, math.ceil(math.log2(n))), 5))
        counts = rng.integers(1, 60, n).astype(np.uint64)
        counts[0] = counts[0] * 50
        L = ora.huffman_lengths(counts, maxlen)
        best = min(sum(int(c) * l for c, l in zip(counts, ls))
                   for ls in itertools.product(range(1, maxlen + 1), repeat=n)
                   if sum(2.0 ** -l for l in ls) <= 1.0)
        assert int((L.astype(np.uint64) * counts).sum()) == best
        assert L.max() <= maxlen


def test_huffman_degenerate_alphabets(ora):
    c = np.zeros(25, np.uint64)
    assert ora.huffman_lengths(c).sum() == 0
    c[7] = 100
    L = ora.huffman_lengths(c)
    assert L[7] == 1 and L.sum() == 1
    # Fibonacci counts need length limiting
    fib = [1, 1]
    while len(fib) < 25:
        fib.append(fib[-1] + fib[-2])
    L = ora.huffman_lengths(np.array(fib, np.uint64), 12)
    assert L.max() == 12
    assert abs(sum(2.0 ** -int(l) for l in L) - 1.0) < 1e-12


def stream_codebook_lengths(b, sec):
    """Code lengths listed in section `sec` of a plain stream (1: bound
    codes, 4: residual codes): the header's slots 20-27 hold the section
    lengths, the sections follow the 256-byte header in order, and a
    codebook is its entry count followed by symbol | length << 16."""
    s = np.frombuffer(bytes(b[:256]), dtype="<u8")
    off = 256 + int(sum(int(s[20 + i]) for i in range(sec)))
    w = np.frombuffer(bytes(b[off:off + int(s[20 + sec])]), dtype="<u4")
    return w[1:1 + int(w[0])] >> 16


def test_long_codewords_round_trip(ora):
    """A field whose residual code needs codewords of 13-16 bits (the
    Huffman code of Sec. V with the 16-bit limit): the stream lists such
    codes, its lengths satisfy Kraft, and decoding restores the field within
    the bound with the lossless vertices bit-exact."""
    import synthfields
    f, _ = synthfields.spiked_field()
    a = f.numpy()
    b, d = ora.compress(a, 1e-3, predictor=0, debug=True)
    L = stream_codebook_lengths(b, 4)
    # every long length occurs: 13, 14, 15 and 16 bits
    assert L.max() == 16 and all((L == n).any() for n in (13, 14, 15, 16))
    assert abs(sum(2.0 ** -int(l) for l in L) - 1.0) < 1e-12
    g = ora.decompress(b)
    _, ea, _ = ora.params(a, 1e-3)
    assert np.abs(g.astype(np.float64) - a).max() <= ea
    ll = np.repeat((d["xcode"] == 24)[None], 2, axis=0).reshape(a.shape)
    assert np.array_equal(g[ll].view(np.uint32), a[ll].view(np.uint32))
