// k_entropy.hip — Huffman stage of the compressor (the "Huffman coding" of
// the framework overview in Sec. V of the paper) and its decoder.
//
// Two canonical codes, one for the bound codes (25 symbols) and one for the
// residual codes (1024 symbols), lengths limited to 12 bits by package-merge
// (leaves ordered by (count, symbol); a leaf precedes a package of equal
// weight).  Symbols are cut into chunks of 1024; every chunk is coded
// MSB-first into its own run of 32-bit words, so encoding and decoding run
// one chunk per workgroup / lane.  The codebook is built by one workgroup
// on the device, so compression needs no host round trip for it.
#include "cpt_device.hpp"
#include "launch.hpp"

namespace cpt {

// -------------------------------------------------------------- histogram
__global__ __launch_bounds__(256) void k_hist(const uint8_t* __restrict__ xcode, const uint32_t* __restrict__ qcode,
                                              size_t N, uint32_t* __restrict__ xhist, uint32_t* __restrict__ qhist) {
  __shared__ uint32_t hx[32];
  __shared__ uint32_t hq[QSYM];
  for (int i = threadIdx.x; i < QSYM; i += 256) hq[i] = 0;
  if (threadIdx.x < 32) hx[threadIdx.x] = 0;
  __syncthreads();
  size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += stride) {
    uint32_t c = xcode[i];
    atomicAdd(&hx[c], 1u);
    if (c != XLOSSLESS) {
      uint32_t q = qcode[i];
      atomicAdd(&hq[q & 0xFFFFu], 1u);
      atomicAdd(&hq[q >> 16], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < QSYM; i += 256)
    if (hq[i]) atomicAdd(&qhist[i], hq[i]);
  if (threadIdx.x < XSYM && hx[threadIdx.x]) atomicAdd(&xhist[threadIdx.x], hx[threadIdx.x]);
}

__global__ void k_zero(uint32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ----------------------------------------------------------- codebook
// One workgroup of 1024 threads builds the length-limited canonical code of
// one alphabet (nsym <= 1024).
constexpr int CB_THREADS = 1024;

__device__ void build_code(const uint32_t* __restrict__ hist, int nsym, HuffTables* __restrict__ out,
                           uint32_t* __restrict__ cb, uint32_t* __restrict__ used_out) {
  __shared__ uint64_t key[1024];          // (count << 11) | symbol, sorted
  __shared__ uint64_t lw[2][2048];        // list weights, double-buffered
  __shared__ uint8_t lf[2][2048];         // list item is a leaf
  __shared__ uint16_t lpos[MAXLEN + 1][1024];  // position of leaf i in list j
  __shared__ int llen[MAXLEN + 1];
  __shared__ int nleaf;
  __shared__ uint8_t clen[1024];
  __shared__ int lcount[MAXLEN + 2];
  __shared__ uint32_t first[MAXLEN + 2];
  __shared__ uint32_t wsum[16];
  const int tid = threadIdx.x;

  // used symbols as sortable keys
  uint32_t c = tid < nsym ? hist[tid] : 0;
  key[tid] = c ? (((uint64_t)c << 11) | (uint64_t)tid) : ~0ull;
  clen[tid] = 0;
  if (tid == 0) nleaf = 0;
  __syncthreads();
  if (c) atomicAdd(&nleaf, 1);
  // bitonic sort of 1024 keys
  for (int k = 2; k <= 1024; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      int ixj = tid ^ j;
      if (ixj > tid) {
        uint64_t a = key[tid], b = key[ixj];
        bool up = (tid & k) == 0;
        if ((a > b) == up) {
          key[tid] = b;
          key[ixj] = a;
        }
      }
    }
  __syncthreads();
  const int n = nleaf;
  if (n == 1) {
    if (tid == 0) clen[key[0] & 2047] = 1;
  } else if (n >= 2) {
    // level 1: the leaves
    if (tid < n) {
      lw[1 & 1][tid] = key[tid] >> 11;
      lf[1 & 1][tid] = 1;
      lpos[1][tid] = (uint16_t)tid;
    }
    if (tid == 0) llen[1] = n;
    __syncthreads();
    for (int j = 2; j <= MAXLEN; j++) {
      const int pb = (j - 1) & 1, nb = j & 1;
      const int np = llen[j - 1] / 2;
      // leaf i goes after the packages strictly lighter than it
      if (tid < n) {
        uint64_t w = key[tid] >> 11;
        int lo = 0, hi = np;  // first package with weight >= w
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          uint64_t pw = lw[pb][2 * mid] + lw[pb][2 * mid + 1];
          if (pw < w) lo = mid + 1; else hi = mid;
        }
        int pos = tid + lo;
        lw[nb][pos] = w;
        lf[nb][pos] = 1;
        lpos[j][tid] = (uint16_t)pos;
      }
      // package q goes after the leaves not heavier than it
      for (int q = tid; q < np; q += CB_THREADS) {
        uint64_t pw = lw[pb][2 * q] + lw[pb][2 * q + 1];
        int lo = 0, hi = n;  // first leaf with weight > pw
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if ((key[mid] >> 11) <= pw) lo = mid + 1; else hi = mid;
        }
        int pos = q + lo;
        lw[nb][pos] = pw;
        lf[nb][pos] = 0;
      }
      if (tid == 0) llen[j] = n + np;
      __syncthreads();
    }
    // selection: the first 2n-2 items of the last list, expanded level by level
    if (tid == 0) {
      int m = 2 * n - 2;
      int cnt[MAXLEN + 1];
      for (int j = MAXLEN; j >= 1; j--) {
        int lo = 0, hi = n;  // leaves with position < m
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if ((int)lpos[j][mid] < m) lo = mid + 1; else hi = mid;
        }
        cnt[j] = lo;
        m = 2 * (m - lo);
      }
      for (int j = 1; j <= MAXLEN; j++) lcount[j] = cnt[j];
    }
    __syncthreads();
    if (tid < n) {
      int l = 0;
      for (int j = 1; j <= MAXLEN; j++) l += tid < lcount[j] ? 1 : 0;
      clen[key[tid] & 2047] = (uint8_t)l;
    }
  }
  __syncthreads();
  // canonical codes: first code per length, then ascending symbols
  if (tid <= MAXLEN + 1) lcount[tid] = 0;
  __syncthreads();
  if (tid < nsym && clen[tid]) atomicAdd(&lcount[clen[tid]], 1);
  __syncthreads();
  if (tid == 0) {
    uint32_t code = 0;
    lcount[0] = 0;
    for (int l = 1; l <= MAXLEN; l++) {
      code = (code + (uint32_t)lcount[l - 1]) << 1;
      first[l] = code;
    }
  }
  __syncthreads();
  // rank of a symbol among used symbols of the same length, and among all
  // used symbols (codebook position), by block prefix counts
  uint32_t l = tid < nsym ? clen[tid] : 0;
  uint32_t usedf = l ? 1u : 0u;
  // prefix over used flag
  {
    int lane = tid & 63, wid = tid >> 6;
    uint32_t x = usedf;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = (uint32_t)__shfl_up((int)x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < 16; w++) {
      if (w < wid) base += wsum[w];
      tot += wsum[w];
    }
    uint32_t rank = base + x - usedf;
    if (usedf) cb[1 + rank] = (uint32_t)tid | (l << 16);
    if (tid == 0) {
      cb[0] = tot;
      *used_out = tot;
    }
    __syncthreads();
  }
  if (tid < nsym) {
    uint32_t code = 0;
    if (l) {
      uint32_t r = 0;
      for (int s = 0; s < tid; s++) r += clen[s] == l ? 1u : 0u;
      code = first[l] + r;
    }
    out->code[tid] = code;
    out->len[tid] = (uint8_t)l;
  }
}

__global__ __launch_bounds__(CB_THREADS) void k_codebooks(const uint32_t* __restrict__ xhist,
                                                          const uint32_t* __restrict__ qhist, HuffTables* xt,
                                                          HuffTables* qt, uint32_t* xcb, uint32_t* qcb,
                                                          uint32_t* used) {
  if (blockIdx.x == 0) build_code(xhist, XSYM, xt, xcb, &used[0]);
  else build_code(qhist, QSYM, qt, qcb, &used[1]);
}

// ------------------------------------------------------ symbol streams
__global__ __launch_bounds__(256) void k_gather_q(const uint8_t* __restrict__ xcode, const uint32_t* __restrict__ qcode,
                                                  const uint32_t* __restrict__ qofs, size_t N,
                                                  uint16_t* __restrict__ qsym) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N || xcode[i] == XLOSSLESS) return;
  uint32_t q = qcode[i];
  size_t o = 2 * (size_t)qofs[i];
  qsym[o] = (uint16_t)(q & 0xFFFFu);
  qsym[o + 1] = (uint16_t)(q >> 16);
}

template <typename S>
__global__ __launch_bounds__(256) void k_chunk_bits(const S* __restrict__ sym, size_t n,
                                                    const HuffTables* __restrict__ t, uint32_t* __restrict__ bits,
                                                    uint32_t* __restrict__ words) {
  __shared__ uint32_t red[256];
  size_t base = (size_t)blockIdx.x * CHUNK;
  uint32_t b = 0;
  for (int i = threadIdx.x; i < CHUNK; i += 256)
    if (base + i < n) b += t->len[sym[base + i]];
  red[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bits[blockIdx.x] = red[0];
    words[blockIdx.x] = (red[0] + 31) / 32;
  }
}

// one workgroup per chunk; 16 consecutive symbols per thread
template <typename S>
__global__ __launch_bounds__(256) void k_encode(const S* __restrict__ sym, size_t n, const HuffTables* __restrict__ t,
                                                const uint32_t* __restrict__ wofs, uint32_t* __restrict__ out) {
  __shared__ uint32_t w[CHUNK * MAXLEN / 32];
  __shared__ uint32_t wsum[4];
  const int per = CHUNK / 256;
  size_t base = (size_t)blockIdx.x * CHUNK + (size_t)threadIdx.x * per;
  for (int i = threadIdx.x; i < CHUNK * MAXLEN / 32; i += 256) w[i] = 0;
  uint32_t codes[per];
  uint8_t lens[per];
  uint32_t mine = 0;
#pragma unroll
  for (int i = 0; i < per; i++) {
    if (base + i < n) {
      S s = sym[base + i];
      codes[i] = t->code[s];
      lens[i] = t->len[s];
    } else {
      codes[i] = 0;
      lens[i] = 0;
    }
    mine += lens[i];
  }
  // exclusive prefix of bit counts over the workgroup
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = mine;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  uint32_t off = x - mine;
  for (int q = 0; q < wid; q++) off += wsum[q];
  uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
  for (int i = 0; i < per; i++) {
    uint32_t l = lens[i];
    if (!l) continue;
    uint32_t c = codes[i];
    uint32_t wi = off >> 5, o = off & 31;
    if (o + l <= 32) {
      atomicOr(&w[wi], c << (32 - o - l));
    } else {
      uint32_t spill = o + l - 32;
      atomicOr(&w[wi], c >> spill);
      atomicOr(&w[wi + 1], c << (32 - spill));
    }
    off += l;
  }
  __syncthreads();
  uint32_t nw = (total + 31) / 32;
  uint32_t* dst = out + wofs[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < nw; i += 256) dst[i] = w[i];
}

// ----------------------------------------------------------- raw values
__global__ __launch_bounds__(256) void k_raw_count(const uint8_t* __restrict__ xcode, const uint32_t* __restrict__ qcode,
                                                   size_t N, uint32_t* __restrict__ cnt, uint32_t* __restrict__ nonll) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  uint32_t c;
  if (xcode[i] == XLOSSLESS) {
    c = 2;
    nonll[i] = 0;
  } else {
    uint32_t q = qcode[i];
    c = ((q & 0xFFFFu) == 0) + ((q >> 16) == 0);
    nonll[i] = 1;
  }
  cnt[i] = c;
}

__global__ __launch_bounds__(256) void k_raw(const float* __restrict__ field, const uint8_t* __restrict__ xcode,
                                             const uint32_t* __restrict__ qcode, const uint32_t* __restrict__ rofs,
                                             size_t N, uint32_t* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  uint32_t o = rofs[i];
  uint32_t bu = __float_as_uint(field[i]), bv = __float_as_uint(field[N + i]);
  if (xcode[i] == XLOSSLESS) {
    out[o] = bu;
    out[o + 1] = bv;
  } else {
    uint32_t q = qcode[i];
    if ((q & 0xFFFFu) == 0) out[o++] = bu;
    if ((q >> 16) == 0) out[o] = bv;
  }
}

// ------------------------------------------------------------- decoding
// LUT entry for every 12-bit prefix: symbol | length << 16; 0xFFFFFFFF when
// no codeword matches.
__global__ __launch_bounds__(1024) void k_build_lut(const uint32_t* __restrict__ cb, size_t cb_words, int nsym,
                                                    uint32_t* __restrict__ lut, uint32_t* __restrict__ err) {
  __shared__ uint8_t len[1024];
  __shared__ int lcount[MAXLEN + 2];
  __shared__ uint32_t first[MAXLEN + 2];
  __shared__ int bad;
  __shared__ uint32_t kraft;
  const int tid = threadIdx.x;
  len[tid] = 0;
  if (tid <= MAXLEN + 1) lcount[tid] = 0;
  if (tid == 0) {
    bad = 0;
    kraft = 0;
  }
  for (int i = tid; i < (1 << MAXLEN); i += 1024) lut[i] = 0xFFFFFFFFu;
  __syncthreads();
  uint32_t used = cb_words >= 1 ? cb[0] : 0;
  if (cb_words < 1 || (size_t)used + 1 != cb_words || used > (uint32_t)nsym) {
    if (tid == 0) atomicOr(err, 1u);
    return;
  }
  if ((uint32_t)tid < used) {
    uint32_t e = cb[1 + tid];
    uint32_t s = e & 0xFFFFu, l = e >> 16;
    uint32_t prev = tid > 0 ? (cb[tid] & 0xFFFFu) : 0;
    if (s >= (uint32_t)nsym || l < 1 || l > MAXLEN || (tid > 0 && s <= prev)) atomicOr((uint32_t*)&bad, 1u);
    else {
      len[s] = (uint8_t)l;
      atomicAdd(&lcount[l], 1);
      atomicAdd(&kraft, 1u << (MAXLEN - l));
    }
  }
  __syncthreads();
  if (bad || kraft > (1u << MAXLEN)) {
    if (tid == 0) atomicOr(err, 1u);
    return;
  }
  if (tid == 0) {
    uint32_t code = 0;
    lcount[0] = 0;
    for (int l = 1; l <= MAXLEN; l++) {
      code = (code + (uint32_t)lcount[l - 1]) << 1;
      first[l] = code;
    }
  }
  __syncthreads();
  if (tid < nsym && len[tid]) {
    uint32_t l = len[tid], r = 0;
    for (int s = 0; s < tid; s++) r += len[s] == l ? 1u : 0u;
    uint32_t code = first[l] + r;
    uint32_t lo = code << (MAXLEN - l), hi = (code + 1) << (MAXLEN - l);
    for (uint32_t i = lo; i < hi && i < (1u << MAXLEN); i++) lut[i] = (uint32_t)tid | (l << 16);
  }
}

__global__ __launch_bounds__(256) void k_words_from_bits(const uint32_t* __restrict__ bits, size_t n,
                                                         uint32_t* __restrict__ words) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) words[i] = (bits[i] + 31) / 32;
}

// one lane per chunk
__global__ __launch_bounds__(256) void k_decode(const uint32_t* __restrict__ lut_g, const uint32_t* __restrict__ cbits,
                                                const uint32_t* __restrict__ wofs, const uint32_t* __restrict__ bs,
                                                size_t bs_words, size_t nsym_total, int alphabet,
                                                uint16_t* __restrict__ out, uint32_t* __restrict__ err) {
  __shared__ uint32_t lut[1 << MAXLEN];
  for (int i = threadIdx.x; i < (1 << MAXLEN); i += 256) lut[i] = lut_g[i];
  __syncthreads();
  size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t nch = (nsym_total + CHUNK - 1) / CHUNK;
  if (c >= nch) return;
  uint32_t nbits = cbits[c];
  size_t w0 = wofs[c];
  size_t nw = (nbits + 31) / 32;
  if (w0 + nw > bs_words || nbits > (uint32_t)CHUNK * MAXLEN) {
    atomicOr(err, 2u);
    return;
  }
  size_t lo = c * CHUNK, hi = lo + CHUNK < nsym_total ? lo + CHUNK : nsym_total;
  uint64_t buf = 0;
  int have = 0;
  size_t wi = 0;
  uint32_t consumed = 0;
  for (size_t i = lo; i < hi; i++) {
    while (have <= 32) {
      uint64_t nxt = wi < nw ? bs[w0 + wi] : 0;
      wi++;
      buf |= nxt << (32 - have);
      have += 32;
    }
    uint32_t peek = (uint32_t)(buf >> (64 - MAXLEN));
    uint32_t e = lut[peek];
    uint32_t l = e >> 16;
    if (e == 0xFFFFFFFFu || consumed + l > nbits || (int)(e & 0xFFFFu) >= alphabet) {
      atomicOr(err, 4u);
      return;
    }
    out[i] = (uint16_t)(e & 0xFFFFu);
    buf <<= l;
    have -= (int)l;
    consumed += l;
  }
  if (consumed != nbits) atomicOr(err, 8u);
}

// ============================================================ launchers
static inline unsigned nblk(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
  if (n) k_zero<<<nblk(n), 256, 0, s>>>(p, n);
}
void launch_hist(const uint8_t* xcode, const uint32_t* qcode, size_t N, uint32_t* xhist, uint32_t* qhist,
                 uint32_t* /*nonll*/, uint32_t* /*nraw*/, hipStream_t s) {
  launch_zero_u32(xhist, 32, s);
  launch_zero_u32(qhist, QSYM, s);
  unsigned g = nblk(N);
  if (g > 2048) g = 2048;
  if (g == 0) g = 1;
  k_hist<<<g, 256, 0, s>>>(xcode, qcode, N, xhist, qhist);
}
void launch_codebooks(const uint32_t* xhist, const uint32_t* qhist, HuffTables* xt, HuffTables* qt, uint32_t* xcb,
                      uint32_t* qcb, uint32_t* used, hipStream_t s) {
  k_codebooks<<<2, CB_THREADS, 0, s>>>(xhist, qhist, xt, qt, xcb, qcb, used);
}
void launch_gather_q(const uint8_t* xcode, const uint32_t* qcode, const uint32_t* qofs, size_t N, uint16_t* qsym,
                     hipStream_t s) {
  if (N) k_gather_q<<<nblk(N), 256, 0, s>>>(xcode, qcode, qofs, N, qsym);
}
void launch_chunk_bits_x(const uint8_t* xcode, size_t N, const HuffTables* t, uint32_t* bits, uint32_t* words,
                         hipStream_t s) {
  size_t nch = (N + CHUNK - 1) / CHUNK;
  if (nch) k_chunk_bits<uint8_t><<<(unsigned)nch, 256, 0, s>>>(xcode, N, t, bits, words);
}
void launch_chunk_bits_q(const uint16_t* qsym, size_t n, const HuffTables* t, uint32_t* bits, uint32_t* words,
                         hipStream_t s) {
  size_t nch = (n + CHUNK - 1) / CHUNK;
  if (nch) k_chunk_bits<uint16_t><<<(unsigned)nch, 256, 0, s>>>(qsym, n, t, bits, words);
}
void launch_encode_x(const uint8_t* xcode, size_t N, const HuffTables* t, const uint32_t* wofs, uint32_t* out,
                     hipStream_t s) {
  size_t nch = (N + CHUNK - 1) / CHUNK;
  if (nch) k_encode<uint8_t><<<(unsigned)nch, 256, 0, s>>>(xcode, N, t, wofs, out);
}
void launch_encode_q(const uint16_t* qsym, size_t n, const HuffTables* t, const uint32_t* wofs, uint32_t* out,
                     hipStream_t s) {
  size_t nch = (n + CHUNK - 1) / CHUNK;
  if (nch) k_encode<uint16_t><<<(unsigned)nch, 256, 0, s>>>(qsym, n, t, wofs, out);
}
void launch_raw_count(const uint8_t* xcode, const uint32_t* qcode, size_t N, uint32_t* cnt, uint32_t* nonll,
                      hipStream_t s) {
  if (N) k_raw_count<<<nblk(N), 256, 0, s>>>(xcode, qcode, N, cnt, nonll);
}
void launch_raw(const float* field, const uint8_t* xcode, const uint32_t* qcode, const uint32_t* rofs, size_t N,
                uint32_t* out, hipStream_t s) {
  if (N) k_raw<<<nblk(N), 256, 0, s>>>(field, xcode, qcode, rofs, N, out);
}
void launch_build_lut(const uint32_t* cb, size_t cb_words, int nsym, uint32_t* lut, uint32_t* err, hipStream_t s) {
  k_build_lut<<<1, 1024, 0, s>>>(cb, cb_words, nsym, lut, err);
}
void launch_words_from_bits(const uint32_t* bits, size_t n, uint32_t* words, hipStream_t s) {
  if (n) k_words_from_bits<<<nblk(n), 256, 0, s>>>(bits, n, words);
}
void launch_decode(const uint32_t* lut, const uint32_t* chunk_bits, const uint32_t* wofs, const uint32_t* bs,
                   size_t bs_words, size_t nsym_total, int alphabet, uint16_t* out, uint32_t* err, hipStream_t s) {
  size_t nch = (nsym_total + CHUNK - 1) / CHUNK;
  if (nch) k_decode<<<nblk(nch), 256, 0, s>>>(lut, chunk_bits, wofs, bs, bs_words, nsym_total, alphabet, out, err);
}

}  // namespace cpt
