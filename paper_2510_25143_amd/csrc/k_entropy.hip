// k_entropy.hip — Huffman stage of the compressor (the "Huffman coding" of
// the framework overview in Sec. V of the paper) and its decoder.
//
// Two canonical codes, one for the bound codes (25 symbols) and one for the
// residual codes (1024 symbols), lengths limited to 16 bits by package-merge
// (leaves ordered by (count, symbol); a leaf precedes a package of equal
// weight).  Symbols are cut into chunks of 1024; every chunk is coded
// MSB-first into its own run of 32-bit words, so encoding and decoding run
// one chunk per workgroup / lane.  The codebook is built by one workgroup
// on the device, so compression needs no host round trip for it.
#include "batch.hpp"
#include "cpt_device.hpp"
#include "launch.hpp"

namespace cpt {

__global__ void k_zero(uint32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ----------------------------------------------------------- codebook
// One workgroup of 1024 threads builds the length-limited canonical code of
// one alphabet (nsym <= 1024) from the sum of the HIST_SLOTS partial
// histograms at hist + s * stride.
constexpr int CB_THREADS = 1024;

__device__ void build_code(const uint32_t* __restrict__ hist, int stride, int nsym, HuffTables* __restrict__ out,
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
  __shared__ uint32_t wlen[CB_THREADS / 64][MAXLEN + 1];
  const int tid = threadIdx.x;

  // used symbols as sortable keys
  uint32_t c = 0;
  if (tid < nsym)
    for (int sl = 0; sl < HIST_SLOTS; sl++) c += hist[(size_t)sl * stride + tid];
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
  // rank among the symbols of the same length before it: ballots inside
  // the wave, per-wave counts for the waves before
  {
    const int lane = tid & 63, wid = tid >> 6;
    const uint64_t below = (1ull << lane) - 1;
    uint32_t r = 0;
    for (int L = 1; L <= MAXLEN; L++) {
      const uint64_t m = __ballot(l == (uint32_t)L);
      if (l == (uint32_t)L) r = (uint32_t)__popcll(m & below);
      if (lane == 0) wlen[wid][L] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (l)
      for (int w = 0; w < wid; w++) r += wlen[w][l];
    if (tid < nsym) {
      out->code[tid] = l ? first[l] + r : 0u;
      out->len[tid] = (uint8_t)l;
    }
  }
}

// ======================================================= batched encoding
// Every kernel below covers all fields of a batch; a workgroup finds its
// field from a prefix table of per-field workgroup counts and skips fields
// whose status is not ok.  Prefix sums run over the concatenated arrays in
// 32-bit arithmetic: a field's own offsets are differences from the value
// at its first element, which are exact modulo 2^32.

// Per-field histograms of the bound codes and residual codes, and per
// vertex the raw-value count (both components of a lossless vertex, else
// the components whose residual code is 0) and the non-lossless indicator.
// gpre[f]: workgroups of HIST_WG vertices of the fields before f; the
// workgroup takes its spans of HIST_SPAN vertices in turn, each thread 16
// consecutive vertices of a span.  The eight residual symbols around
// QR (residuals -4 .. 3) and the bound codes 0 .. 7, which take most
// vertices, are counted in packed 8-bit fields of a thread's registers and
// summed per wave; only the other symbols are added to the shared
// histograms, so few lanes of a wave add to one LDS word at once.
constexpr int HIST_SPAN = (int)HIST_SPAN_VERTICES;
static_assert(HIST_SPAN == 256 * 16, "16 consecutive vertices per thread");
constexpr uint32_t HQ_LO = QR - 4;  // first residual symbol with a packed counter
constexpr int HIST_WG = (int)HIST_WG_VERTICES;  // vertices per histogram workgroup: four spans
static_assert(HIST_WG % HIST_SPAN == 0 && HIST_WG / HIST_SPAN <= 4, "packed counters hold four spans");

// Sum over the wave, every lane enabled (the same value in every lane).
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
  v = row16_sum(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// Adds the eight packed 8-bit counters of every lane to h[0..7] (each wave
// total stays below 2^16: at most 64 lanes times 128 symbols).
__device__ __forceinline__ void add_packed(uint32_t* h, uint64_t c) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t w = (uint32_t)((c >> (16 * k)) & 0xFFu) | ((uint32_t)((c >> (16 * k + 8)) & 0xFFu) << 16);
    const uint32_t tot = wave_total(w);
    if ((threadIdx.x & 63) == 0) {
      if (tot & 0xFFFFu) atomicAdd(&h[2 * k], tot & 0xFFFFu);
      if (tot >> 16) atomicAdd(&h[2 * k + 1], tot >> 16);
    }
  }
}

// The bound and residual codes of the run of 16 vertices starting at field
// vertex i0 (16-byte loads where aligned); 0xFF / 0 past the field's end hi.
__device__ __forceinline__ void load_run(const uint8_t* __restrict__ xcode, const uint32_t* __restrict__ qcode,
                                         size_t base, size_t i0, size_t hi, uint8_t xc[16], uint32_t qc[16]) {
  const bool full = i0 + 16 <= hi && ((base + i0) & 15) == 0;
  if (full) {
    const uint4 xa = *(const uint4*)(xcode + base + i0);
    const uint32_t xw[4] = {xa.x, xa.y, xa.z, xa.w};
#pragma unroll
    for (int j = 0; j < 16; j++) xc[j] = (uint8_t)(xw[j >> 2] >> (8 * (j & 3)));
    const uint4* q4 = (const uint4*)(qcode + base + i0);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint4 w = q4[j];
      qc[4 * j] = w.x;
      qc[4 * j + 1] = w.y;
      qc[4 * j + 2] = w.z;
      qc[4 * j + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const bool in = i0 + j < hi;
      xc[j] = in ? xcode[base + i0 + j] : (uint8_t)0xFF;
      qc[j] = in ? qcode[base + i0 + j] : 0u;
    }
  }
}

__global__ __launch_bounds__(256) void k_hist_b(const FieldDesc* __restrict__ D, const long long* __restrict__ gpre,
                                                int n, const uint8_t* __restrict__ xcode,
                                                const uint32_t* __restrict__ qcode, uint32_t* __restrict__ xhist,
                                                uint32_t* __restrict__ qhist, uint32_t* __restrict__ sr,
                                                uint32_t* __restrict__ sn) {
  __shared__ uint32_t hx[32];
  __shared__ uint32_t hq[QSYM];
  const int f = find_field(gpre, n, blockIdx.x);
  const FieldDesc& d = D[f];
  const size_t wlo = (size_t)((long long)blockIdx.x - gpre[f]) * HIST_WG;
  const size_t N = (size_t)d.N, whi = wlo + HIST_WG < N ? wlo + HIST_WG : N;
  const size_t base = (size_t)d.voff;
  if (d.status) {
    for (size_t i = wlo + 16 * threadIdx.x; i < whi; i += 16 * 256) {
      sr[d.ro + i / 16] = 0;
      sn[d.ro + i / 16] = 0;
    }
    return;
  }
  for (int i = threadIdx.x; i < QSYM; i += 256) hq[i] = 0;
  if (threadIdx.x < 32) hx[threadIdx.x] = 0;
  __syncthreads();
  // packed counters over all spans of the workgroup: bound codes 0..7,
  // residual symbols HQ_LO..HQ_LO+7 (at most 64 vertices per thread, so no
  // 8-bit field passes 128)
  uint64_t cx = 0, cq = 0;
  for (int sp = 0; sp < HIST_WG / HIST_SPAN; sp++) {
    const size_t lo = wlo + (size_t)sp * HIST_SPAN;
    if (lo >= whi) break;
    const size_t hi = lo + HIST_SPAN < whi ? lo + HIST_SPAN : whi;
    const size_t i0 = lo + (size_t)threadIdx.x * 16;
    uint8_t xc[16];
    uint32_t qc[16];
    load_run(xcode, qcode, base, i0, hi, xc, qc);
    uint32_t rsum = 0, nsum = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const uint32_t c = xc[j];
      if (c == 0xFF) continue;  // past the end
      if (c < 8) cx += 1ull << (8 * c);
      else atomicAdd(&hx[c], 1u);
      if (c == XLOSSLESS) {
        rsum += 2;
      } else {
        const uint32_t u = qc[j] & 0xFFFFu, v = qc[j] >> 16;
        const uint32_t du = u - HQ_LO, dv = v - HQ_LO;
        if (du < 8) cq += 1ull << (8 * du);
        else atomicAdd(&hq[u], 1u);
        if (dv < 8) cq += 1ull << (8 * dv);
        else atomicAdd(&hq[v], 1u);
        rsum += (u == 0) + (v == 0);
        nsum += 1;
      }
    }
    if (i0 < hi) {
      sr[d.ro + i0 / 16] = rsum;
      sn[d.ro + i0 / 16] = nsum;
    }
  }
  add_packed(hx, cx);
  add_packed(hq + HQ_LO, cq);
  __syncthreads();
  // the field's histogram copy this workgroup adds to (HIST_SLOTS per field,
  // summed by the codebook kernel), so that few workgroups queue on one word
  const long long slot = (long long)f * HIST_SLOTS + ((long long)blockIdx.x - gpre[f]) % HIST_SLOTS;
  for (int i = threadIdx.x; i < QSYM; i += 256)
    if (hq[i]) atomicAdd(&qhist[(size_t)slot * QSYM + i], hq[i]);
  if (threadIdx.x < XSYM && hx[threadIdx.x]) atomicAdd(&xhist[(size_t)slot * 32 + threadIdx.x], hx[threadIdx.x]);
}

// two workgroups per field: the bound-code and the residual-code codebook
__global__ __launch_bounds__(CB_THREADS) void k_codebooks_b(const FieldDesc* __restrict__ D,
                                                            const uint32_t* __restrict__ xhist,
                                                            const uint32_t* __restrict__ qhist, HuffTables* xt,
                                                            HuffTables* qt, uint32_t* xcb, uint32_t* qcb,
                                                            uint32_t* used) {
  const int f = blockIdx.x >> 1;
  if (D[f].status) return;
  if ((blockIdx.x & 1) == 0)
    build_code(xhist + (size_t)f * HIST_SLOTS * 32, 32, XSYM, xt + f, xcb + (size_t)f * 32, &used[2 * f]);
  else
    build_code(qhist + (size_t)f * HIST_SLOTS * QSYM, QSYM, QSYM, qt + f, qcb + (size_t)f * (QSYM + 4),
               &used[2 * f + 1]);
}

// Four consecutive vertices per lane (1024 per workgroup), so a run of 16
// vertices is one DPP quad: every residual-coded vertex puts its two
// symbols, its 32-bit residual code, at its run's offset plus the coded
// vertices before it in the run (symbol pairs start at even positions of
// the chunk-aligned symbol array).  Four workgroups per histogram span of
// hpre; those wholly past a field's end only take part in no store.  The
// workgroup's residual codes form one contiguous run of at most 1024 words:
// they are placed in LDS first and written out with coalesced stores (a
// word outside that window, which consistent prefix sums never give, is
// stored directly).
__global__ __launch_bounds__(256) void k_gather_q_b(const FieldDesc* __restrict__ D,
                                                    const long long* __restrict__ hpre, int n,
                                                    const uint8_t* __restrict__ xcode,
                                                    const uint32_t* __restrict__ qcode,
                                                    const uint32_t* __restrict__ sq, uint16_t* __restrict__ qsym) {
  static_assert(HIST_SPAN_VERTICES == 4 * 1024, "four gather workgroups per histogram span");
  const int f = find_field(hpre, n, blockIdx.x >> 2);
  const FieldDesc& d = D[f];
  const size_t i0 = (size_t)((long long)blockIdx.x - 4 * hpre[f]) * 1024 + 4 * (size_t)threadIdx.x;
  const size_t N = (size_t)d.N;
  const bool live = !d.status && i0 < N;
  uint32_t xc[4], qc[4];
  const size_t g = d.voff + (live ? i0 : 0);
  if (live && i0 + 4 <= N && (g & 3) == 0) {
    const uint32_t xw = *reinterpret_cast<const uint32_t*>(xcode + g);
    const uint4 qw = *reinterpret_cast<const uint4*>(qcode + g);
#pragma unroll
    for (int k = 0; k < 4; k++) xc[k] = (xw >> (8 * k)) & 0xFFu;
    qc[0] = qw.x;
    qc[1] = qw.y;
    qc[2] = qw.z;
    qc[3] = qw.w;
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const bool in = live && i0 + k < N;
      xc[k] = in ? xcode[g + k] : (uint32_t)XLOSSLESS;
      qc[k] = in ? qcode[g + k] : 0u;
    }
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) cnt += xc[k] != XLOSSLESS ? 1u : 0u;
  // coded vertices of the lanes before this one in its quad
  const int qi = threadIdx.x & 3;
  const uint32_t t1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cnt, 0x90, 0xF, 0xF, true);  // quad_perm [0,0,1,2]
  const uint32_t t2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cnt, 0x40, 0xF, 0xF, true);  // quad_perm [0,0,0,1]
  const uint32_t t3 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cnt, 0x00, 0xF, 0xF, true);  // quad_perm [0,0,0,0]
  const uint32_t before = (qi >= 1 ? t1 : 0u) + (qi >= 2 ? t2 : 0u) + (qi >= 3 ? t3 : 0u);
  __shared__ uint32_t obuf[1024];
  __shared__ uint32_t oend[4], ostart;
  uint32_t* out = reinterpret_cast<uint32_t*>(qsym + (size_t)d.cqb * CHUNK);
  const uint32_t o = live ? (sq[d.ro + i0 / 16] - sq[d.ro]) + before : 0u;
  uint32_t e = live ? o + cnt : 0u;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) e = max(e, (uint32_t)__shfl_xor((int)e, m));
  if ((threadIdx.x & 63) == 0) oend[threadIdx.x >> 6] = e;
  if (threadIdx.x == 0) ostart = o;
  __syncthreads();
  const uint32_t o0 = ostart, o1 = max(max(oend[0], oend[1]), max(oend[2], oend[3]));
  const uint32_t nw = o1 > o0 ? min(o1 - o0, 1024u) : 0u;
  if (live) {
    uint32_t oo = o;
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (xc[k] != XLOSSLESS) {
        const uint32_t i = oo - o0;
        if (i < nw) obuf[i] = qc[k];
        else out[oo] = qc[k];
        oo++;
      }
  }
  __syncthreads();
  for (uint32_t w = threadIdx.x; w < nw; w += 256) out[o0 + w] = obuf[w];
}

// residual symbols and raw values per field, from the prefix sums
__global__ void k_totals_b(FieldDesc* __restrict__ D, int n, const uint32_t* __restrict__ sn,
                           const uint32_t* __restrict__ sq, const uint32_t* __restrict__ sr,
                           const uint32_t* __restrict__ sro) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  FieldDesc& d = D[f];
  if (d.status) {
    d.nq = d.nraw = d.nchq = 0;
    return;
  }
  const size_t a = d.ro, z = d.ro + (d.N + 15) / 16 - 1;
  const uint32_t nl = sq[z] + sn[z] - sq[a];
  const uint32_t nr = sro[z] + sr[z] - sro[a];
  d.nq = 2 * (long long)nl;
  d.nraw = nr;
  d.nchq = (d.nq + CHUNK - 1) / CHUNK;
}

// bits and 32-bit words of every chunk; chunks past a field's last get 0
// One wave per chunk, four chunks per workgroup (chunk c = 4 blockIdx + wave
// of the concatenated chunks; cpre: chunks of the fields before f).  A lane
// sums the code lengths of symbols lane + 64 k: 16-byte loads of 8 residual
// or 16 bound symbols where the chunk is aligned, single loads otherwise.
// Residual code lengths are looked up in a per-wave LDS copy of the field's
// 1024-entry length table (lanes read it at scattered symbols; bound codes
// touch only the table's first 32 bytes and read it in place).
template <bool RESID>
__global__ __launch_bounds__(256) void k_chunk_bits_b(const FieldDesc* __restrict__ D,
                                                      const long long* __restrict__ cpre, int n, long long ctot,
                                                      const uint8_t* __restrict__ xcode,
                                                      const uint16_t* __restrict__ qsym,
                                                      const HuffTables* __restrict__ tabs,
                                                      uint32_t* __restrict__ bits, uint32_t* __restrict__ words) {
  __shared__ __align__(16) uint8_t ltab[4][1024];
  const long long c = 4 * (long long)blockIdx.x + (threadIdx.x >> 6);
  if (c >= ctot) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int f = find_field(cpre, n, c);
  const FieldDesc& d = D[f];
  const long long lc = c - cpre[f];
  const size_t slot = (size_t)(RESID ? d.cqb : d.cxb) + lc;
  if (RESID) {
    reinterpret_cast<uint4*>(ltab[wv])[lane] = reinterpret_cast<const uint4*>(tabs[f].len)[lane];
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  const long long nsym = d.status ? 0 : (RESID ? d.nq : d.N);
  const long long base = lc * CHUNK;
  const long long cnt = nsym - base < CHUNK ? nsym - base : CHUNK;  // symbols in this chunk (<= 0: none)
  const uint8_t* len = tabs[f].len;
  const uint8_t* lw = ltab[wv];
  uint32_t b = 0;
  if (cnt > 0) {
    constexpr int PER = RESID ? 8 : 16;  // symbols per 16-byte load
    const void* src = RESID ? (const void*)(qsym + (size_t)d.cqb * CHUNK + base) : (const void*)(xcode + d.voff + base);
    if (cnt == CHUNK && ((uintptr_t)src & 15) == 0) {
      const uint4* v = reinterpret_cast<const uint4*>(src);
      uint4 w[CHUNK / PER / 64];
#pragma unroll
      for (int k = 0; k < CHUNK / PER / 64; k++) w[k] = v[lane + 64 * k];
#pragma unroll
      for (int k = 0; k < CHUNK / PER / 64; k++) {
        const uint32_t q[4] = {w[k].x, w[k].y, w[k].z, w[k].w};
#pragma unroll
        for (int h = 0; h < 4; h++) {
          if (RESID) {
            b += lw[q[h] & 0xFFFFu];
            b += lw[q[h] >> 16];
          } else {
            b += len[q[h] & 0xFFu];
            b += len[(q[h] >> 8) & 0xFFu];
            b += len[(q[h] >> 16) & 0xFFu];
            b += len[q[h] >> 24];
          }
        }
      }
    } else {
      for (long long i = lane; i < cnt; i += 64)
        b += RESID ? lw[qsym[(size_t)d.cqb * CHUNK + base + i]] : len[xcode[d.voff + base + i]];
    }
  }
  b = row16_sum(b);
  b = (uint32_t)__builtin_amdgcn_readlane((int)b, 0) + (uint32_t)__builtin_amdgcn_readlane((int)b, 16) +
      (uint32_t)__builtin_amdgcn_readlane((int)b, 32) + (uint32_t)__builtin_amdgcn_readlane((int)b, 48);
  if (lane == 0) {
    bits[slot] = b;
    words[slot] = (b + 31) / 32;
  }
}

// One wave per chunk as above, CHUNK / 64 = 16 consecutive symbols per lane
// (16-byte loads where the chunk is aligned); the chunk's words go to the
// field's bitstream section.  Residual codes are looked up in a per-wave LDS
// copy of the field's table, each entry code | length << 16.
template <bool RESID>
__global__ __launch_bounds__(256) void k_encode_b(const FieldDesc* __restrict__ D, const long long* __restrict__ cpre,
                                                  int n, long long ctot, const uint8_t* __restrict__ xcode,
                                                  const uint16_t* __restrict__ qsym,
                                                  const HuffTables* __restrict__ tabs,
                                                  const uint32_t* __restrict__ wofs) {
  constexpr int NW = CHUNK * MAXLEN / 32, PER = CHUNK / 64;
  static_assert(MAXLEN <= 16 && QSYM == 64 * PER, "32-bit table entries, 16 per lane");
  __shared__ uint32_t wbuf[4][NW];
  __shared__ __align__(16) uint32_t ctab[4][QSYM];
  const long long c = 4 * (long long)blockIdx.x + (threadIdx.x >> 6);
  if (c >= ctot) return;
  const int lane = threadIdx.x & 63;
  uint32_t* w = wbuf[threadIdx.x >> 6];
  const int f = find_field(cpre, n, c);
  const FieldDesc& d = D[f];
  const long long lc = c - cpre[f];
  const long long nsym = RESID ? d.nq : d.N;
  if (d.status || lc * CHUNK >= nsym) return;
  const HuffTables* t = tabs + f;
  uint32_t* ct = ctab[threadIdx.x >> 6];
  if (RESID) {
    const uint4* cq = reinterpret_cast<const uint4*>(t->code) + 4 * lane;
    const uint4 c0 = cq[0], c1 = cq[1], c2 = cq[2], c3 = cq[3];
    const uint4 l4 = reinterpret_cast<const uint4*>(t->len)[lane];
    const uint32_t cv[16] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w,
                             c2.x, c2.y, c2.z, c2.w, c3.x, c3.y, c3.z, c3.w};
    const uint32_t lv[4] = {l4.x, l4.y, l4.z, l4.w};
    uint32_t e[16];
#pragma unroll
    for (int i = 0; i < 16; i++) e[i] = cv[i] | (((lv[i >> 2] >> (8 * (i & 3))) & 0xFFu) << 16);
#pragma unroll
    for (int i = 0; i < 4; i++)
      reinterpret_cast<uint4*>(ct)[4 * lane + i] = make_uint4(e[4 * i], e[4 * i + 1], e[4 * i + 2], e[4 * i + 3]);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  const size_t cb = (size_t)(RESID ? d.cqb : d.cxb);
  const long long base = lc * CHUNK + (long long)lane * PER;
  const long long cnt = nsym - lc * CHUNK < CHUNK ? nsym - lc * CHUNK : CHUNK;
  for (int i = lane; i < NW; i += 64) w[i] = 0;
  uint32_t sym[PER];
  const void* src = RESID ? (const void*)(qsym + cb * CHUNK + lc * CHUNK) : (const void*)(xcode + d.voff + lc * CHUNK);
  if (cnt == CHUNK && ((uintptr_t)src & 15) == 0) {
    if (RESID) {
      const uint4* v = reinterpret_cast<const uint4*>(src) + 2 * lane;
      const uint4 a = v[0], bq = v[1];
      const uint32_t h[8] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w};
#pragma unroll
      for (int i = 0; i < 8; i++) {
        sym[2 * i] = h[i] & 0xFFFFu;
        sym[2 * i + 1] = h[i] >> 16;
      }
    } else {
      const uint4 a = reinterpret_cast<const uint4*>(src)[lane];
      const uint32_t h[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int i = 0; i < 16; i++) sym[i] = (h[i >> 2] >> (8 * (i & 3))) & 0xFFu;
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; i++)
      sym[i] = base + i < nsym ? (RESID ? (uint32_t)qsym[cb * CHUNK + base + i] : (uint32_t)xcode[d.voff + base + i])
                               : 0xFFFFFFFFu;
  }
  uint32_t codes[PER];
  uint8_t lens[PER];
  uint32_t mine = 0;
#pragma unroll
  for (int i = 0; i < PER; i++) {
    const bool in = sym[i] != 0xFFFFFFFFu;
    if (RESID) {
      const uint32_t e = in ? ct[sym[i]] : 0u;
      codes[i] = e & 0xFFFFu;
      lens[i] = (uint8_t)(e >> 16);
    } else {
      codes[i] = in ? t->code[sym[i]] : 0u;
      lens[i] = in ? t->len[sym[i]] : (uint8_t)0;
    }
    mine += lens[i];
  }
  // exclusive prefix of bit counts over the wave
  const uint32_t incl = wave_inclusive(mine);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  uint32_t off = incl - mine;
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
  for (int i = 0; i < PER; i++) {
    const uint32_t l = lens[i];
    if (!l) continue;
    const uint32_t cw = codes[i];
    const uint32_t wi = off >> 5, o = off & 31;
    if (o + l <= 32) {
      atomicOr(&w[wi], cw << (32 - o - l));
    } else {
      const uint32_t spill = o + l - 32;
      atomicOr(&w[wi], cw >> spill);
      atomicOr(&w[wi + 1], cw << (32 - spill));
    }
    off += l;
  }
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint32_t nw = (total + 31) / 32;
  uint32_t* dst = (uint32_t*)(d.out + d.off[RESID ? 6 : 3]) + (wofs[cb + lc] - wofs[cb]);
  for (uint32_t i = lane; i < nw; i += 64) dst[i] = w[i];
}

// Stream layout of every field: section lengths and offsets, total length,
// capacity check, and the header.
__global__ __launch_bounds__(64) void k_layout_b(FieldDesc* __restrict__ D, const uint32_t* __restrict__ used,
                                                 const uint32_t* __restrict__ xwords,
                                                 const uint32_t* __restrict__ xwofs,
                                                 const uint32_t* __restrict__ qwords,
                                                 const uint32_t* __restrict__ qwofs) {
  __shared__ uint64_t slot[HDR_SLOTS];
  __shared__ int ok;
  const int f = blockIdx.x;
  FieldDesc& d = D[f];
  if (d.status) {
    if (threadIdx.x == 0) d.len = 0;
    return;
  }
  if (threadIdx.x == 0) {
    const FieldParams& p = d.p;
    const size_t xa = d.cxb, xz = d.cxb + d.nchx - 1;
    const uint32_t words_x = xwofs[xz] + xwords[xz] - xwofs[xa];
    const size_t qcap = (size_t)(2 * d.N + CHUNK - 1) / CHUNK;
    const size_t qa = d.cqb, qz = d.cqb + qcap - 1;
    const uint32_t words_q = qwofs[qz] + qwords[qz] - qwofs[qa];
    const long long sec[8] = {4 * d.mwords,         4 * (1 + (long long)used[2 * f]),     4 * d.nchx,
                              4 * (long long)words_x, 4 * (1 + (long long)used[2 * f + 1]), 4 * d.nchq,
                              4 * (long long)words_q, 4 * d.nraw};
    long long total = HDR_BYTES;
    for (int i = 0; i < 8; i++) {
      d.sec[i] = sec[i];
      d.off[i] = total;
      total += sec[i];
    }
    d.len = total;
    ok = d.out != nullptr && total <= d.cap;
    if (!ok) {
      d.status = STATUS_ECAPACITY;
      d.reason = REASON_CAPACITY;
    }
    uint64_t ebits = (uint64_t)__double_as_longlong(d.eb_abs);
    const uint64_t s[HDR_SLOTS] = {STREAM_MAGIC | (STREAM_VERSION << 32), (uint64_t)p.H, (uint64_t)p.W,
                                   (uint64_t)p.T, (uint64_t)(int64_t)p.k, ebits, (uint64_t)p.eps, (uint64_t)QR,
                                   (uint64_t)TILE, (uint64_t)p.predictor, (uint64_t)p.bt, (uint64_t)p.K,
                                   (uint64_t)p.cx, (uint64_t)p.sx, (uint64_t)p.cy, (uint64_t)p.sy, (uint64_t)NMAX,
                                   (uint64_t)CHUNK, (uint64_t)MAXLEN, (uint64_t)SL_STRIDE, (uint64_t)sec[0],
                                   (uint64_t)sec[1], (uint64_t)sec[2], (uint64_t)sec[3], (uint64_t)sec[4],
                                   (uint64_t)sec[5], (uint64_t)sec[6], (uint64_t)sec[7], (uint64_t)d.nq,
                                   (uint64_t)d.nraw, (uint64_t)total, 0};
    for (int i = 0; i < HDR_SLOTS; i++) slot[i] = s[i];
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (ok && i < HDR_SLOTS) {
    uint32_t* o = (uint32_t*)d.out;
    o[2 * i] = (uint32_t)(slot[i] & 0xFFFFFFFFu);
    o[2 * i + 1] = (uint32_t)(slot[i] >> 32);
  }
}

// small sections: predictor classes (bit-packed LSB-first), both codebooks
// and both chunk tables; grid (n, SB)
__global__ __launch_bounds__(256) void k_sections_b(const FieldDesc* __restrict__ D, const uint8_t* __restrict__ modes,
                                                    const uint32_t* __restrict__ xcb, const uint32_t* __restrict__ qcb,
                                                    const uint32_t* __restrict__ used,
                                                    const uint32_t* __restrict__ xbits,
                                                    const uint32_t* __restrict__ qbits) {
  const int f = blockIdx.x;
  const FieldDesc& d = D[f];
  if (d.status) return;
  const size_t step = (size_t)gridDim.y * 256, first = (size_t)blockIdx.y * 256 + threadIdx.x;
  uint32_t* out = (uint32_t*)d.out;
  const int mb = d.K == 4 ? 2 : (d.K == 2 ? 1 : 0);
  const size_t nblk = (size_t)d.ndec * d.tx * d.ty;
  const uint8_t* m = modes + d.mbase;
  uint32_t* o0 = out + d.off[0] / 4;
  for (size_t w = first; w < (size_t)d.mwords; w += step) {
    uint32_t v = 0;
    for (int b = 0; b < 32; b++) {
      size_t bit = w * 32 + b;
      size_t blk = bit / mb;
      int k = (int)(bit % mb);
      if (blk < nblk && ((m[blk] >> k) & 1)) v |= 1u << b;
    }
    o0[w] = v;
  }
  const size_t ux = 1 + used[2 * f], uq = 1 + used[2 * f + 1];
  for (size_t w = first; w < ux; w += step) out[d.off[1] / 4 + w] = xcb[(size_t)f * 32 + w];
  for (size_t w = first; w < uq; w += step) out[d.off[4] / 4 + w] = qcb[(size_t)f * (QSYM + 4) + w];
  for (size_t w = first; w < (size_t)d.nchx; w += step) out[d.off[2] / 4 + w] = xbits[d.cxb + w];
  for (size_t w = first; w < (size_t)d.nchq; w += step) out[d.off[5] / 4 + w] = qbits[d.cqb + w];
}

// raw words, one thread per run of 16 vertices: two per lossless vertex,
// one per unpredictable component, from the run's offset on in vertex order.
// The run's raw-word count sr (from the histogram pass) decides what is
// read: nothing when it is zero, only the bound codes when it is twice the
// lossless vertices (no unpredictable component), else the residual codes
// as well.
__global__ __launch_bounds__(256) void k_raw_b(const FieldDesc* __restrict__ D, const long long* __restrict__ hpre,
                                               int n, const uint8_t* __restrict__ xcode,
                                               const uint32_t* __restrict__ qcode, const uint32_t* __restrict__ sr,
                                               const uint32_t* __restrict__ sro) {
  const int f = find_field(hpre, n, blockIdx.x);
  const FieldDesc& d = D[f];
  if (d.status) return;
  const size_t lo = (size_t)((long long)blockIdx.x - hpre[f]) * HIST_SPAN;
  const size_t N = (size_t)d.N, hi = lo + HIST_SPAN < N ? lo + HIST_SPAN : N;
  const size_t i0 = lo + (size_t)threadIdx.x * 16;
  if (i0 >= hi) return;
  const uint32_t rw = sr[d.ro + i0 / 16];
  if (rw == 0) return;
  const size_t g = (size_t)d.voff + i0;
  const bool full = i0 + 16 <= hi && (g & 15) == 0;
  uint8_t xc[16];
  if (full) {
    const uint4 xa = *(const uint4*)(xcode + g);
    const uint32_t xw[4] = {xa.x, xa.y, xa.z, xa.w};
#pragma unroll
    for (int j = 0; j < 16; j++) xc[j] = (uint8_t)(xw[j >> 2] >> (8 * (j & 3)));
  } else {
#pragma unroll
    for (int j = 0; j < 16; j++) xc[j] = i0 + j < hi ? xcode[g + j] : (uint8_t)0xFF;
  }
  uint32_t nll = 0;
#pragma unroll
  for (int j = 0; j < 16; j++) nll += xc[j] == XLOSSLESS ? 1u : 0u;
  uint32_t qc[16];
#pragma unroll
  for (int j = 0; j < 16; j++) qc[j] = 0xFFFFFFFFu;  // no zero half: predictable
  if (rw != 2 * nll) {
    if (full) {
      const uint4* q4 = (const uint4*)(qcode + g);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const uint4 w = q4[j];
        qc[4 * j] = w.x;
        qc[4 * j + 1] = w.y;
        qc[4 * j + 2] = w.z;
        qc[4 * j + 3] = w.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; j++)
        if (i0 + j < hi) qc[j] = qcode[g + j];
    }
  }
  uint32_t* out = (uint32_t*)(d.out + d.off[7]);
  uint32_t o = sro[d.ro + i0 / 16] - sro[d.ro];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const size_t i = i0 + j;
    if (xc[j] == XLOSSLESS) {
      out[o] = __float_as_uint(d.field[i]);
      out[o + 1] = __float_as_uint(d.field[N + i]);
      o += 2;
    } else if (xc[j] < XLOSSLESS) {
      if ((qc[j] & 0xFFFFu) == 0) out[o++] = __float_as_uint(d.field[i]);
      if ((qc[j] >> 16) == 0) out[o++] = __float_as_uint(d.field[N + i]);
    }
  }
}

// ------------------------------------------------------------- decoding
// The decoding table of one alphabet (layout: LUT_* in cpt_device.hpp).
// Called by 1024 threads.  The codebook lists (symbol, length) in
// increasing symbol order; a symbol's canonical code is first[l] plus its
// rank among the symbols of length l.  Ranks come from wave ballots; the
// codes, left-aligned to MAXLEN bits, are laid out in canonical order (their
// starts then increase), and every 12-bit prefix finds by binary search the
// last code starting at or before the end of its 16-position window: a code
// of at most 12 bits covers the whole window (its start is a multiple of
// 16), a longer one makes the prefix LUT_LONG, and a window no code reaches
// is LUT_BAD.  An invalid codebook leaves every entry LUT_BAD.
__device__ void build_lut(const uint32_t* __restrict__ cb, size_t cb_words, int nsym, uint32_t* __restrict__ lut,
                          uint32_t* __restrict__ err) {
  __shared__ int lcount[MAXLEN + 2];
  __shared__ uint32_t first[MAXLEN + 2], lbase[MAXLEN + 2];
  __shared__ uint32_t wcnt[16][MAXLEN + 1];
  __shared__ uint32_t sstart[1024], sval[1024];
  __shared__ int bad;
  __shared__ uint32_t kraft;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid <= MAXLEN + 1) lcount[tid] = 0;
  if (tid == 0) {
    bad = 0;
    kraft = 0;
  }
  // no long codes until the table says otherwise
  if (tid < LUT_SYMS - LUT_FIRST) lut[LUT_FIRST + tid] = 0u;
  __syncthreads();
  const uint32_t used = cb_words >= 1 ? cb[0] : 0;
  if (cb_words < 1 || (size_t)used + 1 != cb_words || used > (uint32_t)nsym) {
    for (int i = tid; i < (1 << LUT_BITS); i += 1024) lut[i] = LUT_BAD;
    if (tid == 0) atomicOr(err, 1u);
    return;
  }
  uint32_t s = 0, l = 0;
  if ((uint32_t)tid < used) {
    const uint32_t e = cb[1 + tid];
    s = e & 0xFFFFu;
    l = e >> 16;
    const uint32_t prev = tid > 0 ? (cb[tid] & 0xFFFFu) : 0;
    if (s >= (uint32_t)nsym || l < 1 || l > MAXLEN || (tid > 0 && s <= prev)) {
      atomicOr((uint32_t*)&bad, 1u);
      l = 0;
    } else {
      atomicAdd(&lcount[l], 1);
      atomicAdd(&kraft, 1u << (MAXLEN - l));
    }
  }
  // rank within the wave among entries of the same length
  uint32_t rank = 0;
  for (int L = 1; L <= MAXLEN; L++) {
    const unsigned long long m = __ballot(l == (uint32_t)L);
    if (l == (uint32_t)L) rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wv][L] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (bad || kraft > (1u << MAXLEN)) {
    for (int i = tid; i < (1 << LUT_BITS); i += 1024) lut[i] = LUT_BAD;
    if (tid == 0) atomicOr(err, 1u);
    return;
  }
  if (tid == 0) {
    uint32_t code = 0, base = 0;
    lcount[0] = 0;
    for (int L = 1; L <= MAXLEN; L++) {
      code = (code + (uint32_t)lcount[L - 1]) << 1;
      first[L] = code;
      lbase[L] = base;
      base += (uint32_t)lcount[L];
    }
  }
  if (l) {
    for (int w = 0; w < wv; w++) rank += wcnt[w][l];
  }
  __syncthreads();
  if (l) {
    const uint32_t ci = lbase[l] + rank;
    sstart[ci] = (first[l] + rank) << (MAXLEN - l);
    sval[ci] = s | (l << 16);
    // the long codes' symbols in canonical order, from index 0
    if (l > (uint32_t)LUT_BITS)
      reinterpret_cast<uint16_t*>(lut + LUT_SYMS)[ci - lbase[LUT_BITS + 1]] = (uint16_t)s;
  }
  if (tid < MAXLEN - LUT_BITS) {
    const int L = LUT_BITS + 1 + tid;
    lut[LUT_FIRST + tid] = first[L];
    lut[LUT_COUNT + tid] = (uint32_t)lcount[L];
    lut[LUT_BASE + tid] = lbase[L] - lbase[LUT_BITS + 1];
  }
  __syncthreads();
  constexpr uint32_t WIN = 1u << (MAXLEN - LUT_BITS);
  for (int i = tid; i < (1 << LUT_BITS); i += 1024) {
    uint32_t v = LUT_BAD;
    const uint32_t ws = (uint32_t)i * WIN, we = ws + WIN - 1;
    if (used > 0 && sstart[0] <= we) {
      int lo = 0, hi = (int)used - 1;  // the last code starting at or before we
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sstart[mid] <= we) lo = mid;
        else hi = mid - 1;
      }
      const uint32_t cl = sval[lo] >> 16, st = sstart[lo];
      if (st > ws || cl > (uint32_t)LUT_BITS) {
        // a long code starts inside the window, or covers its start
        if (st > ws || ws < st + (1u << (MAXLEN - cl))) v = LUT_LONG;
      } else if (ws < st + (1u << (MAXLEN - cl))) {
        v = sval[lo];
      }
    }
    lut[i] = v;
  }
}

// One lane per chunk.  Lanes decode DEC_STEP symbols at a time into a
// per-wave staging buffer, then the wave writes the 64 chunks' pieces as
// 32-bit words, each piece contiguous (16 lanes per 64-byte piece).  A
// piece of DEC_STEP symbols consumes at most DEC_STEP * MAXLEN bits, which
// takes at most DEC_WIN refills of the 64-bit bit buffer (one more than the
// bits' word count covers a buffer that starts the piece empty), so before
// each piece every lane fetches the next DEC_WIN words of its chunk into its
// window in LDS, all loads in flight together and one wait, and the buffer
// refills from there.
constexpr int DEC_STEP = 32;
constexpr int DEC_WIN = (DEC_STEP * MAXLEN + 31) / 32 + 1;
// chunks cfirst .. cfirst + 255 of one stream (the workgroup's share)
__device__ __forceinline__ void decode_chunks(const uint32_t* __restrict__ lut_g, const uint32_t* __restrict__ cbits,
                              const uint32_t* __restrict__ wofs, uint32_t wbase, const uint32_t* __restrict__ bs,
                              size_t bs_words, size_t nsym_total, uint16_t* __restrict__ out,
                              uint32_t* __restrict__ err, size_t cfirst) {
  __shared__ __align__(16) uint32_t lut[LUT_WORDS];
  __shared__ uint32_t stage[4][64][DEC_STEP / 2 + 1];  // per wave, per lane: DEC_STEP symbols
  __shared__ uint32_t win[4][64][DEC_WIN];             // per wave, per lane: the piece's words
  {
    static_assert(LUT_WORDS % 4 == 0, "the table is copied in 16-byte pieces");
    constexpr int NV = LUT_WORDS / 4, NL = (NV + 255) / 256;
    uint4 lv[NL];
#pragma unroll
    for (int k = 0; k < NL; k++)
      if (threadIdx.x + 256 * k < NV) lv[k] = reinterpret_cast<const uint4*>(lut_g)[threadIdx.x + 256 * k];
#pragma unroll
    for (int k = 0; k < NL; k++)
      if (threadIdx.x + 256 * k < NV) reinterpret_cast<uint4*>(lut)[threadIdx.x + 256 * k] = lv[k];
  }
  __syncthreads();
  const uint16_t* lsym = reinterpret_cast<const uint16_t*>(lut + LUT_SYMS);
  // the long-code ranges of the workgroup's alphabet, held in registers
  // (read after the barrier that completes the copy)
  uint32_t lfirst[MAXLEN - LUT_BITS], lcnt[MAXLEN - LUT_BITS], lbas[MAXLEN - LUT_BITS];
#pragma unroll
  for (int i = 0; i < MAXLEN - LUT_BITS; i++) {
    lfirst[i] = lut[LUT_FIRST + i];
    lcnt[i] = lut[LUT_COUNT + i];
    lbas[i] = lut[LUT_BASE + i];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t nch = (nsym_total + CHUNK - 1) / CHUNK;
  const size_t c0 = cfirst + (size_t)wv * 64;  // first chunk of this wave
  if (c0 >= nch) return;  // whole wave past the end
  const size_t c = c0 + lane;
  bool live = c < nch;
  uint32_t nbits = 0;
  size_t w0 = 0, nw = 0;
  if (live) {
    nbits = cbits[c];
    w0 = wofs[c] - wbase;
    nw = (nbits + 31) / 32;
    if (w0 + nw > bs_words || nbits > (uint32_t)CHUNK * MAXLEN) {
      atomicOr(err, 2u);
      live = false;
    }
  }
  if (!live) nw = 0;
  const size_t lo = c * CHUNK;
  const size_t hi = live ? (lo + CHUNK < nsym_total ? lo + CHUNK : nsym_total) : lo;
  const uint32_t* cw = bs + w0;  // the chunk's words (only the first nw are read)
  uint32_t* mywin = win[wv][lane];
  uint64_t buf = 0;
  int have = 0;
  uint32_t wi = 0;  // next word of the chunk to enter the bit buffer
  uint32_t consumed = 0;
  bool bad = false;
  for (int base = 0; base < CHUNK; base += DEC_STEP) {
    // the words wi .. wi + DEC_WIN - 1 that this piece may need (0 past the
    // chunk's end)
    uint32_t wl[DEC_WIN];
#pragma unroll
    for (int k = 0; k < DEC_WIN; k++) wl[k] = nw > 0 ? cw[wi + k < nw ? wi + k : 0] : 0u;
#pragma unroll
    for (int k = 0; k < DEC_WIN; k++) mywin[k] = wi + k < nw ? wl[k] : 0u;
    const uint32_t wbeg = wi;
    // symbols of this piece in the lane's chunk
    const int navail = lo + base < hi ? (int)min((size_t)DEC_STEP, hi - (lo + base)) : 0;
    // decode this lane's next DEC_STEP symbols into the staging buffer (the
    // table holds only symbols of the alphabet: the codebook was checked)
    uint32_t pair = 0;
    for (int k = 0; k < DEC_STEP; k++) {
      uint32_t sym = 0;
      if (!bad && k < navail) {
        if (have <= 32) {
          buf |= (uint64_t)mywin[wi - wbeg] << (32 - have);
          wi++;
          have += 32;
        }
        uint32_t e = lut[(uint32_t)(buf >> (64 - LUT_BITS))];
        if (e == LUT_LONG) {
          // a code of 13..16 bits: the length whose canonical range holds
          // the window's prefix of that length (codes are prefix-free, so
          // at most one does; the shortest is kept)
          const uint32_t w16 = (uint32_t)(buf >> (64 - MAXLEN));
          uint32_t idx = 0, L = 0;
#pragma unroll
          for (int i = MAXLEN - LUT_BITS - 1; i >= 0; i--) {
            const uint32_t dlt = (w16 >> (MAXLEN - LUT_BITS - 1 - i)) - lfirst[i];
            if (dlt < lcnt[i]) {
              idx = lbas[i] + dlt;
              L = (uint32_t)(LUT_BITS + 1 + i);
            }
          }
          e = L ? ((uint32_t)lsym[min(idx, 1023u)] | (L << 16)) : LUT_BAD;
        }
        const uint32_t l = e >> 16;
        if (e == LUT_BAD || consumed + l > nbits) {
          atomicOr(err, 4u);
          bad = true;
        } else {
          sym = e & 0xFFFFu;
          buf <<= l;
          have -= (int)l;
          consumed += l;
        }
      }
      if (k & 1) stage[wv][lane][k >> 1] = pair | (sym << 16);
      else pair = sym;
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // write: piece (chunk c0 + q, symbols base .. base + DEC_STEP) as 16 words;
    // when every chunk of the wave is whole, 32-bit offsets from one base
    if ((c0 + 64) * CHUNK <= nsym_total) {
      uint32_t* ow = reinterpret_cast<uint32_t*>(out + c0 * CHUNK + base);
      for (int d = lane; d < 64 * (DEC_STEP / 2); d += 64) {
        const int q = d / (DEC_STEP / 2), w = d - q * (DEC_STEP / 2);
        ow[q * (CHUNK / 2) + w] = stage[wv][q][w];
      }
    } else {
      for (int d = lane; d < 64 * (DEC_STEP / 2); d += 64) {
        const int q = d / (DEC_STEP / 2), w = d - q * (DEC_STEP / 2);
        const size_t cc = c0 + q;
        if (cc >= nch) continue;
        const size_t s0 = cc * CHUNK + base + 2 * w;
        const size_t top = cc * CHUNK + CHUNK < nsym_total ? cc * CHUNK + CHUNK : nsym_total;
        const uint32_t v = stage[wv][q][w];
        if (s0 + 1 < top) {
          *(uint32_t*)(out + s0) = v;
        } else if (s0 < top) {
          out[s0] = (uint16_t)(v & 0xFFFFu);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  if (live && !bad && consumed != nbits) atomicOr(err, 8u);
}

// ===================================================== batched decoding
// Every kernel covers all streams of a batch; a workgroup finds its stream
// from a prefix table; error bits are recorded per stream.
__global__ __launch_bounds__(256) void k_unpack_modes_b(DecDesc* __restrict__ D, const long long* __restrict__ mpre,
                                                        int n, uint8_t* __restrict__ modes) {
  const int f = find_field(mpre, n, blockIdx.x);
  DecDesc& d = D[f];
  const size_t i = (size_t)((long long)blockIdx.x - mpre[f]) * 256 + threadIdx.x;
  if (i >= (size_t)d.nblk) return;
  const uint32_t* in = d.sec[0];
  uint32_t v = 0;
  for (int k = 0; k < d.mb; k++) {
    const size_t bit = i * d.mb + k;
    v |= ((in[bit / 32] >> (bit % 32)) & 1u) << k;
  }
  if ((int)v >= d.p.K) atomicOr(&d.err, 256u);
  modes[d.mbase + i] = (uint8_t)v;
}

__global__ __launch_bounds__(1024) void k_build_lut_b(DecDesc* __restrict__ D, uint32_t* __restrict__ luts) {
  const int f = blockIdx.x >> 1, a = blockIdx.x & 1;
  DecDesc& d = D[f];
  build_lut(d.sec[a ? 4 : 1], (size_t)d.secw[a ? 4 : 1], a ? QSYM : XSYM, luts + (size_t)blockIdx.x * LUT_WORDS,
            &d.err);
}

// words of every chunk from its bit count (chunk table of the stream)
template <bool RESID>
__global__ __launch_bounds__(256) void k_words_from_bits_b(const DecDesc* __restrict__ D,
                                                           const long long* __restrict__ cpre, int n, long long tot,
                                                           uint32_t* __restrict__ words) {
  const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
  if (c >= tot) return;
  const int f = find_field(cpre, n, c);
  const DecDesc& d = D[f];
  const long long lc = c - cpre[f];
  words[c] = (d.sec[RESID ? 5 : 2][lc] + 31) / 32;
}

// Both code streams of every stream in one launch: the first dxblocks
// workgroups decode bound codes, the rest residual codes (256 chunks each;
// dxpre / dqpre: workgroups of the streams before f).  Either alone leaves
// the chip with one or two waves per SIMD; together they overlap.
__global__ __launch_bounds__(256) void k_decode_b(DecDesc* __restrict__ D, const long long* __restrict__ dxpre,
                                                  long long dxblocks, const long long* __restrict__ dqpre, int n,
                                                  const uint32_t* __restrict__ luts,
                                                  const uint32_t* __restrict__ xwofs,
                                                  const uint32_t* __restrict__ qwofs, uint16_t* __restrict__ xs,
                                                  uint16_t* __restrict__ qs) {
  const bool resid = (long long)blockIdx.x >= dxblocks;
  const long long b = resid ? (long long)blockIdx.x - dxblocks : (long long)blockIdx.x;
  const long long* pre = resid ? dqpre : dxpre;
  const int f = find_field(pre, n, b);
  DecDesc& d = D[f];
  const uint32_t* wofs = resid ? qwofs : xwofs;
  const size_t cb = (size_t)(resid ? d.cqb : d.cxb);
  const size_t cfirst = (size_t)(b - pre[f]) * 256;
  decode_chunks(luts + (size_t)(2 * f + (resid ? 1 : 0)) * LUT_WORDS, d.sec[resid ? 5 : 2], wofs + cb, wofs[cb],
                d.sec[resid ? 6 : 3], (size_t)d.secw[resid ? 6 : 3], (size_t)(resid ? d.nq : d.N),
                resid ? qs + (size_t)d.qsb : xs + (size_t)d.voff, &d.err, cfirst);
}

// One thread per segment (block row): its stream, the segment within the
// stream, the segment's first vertex g0 and its length (16, or less at the
// right edge).  A stream has fewer than 2^31 segments: 32-bit divisions.
struct SegRow {
  int f;
  unsigned ls, len;
  size_t g0;
  bool live;
};
__device__ __forceinline__ SegRow seg_row(const DecDesc* __restrict__ D, const long long* __restrict__ spre, int n) {
  SegRow q;
  q.f = find_field(spre, n, blockIdx.x);
  const DecDesc& d = D[q.f];
  const long long ls = ((long long)blockIdx.x - spre[q.f]) * 256 + threadIdx.x;
  q.live = ls < d.nseg;
  q.ls = q.live ? (unsigned)ls : 0u;
  const unsigned tx = (unsigned)d.p.tx, H = (unsigned)d.p.H, W = (unsigned)d.p.W;
  const unsigned ty = q.ls / tx, t = ty / H;
  const unsigned bx = q.ls - ty * tx, y = ty - t * H;
  q.len = min(16u, W - 16 * bx);
  q.g0 = ((size_t)t * H + y) * W + 16 * bx;
  return q;
}

// the segment's bound codes (16-byte loads where the row is aligned)
__device__ __forceinline__ void seg_codes(const uint16_t* __restrict__ p, unsigned len, uint32_t c[16]) {
  if (len == 16 && ((uintptr_t)p & 15) == 0) {
    const uint4 a = reinterpret_cast<const uint4*>(p)[0], b = reinterpret_cast<const uint4*>(p)[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int j = 0; j < 8; j++) {
      c[2 * j] = w[j] & 0xFFFFu;
      c[2 * j + 1] = w[j] >> 16;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; j++) c[j] = (unsigned)j < len ? p[j] : (uint32_t)XLOSSLESS;
  }
}

// residual-coded vertices per segment; a bound code above 24 is an error
__global__ __launch_bounds__(256) void k_seg_nonll_b(DecDesc* __restrict__ D, const long long* __restrict__ spre,
                                                     int n, const uint16_t* __restrict__ xs,
                                                     uint32_t* __restrict__ sn) {
  const SegRow q = seg_row(D, spre, n);
  if (!q.live) return;
  DecDesc& d = D[q.f];
  uint32_t c[16];
  seg_codes(xs + d.voff + q.g0, q.len, c);
  uint32_t cnt = 0;
  bool over = false;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const bool in = (unsigned)j < q.len;
    over |= in && c[j] > XLOSSLESS;
    cnt += in && c[j] < XLOSSLESS ? 1u : 0u;
  }
  if (over) atomicOr(&d.err, 16u);
  sn[d.soff + q.ls] = cnt;
}

// raw words per segment (two for a lossless vertex, one per unpredictable
// component); a residual position past the stream's symbols or a bound too
// small for its code is an error.  Symbol pairs start at even positions of
// an even-aligned array, so each pair is one 32-bit word.  The 256
// consecutive segments of a workgroup (one field) own one contiguous run of
// pairs, at most 16 per segment; the workgroup first copies that run into
// LDS with coalesced loads, and each thread then reads its pairs from there
// (a pair outside the copied run, which consistent prefix sums never give,
// is read from memory).
constexpr int SEG_RAW_WORDS = 256 * 16;
__global__ __launch_bounds__(256) void k_seg_raw_b(DecDesc* __restrict__ D, const long long* __restrict__ spre, int n,
                                                   const uint16_t* __restrict__ xs, const uint16_t* __restrict__ qs,
                                                   const uint32_t* __restrict__ sq, uint32_t* __restrict__ sr) {
  __shared__ uint32_t run[SEG_RAW_WORDS];
  __shared__ uint32_t wend[4];
  const SegRow q = seg_row(D, spre, n);
  DecDesc& d = D[q.f];
  uint32_t c[16];
  if (q.live) {
    seg_codes(xs + d.voff + q.g0, q.len, c);
  } else {
#pragma unroll
    for (int j = 0; j < 16; j++) c[j] = XLOSSLESS;
  }
  const uint32_t* qq = reinterpret_cast<const uint32_t*>(qs + d.qsb);
  const uint32_t o0 = q.live ? 2u * (sq[d.soff + q.ls] - sq[d.soff]) : 0u;
  uint32_t coded = 0;
#pragma unroll
  for (int j = 0; j < 16; j++) coded += (unsigned)j < q.len && c[j] < XLOSSLESS ? 1u : 0u;
  // the run: from the first segment's first pair to the furthest pair end
  uint32_t e = q.live ? o0 + 2u * coded : 0u;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) e = max(e, (uint32_t)__shfl_xor((int)e, m));
  if ((threadIdx.x & 63) == 0) wend[threadIdx.x >> 6] = e;
  __shared__ uint32_t wlo;
  if (threadIdx.x == 0) wlo = o0 >> 1;
  __syncthreads();
  const uint32_t w0 = wlo;
  const uint32_t pend = max(max(wend[0], wend[1]), max(wend[2], wend[3]));
  const uint32_t wlim = min(pend, (uint32_t)min(d.nq, (long long)0xFFFFFFFF)) >> 1;
  const uint32_t nw = wlim > w0 ? min(wlim - w0, (uint32_t)SEG_RAW_WORDS) : 0u;
  {  // all sixteen loads of a thread in flight together
    uint32_t v[SEG_RAW_WORDS / 256];
#pragma unroll
    for (int k = 0; k < SEG_RAW_WORDS / 256; k++) {
      const uint32_t w = threadIdx.x + 256u * k;
      v[k] = w < nw ? qq[w0 + w] : 0u;
    }
#pragma unroll
    for (int k = 0; k < SEG_RAW_WORDS / 256; k++) {
      const uint32_t w = threadIdx.x + 256u * k;
      if (w < nw) run[w] = v[k];
    }
  }
  __syncthreads();
  if (!q.live) return;
  // every coded vertex's symbol pair (an index past the stream's symbols is
  // an error and reads nothing)
  uint32_t pr[16];
  uint32_t ok = 0, r = 0;
  bool bad = false;
  long long o = o0;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const bool inrow = (unsigned)j < q.len;
    const bool cd = inrow && c[j] < XLOSSLESS;
    const bool in = cd && (d.p.eps >> c[j]) >= 1 && o + 2 <= d.nq;
    bad |= cd && !in;
    ok |= in ? 1u << j : 0u;
    const uint32_t i = (uint32_t)(o >> 1) - w0;
    pr[j] = in ? (i < nw ? run[i] : qq[o >> 1]) : 0xFFFFFFFFu;
    o += cd ? 2 : 0;
    r += inrow && c[j] == XLOSSLESS ? 2u : 0u;
  }
#pragma unroll
  for (int j = 0; j < 16; j++)
    if ((ok >> j) & 1u) r += ((pr[j] & 0xFFFFu) == 0) + ((pr[j] >> 16) == 0);
  if (bad) atomicOr(&d.err, 32u);
  sr[d.soff + q.ls] = r;
}

// the stream's totals against its header: bitstream words, residual
// symbols, raw values; no error bit.  Reconstruction runs only for streams
// that pass, so that every offset it follows stays inside the stream.
__global__ void k_dec_check_b(DecDesc* __restrict__ D, int n, const uint32_t* __restrict__ xw,
                              const uint32_t* __restrict__ xwofs, const uint32_t* __restrict__ qw,
                              const uint32_t* __restrict__ qwofs, const uint32_t* __restrict__ sn,
                              const uint32_t* __restrict__ sq, const uint32_t* __restrict__ sr,
                              const uint32_t* __restrict__ sro) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  DecDesc& d = D[f];
  if (d.status) return;
  uint32_t e = d.err;
  const size_t xa = d.cxb, xz = d.cxb + d.nchx - 1;
  const uint32_t words_x = d.nchx > 0 ? xwofs[xz] + xw[xz] - xwofs[xa] : 0;
  uint32_t words_q = 0;
  if (d.nchq > 0) {
    const size_t qa = d.cqb, qz = d.cqb + d.nchq - 1;
    words_q = qwofs[qz] + qw[qz] - qwofs[qa];
  }
  const size_t a = d.soff, z = d.soff + d.nseg - 1;
  const uint32_t nl = sq[z] + sn[z] - sq[a];
  const uint32_t nr = sro[z] + sr[z] - sro[a];
  if ((long long)words_x != d.secw[3] || (long long)words_q != d.secw[6]) e |= 512u;
  if (2 * (long long)nl != d.nq || (long long)nr != d.nraw) e |= 1024u;
  d.err = e;
  if (e) d.status = -3;  // CPT_ECORRUPT
}

// ============================================================ launchers
static inline unsigned nblk(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
  if (n) k_zero<<<nblk(n), 256, 0, s>>>(p, n);
}
void launch_codes_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* hpre,
                    long long hblocks, const long long* gpre, long long gblocks, long long Rtot, hipStream_t s) {
  launch_zero_u32(E.xhist, 32 * (size_t)HIST_SLOTS * n, s);
  launch_zero_u32(E.qhist, QSYM * (size_t)HIST_SLOTS * n, s);
  if (gblocks > 0)
    k_hist_b<<<(unsigned)gblocks, 256, 0, s>>>(D, gpre, n, B.xcode, B.qcode, E.xhist, E.qhist, E.sr, E.sn);
  k_codebooks_b<<<2 * n, CB_THREADS, 0, s>>>(D, E.xhist, E.qhist, E.xt, E.qt, E.xcb, E.qcb, E.used);
  if (gblocks <= 0) return;
  uint32_t* tot = E.part;  // two scratch words ahead of the scan partials
  launch_scan(E.sn, (size_t)Rtot, E.sq, E.part + 4, tot, s);
  launch_scan(E.sr, (size_t)Rtot, E.sro, E.part + 4, tot + 1, s);
  k_totals_b<<<nblk(n, 64), 64, 0, s>>>(D, n, E.sn, E.sq, E.sr, E.sro);
  k_gather_q_b<<<(unsigned)(4 * hblocks), 256, 0, s>>>(D, hpre, n, B.xcode, B.qcode, E.sq, E.qsym);
}

void launch_chunks_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* cxpre,
                     long long cxtot, const long long* cqpre, long long cqtot, hipStream_t s) {
  uint32_t* tot = E.part;
  if (cxtot > 0) {
    k_chunk_bits_b<false><<<(unsigned)((cxtot + 3) / 4), 256, 0, s>>>(D, cxpre, n, cxtot, B.xcode, E.qsym, E.xt,
                                                                        E.xbits, E.xwords);
    launch_scan(E.xwords, (size_t)cxtot, E.xwofs, E.part + 4, tot + 2, s);
  }
  if (cqtot > 0) {
    k_chunk_bits_b<true><<<(unsigned)((cqtot + 3) / 4), 256, 0, s>>>(D, cqpre, n, cqtot, B.xcode, E.qsym, E.qt,
                                                                       E.qbits, E.qwords);
    launch_scan(E.qwords, (size_t)cqtot, E.qwofs, E.part + 4, tot + 3, s);
  }
  k_layout_b<<<n, 64, 0, s>>>(D, E.used, E.xwords, E.xwofs, E.qwords, E.qwofs);
}

void launch_assemble_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* cxpre,
                       long long cxtot, const long long* cqpre, long long cqtot, const long long* hpre,
                       long long hblocks, hipStream_t s) {
  k_sections_b<<<dim3(n, 16), 256, 0, s>>>(D, B.modes, E.xcb, E.qcb, E.used, E.xbits, E.qbits);
  if (cxtot > 0)
    k_encode_b<false><<<(unsigned)((cxtot + 3) / 4), 256, 0, s>>>(D, cxpre, n, cxtot, B.xcode, E.qsym, E.xt, E.xwofs);
  if (cqtot > 0)
    k_encode_b<true><<<(unsigned)((cqtot + 3) / 4), 256, 0, s>>>(D, cqpre, n, cqtot, B.xcode, E.qsym, E.qt, E.qwofs);
  if (hblocks > 0) k_raw_b<<<(unsigned)hblocks, 256, 0, s>>>(D, hpre, n, B.xcode, B.qcode, E.sr, E.sro);
}
void launch_decode_front_b(DecDesc* D, int n, const DecodeBufs& B, const long long* mpre, long long mblocks,
                           const long long* cxpre, long long cxtot, const long long* cqpre, long long cqtot,
                           hipStream_t s) {
  if (mblocks > 0) k_unpack_modes_b<<<(unsigned)mblocks, 256, 0, s>>>(D, mpre, n, B.modes);
  k_build_lut_b<<<2 * n, 1024, 0, s>>>(D, B.lut);
  if (cxtot > 0) {
    k_words_from_bits_b<false><<<nblk((size_t)cxtot), 256, 0, s>>>(D, cxpre, n, cxtot, B.xw);
    launch_scan(B.xw, (size_t)cxtot, B.xwofs, B.part + 4, B.part, s);
  }
  if (cqtot > 0) {
    k_words_from_bits_b<true><<<nblk((size_t)cqtot), 256, 0, s>>>(D, cqpre, n, cqtot, B.qw);
    launch_scan(B.qw, (size_t)cqtot, B.qwofs, B.part + 4, B.part + 1, s);
  }
}

void launch_decode_b(DecDesc* D, int n, const DecodeBufs& B, const long long* dxpre, long long dxblocks,
                     const long long* dqpre, long long dqblocks, const long long* spre, long long sblocks,
                     long long Stot, long long CX, long long CQ, hipStream_t s) {
  if (dxblocks + dqblocks > 0)
    k_decode_b<<<(unsigned)(dxblocks + dqblocks), 256, 0, s>>>(D, dxpre, dxblocks, dqpre, n, B.lut, B.xwofs, B.qwofs,
                                                                B.xs, B.qs);
  if (sblocks <= 0) return;
  k_seg_nonll_b<<<(unsigned)sblocks, 256, 0, s>>>(D, spre, n, B.xs, B.sn);
  launch_scan(B.sn, (size_t)Stot, B.sq, B.part + 4, B.part + 2, s);
  k_seg_raw_b<<<(unsigned)sblocks, 256, 0, s>>>(D, spre, n, B.xs, B.qs, B.sq, B.sr);
  launch_scan(B.sr, (size_t)Stot, B.sro, B.part + 4, B.part + 3, s);
  k_dec_check_b<<<nblk((size_t)n, 64), 64, 0, s>>>(D, n, B.xw, B.xwofs, B.qw, B.qwofs, B.sn, B.sq, B.sr, B.sro);
}

}  // namespace cpt
