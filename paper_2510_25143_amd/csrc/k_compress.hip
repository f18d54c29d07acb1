// k_compress.hip — the compression hot loop: per-block predictor choice and
// the per-vertex bound, prediction, quantization and write-back.
//
// Order (reproducible by construction): for every frame t, three colour
// phases; phase c processes every 16x16 block with (bx + by) mod 3 == c.
// Blocks of one colour share no face, so they are processed independently
// (one or two per workgroup).  Inside a block the vertices are taken in
// raster order; with the main-diagonal triangulation the raster
// predecessors of a vertex are exactly its neighbours on earlier
// anti-diagonals, so the block is swept along its 31 anti-diagonals, each
// one processed in parallel.
//
// Per vertex (Alg. 3 and Alg. 4 of the paper): a vertex on a crossed face of
// the original field is stored losslessly; otherwise its bound is the
// minimum of eps' and the Alg. 2 bound of each of its (up to 36) faces,
// evaluated on the current values — reconstructed where already processed,
// original elsewhere.  22 of the 36 faces never touch the left, upper or
// upper-left neighbour of the vertex (its raster predecessors); their bounds
// are computed for the whole block in parallel first.  The other 14 are
// computed during the sweep, one face per lane, sixteen lanes per vertex.
#include <type_traits>

#include "batch.hpp"
#include "cpt_device.hpp"
#include "launch.hpp"
#include "predict.hpp"

namespace cpt {

static_assert(make_face_table().n == 36, "36 incident faces per interior vertex");

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int lorenzo_local(const int2 (*C)[TILE], const int2 (*P)[TILE], int lx, int ly,
                                             bool has_prev, int comp) {
  auto g = [&](const int2 (*A)[TILE], int i, int j) -> int {
    if (i < 0 || j < 0) return 0;
    return comp ? A[j][i].y : A[j][i].x;
  };
  int s = g(C, lx - 1, ly) + g(C, lx, ly - 1) - g(C, lx - 1, ly - 1);
  if (has_prev) s += g(P, lx, ly) - g(P, lx - 1, ly) - g(P, lx, ly - 1) + g(P, lx - 1, ly - 1);
  return s;
}

__device__ __forceinline__ int64_t featq_num(int64_t num, int64_t den) {
  if (den <= 0) return 0;
  int64_t q = floor_div64(num * 256, den);
  return q < -65536 ? -65536 : (q > 65536 ? 65536 : q);
}

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------ mode choice
// One wave decides the predictor class of one block of a decision frame.
// Exhaustive trial: each candidate is micro-encoded over the block with the
// global bound eps' (Sec. VI-B): Lorenzo writes its reconstruction back to a
// candidate buffer (anti-diagonal sweep), semi-Lagrangian reads only the
// previous frame.  The rate score of each candidate uses the codes on the
// stride-2 subgrid.  The choice reads only the block's own values of frame t
// and the final frame t-1, so it may run right before the block's own colour
// phase.  A single wave per block keeps every block of a frame resident at
// once; the sequential Lorenzo sweep sets the block's latency.
struct ModesSmem {
  int2 C[TILE][TILE];
  int2 P[TILE][TILE];
  int64_t R[4];
  union {
    struct {  // features and selector activations
      float fin[10];
      float h1[64], h2[64], lg[4];
    };
    int2 PT[TILE][TILE];             // Lorenzo trial: frame t-1 part of each prediction
    alignas(16) uint32_t hist[256];  // rate: one class at a time, 1024 codes, one byte each
  };
  int16_t SAMP[4][128];
  int T[129];  // T[h] = floor(h log2 h 2^16) for h <= 128 (< 2^26)
  int cls;
};
static_assert(QSYM == 4 * 256, "one histogram byte per residual code");
static_assert(sizeof(ModesSmem) <= 9216, "sixteen one-wave blocks share a compute unit's LDS");

// LDS writes of one lane become visible to the other lanes of its wave
// (the wave's LDS operations complete in order; this keeps the compiler from
// reordering across it)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Sum over the wave, every lane enabled: DPP row rotations give each lane
// its 16-lane row's sum, then the four rows are added.
__device__ __forceinline__ int wave_sum(int v) {
  v += __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row_ror:8
  v += __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, true);  // row_ror:4
  v += __builtin_amdgcn_mov_dpp(v, 0x122, 0xF, 0xF, true);  // row_ror:2
  v += __builtin_amdgcn_mov_dpp(v, 0x121, 0xF, 0xF, true);  // row_ror:1
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
         __builtin_amdgcn_readlane(v, 48);
}

// The same for fp64 values (both halves through DPP): exact for integers
// whose partial sums stay below 2^53.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0x128>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x122>(v);
  v += dpp_f64<0x121>(v);
  return readlane_f64(v, 0) + readlane_f64(v, 16) + readlane_f64(v, 32) + readlane_f64(v, 48);
}
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0x128>(v));
  v = fmax(v, dpp_f64<0x124>(v));
  v = fmax(v, dpp_f64<0x122>(v));
  v = fmax(v, dpp_f64<0x121>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  for (int o = 32; o > 0; o >>= 1) v = op(v, (T)__shfl_xor(v, o));
  return v;
}

// cur, flags: the field's arrays; mrow: its predictor classes of frame t's
// group (block by * tx + bx); feats: the group's feature rows or null.
// Called by the 64 lanes of one wave (threads 0..63 of the workgroup), with
// no workgroup barrier inside; returns the class of the block.
__device__ int block_mode(ModesSmem& S, const int2* __restrict__ cur, const uint8_t* __restrict__ flags,
                          const FieldParams& p, int t, int bx, int by, const int64_t* __restrict__ tlog,
                          const uint16_t* __restrict__ selw, uint8_t* mrow, float* __restrict__ feats) {
  auto& C = S.C;
  auto& P = S.P;
  auto& SAMP = S.SAMP;
  const int lane = threadIdx.x & 63;
  const int x0 = bx * TILE, y0 = by * TILE;
  const int H = p.H, W = p.W;
  const size_t HW = (size_t)H * W;
  const int2* cf = cur + (size_t)t * HW;
  const int2* pf = cur + (size_t)(t - 1) * HW;
  const SLConst slc{p.cx, p.sx, p.cy, p.sy};
  const int eps = p.eps;
  // all loads of the block and the table are issued before the first wait
  int2 cv[4], pv[4];
  uint32_t vm = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int v = lane + 64 * k, x = x0 + (v & 15), y = y0 + (v >> 4);
    const bool valid = (x < W) & (y < H);
    vm |= valid ? 1u << k : 0u;
    const size_t gi = valid ? (size_t)y * W + x : 0;
    cv[k] = cf[gi];
    pv[k] = pf[gi];
  }
  int64_t tv[3];
#pragma unroll
  for (int k = 0; k < 3; k++) tv[k] = tlog[min(lane + 64 * k, 128)];
  // lossless flags of the block, for the features
  const bool need_feats = feats != nullptr || p.predictor == 4;
  uint32_t fv = 0;
  if (need_feats) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int v = lane + 64 * k, x = x0 + (v & 15), y = y0 + (v >> 4);
      fv |= (flags[(size_t)t * HW + (((x < W) & (y < H)) ? (size_t)y * W + x : 0)] ? 1u : 0u) << k;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int v = lane + 64 * k;
    const bool valid = (vm >> k) & 1u;
    C[v >> 4][v & 15] = valid ? cv[k] : make_int2(0, 0);
    P[v >> 4][v & 15] = valid ? pv[k] : make_int2(0, 0);
  }
#pragma unroll
  for (int k = 0; k < 3; k++)
    if (lane + 64 * k <= 128) S.T[lane + 64 * k] = (int)tv[k];
  for (int i = lane; i < p.K * 128; i += 64) (&SAMP[0][0])[i] = -1;
  wave_sync();
  // frame t-1 at a domain vertex, from global memory (cache hits: the
  // block was just loaded)
  auto Fprev = [&](int xx, int yy) { return pf[(size_t)yy * W + xx]; };

  // ---------------- block features (also the selector's input)
  int cls_learned = -1;
  if (need_feats) {
    const int64_t s = eps > 1 ? eps : 1;
    int64_t S0 = 0, S1 = 0, S2 = 0, Dm = 0, Ds = 0, Sx = 0, Sy = 0, nf = 0, S6 = 0, S7 = 0, n = 0, m = 0;
    for (int k = 0; k < 4; k++) {
      const int v = lane + 64 * k, lx = v & 15, ly = v >> 4, x = x0 + lx, y = y0 + ly;
      if (!(x < W && y < H)) continue;
      const int2 X = C[ly][lx], Pv = P[ly][lx];
      n += 1;
      S0 += (int64_t)iabs(X.x - Pv.x) + iabs(X.y - Pv.y);
      const int lu = lorenzo_local(C, P, lx, ly, true, 0), lv = lorenzo_local(C, P, lx, ly, true, 1);
      const int64_t r3 = (int64_t)iabs(X.x - lu) + iabs(X.y - lv);
      S1 += r3;
      if (lx + 1 < TILE && x + 1 < W) S2 += (int64_t)iabs(C[ly][lx + 1].x - X.x) + iabs(C[ly][lx + 1].y - X.y);
      if (ly + 1 < TILE && y + 1 < H) S2 += (int64_t)iabs(C[ly + 1][lx].x - X.x) + iabs(C[ly + 1][lx].y - X.y);
      const int64_t DCAP = (int64_t)1 << 40;
      const int64_t dx = clamp64(sl_disp(Pv.x, p.cx, p.sx), -DCAP, DCAP);
      const int64_t dy = clamp64(sl_disp(Pv.y, p.cy, p.sy), -DCAP, DCAP);
      const int64_t ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
      const int64_t d = ax > ay ? ax : ay;
      Dm = Dm > d ? Dm : d;
      Ds += d;
      Sx += dx;
      Sy += dy;
      nf += (fv >> k) & 1u;
      if ((lx & 3) == 0 && (ly & 3) == 0) {
        int pu, pv;
        sl_predict_f(Fprev, H, W, x, y, slc, 2, &pu, &pv);
        S6 += (int64_t)iabs(X.x - pu) + iabs(X.y - pv);
        S7 += r3;
        m += 1;
      }
    }
    // wave sums and the maximum, exact in fp64: every partial sum is an
    // integer below 2^49
    auto sum = [](int64_t v) { return (int64_t)wave_sum_f64((double)v); };
    S0 = sum(S0);
    S1 = sum(S1);
    S2 = sum(S2);
    Dm = (int64_t)wave_max_f64((double)Dm);
    Ds = sum(Ds);
    Sx = sum(Sx);
    Sy = sum(Sy);
    nf = sum(nf);
    S6 = sum(S6);
    S7 = sum(S7);
    n = sum(n);
    m = sum(m);
    // lane i < 10 forms feature i (one exact division each, side by side)
    if (lane < 10) {
      const int64_t num[10] = {S0, S1, S2, Dm, Ds, nf, S6, S7, Sx, Sy};
      const int64_t den[10] = {2 * n * s, 2 * n * s, 2 * n * s, 65536,     n * 65536,
                               n,         2 * m * s, 2 * m * s, n * 65536, n * 65536};
      int64_t a = 0, b = 1;
#pragma unroll
      for (int i = 0; i < 10; i++)
        if (lane == i) {
          a = num[i];
          b = den[i];
        }
      S.fin[lane] = (float)featq_num(a, b) / 256.0f;
    }
    wave_sync();
    const size_t bi = (size_t)by * p.tx + bx;
    if (feats != nullptr && lane < 10) feats[bi * 10 + lane] = S.fin[lane];
    if (p.predictor == 4) {
      // 10-64-64-4 MLP, bf16 weights, fp32 fused multiply-add in input order;
      // a unit's weight row is read in 32-bit (layer 1) or 128-bit pieces
      // (the weights are 16-byte aligned, every row offset a multiple of 4
      // or 16 bytes), low half first
      {
        const uint32_t* w1 = reinterpret_cast<const uint32_t*>(selw + lane * 10);
        uint32_t wr[5];
#pragma unroll
        for (int i = 0; i < 5; i++) wr[i] = w1[i];
        float a = bf16f(selw[640 + lane]);
#pragma unroll
        for (int i = 0; i < 5; i++) {
          a = fmaf(bf16f((uint16_t)(wr[i] & 0xFFFFu)), S.fin[2 * i], a);
          a = fmaf(bf16f((uint16_t)(wr[i] >> 16)), S.fin[2 * i + 1], a);
        }
        S.h1[lane] = a > 0.0f ? a : 0.0f;
      }
      wave_sync();
      auto dense64 = [&](const uint16_t* row, const float* in, float a) {
        const uint4* w = reinterpret_cast<const uint4*>(row);
        uint4 wr[8];
#pragma unroll
        for (int i = 0; i < 8; i++) wr[i] = w[i];
#pragma unroll
        for (int i = 0; i < 8; i++) {
          const uint32_t h[4] = {wr[i].x, wr[i].y, wr[i].z, wr[i].w};
#pragma unroll
          for (int k = 0; k < 4; k++) {
            a = fmaf(bf16f((uint16_t)(h[k] & 0xFFFFu)), in[8 * i + 2 * k], a);
            a = fmaf(bf16f((uint16_t)(h[k] >> 16)), in[8 * i + 2 * k + 1], a);
          }
        }
        return a;
      };
      {
        const float a = dense64(selw + 704 + lane * 64, S.h1, bf16f(selw[4800 + lane]));
        S.h2[lane] = a > 0.0f ? a : 0.0f;
      }
      wave_sync();
      if (lane < 4) S.lg[lane] = dense64(selw + 4864 + lane * 64, S.h2, bf16f(selw[5120 + lane]));
      wave_sync();
      int best = 0;
      for (int c = 1; c < 4; c++)
        if (S.lg[c] > S.lg[best]) best = c;
      cls_learned = best;
    }
  }
  if (p.predictor == 4) {
    if (lane == 0) mrow[(size_t)by * p.tx + bx] = (uint8_t)cls_learned;
    return cls_learned;
  }

  // ---------------- exhaustive trial over the K candidates
  // Lorenzo: lanes 0-15 sweep the rows of u, lanes 16-31 those of v, carrying
  // the candidate reconstructions in registers; then every lane takes
  // semi-Lagrangian candidates (class, stride-2 point).  Codes of the
  // stride-2 subgrid go to SAMP[class][0..127] (slot 2 i + component of
  // subgrid point i; -1 when absent).
  {
    // the frame t-1 part of every vertex's prediction first (tile-local)
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int v = lane + 64 * k, lx = v & 15, ly = v >> 4;
      const int2 z = make_int2(0, 0);
      const int2 pc = P[ly][lx], pl = lx > 0 ? P[ly][lx - 1] : z, pu = ly > 0 ? P[ly - 1][lx] : z;
      const int2 plu = (lx > 0 && ly > 0) ? P[ly - 1][lx - 1] : z;
      S.PT[ly][lx] = make_int2(pc.x - pl.x - pu.x + plu.x, pc.y - pl.y - pu.y + plu.y);
    }
    wave_sync();
    // A lane keeps its own last reconstruction (the left neighbour of its
    // next vertex); the row above arrives from the previous lane of the same
    // 16-lane DPP row by a row shift of that lane's last value.  All 64 lanes
    // step together (DPP reads need active source lanes); lanes 32-63 have
    // no vertices.
    const int c = (lane >> 4) & 1, row = lane & 15;
    const bool rowok = lane < 2 * TILE && y0 + row < H;
    const int cend = min(TILE, W - x0);
    const int* PTc = &S.PT[row][0].x + c;
    const int* Cc = &C[row][0].x + c;
    int last = 0, upl = 0;
    for (int d = 0; d < 2 * TILE - 1; d++) {
      const int col = d - row, cc = min(max(col, 0), TILE - 1);
      const int pt = PTc[2 * cc], xv = Cc[2 * cc];
      const int up = __builtin_amdgcn_update_dpp(0, last, 0x111, 0xF, 0xF, true);  // row_shr:1
      if (rowok && (unsigned)col < (unsigned)cend) {
        const int sm = (col > 0 ? last : 0) + (row > 0 ? up : 0) - (col > 0 && row > 0 ? upl : 0) + pt;
        int rec;
        const int q = quantize(xv, sm, eps, &rec);
        last = rec;
        if (((row | col) & 1) == 0) SAMP[0][2 * ((row >> 1) * 8 + (col >> 1)) + c] = q;
      }
      upl = up;
    }
  }
  for (int task = lane; task < 64 * (p.K - 1); task += 64) {
    const int cls = 1 + (task >> 6), pt = task & 63;
    const int sx = 2 * (pt & 7), sy = 2 * (pt >> 3);
    if (x0 + sx < W && y0 + sy < H) {
      const int2 Xs = C[sy][sx];
      int pu, pv, ru, rv;
      sl_predict_f(Fprev, H, W, x0 + sx, y0 + sy, slc, class_dmax(p.K, cls), &pu, &pv);
      SAMP[cls][2 * pt] = quantize(Xs.x, pu, eps, &ru);
      SAMP[cls][2 * pt + 1] = quantize(Xs.y, pv, eps, &rv);
    }
  }
  wave_sync();
  // rate score per candidate: a byte histogram of the class's 128 codes
  // (counts <= 128); the lane whose atomic add finds a code's count still 0
  // holds its first occurrence and adds T[final count] for it.  Sums fit in
  // 32 bits: T[h] < 2^26 and the first occurrences add up to at most T[128].
  for (int cls = 0; cls < p.K; cls++) {
    reinterpret_cast<uint4*>(S.hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
    const int a0 = SAMP[cls][lane], a1 = SAMP[cls][lane + 64];
    const int s0 = 8 * (a0 & 3), s1 = 8 * (a1 & 3);
    bool f0 = false, f1 = false;
    if (a0 > 0) f0 = ((atomicAdd(&S.hist[a0 >> 2], 1u << s0) >> s0) & 0xFFu) == 0u;
    if (a1 > 0) f1 = ((atomicAdd(&S.hist[a1 >> 2], 1u << s1) >> s1) & 0xFFu) == 0u;
    wave_sync();
    int tsum = 0;
    if (f0) tsum += S.T[(S.hist[a0 >> 2] >> s0) & 0xFFu];
    if (f1) tsum += S.T[(S.hist[a1 >> 2] >> s1) & 0xFFu];
    tsum = wave_sum(tsum);
    // valid codes in the low half, unpredictable ones in the high half
    const int cnt = wave_sum((a0 > 0) + (a1 > 0) + (((a0 == 0) + (a1 == 0)) << 16));
    if (lane == 0) {
      const int n = cnt & 0xFFFF, L = cnt >> 16;
      const int h0 = n > 0 ? floor_div32(S.T[n] - tsum, n) : 0;
      const int pen = (n + L) > 0 ? floor_div32(16 * 65536 * L, n + L) : 0;
      const int lgK = p.K == 4 ? 2 : 1;
      const int meta = floor_div32(65536 * lgK, 512 * p.bt);
      S.R[cls] = (int64_t)h0 + pen + meta;
    }
    wave_sync();
  }
  if (lane == 0) {
    int best = 1;
    for (int c = 2; c < p.K; c++)
      if (S.R[c] < S.R[best]) best = c;
    const int cls = 1000 * (S.R[0] - S.R[best]) > 3 * S.R[0] ? best : 0;
    mrow[(size_t)by * p.tx + bx] = (uint8_t)cls;
    S.cls = cls;
  }
  wave_sync();
  return S.cls;
}

// --------------------------------------------------------------- the phase
// The 14 space-time neighbours of a vertex; the first three are the raster
// predecessors inside the block (they change during the sweep).
struct NbrTable {
  int8_t dx[14], dy[14], dt[14];
};
constexpr NbrTable NBR = {{-1, 0, -1, 1, 0, 1, 0, -1, 0, -1, 0, 1, 0, 1},
                          {0, -1, -1, 0, 1, 1, 0, 0, -1, -1, 0, 0, 1, 1},
                          {0, 0, 0, 0, 0, 0, -1, -1, -1, -1, 1, 1, 1, 1}};

constexpr int nbr_index(uint8_t packed) {
  for (int j = 0; j < 14; j++)
    if (pack_off(NBR.dx[j], NBR.dy[j], NBR.dt[j]) == packed) return j;
  return -1;
}
struct PairTable {
  int8_t a[36], b[36];
};
constexpr PairTable make_pairs() {
  PairTable P{};
  FaceTable T = make_face_table();
  for (int f = 0; f < 36; f++) {
    P.a[f] = (int8_t)nbr_index(T.a[f]);
    P.b[f] = (int8_t)nbr_index(T.b[f]);
  }
  return P;
}
constexpr PairTable PAIRS = make_pairs();
struct DynPairs {
  int8_t a[16], b[16];
};
constexpr DynPairs make_dyn_pairs() {
  DynPairs D{};
  int n = 0;
  for (int f = 0; f < 36; f++)
    if (PAIRS.a[f] < 3 || PAIRS.b[f] < 3) {
      D.a[n] = PAIRS.a[f];
      D.b[n] = PAIRS.b[f];
      n++;
    }
  for (; n < 16; n++) {
    D.a[n] = -1;
    D.b[n] = -1;
  }
  return D;
}
struct StaticPairs {
  int8_t a[22], b[22];
};
constexpr StaticPairs make_static_pairs() {
  StaticPairs S{};
  int n = 0;
  for (int f = 0; f < 36; f++)
    if (PAIRS.a[f] >= 3 && PAIRS.b[f] >= 3) {
      S.a[n] = PAIRS.a[f];
      S.b[n] = PAIRS.b[f];
      n++;
    }
  return S;
}
constexpr StaticPairs SPAIRS = make_static_pairs();
constexpr int count_static() {
  int n = 0;
  for (int f = 0; f < 36; f++) n += (PAIRS.a[f] >= 3 && PAIRS.b[f] >= 3) ? 1 : 0;
  return n;
}
static_assert(count_static() == 22, "22 faces avoid the raster predecessors");
// The same 22 faces in four trails (each face oriented so that its first
// neighbour is the previous face's second wherever the trail continues):
// 18 faces reuse a neighbour's value, determinant with the vertex, norm and
// sign tests.  The bound of a face is symmetric in its two neighbours and
// the running minimum does not depend on the order of the faces.
constexpr StaticPairs STRAIL = {{3, 5, 4, 13, 3, 11, 13, 12, 4, 6, 3, 8, 6, 5, 13, 10, 12, 9, 7, 6, 9, 7},
                                {5, 4, 13, 3, 11, 13, 12, 4, 6, 3, 8, 6, 5, 13, 10, 11, 10, 8, 6, 9, 7, 4}};
constexpr bool trail_covers_static() {
  for (int f = 0; f < 22; f++) {
    int hits = 0;
    for (int k = 0; k < 22; k++)
      hits += ((STRAIL.a[k] == SPAIRS.a[f] && STRAIL.b[k] == SPAIRS.b[f]) ||
               (STRAIL.a[k] == SPAIRS.b[f] && STRAIL.b[k] == SPAIRS.a[f]))
                  ? 1
                  : 0;
    if (hits != 1) return false;
  }
  return true;
}
static_assert(trail_covers_static(), "the trails hold every static face once");
static_assert(make_pairs().a[0] >= 0 && make_dyn_pairs().a[13] >= 0 && make_dyn_pairs().a[14] < 0,
              "face and neighbour tables are consistent");
// Lane j's sweep face as one word: bit 0 set for the 14 lanes with a face,
// then the offsets (dx, dy, dt) + 1 of its two neighbours, two bits each
// (zero offsets for the two lanes without a face).
struct DynLanes {
  uint32_t e[16];
};
constexpr DynLanes make_dyn_lanes() {
  DynLanes L{};
  const DynPairs D = make_dyn_pairs();
  for (int j = 0; j < 16; j++) {
    const int fa = D.a[j], fb = D.b[j];
    if (fa < 0) {
      L.e[j] = 1u << 1 | 1u << 3 | 1u << 5 | 1u << 7 | 1u << 9 | 1u << 11;  // zero offsets, no face
      continue;
    }
    L.e[j] = 1u | (uint32_t)(NBR.dx[fa] + 1) << 1 | (uint32_t)(NBR.dy[fa] + 1) << 3 | (uint32_t)(NBR.dt[fa] + 1) << 5 |
             (uint32_t)(NBR.dx[fb] + 1) << 7 | (uint32_t)(NBR.dy[fb] + 1) << 9 | (uint32_t)(NBR.dt[fb] + 1) << 11;
  }
  return L;
}
__constant__ DynLanes c_dynlanes = make_dyn_lanes();

// Running minimum of Alg. 2 bounds.  For the face (me, n0, n1) with
// d0 = det(me, n0), d1 = det(me, n1):  Alg. 2 returns 0 when M = d0 - d1 +
// det(n0, n1) is 0 or a neighbour is the zero vector; otherwise the minimum
// of floor((N-1)/D) over (|M|, |u1-u0|+|v0-v1|), (|d1|, |u1|+|v1|),
// (|d0|, |u0|+|v0|), raised to |u2|-1 (|v2|-1) when the u (v) components
// share a strict sign.  A face whose raise already reaches the running
// minimum xi cannot lower it, so its quotients are skipped; a quotient is
// only evaluated when it beats the current value (N - 1 < e D, exact).
// The operands are fixed-point integers below 2^25 held as fp64 values, so
// every sum, difference, absolute value and product below is exact and the
// comparisons decide exactly as in integers.  N is a non-negative integer;
// for N = 0 the estimate ends at -1 and the final max gives the 0 of
// Alg. 2.  The one-step correction of the fp64 reciprocal estimate is a
// select, not a branch.
__device__ __forceinline__ void lower_to(int& e, double& ed, double N, double D) {
  if (N > ed * D) return;  // integers: N - 1 >= e D
  const double n1 = N - 1.0;
  int q = (int)(n1 * __builtin_amdgcn_rcp(D));
  const double r = n1 - (double)q * D;
  q += (r >= D ? 1 : 0) - (r < 0.0 ? 1 : 0);
  e = max(q, 0);
  ed = (double)e;
}

__device__ __forceinline__ double det2d(double2 a, double2 b) { return fma(a.x, b.y, -(a.y * b.x)); }

// What the raise of Alg. 2 needs of the vertex itself besides its value:
// |component| - 1.
// The sign tests read the high words of the fp64 values: an integer-valued
// double that is not -0 is positive, zero or negative exactly as its high
// word is as an int32.  mx (my) is -1 when the vertex's u (v) is negative,
// else 0; a neighbour component shares the vertex's strict sign when its
// high word xor mx is positive (for a zero vertex component the raise term
// is -1 and the test does not matter).
struct MeSign {
  int rx, ry, mx, my;
};
__device__ __forceinline__ int hiw(double v) { return __double2hiint(v); }
__device__ __forceinline__ MeSign me_sign(double2 me) {
  return MeSign{(int)fabs(me.x) - 1, (int)fabs(me.y) - 1, hiw(me.x) >> 31, hiw(me.y) >> 31};
}

// Running minimum with the Alg. 2 bound of the face (me, n0, n1).  A
// component's raise applies when n0 and n1 share the strict sign of the
// vertex's own component, i.e. both products with it are positive (exact:
// the products stay below 2^50).
__device__ __forceinline__ void face_update(int& xi, double2 me, const MeSign& ms, double2 n0, double2 n1) {
  const double d0 = det2d(me, n0), d1 = det2d(me, n1);
  const double M = (d0 - d1) + det2d(n0, n1);
  const double a0 = fabs(n0.x) + fabs(n0.y), a1 = fabs(n1.x) + fabs(n1.y);
  if (M == 0.0 || a0 == 0.0 || a1 == 0.0) {
    xi = 0;
    return;
  }
  const bool sx = min(hiw(n0.x) ^ ms.mx, hiw(n1.x) ^ ms.mx) > 0;
  const bool sy = min(hiw(n0.y) ^ ms.my, hiw(n1.y) ^ ms.my) > 0;
  const int relax = max(sx ? ms.rx : -1, sy ? ms.ry : -1);
  if (relax >= xi) return;
  int e = xi;
  double ed = (double)xi;
  lower_to(e, ed, fabs(M), fabs(n1.x - n0.x) + fabs(n0.y - n1.y));
  lower_to(e, ed, fabs(d1), a1);
  lower_to(e, ed, fabs(d0), a0);
  xi = min(xi, max(e, relax));
}

// A neighbour of the vertex as the face bounds use it: its value, the
// determinant with the vertex, |u| + |v|, and whether each component shares
// the vertex's strict sign.
struct NbrQ {
  double2 n;
  double d, a;
  bool sx, sy;
};
__device__ __forceinline__ NbrQ nbr_q(double2 n, double2 me, const MeSign& ms) {
  return NbrQ{n, det2d(me, n), fabs(n.x) + fabs(n.y), (hiw(n.x) ^ ms.mx) > 0, (hiw(n.y) ^ ms.my) > 0};
}

// face_update for neighbours given with their per-neighbour terms
__device__ __forceinline__ void face_update_q(int& xi, const MeSign& ms, const NbrQ& A, const NbrQ& B) {
  const double M = (A.d - B.d) + det2d(A.n, B.n);
  if (M == 0.0 || A.a == 0.0 || B.a == 0.0) {
    xi = 0;
    return;
  }
  const int relax = max(A.sx && B.sx ? ms.rx : -1, A.sy && B.sy ? ms.ry : -1);
  if (relax >= xi) return;
  int e = xi;
  double ed = (double)xi;
  lower_to(e, ed, fabs(M), fabs(B.n.x - A.n.x) + fabs(A.n.y - B.n.y));
  lower_to(e, ed, fabs(B.d), B.a);
  lower_to(e, ed, fabs(A.d), A.a);
  xi = min(xi, max(e, relax));
}

// The block's neighbourhood as exact fp64 integers.  Faces reach frame t-1
// only at offsets (-1..0, -1..0) and frame t+1 only at (0..1, 0..1), so those
// two frames are staged one-sided (17 x 17), frame t with the full halo.
// Indices: V0[1 + y - y0][1 + x - x0], V1 the same, V2[y - y0][x - x0].
constexpr int HALO1 = TILE + 1;
struct TileInfo {
  int x0, y0, H, W, T, eps, cls, valid;
};
struct PhaseSmem {
  double2 V0[HALO1][HALO1];  // frame t-1, x in [x0-1, x0+15], y in [y0-1, y0+15]
  double2 V1[HALO][HALO];    // frame t, [x0-1, x0+16] x [y0-1, y0+16]
  double2 V2[HALO1][HALO1];  // frame t+1, [x0, x0+16] x [y0, y0+16]
  // bound from the faces fixed for the whole sweep (-1 = lossless); the
  // sweep reads a vertex's entry once, then stores its residual codes there
  int XQ[TILE][TILE];
  // |u| - 1, |v| - 1 of each vertex (its raise terms); the sweep reads them
  // once, then stores the bound code and the bound there
  int2 MS[TILE][TILE];
  int2 SLP[TILE][TILE];      // semi-Lagrangian predictions, or the fixed part of the Lorenzo prediction
  TileInfo info;             // what the sweep needs of the block when a workgroup holds several
};
static_assert(sizeof(PhaseSmem) <= 160 * 1024 / 8, "eight blocks share a compute unit's LDS");

// The halo cells of the three staged frames, one entry each: index into the
// contiguous V0, V1, V2 range (bits 0-9), x and y offset from the block's
// first vertex plus one (bits 10-14 and 15-19), frame 0, 1, 2 for t-1, t,
// t+1 (bits 20-21), and whether the cell is loaded (bit 22).  Frame t-1
// needs the row above and the column left of the block, frame t+1 the row
// below and the column right of it, frame t the whole ring; the two ring
// corners of frame t that belong to blocks of the same colour are never
// read and only cleared.
constexpr int NHALO = 2 * (HALO1 + TILE) + (4 * HALO - 4);
struct HaloTable {
  uint32_t e[NHALO];
};
constexpr uint32_t halo_entry(int f, int hy, int hx, bool load) {
  const int flat = f == 0 ? hy * HALO1 + hx : (f == 1 ? HALO1 * HALO1 + hy * HALO + hx : HALO1 * HALO1 + HALO * HALO + hy * HALO1 + hx);
  const int ox = f == 2 ? hx + 1 : hx, oy = f == 2 ? hy + 1 : hy;
  return (uint32_t)flat | (uint32_t)ox << 10 | (uint32_t)oy << 15 | (uint32_t)f << 20 | (load ? 1u : 0u) << 22;
}
constexpr HaloTable make_halo() {
  HaloTable H{};
  int n = 0;
  for (int hx = 0; hx < HALO1; hx++) H.e[n++] = halo_entry(0, 0, hx, true);
  for (int hy = 1; hy < HALO1; hy++) H.e[n++] = halo_entry(0, hy, 0, true);
  for (int hx = 0; hx < HALO - 1; hx++) H.e[n++] = halo_entry(1, 0, hx, true);
  for (int hx = 1; hx < HALO; hx++) H.e[n++] = halo_entry(1, HALO - 1, hx, true);
  for (int hy = 1; hy < HALO - 1; hy++) H.e[n++] = halo_entry(1, hy, 0, true);
  for (int hy = 1; hy < HALO - 1; hy++) H.e[n++] = halo_entry(1, hy, HALO - 1, true);
  for (int hx = 0; hx < HALO1; hx++) H.e[n++] = halo_entry(2, TILE, hx, true);
  for (int hy = 0; hy < TILE; hy++) H.e[n++] = halo_entry(2, hy, TILE, true);
  H.e[n++] = halo_entry(1, 0, HALO - 1, false);
  H.e[n++] = halo_entry(1, HALO - 1, 0, false);
  return H;
}
constexpr bool halo_covers_ring() {
  // every staged cell is either one thread's own cell or exactly one entry
  bool seen[HALO1 * HALO1 * 2 + HALO * HALO] = {};
  for (int v = 0; v < TILE * TILE; v++) {
    const int vy = v / TILE, vx = v % TILE;
    seen[(vy + 1) * HALO1 + vx + 1] = true;
    seen[HALO1 * HALO1 + (vy + 1) * HALO + vx + 1] = true;
    seen[HALO1 * HALO1 + HALO * HALO + vy * HALO1 + vx] = true;
  }
  const HaloTable H = make_halo();
  for (int i = 0; i < NHALO; i++) {
    const int flat = (int)(H.e[i] & 1023);
    if (seen[flat]) return false;
    seen[flat] = true;
  }
  for (bool b : seen)
    if (!b) return false;
  return true;
}
static_assert(NHALO == 134 && halo_covers_ring(), "the halo table and the threads' own cells cover the staged frames once");
static_assert(offsetof(PhaseSmem, V1) == sizeof(double2) * HALO1 * HALO1 &&
                  offsetof(PhaseSmem, V2) == sizeof(double2) * (HALO1 * HALO1 + HALO * HALO),
              "a halo entry's index runs over V0, V1, V2 as one range");
__constant__ HaloTable c_halo = make_halo();

// frame 0, 1, 2 (t-1, t, t+1) at halo indices (hy, hx) of the 18 x 18 frame
// around the block, (1, 1) being the block's first vertex
__device__ __forceinline__ double2* vslot(PhaseSmem& S, int f, int hy, int hx) {
  return f == 0 ? &S.V0[hy][hx] : (f == 1 ? &S.V1[hy][hx] : &S.V2[hy - 1][hx - 1]);
}

union TileSmem {
  ModesSmem m;
  PhaseSmem p;
};

// NB blocks of frame t, one per 256 threads: the thread's own block is
// (bx, by) with predictor class *clsp, or cls0 when clsp is null; cur,
// flags, xcode, qcode and xi_dbg point at that block's field's arrays, and
// valid is false for a slot without a block (it only keeps the barriers).
// Staging, the static faces and the results are per block; in the sweep a
// wave holds 4 / NB rows of every block, so that with several blocks its
// rows share their anti-diagonal steps.  Called by all 256 NB threads; ends
// with a barrier, so the shared memory may be reused at once.
template <int NB>
__device__ __forceinline__ void phase_tile(PhaseSmem* SS, bool valid, int2* __restrict__ cur,
                                           const uint8_t* __restrict__ flags, const FieldParams& p, int t, int bx,
                                           int by, int cls0, const uint8_t* __restrict__ clsp,
                                           uint8_t* __restrict__ xcode, uint32_t* __restrict__ qcode,
                                           int32_t* __restrict__ xi_dbg) {
  static_assert(NB == 1 || NB == 2 || NB == 4, "a wave holds 4 / NB rows of each block");
  const int tid = threadIdx.x;
  const int lt = NB == 1 ? tid : (tid & 255);  // thread within its own block
  PhaseSmem& S = SS[NB == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 8)];
  auto& V0 = S.V0;
  auto& V1 = S.V1;
  auto& XS = S.XQ;
  auto& MS = S.MS;
  auto& SLP = S.SLP;
  const int H = p.H, W = p.W, T = p.T;
  const size_t HW = (size_t)H * W;
  const int x0 = bx * TILE, y0 = by * TILE;
  const int eps = p.eps;
  const int vx = lt & 15, vy = lt >> 4;
  const bool vin = valid && x0 + vx < W && y0 + vy < H;

  // this lane's sweep face, read with the frame loads
  const uint32_t dyn = c_dynlanes.e[tid & 15];

  // ---- stage frames t-1, t, t+1.  Every thread loads its own vertex's cell
  // of the three frames, and threads 0 .. NHALO-1 one halo cell each (from
  // a table); cells outside the domain or the frame range are staged as 0.
  // All loads of a thread are issued before the first one is waited for.
  const size_t own = (size_t)(y0 + vy) * W + (x0 + vx);
  const int2* f0 = cur + (size_t)(t > 0 ? t - 1 : 0) * HW;
  const int2* f1 = cur + (size_t)t * HW;
  const int2* f2 = cur + (size_t)(t + 1 < T ? t + 1 : t) * HW;
  const bool ld0 = vin & (t > 0), ld2 = vin & (t + 1 < T);
  const int2 c0 = f0[ld0 ? own : 0], c1 = f1[vin ? own : 0], c2 = f2[ld2 ? own : 0];
  int2 ch = make_int2(0, 0);
  int hslot = -1;
  if (valid && lt < NHALO) {
    const uint32_t e = c_halo.e[lt];
    const int f = (int)(e >> 20) & 3;
    const int gx = x0 + (int)((e >> 10) & 31) - 1, gy = y0 + (int)((e >> 15) & 31) - 1, tt = t - 1 + f;
    const bool ld = ((e >> 22) & 1u) & (gx >= 0) & (gx < W) & (gy >= 0) & (gy < H) & (tt >= 0) & (tt < T);
    ch = cur[ld ? (size_t)tt * HW + (size_t)gy * W + gx : 0];
    if (!ld) ch = make_int2(0, 0);
    hslot = (int)(e & 1023);
  }
  // this thread's lossless flag and the block's class (when read here), with
  // the frame loads in flight
  const uint8_t fl = flags[vin ? (size_t)t * HW + own : 0];
  const int cls = (valid && clsp) ? (int)*clsp : cls0;
  const bool lossless = !vin || fl != 0;
  auto dbl = [](int2 v) { return make_double2((double)v.x, (double)v.y); };
  const double2 z2 = make_double2(0.0, 0.0);
  V0[vy + 1][vx + 1] = ld0 ? dbl(c0) : z2;
  V1[vy + 1][vx + 1] = vin ? dbl(c1) : z2;
  S.V2[vy][vx] = ld2 ? dbl(c2) : z2;
  if (hslot >= 0) (&V0[0][0])[hslot] = dbl(ch);
  const int dmax = p.predictor == 1 ? 2 : class_dmax(p.K, cls);
  __syncthreads();

  // ---- faces whose other vertices stay fixed during the sweep
  {
    const int lx = vx, ly = vy, x = x0 + lx, y = y0 + ly;
    int xi = -1;
    int2 msv = make_int2(0, 0);
    if (vin) {
      if (!lossless) {
        xi = eps;
        const double2 me = V1[ly + 1][lx + 1];
        const MeSign ms = me_sign(me);
        msv = make_int2(ms.rx, ms.ry);
        // Faces through a raster predecessor (left, up, up-left) are all
        // evaluated in the sweep, also where that neighbour lies outside the
        // block; the other 22 are evaluated here for every vertex alike.
        // whether neighbour j lies in the domain, from six per-lane tests
        const bool xl = x > 0, xr = x + 1 < W, yl = y > 0, yr = y + 1 < H, tl = t > 0, tr = t + 1 < T;
        auto inside = [&](int j) {
          const int dx = NBR.dx[j], dy = NBR.dy[j], dt = NBR.dt[j];
          return (dx < 0 ? xl : (dx > 0 ? xr : true)) & (dy < 0 ? yl : (dy > 0 ? yr : true)) &
                 (dt < 0 ? tl : (dt > 0 ? tr : true));
        };
        auto nv = [&](int j) { return *vslot(S, 1 + NBR.dt[j], ly + 1 + NBR.dy[j], lx + 1 + NBR.dx[j]); };
        NbrQ prev = nbr_q(nv(STRAIL.a[0]), me, ms);
#pragma unroll
        for (int k = 0; k < 22; k++) {
          const int a = STRAIL.a[k], b = STRAIL.b[k];
          // the shared neighbour's value is read again from LDS (no VALU
          // work); its derived terms carry over in registers
          NbrQ A = (k > 0 && a == STRAIL.b[k > 0 ? k - 1 : 0]) ? prev : nbr_q(nv(a), me, ms);
          A.n = nv(a);
          const NbrQ B = nbr_q(nv(b), me, ms);
          prev = B;
          if (!(inside(a) & inside(b))) continue;
          face_update_q(xi, ms, A, B);
          // keep each face's loads with the face (fewer live registers)
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
      }
      if (cls == 0) {
        // the frame t-1 part of the 3-D Lorenzo prediction, less the halo
        // cells of frame t that the sweep's sum left + up - upper-left reads
        // at the block's left and top edges: the prediction counts them as
        // 0, and they do not change during the sweep (all sums exact)
        const double2 z = make_double2(0.0, 0.0);
        const double2 pc = V0[ly + 1][lx + 1];
        const double2 pl = lx > 0 ? V0[ly + 1][lx] : z;
        const double2 pu = ly > 0 ? V0[ly][lx + 1] : z;
        const double2 plu = (lx > 0 && ly > 0) ? V0[ly][lx] : z;
        const double2 hl = lx == 0 ? V1[ly + 1][lx] : z;
        const double2 hu = ly == 0 ? V1[ly][lx + 1] : z;
        const double2 hlu = (lx == 0 || ly == 0) ? V1[ly][lx] : z;
        SLP[ly][lx] = make_int2((int)(((pc.x - pl.x) - (pu.x - plu.x)) - ((hl.x + hu.x) - hlu.x)),
                                (int)(((pc.y - pl.y) - (pu.y - plu.y)) - ((hl.y + hu.y) - hlu.y)));
      } else {
        // the samples of frame t-1 from global memory (cache hits: the
        // block's neighbourhood was just loaded), its value at the vertex
        // from the staged copy
        const int2* prev = cur + (size_t)(t - 1) * HW;
        auto F = [&](int xx, int yy) { return prev[(size_t)yy * W + xx]; };
        const double2 gc = V0[ly + 1][lx + 1];
        int pu, pv;
        sl_predict_g(F, H, W, x, y, make_int2((int)gc.x, (int)gc.y), SLConst{p.cx, p.sx, p.cy, p.sy}, dmax, &pu,
                     &pv);
        SLP[ly][lx] = make_int2(pu, pv);
      }
    }
    XS[ly][lx] = xi;
    MS[ly][lx] = msv;
  }
  if (NB > 1 && lt == 0) S.info = TileInfo{x0, y0, H, W, T, eps, cls, valid ? 1 : 0};
  __syncthreads();

  // ---- anti-diagonal sweep: row g of the block, lane j takes the j-th face
  // that meets a raster predecessor; lanes 0 and 1 then quantize u and v
  const int j = tid & 15;
  const int g = NB == 1 ? tid >> 4 : (tid >> 6) * (4 / NB) + ((tid >> 4) & 3) / NB;
  PhaseSmem& Sw = SS[NB == 1 ? 0 : ((tid >> 4) & 3) % NB];
  int bx0 = x0, by0 = y0, bH = H, bW = W, bT = T, beps = eps, bcls = cls;
  bool bvalid = valid;
  if constexpr (NB > 1) {
    const TileInfo I = Sw.info;
    bx0 = I.x0, by0 = I.y0, bH = I.H, bW = I.W, bT = I.T, beps = I.eps, bcls = I.cls, bvalid = I.valid != 0;
  }
  const int y = by0 + g;
  const bool has_face = dyn & 1u;
  const int axo = (int)((dyn >> 1) & 3) - 1, ayo = (int)((dyn >> 3) & 3) - 1, ato = (int)((dyn >> 5) & 3) - 1;
  const int bxo = (int)((dyn >> 7) & 3) - 1, byo = (int)((dyn >> 9) & 3) - 1, bto = (int)((dyn >> 11) & 3) - 1;
  const int comp = j & 1;
  // y and t of this lane's face do not change during the sweep
  const bool face_yt = has_face && y + ayo >= 0 && y + ayo < bH && t + ato >= 0 && t + ato < bT && y + byo >= 0 &&
                       y + byo < bH && t + bto >= 0 && t + bto < bT;
  // columns of the block with a vertex [0, aend), and those where this
  // lane's face has both neighbours inside the domain [flo, fhi)
  const int aend = bvalid && y < bH ? min(TILE, bW - bx0) : 0;
  const int flo = max(max(-min(axo, bxo), 0) - bx0, 0);
  const int fhi = face_yt ? max(min(bW - max(max(axo, bxo), 0) - bx0, TILE), flo) : flo;
  auto& V1w = Sw.V1;
  auto& XSw = Sw.XQ;
  auto& MSw = Sw.MS;
  const double2* Vme = &V1w[g + 1][1];
  // rows of this lane's two face neighbours (only a face of frame t reaches
  // the column before the block; the lanes without a face read frame t)
  const double2* Va = vslot(Sw, 1 + ato, g + 1 + ayo, 1 + axo);
  const double2* Vb = vslot(Sw, 1 + bto, g + 1 + byo, 1 + bxo);
  // component comp of the left, upper and upper-left neighbours and of the
  // fixed prediction term, at index lx (rows of pairs: stride 2)
  const double* Ql = &V1w[g + 1][0].x + comp;
  const double* Qu = &V1w[g][1].x + comp;
  const double* Qlu = &V1w[g][0].x + comp;
  const int* Qp = (const int*)&Sw.SLP[g][0] + comp;
  // wave wv holds rows R wv .. R wv + R - 1 of each block (R = 4 / NB),
  // which have vertices on the anti-diagonals R wv .. R wv + R + 14; on the
  // others it only keeps the workgroup's barrier count
  constexpr int R = 4 / NB;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int dlo = R * wv, dhi = R * wv + R - 1 + TILE;
  for (int d = 0; d < dlo; d++) __syncthreads();
  for (int d = dlo; d < dhi; d++) {
    const int lx = d - g;
    const bool active = (unsigned)lx < (unsigned)aend;
    // every value the step reads is final after the last barrier: read them
    // all at once (at a clamped column for the idle lanes)
    const int lc = min(max(lx, 0), TILE - 1);
    const int xs = XSw[g][lc];
    const int2 msw = MSw[g][lc];
    const double2 me = Vme[lc], pa = Va[lc], pb = Vb[lc];
    const double l = Ql[2 * lc], u = Qu[2 * lc], lu = Qlu[2 * lc];
    const int pt = Qp[2 * lc];
    int e = beps;
    if (active) {
      e = xs >= 0 ? xs : beps;
      if (xs >= 0 && (unsigned)(lx - flo) < (unsigned)(fhi - flo)) face_update(e, me, MeSign{msw.x, msw.y, hiw(me.x) >> 31, hiw(me.y) >> 31}, pa, pb);
    }
    e = row16_min(e);
    if (active && j < 2) {
      const int xi = xs < 0 ? 0 : min(xs, e);
      const int code = xi_code(beps, xi);
      int qc = 0;
      if (code != XLOSSLESS) {
        const int xt = beps >> code;
        // 3-D Lorenzo (the fixed term already cancels the halo cells read
        // at the block's edges) or the semi-Lagrangian prediction
        const int pred = bcls == 0 ? (int)((l + u) - lu) + pt : pt;
        int rec;
        qc = quantize((int)(comp ? me.y : me.x), pred, xt, &rec);
        ((double*)&V1w[g + 1][lx + 1])[comp] = (double)rec;
      }
      // this vertex's entries of XQ and MS were read at the top of this step
      // and are not read again: its outputs take their place
      ((uint16_t*)&XSw[g][lx])[comp] = (uint16_t)qc;
      (&MSw[g][lx].x)[comp] = comp ? xi : code;
    }
    __syncthreads();
  }
  for (int d = dhi; d < 2 * TILE - 1; d++) __syncthreads();

  // ---- results of the block, one coalesced write per array
  {
    const int lx = lt & 15, ly = lt >> 4, x = x0 + lx, yy = y0 + ly;
    if (valid && x < W && yy < H) {
      const size_t gv = (size_t)t * HW + (size_t)yy * W + x;
      const double2 r = V1[ly + 1][lx + 1];
      const int2 cx = MS[ly][lx];
      cur[gv] = make_int2((int)r.x, (int)r.y);
      xcode[gv] = (uint8_t)cx.x;
      qcode[gv] = (uint32_t)XS[ly][lx];
      if (xi_dbg) xi_dbg[gv] = cx.y;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------- batched launches
// Block (bx, by) of colour c from the index li of a field's column-padded
// phase grid; false for the padding.
__device__ __forceinline__ bool phase_block(long long li, int tx, int c, int* bx, int* by) {
  const int pc = phase_cols(tx);
  const int y = (int)(li / pc), xi = (int)(li - (long long)y * pc);
  const int b0 = ((c - y) % 3 + 3) % 3;
  *bx = b0 + 3 * xi;
  *by = y;
  return *bx < tx;
}

// Workgroups are dealt to the chip's eight XCDs in turn (workgroup i to XCD
// i mod 8), each with its own L2.  The n workgroups of one field take the
// field's blocks so that those dealt to one XCD form one contiguous run of
// the row-major block order: every XCD keeps a band of block rows in every
// colour phase and frame, and finds the halo and the neighbouring frames in
// its own L2.  A bijection of [0, n).
__device__ __forceinline__ long long xcd_band(long long li, long long n) {
  const long long k = li & 7, q = li >> 3, base = n >> 3, rem = n & 7;
  return k * base + (k < rem ? k : rem) + q;
}

// Class of block (bx, by) of frame t, then its phase.  mstate says whether
// frame t uses decided classes and whether this call decides them.  S is
// the workgroup's TileSmem with DECIDE (one block per workgroup), else its
// NB PhaseSmem; valid is false for a slot without a block.
template <bool DECIDE, int NB, typename Smem>
__device__ __forceinline__ void run_block(Smem* S, bool valid, const BatchView& B, const FieldDesc& d,
                                          const FieldParams& p, int t, int bx, int by, int mstate, int gidx) {
  int2* cur = B.cur + d.voff;
  const uint8_t* flags = B.flags + d.voff;
  // the class is either known here or read from clsp inside the phase,
  // after the frame loads are under way
  int cls = 0;
  const uint8_t* clsp = nullptr;
  if (t >= 1) {
    if (p.predictor == 1) {
      cls = 1;
    } else if (mstate != MODES_NONE) {
      uint8_t* mrow = B.modes + d.mbase + (size_t)gidx * p.tx * p.ty;
      if constexpr (DECIDE) {
        if (mstate == MODES_DECIDE) {
          float* feats = d.feats_dbg ? d.feats_dbg + (size_t)gidx * p.tx * p.ty * 10 : nullptr;
          if (threadIdx.x < 64) {
            const int c = block_mode(S->m, cur, flags, p, t, bx, by, B.tlog, B.selw, mrow, feats);
            if (threadIdx.x == 0) S->m.cls = c;
          }
          __syncthreads();
          cls = S->m.cls;
          __syncthreads();
        } else {
          clsp = mrow + (size_t)by * p.tx + bx;
        }
      } else {
        clsp = mrow + (size_t)by * p.tx + bx;
      }
    }
  }
  if constexpr (DECIDE)
    phase_tile<1>(&S->p, valid, cur, flags, p, t, bx, by, cls, clsp, B.xcode + d.voff, B.qcode + d.voff, d.xi_dbg);
  else
    phase_tile<NB>(S, valid, cur, flags, p, t, bx, by, cls, clsp, B.xcode + d.voff, B.qcode + d.voff, d.xi_dbg);
}

// predictor classes of frame t for every block of the first m fields of the
// launch order; pre[j] = blocks of the fields before j
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_modes_b(BatchView B, const long long* __restrict__ pre, int m, int t,
                                                int gidx) {
  __shared__ ModesSmem S;
  const int j = find_field(pre, m, blockIdx.x);
  const FieldDesc& d = B.D[j == 0 ? B.ord0 : B.ord[j]];
  if (d.status) return;
  const FieldParams p = d.p;
  const long long li = xcd_band((long long)blockIdx.x - pre[j], pre[j + 1] - pre[j]);
  const int by = (int)(li / p.tx), bx = (int)(li - (long long)by * p.tx);
  uint8_t* mrow = B.modes + d.mbase + (size_t)gidx * p.tx * p.ty;
  float* feats = d.feats_dbg ? d.feats_dbg + (size_t)gidx * p.tx * p.ty * 10 : nullptr;
  block_mode(S, B.cur + d.voff, B.flags + d.voff, p, t, bx, by, B.tlog, B.selw, mrow, feats);
}

// colour phase c of frame t over the first m fields of the launch order
// (nblocks blocks of column-padded phase grids); with DECIDE the classes of
// a decision frame are chosen in the same launch.  A workgroup of 256 NB
// threads takes NB consecutive blocks of the launch (NB > 1 only without
// DECIDE); the workgroups are banded over the XCDs.
template <bool DECIDE, int NB>
__global__ __launch_bounds__(256 * NB) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_phase_b(
    BatchView B, const long long* __restrict__ pre, int m, int t, int c, int mstate, int gidx, long long nblocks) {
  static_assert(NB == 1 || !DECIDE, "the fused predictor choice takes one block per workgroup");
  if constexpr (NB == 1) {
    using Smem = typename std::conditional<DECIDE, TileSmem, PhaseSmem>::type;
    __shared__ Smem S;
    const int j = find_field(pre, m, blockIdx.x);
    const FieldDesc& d = B.D[j == 0 ? B.ord0 : B.ord[j]];
    if (d.status) return;
    const FieldParams p = d.p;
    int bx, by;
    if (!phase_block(xcd_band((long long)blockIdx.x - pre[j], pre[j + 1] - pre[j]), p.tx, c, &bx, &by)) return;
    run_block<DECIDE, 1>(&S, true, B, d, p, t, bx, by, mstate, gidx);
  } else {
    // every slot keeps the barriers, with or without a block
    __shared__ PhaseSmem S[NB];
    // the slot of the wave's own block (uniform over the wave)
    const int bs = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 8));
    const long long li = xcd_band(blockIdx.x, (nblocks + NB - 1) / NB) * NB + bs;
    bool valid = li < nblocks;
    const int j = find_field(pre, m, valid ? li : nblocks - 1);
    const FieldDesc& d = B.D[j == 0 ? B.ord0 : B.ord[j]];
    const FieldParams p = d.p;
    int bx = 0, by = 0;
    valid = valid && !d.status && phase_block(li - pre[j], p.tx, c, &bx, &by);
    run_block<false, NB>(S, valid, B, d, p, t, bx, by, mstate, gidx);
  }
}

// ------------------------------------------------------ persistent schedule
// Work items are groups of up to `group` blocks of one stage (field, frame,
// colour).  Items are numbered stage round by stage round (round r holds
// stage r of every field that has one), so every item depends only on items
// with smaller numbers.  A workgroup takes the next number, waits until its
// field has finished all items of earlier stages (done[f] >= need), runs
// the blocks and counts the item as done.  Items are taken in increasing
// order by running workgroups, so every wait ends.
//
// Polling uses relaxed loads: an acquire load would invalidate the caches
// every workgroup of the chip shares on each poll.  One acquire fence per
// wave follows the wait, one release fence per wave precedes the count.
// A wait longer than `budget` wall-clock ticks raises ctl[1], and every
// workgroup leaves.
__device__ __forceinline__ unsigned ld_relaxed(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_persist(
    BatchView B, const SchedSeg* __restrict__ seg, const long long* __restrict__ sstart, int nseg,
    long long nitems, int group, unsigned* done, unsigned* ctl, unsigned long long budget) {
  __shared__ TileSmem S;
  __shared__ unsigned s_item;
  __shared__ int s_go;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      const unsigned it = atomicAdd(&ctl[0], 1u);
      int go = 0;
      if ((long long)it < nitems && !ld_relaxed(&ctl[1])) {
        const int j = find_field(sstart, nseg, it);
        const unsigned f = (unsigned)seg[j].f, need = seg[j].need;
        go = 1;
        if (ld_relaxed(&done[f]) < need) {
          const unsigned long long t0 = wall_clock64();
          int nap = 1;
          while (ld_relaxed(&done[f]) < need) {
            if (ld_relaxed(&ctl[1]) || wall_clock64() - t0 > budget) {
              atomicOr(&ctl[1], 1u);
              go = 0;
              break;
            }
            if (nap == 1) __builtin_amdgcn_s_sleep(1);
            else if (nap == 2) __builtin_amdgcn_s_sleep(4);
            else __builtin_amdgcn_s_sleep(16);
            nap = nap < 3 ? nap + 1 : 3;
          }
        }
      }
      s_item = it;
      s_go = go;
    }
    __syncthreads();
    if (!s_go) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const long long it = s_item;
    const int j = find_field(sstart, nseg, it);
    const SchedSeg sg = seg[j];
    const FieldDesc& d = B.D[sg.f];
    if (!d.status) {
      const FieldParams p = d.p;
      const long long li0 = (it - sstart[j]) * group;
      for (int g = 0; g < group; g++) {
        const long long li = li0 + g;
        if (li >= sg.nb) break;
        int bx, by;
        if (phase_block(li, p.tx, sg.c, &bx, &by)) run_block<true, 1>(&S, true, B, d, p, sg.t, bx, by, sg.mstate, sg.gidx);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&done[sg.f], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ============================================================ launchers
void launch_modes_b(const BatchView& B, const long long* pre, int m, long long nblocks, int t, int gidx,
                    hipStream_t s) {
  if (nblocks > 0) k_modes_b<<<(unsigned)nblocks, 64, 0, s>>>(B, pre, m, t, gidx);
}

void launch_phase_b(const BatchView& B, const long long* pre, int m, long long nblocks, int t, int c,
                    int mstate, int gidx, bool fused, int nb, hipStream_t s) {
  if (nblocks <= 0) return;
  if (fused) k_phase_b<true, 1><<<(unsigned)nblocks, 256, 0, s>>>(B, pre, m, t, c, mstate, gidx, nblocks);
  else if (nb == 1) k_phase_b<false, 1><<<(unsigned)nblocks, 256, 0, s>>>(B, pre, m, t, c, mstate, gidx, nblocks);
  else k_phase_b<false, 2><<<(unsigned)((nblocks + 1) / 2), 512, 0, s>>>(B, pre, m, t, c, mstate, gidx, nblocks);
}

int persist_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist, 256, 0) != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

void launch_persist(const BatchView& B, const SchedSeg* seg, const long long* sstart, int nseg, long long nitems,
                    int group, int grid, unsigned* done, unsigned* ctl, hipStream_t s) {
  // wait budget: two seconds of the device's constant-rate wall clock
  static unsigned long long budget = 0;
  if (!budget) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    budget = 2000ull * (unsigned long long)khz;
  }
  if (nitems > 0 && grid > 0) k_persist<<<grid, 256, 0, s>>>(B, seg, sstart, nseg, nitems, group, done, ctl, budget);
}

}  // namespace cpt
