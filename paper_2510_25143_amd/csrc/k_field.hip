// k_field.hip — field-level kernels: value range, fixed-point conversion,
// SoS edge signs, space-time face masks (critical-point extraction), lossless
// flags, compaction of crossed faces, device-wide exclusive scan and the
// before/after comparison.
//
// Extraction follows Sec. III-C/E/F of the paper: every prism over a
// main-diagonal triangle is split into three tetrahedra; a face is crossed
// when the origin lies in the simulated-simplicity perturbation of its three
// vector values.  Each vertex owns twelve faces and seven edges (the three
// spatial edges to +x, +y, +x+y, the time edge, and the three diagonals to
// the +x, +y, +x+y vertices of the next frame); a face is decided from the
// SoS signs of its three edges, each computed once by the edge's owner.
#include <math.h>

#include "batch.hpp"
#include "cpt_device.hpp"
#include "launch.hpp"

namespace cpt {

// ----------------------------------------------------------------- range
__device__ __forceinline__ int ordered_key(uint32_t b) {
  int s = (int)b;
  return s >= 0 ? s : (s ^ 0x7FFFFFFF);
}

__global__ void k_range_init(int* r) {
  if (threadIdx.x == 0) {
    r[0] = 0x7FFFFFFF;   // min key
    r[1] = (int)0x80000000;  // max key
    r[2] = 0;            // max |x| bits
    r[3] = 0;            // non-finite seen
  }
}

__device__ __forceinline__ void range_acc(uint32_t b, int& mn, int& mx, uint32_t& ma, uint32_t& bad) {
  if (((b >> 23) & 0xFFu) == 0xFFu) bad = 1;
  int key = ordered_key(b);
  mn = min(mn, key);
  mx = max(mx, key);
  ma = max(ma, b & 0x7FFFFFFFu);
}

// min, max (as ordered keys), max |x| bits and a non-finite flag; four
// floats per load
__global__ __launch_bounds__(256) void k_range(const float* __restrict__ x, size_t n, int* r) {
  int mn = 0x7FFFFFFF, mx = (int)0x80000000;
  uint32_t ma = 0, bad = 0;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t n4 = ((uintptr_t)x & 15) == 0 ? n / 4 : 0;
  const uint4* x4 = (const uint4*)x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    uint4 v = x4[i];
    range_acc(v.x, mn, mx, ma, bad);
    range_acc(v.y, mn, mx, ma, bad);
    range_acc(v.z, mn, mx, ma, bad);
    range_acc(v.w, mn, mx, ma, bad);
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    range_acc(__float_as_uint(x[i]), mn, mx, ma, bad);
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, __shfl_xor(mn, o));
    mx = max(mx, __shfl_xor(mx, o));
    ma = max(ma, (uint32_t)__shfl_xor((int)ma, o));
    bad |= (uint32_t)__shfl_xor((int)bad, o);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&r[0], mn);
    atomicMax(&r[1], mx);
    atomicMax((unsigned int*)&r[2], ma);
    if (bad) atomicOr(&r[3], 1);
  }
}

// --------------------------------------------------------- lossless flags
// INC[o]: face types whose vertex set contains offset o = (ox,oy,ot) from the
// owner; a vertex is lossless when any face through it is crossed.
struct IncTable {
  uint16_t m[8];
};
constexpr IncTable make_inc() {
  IncTable I{};
  for (int o = 0; o < 8; o++) {
    uint16_t m = 0;
    for (int f = 0; f < 12; f++)
      for (int i = 0; i < 3; i++)
        if (FTYPE[f][i][0] == (o & 1) && FTYPE[f][i][1] == ((o >> 1) & 1) && FTYPE[f][i][2] == ((o >> 2) & 1))
          m |= (uint16_t)(1u << f);
    I.m[o] = m;
  }
  return I;
}
__constant__ IncTable c_inc = make_inc();

// ------------------------------------------------------- batched field pass
// per-field range slots: min key, max key, max |x| bits, non-finite seen.
// Each field has RANGE_SLOTS slots a cache line apart; workgroup w adds to
// slot w mod RANGE_SLOTS, so the atomics of many workgroups do not queue on
// one line.
__device__ __forceinline__ int4* range_slot(int4* r, int f, long long s) {
  return r + ((size_t)f * RANGE_SLOTS + (size_t)s) * RANGE_SLOT_STRIDE;
}
__global__ void k_range_init_b(int4* __restrict__ r, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * RANGE_SLOTS) *range_slot(r, i / RANGE_SLOTS, i % RANGE_SLOTS) = make_int4(0x7FFFFFFF, (int)0x80000000, 0, 0);
}

// rpre[f]: workgroups of the fields before f, each covering RANGE_SPAN
// floats; one reduction per workgroup, then one atomic per quantity into the
// workgroup's slot
constexpr int RANGE_SPAN = (int)RANGE_SPAN_FLOATS;
__global__ __launch_bounds__(256) void k_range_b(const FieldDesc* __restrict__ D, const long long* __restrict__ rpre,
                                                 int n, int4* __restrict__ r) {
  __shared__ int4 part[4];
  const int f = find_field(rpre, n, blockIdx.x);
  const float* x = D[f].field;
  const size_t nf = 2 * (size_t)D[f].N;
  const size_t lo = (size_t)((long long)blockIdx.x - rpre[f]) * RANGE_SPAN;
  const size_t hi = lo + RANGE_SPAN < nf ? lo + RANGE_SPAN : nf;
  int mn = 0x7FFFFFFF, mx = (int)0x80000000;
  uint32_t ma = 0, bad = 0;
  if (((uintptr_t)x & 15) == 0 && hi - lo == RANGE_SPAN) {
    const uint4* x4 = (const uint4*)(x + lo);
#pragma unroll 4
    for (int k = 0; k < RANGE_SPAN / 1024; k++) {
      uint4 v = x4[k * 256 + threadIdx.x];
      range_acc(v.x, mn, mx, ma, bad);
      range_acc(v.y, mn, mx, ma, bad);
      range_acc(v.z, mn, mx, ma, bad);
      range_acc(v.w, mn, mx, ma, bad);
    }
  } else {
    for (size_t i = lo + threadIdx.x; i < hi; i += 256) range_acc(__float_as_uint(x[i]), mn, mx, ma, bad);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, __shfl_xor(mn, o));
    mx = max(mx, __shfl_xor(mx, o));
    ma = max(ma, (uint32_t)__shfl_xor((int)ma, o));
    bad |= (uint32_t)__shfl_xor((int)bad, o);
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = make_int4(mn, mx, (int)ma, (int)bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; w++) {
      mn = min(mn, part[w].x);
      mx = max(mx, part[w].y);
      ma = max(ma, (uint32_t)part[w].z);
      bad |= (uint32_t)part[w].w;
    }
    int4* q = range_slot(r, f, ((long long)blockIdx.x - rpre[f]) % RANGE_SLOTS);
    atomicMin(&q->x, mn);
    atomicMax(&q->y, mx);
    atomicMax((unsigned int*)&q->z, ma);
    if (bad) atomicOr(&q->w, 1);
  }
}

__device__ __forceinline__ double key_value(int key) {
  int s = key >= 0 ? key : (key ^ 0x7FFFFFFF);
  return (double)__int_as_float(s);
}

// Semi-Lagrangian displacement factor (Sec. VI-A in Q16 fixed point): the
// displacement of a fixed-point velocity u is floor(u c / 2^s) cells in Q16,
// where c / 2^s is r 2^(16-k) (r = dt/dx, the grid's time step over spacing)
// rounded to 31 significant bits: c in [2^30, 2^31), round half to even.
// Two limits: s is at most 62 (c then shorter, possibly 0, and a factor of 0
// is stored as c = s = 0), and a factor of 2^31 - 1 or more saturates to
// c = 2^31 - 1, s = 0.  Worked on the double's bits: r = m 2^ex with an
// integer significand m normalised into [2^52, 2^53).
__device__ void sl_factor_dev(double r, int k, int64_t* c, int64_t* s) {
  const uint64_t bits = (uint64_t)__double_as_longlong(r);
  const int E = (int)((bits >> 52) & 0x7FF);
  uint64_t m = bits & ((1ull << 52) - 1);
  int ex;
  if (E == 0) {
    ex = -1074;
  } else {
    m |= 1ull << 52;
    ex = E - 1075;
  }
  if (m == 0) {  // r = 0: no displacement
    *c = 0;
    *s = 0;
    return;
  }
  const int lz = __clzll((long long)m) - 11;
  m <<= lz;
  ex -= lz;
  const int p = ex + 16 - k;  // r 2^(16-k) = m 2^p
  int sh = -p - 22;  // c = m 2^-22 rounded, c 2^-sh = m 2^p
  int rs = 22;
  if (sh > 62) {
    rs += sh - 62;
    sh = 62;
  }
  uint64_t q = 0;
  if (rs < 64) {
    q = m >> rs;
    const uint64_t rem = m & ((1ull << rs) - 1), half = 1ull << (rs - 1);
    if (rem > half || (rem == half && (q & 1))) q++;
  }
  if (q == (1ull << 31)) {  // rounding carried into bit 31
    q = 1ull << 30;
    sh -= 1;
  }
  if (sh < 0) {  // the factor is 2^31 or more
    *c = 2147483647;
    *s = 0;
    return;
  }
  if (q == 0) sh = 0;
  *c = (int64_t)q;
  *s = sh;
}

// Per-field parameters from the value range (Sec. VI of the paper, fixed
// point): k = 23 - e for max|x| = m 2^e, m in [0.5, 1), at most 120;
// eps' = floor(eb_abs 2^k - 1/2), at most 2^23 - 1.  Every step is exact in
// double precision.
__global__ void k_params_b(FieldDesc* __restrict__ D, const int4* __restrict__ r, int n) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  FieldDesc& d = D[f];
  d.status = 0;
  d.reason = REASON_NONE;
  int4 R = *range_slot(const_cast<int4*>(r), f, 0);
  for (int i = 1; i < RANGE_SLOTS; i++) {
    const int4 q = *range_slot(const_cast<int4*>(r), f, i);
    R.x = min(R.x, q.x);
    R.y = max(R.y, q.y);
    R.z = (int)max((uint32_t)R.z, (uint32_t)q.z);
    R.w |= q.w;
  }
  const double mn = key_value(R.x), mx = key_value(R.y);
  // max|x| = 0.f 2^e with the leading fraction bit set: e from the float's
  // exponent field (normal) or from the position of the leading significand
  // bit (subnormal); k = 23 - e puts max|x| 2^k in [2^22, 2^23)
  const uint32_t mab = (uint32_t)R.z, mexp = mab >> 23, mman = mab & 0x7FFFFFu;
  int kk = 23;
  if (R.w) {
    d.status = STATUS_EINVAL;
    d.reason = REASON_NONFINITE;
  } else if (mexp >= 127 + 100) {
    d.status = STATUS_EINVAL;
    d.reason = REASON_MAGNITUDE;
  } else if (mab != 0) {
    const int e = mexp ? (int)mexp - 126 : (32 - __clz((int)mman)) - 149;
    kk = min(23 - e, 120);
  }
  // eps' = floor(eb_abs 2^k - 1/2) in [0, 2^23 - 1]: the half unit absorbs
  // the rounding of the conversion, so |x - x'| <= eb_abs in field units
  const double a = d.eb_mode == 0 ? d.eb * (mx - mn) : d.eb;
  const double sc = floor(ldexp(a, kk) - 0.5);
  const int64_t ep = sc <= 0.0 ? 0 : (sc >= 8388607.0 ? 8388607 : (int64_t)sc);
  FieldParams p;
  p.H = d.H;
  p.W = d.W;
  p.T = d.T;
  p.k = kk;
  p.eps = (int)ep;
  p.tx = d.tx;
  p.ty = d.ty;
  p.predictor = d.predictor;
  p.K = d.K;
  p.bt = d.bt;
  sl_factor_dev(d.dt_dx, kk, &p.cx, &p.sx);
  sl_factor_dev(d.dt_dy, kk, &p.cy, &p.sy);
  d.p = p;
  d.eb_abs = a;
}

// ------------------------------------------------------ fused field pass
// One workgroup per 32x16 tile of one field marches through the frames:
// per frame it converts the tile (plus halo) to fixed point, computes the
// SoS edge signs, the face masks and the lossless flags in shared memory,
// and writes only the fixed-point values and the flags.  At step s the
// edges of frame s+1 need frames s+1 and s+2, the masks of frame s need the
// edges of s and s+1, the flags of frame s need the masks of s and s-1; two
// frames of each are kept.  Halos: values [-1, 34) x [-1, 18), edges
// [-1, 33) x [-1, 17), masks [-1, 32) x [-1, 16) relative to the tile.
// The tile is an execution parameter: every shape gives the same output.
// Three shapes are built (FP_SHAPE_TW / FP_SHAPE_TH in batch.hpp), each with
// at most 768 halo values, so that three per thread cover them.
template <int TW, int TH>
struct FpShape {
  static constexpr int CW = TW + 3, CH = TH + 3;  // values
  static constexpr int EW = TW + 2, EH = TH + 2;  // edge cells
  static constexpr int MW = TW + 1, MH = TH + 1;  // mask cells
  static constexpr int NC = CW * CH;
  static_assert(NC <= 3 * 256, "three halo values per thread");
};

template <int TW, int TH>
struct FieldPassSmem {
  using Sh = FpShape<TW, TH>;
  int2 cur[2][Sh::CH][Sh::CW];
  uint8_t edg[2][Sh::EH][Sh::EW];
  uint32_t msk[2][Sh::MH][Sh::MW];
};

// A, B: values of frames t and t + 1 as flat [CH][CW] arrays; c: the
// owner's flat index
template <int FP_CW>
__device__ __forceinline__ uint32_t fp_edges(const int2* A, const int2* B, int c, bool px, bool py, bool pt) {
  const int2 a = A[c];
  uint32_t e = 0;
  if (px) e |= (sos_sign(a.x, a.y, A[c + 1].x, A[c + 1].y) > 0) << 0;
  if (py) e |= (sos_sign(a.x, a.y, A[c + FP_CW].x, A[c + FP_CW].y) > 0) << 1;
  if (px && py) e |= (sos_sign(a.x, a.y, A[c + FP_CW + 1].x, A[c + FP_CW + 1].y) > 0) << 2;
  if (pt) {
    e |= (sos_sign(a.x, a.y, B[c].x, B[c].y) > 0) << 3;
    if (px) e |= (sos_sign(a.x, a.y, B[c + 1].x, B[c + 1].y) > 0) << 4;
    if (py) e |= (sos_sign(a.x, a.y, B[c + FP_CW].x, B[c + FP_CW].y) > 0) << 5;
    if (px && py) e |= (sos_sign(a.x, a.y, B[c + FP_CW + 1].x, B[c + FP_CW + 1].y) > 0) << 6;
  }
  return e;
}

// The twelve face tests of a cell side by side.  Face f is crossed when
// the signs of its edges ab and bc agree and differ from that of ac; bit f
// of X, Y, Z holds the sign of ab, bc, ac.  X and Z come from the owner's
// own seven edge bits (table xz: X in bits 0-11, Z in bits 16-27), Y from
// the edges of the neighbouring cells.  Faces whose prism leaves the
// domain are masked out; the sign of a crossed face is that of ab.
__device__ __forceinline__ uint32_t fp_xz(uint32_t ea) {
  constexpr int xb[12] = {0, 1, 0, 4, 1, 5, 0, 3, 1, 3, 2, 3};
  constexpr int zb[12] = {2, 2, 6, 6, 6, 6, 4, 4, 5, 5, 6, 6};
  uint32_t x = 0, z = 0;
#pragma unroll
  for (int f = 0; f < 12; f++) {
    x |= ((ea >> xb[f]) & 1u) << f;
    z |= ((ea >> zb[f]) & 1u) << f;
  }
  return x | (z << 16);
}

// The faces of a cell that stay inside the domain: the two in the frame
// need the cell's x and y successors, the others also the next frame.
__device__ __forceinline__ uint32_t fp_valid(bool px, bool py, bool pt) {
  return (px && py ? 0x003u : 0u) | (px && py && pt ? 0xC3Cu : 0u) | (px && pt ? 0x0C0u : 0u) |
         (py && pt ? 0x300u : 0u);
}

// E0, E1: edge bytes of frames t and t + 1 as flat [EH][EW] arrays;
// e: the owner's flat index; valid: fp_valid of the cell
template <int FP_EW>
__device__ __forceinline__ uint32_t fp_mask(const uint8_t* E0, const uint8_t* E1, const uint32_t* __restrict__ xz,
                                            int e, uint32_t valid) {
  if (!valid) return 0;
  const uint32_t ea = E0[e], eb = E0[e + 1], ec = E0[e + FP_EW], ed = E0[e + FP_EW + 1];
  const uint32_t ea1 = E1[e], eb1 = E1[e + 1], ec1 = E1[e + FP_EW];
  const uint32_t t = xz[ea & 127u];
  const uint32_t X = t & 0xFFFu, Z = t >> 16;
#define B(e, k, f) ((((e) >> (k)) & 1u) << (f))
  const uint32_t Y = B(eb, 1, 0) | B(ec, 0, 1) | B(eb, 5, 2) | B(eb1, 1, 3) | B(ec, 4, 4) | B(ec1, 0, 5) |
                     B(eb, 3, 6) | B(ea1, 0, 7) | B(ec, 3, 8) | B(ea1, 1, 9) | B(ed, 3, 10) | B(ea1, 2, 11);
#undef B
  const uint32_t crossed = ~(X ^ Y) & (Z ^ Y) & valid;
  return crossed | ((X & crossed) << 12);
}

// One 32x16 tile at (x0, y0) of a field marching through its frames.  With
// MASKS false it writes the tile's fixed-point values (cur) and lossless
// flags; with MASKS true only its face masks (twelve crossed-face bits and
// their signs per vertex, as the extraction numbers them).
template <bool MASKS, int FP_TW, int FP_TH>
__device__ __forceinline__ void fieldpass_tile(FieldPassSmem<FP_TW, FP_TH>& S, uint32_t* xz,
                                               const float* __restrict__ field, int H, int W, int T, int k, int x0,
                                               int y0, int2* __restrict__ cur, uint8_t* __restrict__ flags,
                                               uint32_t* __restrict__ masks) {
  using Sh = FpShape<FP_TW, FP_TH>;
  constexpr int FP_CW = Sh::CW, FP_EW = Sh::EW, FP_EH = Sh::EH, FP_MW = Sh::MW, FP_MH = Sh::MH, FP_NC = Sh::NC;
  const size_t HW = (size_t)H * W, N = HW * (size_t)T;
  const float* fu = field;
  const float* fv = field + N;
  const int tid = threadIdx.x;

  // Per-thread offsets of halo values j = tid + 256 q (flat [FP_CH][FP_CW]
  // index j) within a frame, fixed over the frames: -1 outside the domain
  // (H W T < 2^31, so they fit 32 bits); bit q of tv: value j is a tile
  // vertex, written out.  Edge and mask cells j = tid + 256 q, three bits
  // each (cell in the domain, its x and y successors in the domain): edge
  // cells in bits 3q of ecell, mask cells in bits 3q of mcell.
  int hoff[3];
  uint32_t tv = 0, ecell = 0, mcell = 0;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const int j = tid + 256 * q;
    const int cy = j / FP_CW, cx = j - cy * FP_CW;
    const int x = x0 + cx - 1, y = y0 + cy - 1;
    const bool in = j < FP_NC && x >= 0 && x < W && y >= 0 && y < H;
    hoff[q] = in ? y * W + x : -1;
    if (in && cx >= 1 && cx <= FP_TW && cy >= 1 && cy <= FP_TH) tv |= 1u << q;
    const int ey = j / FP_EW, ex = j - ey * FP_EW, ux = x0 + ex - 1, uy = y0 + ey - 1;
    if (ux >= 0 && ux < W && uy >= 0 && uy < H)
      ecell |= (1u | (ux + 1 < W ? 2u : 0u) | (uy + 1 < H ? 4u : 0u)) << (3 * q);
    const int my = j / FP_MW, mx = j - my * FP_MW, vx = x0 + mx - 1, vy = y0 + my - 1;
    if (vx >= 0 && vx < W && vy >= 0 && vy < H)
      mcell |= (1u | (vx + 1 < W ? 2u : 0u) | (vy + 1 < H ? 4u : 0u)) << (3 * q);
  }

  // halo values of frame t: fixed-point pairs (0 outside the domain)
  float ru[3], rv[3];
  auto fetch = [&](int t) {
    const float* pu = fu + (size_t)t * HW;
    const float* pv = fv + (size_t)t * HW;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      ru[q] = rv[q] = 0.f;
      if (t < T && hoff[q] >= 0) {
        ru[q] = pu[hoff[q]];
        rv[q] = pv[hoff[q]];
      }
    }
  };
  auto store = [&](int t) {
    int2* sc = &S.cur[t & 1][0][0];
    int2* pc = MASKS ? nullptr : cur + (size_t)t * HW;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const int j = tid + 256 * q;
      if (j >= FP_NC) continue;
      const bool in = t < T && hoff[q] >= 0;
      const int2 v = in ? make_int2(to_fixed(ru[q], k), to_fixed(rv[q], k)) : make_int2(0, 0);
      sc[j] = v;
      if (!MASKS && in && (tv >> q & 1u)) pc[hoff[q]] = v;
    }
  };
  auto edges_of = [&](int t) {  // edges of frame t (t + 1 < T uses frame t + 1)
    const int2* A = &S.cur[t & 1][0][0];
    const int2* B = &S.cur[(t + 1) & 1][0][0];
    uint8_t* E = &S.edg[t & 1][0][0];
    const bool pt = t + 1 < T;
    uint32_t c = ecell;
    for (int j = tid; j < FP_EW * FP_EH; j += 256, c >>= 3) {
      uint32_t e = 0;
      if (c & 1u) e = fp_edges<FP_CW>(A, B, j + j / FP_EW, c & 2u, c & 4u, pt);
      E[j] = (uint8_t)e;
    }
  };

  if (tid < 128) xz[tid] = fp_xz((uint32_t)tid);
  // the masks of "frame -1" are empty, so the flags of frame 0 read zeros
  // there (cells outside the domain hold zero masks as well)
  for (int j = tid; j < FP_MW * FP_MH; j += 256) (&S.msk[1][0][0])[j] = 0u;
  // prologue: frames 0 and 1, edges of frame 0
  fetch(0);
  store(0);
  fetch(1);
  store(1);
  fetch(2);
  __syncthreads();
  edges_of(0);
  __syncthreads();
  for (int s = 0; s < T; s++) {
    // values of frame s + 2 (loaded during the previous step), then start
    // loading frame s + 3
    if (s + 2 < T) store(s + 2);
    fetch(s + 3);
    __syncthreads();
    if (s + 1 < T) edges_of(s + 1);
    __syncthreads();
    // masks of frame s
    {
      const uint8_t* E0 = &S.edg[s & 1][0][0];
      const uint8_t* E1 = &S.edg[(s + 1) & 1][0][0];
      uint32_t* M = &S.msk[s & 1][0][0];
      const bool pt = s + 1 < T;
      uint32_t c = mcell;
      for (int j = tid; j < FP_MW * FP_MH; j += 256, c >>= 3) {
        M[j] = fp_mask<FP_EW>(E0, E1, xz, j + j / FP_MW, (c & 1u) ? fp_valid(c & 2u, c & 4u, pt) : 0u);
      }
    }
    __syncthreads();
    if constexpr (MASKS) {
      // the face masks of the tile's vertices of frame s
      uint32_t* pm = masks + (size_t)s * HW;
      for (int j = tid; j < FP_TW * FP_TH; j += 256) {
        const int iy = j / FP_TW, ix = j - iy * FP_TW;
        const int x = x0 + ix, y = y0 + iy;
        if (x < W && y < H) pm[(size_t)y * W + x] = S.msk[s & 1][iy + 1][ix + 1];
      }
    } else {
      // lossless flags of frame s: any crossed face through the vertex
      uint8_t* pf = flags + (size_t)s * HW;
      for (int j = tid; j < FP_TW * FP_TH; j += 256) {
        const int iy = j / FP_TW, ix = j - iy * FP_TW;
        const int x = x0 + ix, y = y0 + iy;
        if (x >= W || y >= H) continue;
        uint32_t any = 0;
#pragma unroll
        for (int o = 0; o < 8; o++) {
          const int ox = o & 1, oy = (o >> 1) & 1, ot = (o >> 2) & 1;
          any |= S.msk[(s - ot) & 1][iy + 1 - oy][ix + 1 - ox] & c_inc.m[o];
        }
        pf[y * W + x] = any ? 1 : 0;
      }
    }
  }
}


// fpre[f]: tiles of the fields before f
template <int TW, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_fieldpass_b(const FieldDesc* __restrict__ D,
                                                     const long long* __restrict__ fpre, int n,
                                                     int2* __restrict__ cur_all, uint8_t* __restrict__ flags_all) {
  __shared__ FieldPassSmem<TW, TH> S;
  __shared__ uint32_t xz[128];  // the X and Z words of the face tests per edge byte of the owner
  const int f = find_field(fpre, n, blockIdx.x);
  const FieldDesc& d = D[f];
  if (d.status) return;
  const int ntx = (d.W + TW - 1) / TW;
  const int tile = (int)((long long)blockIdx.x - fpre[f]);
  fieldpass_tile<false, TW, TH>(S, xz, d.field, d.H, d.W, d.T, d.p.k, (tile % ntx) * TW, (tile / ntx) * TH,
                                cur_all + d.voff, flags_all + d.voff, nullptr);
}

// Face masks of one field on the grid 2^k, one workgroup per 32x16 tile.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_maskpass(
    const float* __restrict__ field, int H, int W, int T, int k, uint32_t* __restrict__ masks) {
  __shared__ FieldPassSmem<32, 16> S;
  __shared__ uint32_t xz[128];
  const int ntx = (W + 31) / 32;
  const int tile = blockIdx.x;
  fieldpass_tile<true, 32, 16>(S, xz, field, H, W, T, k, (tile % ntx) * 32, (tile / ntx) * 16, nullptr, nullptr,
                               masks);
}

// ------------------------------------------------------------- compaction
__global__ __launch_bounds__(256) void k_count_faces(const uint32_t* __restrict__ masks, size_t N,
                                                     uint32_t* __restrict__ cnt) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) cnt[i] = __popc(masks[i] & 0xFFFu);
}

__global__ __launch_bounds__(256) void k_write_codes(const uint32_t* __restrict__ masks,
                                                     const uint32_t* __restrict__ ofs, size_t N,
                                                     uint64_t* __restrict__ codes, size_t cap) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t m = masks[i];
  if (!(m & 0xFFFu)) return;
  size_t o = ofs[i];
  for (int f = 0; f < 12; f++)
    if (m & (1u << f)) {
      if (o < cap) codes[o] = (((uint64_t)i * 12 + f) << 1) | ((m >> (12 + f)) & 1u);
      o++;
    }
}

// ------------------------------------------------------------------ scan
// Exclusive scan of n uint32 values in three passes; blocks of 256 threads
// own 2048 consecutive values.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;

__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[4];
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < 4; w++) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, size_t n,
                                                     uint32_t* __restrict__ part) {
  size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
  if (base + SCAN_ITEMS <= n) {
    const uint4* p4 = (const uint4*)(in + base);
    const uint4 a = p4[0], b = p4[1];
    s = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
  } else {
    for (int j = 0; j < SCAN_ITEMS; j++)
      if (base + j < n) s += in[base + j];
  }
  uint32_t tot;
  block_exclusive(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// exclusive scan of the nb partials by one workgroup of 1024 threads, each
// owning a run of consecutive partials
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* __restrict__ part, size_t nb,
                                                        uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[16];
  const size_t per = (nb + 1023) / 1024;
  const size_t lo = (size_t)threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
  uint32_t s = 0;
  for (size_t i = lo; i < hi; i++) s += part[i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = s;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  uint32_t carry = 0, tot = 0;
  for (int w = 0; w < 16; w++) {
    if (w < wid) carry += wsum[w];
    tot += wsum[w];
  }
  uint32_t run = carry + x - s;
  for (size_t i = lo; i < hi; i++) {
    const uint32_t v = part[i];
    part[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, size_t n,
                                                    const uint32_t* __restrict__ part,
                                                    uint32_t* __restrict__ out) {
  size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  const bool full = base + SCAN_ITEMS <= n;
  if (full) {
    const uint4* p4 = (const uint4*)(in + base);
    const uint4 a = p4[0], b = p4[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) v[j] = base + j < n ? in[base + j] : 0;
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) s += v[j];
  uint32_t tot;
  uint32_t ex = block_exclusive(s, &tot) + part[blockIdx.x];
  uint32_t o[SCAN_ITEMS];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    o[j] = ex;
    ex += v[j];
  }
  if (full) {
    uint4* q4 = (uint4*)(out + base);
    q4[0] = make_uint4(o[0], o[1], o[2], o[3]);
    q4[1] = make_uint4(o[4], o[5], o[6], o[7]);
  } else {
    for (int j = 0; j < SCAN_ITEMS; j++)
      if (base + j < n) out[base + j] = o[j];
  }
}

// ---------------------------------------------------------------- compare
__global__ __launch_bounds__(256) void k_compare(const uint32_t* __restrict__ ma, const uint32_t* __restrict__ mb,
                                                 const float* __restrict__ a, const float* __restrict__ b,
                                                 size_t N, unsigned long long* __restrict__ fc,
                                                 double* __restrict__ part) {
  // part[3*block]: max |a-b|, sum (a-b)^2 (fixed order within a block)
  __shared__ double smax[256], ssum[256];
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dm = 0.0, ds = 0.0;
  uint32_t ft = 0, fs = 0;
  if (i < N) {
    uint32_t x = ma[i] ^ mb[i];
    uint32_t crossed = ma[i] & 0xFFFu;
    uint32_t bad = (x & 0xFFFu) | ((x >> 12) & crossed & 0xFFFu);
    ft = __popc(bad & 3u);
    fs = __popc(bad & ~3u);
    for (int c = 0; c < 2; c++) {
      double d = fabs((double)a[c * N + i] - (double)b[c * N + i]);
      dm = fmax(dm, d);
      ds = fma(d, d, ds);
    }
  }
  if (ft) atomicAdd(&fc[0], (unsigned long long)ft);
  if (fs) atomicAdd(&fc[1], (unsigned long long)fs);
  smax[threadIdx.x] = dm;
  ssum[threadIdx.x] = ds;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smax[0];
    part[2 * blockIdx.x + 1] = ssum[0];
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ============================================================ launchers
static inline unsigned nblk(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_range(const float* x, size_t n, int* r, hipStream_t s) {
  k_range_init<<<1, 64, 0, s>>>(r);
  unsigned g = nblk((n + 3) / 4);
  if (g > 2048) g = 2048;
  if (g == 0) g = 1;
  k_range<<<g, 256, 0, s>>>(x, n, r);
}
void launch_maskpass(const float* f, int H, int W, int T, int k, uint32_t* masks, hipStream_t s) {
  const long long tiles = (long long)((W + 31) / 32) * ((H + 15) / 16);
  if (tiles > 0 && T > 0) k_maskpass<<<(unsigned)tiles, 256, 0, s>>>(f, H, W, T, k, masks);
}
size_t scan_partials_size(size_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }
void launch_scan(const uint32_t* in, size_t n, uint32_t* out, uint32_t* part, uint32_t* total, hipStream_t s) {
  size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) {
    k_scan_partials<<<1, 1024, 0, s>>>(part, 0, total);
    return;
  }
  k_scan_reduce<<<(unsigned)nb, 256, 0, s>>>(in, n, part);
  k_scan_partials<<<1, 1024, 0, s>>>(part, nb, total);
  k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(in, n, part, out);
}
void launch_count_faces(const uint32_t* masks, size_t N, uint32_t* cnt, hipStream_t s) {
  k_count_faces<<<nblk(N), 256, 0, s>>>(masks, N, cnt);
}
void launch_write_codes(const uint32_t* masks, const uint32_t* ofs, size_t N, uint64_t* codes, size_t cap,
                        hipStream_t s) {
  k_write_codes<<<nblk(N), 256, 0, s>>>(masks, ofs, N, codes, cap);
}
size_t compare_partials(size_t N) { return nblk(N); }

void launch_params_b(FieldDesc* D, int n, const long long* rpre, long long rblocks, int4* range, hipStream_t s) {
  k_range_init_b<<<nblk((size_t)n * RANGE_SLOTS, 64), 64, 0, s>>>(range, n);
  if (rblocks > 0) k_range_b<<<(unsigned)rblocks, 256, 0, s>>>(D, rpre, n, range);
  k_params_b<<<nblk(n, 64), 64, 0, s>>>(D, range, n);
}
static_assert(FP_SHAPES == 3 && FP_SHAPE_TW[0] == 32 && FP_SHAPE_TH[0] == 16 && FP_SHAPE_TW[1] == 64 &&
                  FP_SHAPE_TH[1] == 8 && FP_SHAPE_TW[2] == 16 && FP_SHAPE_TH[2] == 32,
              "the instantiated tile shapes");
void launch_fieldpass_b(FieldDesc* D, int n, const long long* rpre, long long rblocks, const long long* fpre,
                        long long fblocks, int4* range, int2* cur, uint8_t* flags, int shape, hipStream_t s) {
  launch_params_b(D, n, rpre, rblocks, range, s);
  if (fblocks <= 0) return;
  if (shape == 1) k_fieldpass_b<64, 8><<<(unsigned)fblocks, 256, 0, s>>>(D, fpre, n, cur, flags);
  else if (shape == 2) k_fieldpass_b<16, 32><<<(unsigned)fblocks, 256, 0, s>>>(D, fpre, n, cur, flags);
  else k_fieldpass_b<32, 16><<<(unsigned)fblocks, 256, 0, s>>>(D, fpre, n, cur, flags);
}
void launch_compare(const uint32_t* ma, const uint32_t* mb, const float* a, const float* b, size_t N,
                    unsigned long long* fc, double* part, hipStream_t s) {
  k_zero_u64<<<1, 64, 0, s>>>(fc, 2);
  k_compare<<<nblk(N), 256, 0, s>>>(ma, mb, a, b, N, fc, part);
}

}  // namespace cpt
