// cpt_device.hpp — device-side constants and exact integer helpers shared by
// the HIP kernels of libcptraj.
//
// Method: "Time-Varying Vector Field Compression with Preserved Critical
// Point Trajectories" (arXiv 2510.25143).  Every predicate below is exact:
// values are 25-bit fixed-point integers, so every 2x2 determinant (< 2^50)
// and every sum of three (< 2^52) is an exact fp64 value, and fp64 FMA runs
// at full vector rate on CDNA4 where 64-bit integer multiply does not.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpt {

constexpr int TILE = 16;         // spatial block edge (blocking and mode choice)
constexpr int QR = 512;          // residual quantization radius
constexpr int QSYM = 2 * QR;     // residual code alphabet, code 0 = unpredictable
constexpr int XSYM = 25;         // bound code alphabet, 24 = lossless
constexpr int XLOSSLESS = 24;
constexpr int MAXLEN = 16;       // longest Huffman codeword
// Decoding table of one alphabet (32-bit words): the entry of every 12-bit
// prefix (symbol | length << 16 for a code of at most 12 bits, LUT_LONG for
// the prefix of longer codes, LUT_BAD where no code starts), then per length
// 13..16 its first canonical code, its number of codes and the index of its
// first symbol in the list of long codes, then that list as 16-bit symbols.
constexpr int LUT_BITS = 12;
constexpr int LUT_FIRST = 1 << LUT_BITS, LUT_COUNT = LUT_FIRST + 4, LUT_BASE = LUT_FIRST + 8;
constexpr int LUT_SYMS = LUT_FIRST + 16;  // word index of the long-code symbol list
constexpr int LUT_WORDS = LUT_SYMS + 512;
constexpr uint32_t LUT_LONG = 0xFFFFFFFEu, LUT_BAD = 0xFFFFFFFFu;
static_assert(MAXLEN - LUT_BITS == 4, "four long-code lengths");
constexpr int CHUNK = 1024;      // symbols per independently decodable chunk
constexpr int NMAX = 32;         // maximum semi-Lagrangian substeps
constexpr int HALO = TILE + 2;   // block plus one-vertex halo

// ---------------------------------------------------------------- integers
__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
  int64_t q = a / b, r = a - q * b;
  return (r != 0 && ((r < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int floor_div32(int a, int b) {  // b > 0
  int q = a / b;
  return (q * b > a) ? q - 1 : q;
}
__device__ __forceinline__ int iabs(int a) { return a < 0 ? -a : a; }

// Exact round-half-even of x * 2^k computed from the float's bits, so that
// the result never depends on the denormal or rounding mode of the ALU.
// Callers guarantee |x| 2^k < 2^24.
__device__ __forceinline__ int to_fixed(float x, int k) {
  uint32_t b = __float_as_uint(x);
  uint32_t e = (b >> 23) & 0xFFu;
  uint32_t m = b & 0x7FFFFFu;
  int ex;
  if (e == 0) {
    ex = -149 + k;
  } else {
    m |= 0x800000u;
    ex = (int)e - 150 + k;
  }
  int r;
  if (ex >= 0) {
    r = ex > 7 ? 0x7FFFFFFF : (int)(m << ex);
  } else {
    int sh = -ex;
    if (sh > 25) {
      r = 0;
    } else {
      uint32_t q = m >> sh, rem = m & ((1u << sh) - 1u), half = 1u << (sh - 1);
      if (rem > half || (rem == half && (q & 1u))) q++;
      r = (int)q;
    }
  }
  return (b >> 31) ? -r : r;
}

// Exact x 2^-k for |x| < 2^25 (all results normal or zero by choice of k).
__device__ __forceinline__ float from_fixed(int x, int k) {
  return ldexpf((float)x, -k);
}

// ------------------------------------------------- simulation of simplicity
// Sign of det(p~, q~) for g_p < g_q with v perturbed by eps^(2^(2g)) and u by
// eps^(2^(2g+1)): first nonzero of (u_p v_q - v_p u_q, -u_q, v_q, u_p, 1).
__device__ __forceinline__ int sos_sign(int up, int vp, int uq, int vq) {
  double d = fma((double)up, (double)vq, -((double)vp * (double)uq));
  if (d != 0.0) return d > 0.0 ? 1 : -1;
  if (uq != 0) return uq < 0 ? 1 : -1;
  if (vq != 0) return vq > 0 ? 1 : -1;
  if (up != 0) return up > 0 ? 1 : -1;
  return 1;
}

// exact 2x2 determinant u_a v_b - v_a u_b of 25-bit integers
__device__ __forceinline__ double det2(int2 a, int2 b) {
  return fma((double)a.x, (double)b.y, -((double)a.y * (double)b.x));
}

// Minimum over each row of 16 lanes (DPP row rotations; every lane of the
// row receives the result).  Called with every lane of the wave enabled, so
// no lane reads outside the row's live values; bound_ctrl lets the compiler
// fold each rotation into the min itself.
__device__ __forceinline__ int row16_min(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true));  // row_ror:8
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, true));  // row_ror:4
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x122, 0xF, 0xF, true));  // row_ror:2
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x121, 0xF, 0xF, true));  // row_ror:1
  return v;
}

// Sums over the 16 lanes of each DPP row, every lane enabled: the row's
// total in every lane, and each lane's exclusive prefix.
__device__ __forceinline__ uint32_t row16_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);  // row_ror:8
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, true);  // row_ror:4
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x122, 0xF, 0xF, true);  // row_ror:2
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x121, 0xF, 0xF, true);  // row_ror:1
  return v;
}
__device__ __forceinline__ uint32_t row16_exclusive(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  return x - v;
}

// Inclusive prefix sum over the wave, every lane enabled: DPP row prefixes,
// then the totals of the rows before (lanes 15, 31, 47) added per row.
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
  const uint32_t t1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 31);
  const uint32_t t2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 47);
  const int row = (int)(threadIdx.x & 63) >> 4;
  return x + (row > 0 ? t0 : 0u) + (row > 1 ? t1 : 0u) + (row > 2 ? t2 : 0u);
}

// Minimum over each quad of 4 lanes (DPP quad permutations).
__device__ __forceinline__ int quad_min(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));  // quad_perm [2,3,0,1]
  return v;
}

// Bound code: smallest q with (eps >> q) <= xi; 24 when xi == 0.
__device__ __forceinline__ int xi_code(int eps, int xi) {
  if (xi <= 0) return XLOSSLESS;
  int q = (32 - __clz(eps)) - (32 - __clz(xi));
  if (q < 0) q = 0;
  if ((eps >> q) > xi) q++;
  return q;
}

// Residual quantization with bin 2 xt + 1; returns the code (0 when the
// component is unpredictable) and writes the reconstruction.  The quotient
// q = floor((x - pred + xt) / w) is estimated in fp32 and corrected to the
// exact value; the component is predictable when 1 - QR <= q <= QR - 1.
// With eps' < 2^23 and |x|, |pred| < 2^28 every step fits in 32 bits, and
// an estimate more than one off only happens far outside that range.
__device__ __forceinline__ int quantize(int x, int pred, int xt, int* recon) {
  const int num = x - pred + xt, w = 2 * xt + 1;
  int q = (int)floorf((float)num * __builtin_amdgcn_rcpf((float)w));
  const int r = num - q * w;
  q += (r >= w ? 1 : 0) - (r < 0 ? 1 : 0);
  if (q < 1 - QR || q > QR - 1) {
    *recon = x;
    return 0;
  }
  *recon = pred + q * w;
  return q + QR;
}

// --------------------------------------------------------- incident faces
// The 36 faces around a vertex as pairs of neighbour offsets (dx, dy, dt),
// each packed as ((dx+1) | (dy+1) << 2 | (dt+1) << 4).  Built from the twelve
// face types: the lower and upper slice triangles of the main-diagonal split,
// the two inner faces of each prism, and two faces on each side quad.
struct FaceTable {
  uint8_t a[36], b[36];
  int n;
};

constexpr int FTYPE[12][3][3] = {
    {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}}, {{0, 0, 0}, {0, 1, 0}, {1, 1, 0}},
    {{0, 0, 0}, {1, 0, 0}, {1, 1, 1}}, {{0, 0, 0}, {1, 0, 1}, {1, 1, 1}},
    {{0, 0, 0}, {0, 1, 0}, {1, 1, 1}}, {{0, 0, 0}, {0, 1, 1}, {1, 1, 1}},
    {{0, 0, 0}, {1, 0, 0}, {1, 0, 1}}, {{0, 0, 0}, {0, 0, 1}, {1, 0, 1}},
    {{0, 0, 0}, {0, 1, 0}, {0, 1, 1}}, {{0, 0, 0}, {0, 0, 1}, {0, 1, 1}},
    {{0, 0, 0}, {1, 1, 0}, {1, 1, 1}}, {{0, 0, 0}, {0, 0, 1}, {1, 1, 1}},
};

constexpr uint8_t pack_off(int dx, int dy, int dt) {
  return (uint8_t)((dx + 1) | ((dy + 1) << 2) | ((dt + 1) << 4));
}

constexpr FaceTable make_face_table() {
  FaceTable T{};
  T.n = 0;
  for (int o = 0; o < 8; o++) {
    int ox = o & 1, oy = (o >> 1) & 1, ot = (o >> 2) & 1;  // vertex offset inside the face
    for (int f = 0; f < 12; f++) {
      int hit = -1;
      for (int i = 0; i < 3; i++)
        if (FTYPE[f][i][0] == ox && FTYPE[f][i][1] == oy && FTYPE[f][i][2] == ot) hit = i;
      if (hit < 0) continue;
      int j = 0;
      uint8_t p[2] = {0, 0};
      for (int i = 0; i < 3; i++)
        if (i != hit) p[j++] = pack_off(FTYPE[f][i][0] - ox, FTYPE[f][i][1] - oy, FTYPE[f][i][2] - ot);
      T.a[T.n] = p[0];
      T.b[T.n] = p[1];
      T.n++;
    }
  }
  return T;
}

__device__ __forceinline__ int off_dx(uint8_t p) { return (int)(p & 3) - 1; }
__device__ __forceinline__ int off_dy(uint8_t p) { return (int)((p >> 2) & 3) - 1; }
__device__ __forceinline__ int off_dt(uint8_t p) { return (int)((p >> 4) & 3) - 1; }

}  // namespace cpt
