// k_decompress.hip — reconstruction of a frame from its decoded codes.
//
// Decompression inverts the prediction and quantization of the compressor:
// each vertex's value is the prediction plus its residual code times
// 2 xi~ + 1 (xi~ = eps' >> bound code), or the stored raw float when the
// vertex is lossless or the component was unpredictable.  Predictions only
// read the block's own frame (Lorenzo) or the previous frame (semi-
// Lagrangian), so every block of a frame is reconstructed independently.
#include "cpt_device.hpp"
#include "launch.hpp"
#include "predict.hpp"

namespace cpt {

__global__ __launch_bounds__(256) void k_dec_nonll(const uint16_t* __restrict__ xs, size_t N,
                                                   uint32_t* __restrict__ nonll) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) nonll[i] = xs[i] != XLOSSLESS ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_dec_counts(const uint16_t* __restrict__ xs, const uint16_t* __restrict__ qs,
                                                    const uint32_t* __restrict__ qofs, size_t N, size_t nq, int eps,
                                                    uint32_t* __restrict__ rcnt, uint32_t* __restrict__ err) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  uint32_t c = xs[i];
  uint32_t r = 0;
  if (c > XLOSSLESS) {
    atomicOr(err, 16u);
  } else if (c == XLOSSLESS) {
    r = 2;
  } else {
    size_t o = 2 * (size_t)qofs[i];
    if ((eps >> c) < 1 || o + 2 > nq) {
      atomicOr(err, 32u);
    } else {
      r = (qs[o] == 0) + (qs[o + 1] == 0);
    }
  }
  rcnt[i] = r;
}

// One wave per block: each lane prepares four vertices (v = lane + 64 k),
// lanes 0-31 then sweep the Lorenzo anti-diagonals, and each lane writes its
// four vertices.  With one wave per block every block of a frame is
// resident at once.
__device__ __forceinline__ void rc_wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__global__ __launch_bounds__(64) void k_reconstruct(int2* __restrict__ cur, float* __restrict__ field,
                                                    const uint16_t* __restrict__ xs, const uint16_t* __restrict__ qs,
                                                    const uint32_t* __restrict__ qofs, const uint32_t* __restrict__ raw,
                                                    const uint32_t* __restrict__ rofs,
                                                    const uint8_t* __restrict__ modes, long long mode_base,
                                                    FieldParams p, int t, uint32_t* __restrict__ err) {
  __shared__ int C[2][TILE][TILE];     // reconstructed fixed-point values (u, v)
  __shared__ int P[2][TILE][TILE];     // previous frame, for the Lorenzo predictor
  __shared__ int DQ[2][TILE][TILE];    // q (2 xi~ + 1) of components still to predict
  __shared__ uint8_t KN[2][TILE][TILE];  // component already known (raw or semi-Lagrangian)
  const int lane = threadIdx.x;
  const int bx = blockIdx.x, by = blockIdx.y;
  const int H = p.H, W = p.W;
  const size_t HW = (size_t)H * W, N = HW * (size_t)p.T;
  int cls = 0;
  if (t >= 1) {
    if (p.predictor == 1) cls = 1;
    else if (mode_base >= 0) cls = modes[(size_t)mode_base + (size_t)by * p.tx + bx];
  }
  const int dmax = p.predictor == 1 ? 2 : class_dmax(p.K, cls);
  int vcode[4], vq[4];
  uint32_t vr[4];
  const int x0 = bx * TILE, y0 = by * TILE;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int v = lane + 64 * k, lx = v & 15, ly = v >> 4;
    const int x = x0 + lx, y = y0 + ly;
    const bool valid = x < W && y < H;
    const size_t gv = (size_t)t * HW + (size_t)y * W + x;
    const int2 pv2 = (valid && t > 0) ? cur[gv - HW] : make_int2(0, 0);
    P[0][ly][lx] = pv2.x;
    P[1][ly][lx] = pv2.y;
  }
  rc_wave_sync();
  // frame t-1 from the staged block where it covers the sample
  const int2* prevf = t > 0 ? cur + (size_t)(t - 1) * HW : cur;
  auto F = [&](int xx, int yy) {
    const int tx_ = xx - x0, ty_ = yy - y0;
    return (tx_ >= 0 && tx_ < TILE && ty_ >= 0 && ty_ < TILE) ? make_int2(P[0][ty_][tx_], P[1][ty_][tx_])
                                                               : prevf[(size_t)yy * W + xx];
  };

  // everything that does not depend on the block's own reconstruction
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int v = lane + 64 * k, lx = v & 15, ly = v >> 4;
    const int x = x0 + lx, y = y0 + ly;
    const bool valid = x < W && y < H;
    const size_t gv = (size_t)t * HW + (size_t)y * W + x;
    vcode[k] = XLOSSLESS;
    vq[k] = 0;
    vr[k] = 0;
    if (!valid) continue;
    const int code = xs[gv];
    uint32_t r = rofs[gv];
    int q[2] = {0, 0}, pr[2] = {0, 0};
    int64_t w = 0;
    if (code != XLOSSLESS) {
      size_t o = 2 * (size_t)qofs[gv];
      q[0] = qs[o];
      q[1] = qs[o + 1];
      w = 2 * (int64_t)(p.eps >> code) + 1;
      if (cls != 0) sl_predict_f(F, H, W, x, y, SLConst{p.cx, p.sx, p.cy, p.sy}, dmax, &pr[0], &pr[1]);
    }
    vcode[k] = code;
    vq[k] = q[0] | (q[1] << 16);
    vr[k] = r;
    for (int c = 0; c < 2; c++) {
      if (code == XLOSSLESS || q[c] == 0) {
        uint32_t b = raw[r++];
        if (((b >> 23) & 0xFFu) == 0xFFu) atomicOr(err, 64u);
        C[c][ly][lx] = to_fixed(__uint_as_float(b), p.k);
        KN[c][ly][lx] = 1;
      } else {
        int64_t dq = (int64_t)(q[c] - QR) * w;
        if (cls != 0) {
          int64_t rv = (int64_t)pr[c] + dq;
          if (rv >= (1 << 25) || rv <= -(1 << 25)) {
            atomicOr(err, 128u);
            rv = 0;
          }
          C[c][ly][lx] = (int)rv;
          KN[c][ly][lx] = 1;
        } else {
          DQ[c][ly][lx] = (int)dq;
          KN[c][ly][lx] = 0;
        }
      }
    }
  }
  rc_wave_sync();

  // Lorenzo blocks: lanes 0-15 sweep the rows of u and lanes 16-31 the rows
  // of v along the anti-diagonals.  A lane keeps its last value (the left
  // neighbour of its next vertex); the row above arrives from the previous
  // lane of the same 16-lane DPP row by a row shift.  All 64 lanes step
  // together (DPP reads need active source lanes).
  if (cls == 0) {
    const int c = (lane >> 4) & 1, row = lane & 15;
    const bool mine = lane < 2 * TILE;
    const bool has_prev = t > 0;
    int last = 0, upl = 0;
    for (int d = 0; d < 2 * TILE - 1; d++) {
      const int col = d - row;
      const int up = __builtin_amdgcn_update_dpp(0, last, 0x111, 0xF, 0xF, true);  // row_shr:1
      if (mine && col >= 0 && col < TILE && bx * TILE + col < W && by * TILE + row < H) {
        if (KN[c][row][col]) {
          last = C[c][row][col];
        } else {
          int s = (col > 0 ? last : 0) + (row > 0 ? up : 0) - (col > 0 && row > 0 ? upl : 0);
          if (has_prev)
            s += P[c][row][col] - (col > 0 ? P[c][row][col - 1] : 0) - (row > 0 ? P[c][row - 1][col] : 0) +
                 (col > 0 && row > 0 ? P[c][row - 1][col - 1] : 0);
          int64_t rv = (int64_t)s + DQ[c][row][col];
          if (rv >= (1 << 25) || rv <= -(1 << 25)) {
            atomicOr(err, 128u);
            rv = 0;
          }
          last = (int)rv;
          C[c][row][col] = last;
        }
      }
      upl = up;
    }
    rc_wave_sync();
  }
  // known raw components are restored bit-exactly; the rest are exact
  // multiples of 2^-k
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int v = lane + 64 * k, lx = v & 15, ly = v >> 4;
    const int x = bx * TILE + lx, y = by * TILE + ly;
    if (!(x < W && y < H)) continue;
    const size_t gv = (size_t)t * HW + (size_t)y * W + x;
    const int u = C[0][ly][lx], vv = C[1][ly][lx];
    cur[gv] = make_int2(u, vv);
    const uint32_t r0 = vr[k];
    float fu, fv;
    if (vcode[k] == XLOSSLESS) {
      fu = __uint_as_float(raw[r0]);
      fv = __uint_as_float(raw[r0 + 1]);
    } else {
      uint32_t r = r0;
      fu = (vq[k] & 0xFFFF) == 0 ? __uint_as_float(raw[r++]) : from_fixed(u, p.k);
      fv = (vq[k] >> 16) == 0 ? __uint_as_float(raw[r]) : from_fixed(vv, p.k);
    }
    field[gv] = fu;
    field[N + gv] = fv;
  }
}

// ============================================================ launchers
static inline unsigned nblk(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void launch_dec_nonll(const uint16_t* xs, size_t N, uint32_t* nonll, hipStream_t s) {
  if (N) k_dec_nonll<<<nblk(N), 256, 0, s>>>(xs, N, nonll);
}
void launch_dec_counts(const uint16_t* xs, const uint16_t* qs, const uint32_t* qofs, size_t N, size_t nq, int eps,
                       uint32_t* rcnt, uint32_t* err, hipStream_t s) {
  if (N) k_dec_counts<<<nblk(N), 256, 0, s>>>(xs, qs, qofs, N, nq, eps, rcnt, err);
}
void launch_reconstruct(int2* cur, float* field, const uint16_t* xs, const uint16_t* qs, const uint32_t* qofs,
                        const uint32_t* raw, const uint32_t* rofs, const uint8_t* modes, long long mode_base,
                        const FieldParams& p, int t, uint32_t* err, hipStream_t s) {
  dim3 grid(p.tx, p.ty);
  k_reconstruct<<<grid, 64, 0, s>>>(cur, field, xs, qs, qofs, raw, rofs, modes, mode_base, p, t, err);
}

}  // namespace cpt
