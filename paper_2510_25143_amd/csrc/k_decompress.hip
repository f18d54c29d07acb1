// k_decompress.hip — reconstruction of a frame from its decoded codes.
//
// Decompression inverts the prediction and quantization of the compressor:
// each vertex's value is the prediction plus its residual code times
// 2 xi~ + 1 (xi~ = eps' >> bound code), or the stored raw float when the
// vertex is lossless or the component was unpredictable.  Predictions only
// read the block's own frame (Lorenzo) or the previous frame (semi-
// Lagrangian), so every block of a frame is reconstructed independently.
#include "batch.hpp"
#include "cpt_device.hpp"
#include "launch.hpp"
#include "predict.hpp"

namespace cpt {

// One wave per block: each lane prepares four vertices (v = lane + 64 k),
// lanes 0-31 then sweep the Lorenzo anti-diagonals, and each lane writes its
// four vertices.  With one wave per block every block of a frame is
// resident at once.  Streams that failed a check are skipped.
__device__ __forceinline__ void rc_wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__global__ __launch_bounds__(64) void k_reconstruct_b(DecDesc* __restrict__ D, const int* __restrict__ ord,
                                                      const long long* __restrict__ pre, int m, int t,
                                                      const long long* __restrict__ mtab, DecodeBufs B) {
  __shared__ int C[2][TILE][TILE];     // reconstructed fixed-point values (u, v)
  __shared__ int P[2][TILE][TILE];     // previous frame, for the Lorenzo predictor
  __shared__ int DQ[2][TILE][TILE];    // q (2 xi~ + 1) of components still to predict
  __shared__ uint8_t KN[2][TILE][TILE];  // component already known (raw or semi-Lagrangian)
  const int j = find_field(pre, m, blockIdx.x);
  DecDesc& d = D[ord[j]];
  if (d.status) return;
  const FieldParams p = d.p;
  const int lane = threadIdx.x;
  const long long li = (long long)blockIdx.x - pre[j];
  const int by = (int)(li / p.tx), bx = (int)(li - (long long)by * p.tx);
  const int H = p.H, W = p.W;
  const size_t HW = (size_t)H * W, N = HW * (size_t)p.T;
  int2* cur = B.cur + d.voff;
  float* field = d.out;
  const uint16_t* xs = B.xs + d.voff;
  const uint16_t* qs = B.qs + d.qsb;
  const uint32_t* qofs = B.qofs + d.voff;
  const uint32_t* rofs = B.rofs + d.voff;
  const uint32_t qbase = qofs[0], rbase = rofs[0];
  const uint32_t* raw = d.sec[7];
  uint32_t* err = &d.err;
  const long long mode_base = mtab[d.mtb + t];
  int cls = 0;
  if (t >= 1) {
    if (p.predictor == 1) cls = 1;
    else if (mode_base >= 0) cls = B.modes[d.mbase + mode_base + (long long)by * p.tx + bx];
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
    uint32_t r = rofs[gv] - rbase;
    int q[2] = {0, 0}, pr[2] = {0, 0};
    int64_t w = 0;
    if (code != XLOSSLESS) {
      size_t o = 2 * (size_t)(qofs[gv] - qbase);
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
    for (int dd = 0; dd < 2 * TILE - 1; dd++) {
      const int col = dd - row;
      const int up = __builtin_amdgcn_update_dpp(0, last, 0x111, 0xF, 0xF, true);  // row_shr:1
      if (mine && col >= 0 && col < TILE && x0 + col < W && y0 + row < H) {
        if (KN[c][row][col]) {
          last = C[c][row][col];
        } else {
          int sm = (col > 0 ? last : 0) + (row > 0 ? up : 0) - (col > 0 && row > 0 ? upl : 0);
          if (has_prev)
            sm += P[c][row][col] - (col > 0 ? P[c][row][col - 1] : 0) - (row > 0 ? P[c][row - 1][col] : 0) +
                  (col > 0 && row > 0 ? P[c][row - 1][col - 1] : 0);
          int64_t rv = (int64_t)sm + DQ[c][row][col];
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
    const int x = x0 + lx, y = y0 + ly;
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
void launch_reconstruct_b(DecDesc* D, const int* ord, const long long* pre, int m, long long nblocks, int t,
                          const long long* mtab, const DecodeBufs& B, hipStream_t s) {
  if (nblocks > 0) k_reconstruct_b<<<(unsigned)nblocks, 64, 0, s>>>(D, ord, pre, m, t, mtab, B);
}

}  // namespace cpt
