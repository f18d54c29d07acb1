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

__global__ __launch_bounds__(256) void k_reconstruct(int2* __restrict__ cur, float* __restrict__ field,
                                                     const uint16_t* __restrict__ xs, const uint16_t* __restrict__ qs,
                                                     const uint32_t* __restrict__ qofs, const uint32_t* __restrict__ raw,
                                                     const uint32_t* __restrict__ rofs,
                                                     const uint8_t* __restrict__ modes, long long mode_base,
                                                     FieldParams p, int t, uint32_t* __restrict__ err) {
  __shared__ int2 C[TILE][TILE];
  __shared__ int2 P[TILE][TILE];
  const int tid = threadIdx.x, lx = tid & 15, ly = tid >> 4;
  const int bx = blockIdx.x, by = blockIdx.y;
  const int x = bx * TILE + lx, y = by * TILE + ly;
  const int H = p.H, W = p.W;
  const size_t HW = (size_t)H * W, N = HW * (size_t)p.T;
  const bool valid = x < W && y < H;
  const size_t gi = (size_t)y * W + x, gv = (size_t)t * HW + gi;
  int cls = 0;
  if (t >= 1) {
    if (p.predictor == 1) cls = 1;
    else if (mode_base >= 0) cls = modes[(size_t)mode_base + (size_t)by * p.tx + bx];
  }
  const int dmax = p.predictor == 1 ? 2 : class_dmax(p.K, cls);
  P[ly][lx] = (valid && t > 0) ? cur[gv - HW] : make_int2(0, 0);
  C[ly][lx] = make_int2(0, 0);

  // everything that does not depend on the block's own reconstruction
  int code = XLOSSLESS, qu = 0, qv = 0, xt = 0, pu = 0, pv = 0;
  uint32_t ro = 0;
  if (valid) {
    code = xs[gv];
    ro = rofs[gv];
    if (code != XLOSSLESS) {
      size_t o = 2 * (size_t)qofs[gv];
      qu = qs[o];
      qv = qs[o + 1];
      xt = p.eps >> code;
      if (cls != 0) sl_predict(cur + (size_t)(t - 1) * HW, H, W, x, y, SLConst{p.cx, p.sx, p.cy, p.sy}, dmax, &pu, &pv);
    }
  }
  auto finish = [&](int pu_, int pv_) {
    int comp_pred[2] = {pu_, pv_};
    int comp_q[2] = {qu, qv};
    int outv[2];
    uint32_t r = ro;
    for (int c = 0; c < 2; c++) {
      float f;
      int fx;
      if (code == XLOSSLESS || comp_q[c] == 0) {
        uint32_t b = raw[r++];
        f = __uint_as_float(b);
        if (((b >> 23) & 0xFFu) == 0xFFu) atomicOr(err, 64u);
        fx = to_fixed(f, p.k);
      } else {
        int64_t rv = (int64_t)comp_pred[c] + (int64_t)(comp_q[c] - QR) * (2 * (int64_t)xt + 1);
        if (rv >= (1 << 25) || rv <= -(1 << 25)) {
          atomicOr(err, 128u);
          rv = 0;
        }
        fx = (int)rv;
        f = from_fixed(fx, p.k);
      }
      outv[c] = fx;
      field[(size_t)c * N + gv] = f;
    }
    C[ly][lx] = make_int2(outv[0], outv[1]);
    cur[gv] = make_int2(outv[0], outv[1]);
  };
  __syncthreads();
  if (cls != 0) {
    if (valid) finish(pu, pv);
    return;
  }
  for (int d = 0; d < 2 * TILE - 1; d++) {
    if (valid && lx + ly == d) {
      int pr[2] = {0, 0};
      if (code != XLOSSLESS) {
        for (int c = 0; c < 2; c++) {
          auto g = [&](const int2 (*A)[TILE], int i, int j) -> int {
            if (i < 0 || j < 0) return 0;
            return c ? A[j][i].y : A[j][i].x;
          };
          pr[c] = g(C, lx - 1, ly) + g(C, lx, ly - 1) - g(C, lx - 1, ly - 1) + g(P, lx, ly) - g(P, lx - 1, ly) -
                  g(P, lx, ly - 1) + g(P, lx - 1, ly - 1);
        }
      }
      finish(pr[0], pr[1]);
    }
    __syncthreads();
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
  k_reconstruct<<<grid, 256, 0, s>>>(cur, field, xs, qs, qofs, raw, rofs, modes, mode_base, p, t, err);
}

}  // namespace cpt
