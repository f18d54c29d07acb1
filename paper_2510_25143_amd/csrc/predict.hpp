// predict.hpp — device predictors shared by compression and decompression.
//
// Semi-Lagrangian predictor (Sec. VI-A of the paper) in Q16 cell units: the
// displacement of a fixed-point velocity u is floor(u c / 2^s), with c/2^s
// approximating dt/dx 2^(16-k); the departure point is traced back from the
// grid point with one RK2 midpoint step when the displacement estimate is at
// most d_max cells, else with N = min(ceil(d_inf/d_max), 32) Euler substeps,
// clamping to the domain after each step; the prediction is the bilinear
// sample (rounded half up) of the previous reconstructed frame there.
#pragma once
#include "cpt_device.hpp"

namespace cpt {

struct SLConst {
  int64_t cx, sx, cy, sy;
};

__device__ __forceinline__ int64_t sl_disp(int64_t u, int64_t c, int64_t s) {
  return (u * c) >> s;  // arithmetic shift = floor
}

__device__ __forceinline__ int64_t clamp64(int64_t a, int64_t lo, int64_t hi) {
  return a < lo ? lo : (a > hi ? hi : a);
}

// Bilinear sample of both components of the previous frame at Q16 (px, py)
// inside the domain; F(x, y) returns its int2 value at a grid point.
template <typename Fetch>
__device__ __forceinline__ void bilinear2f(const Fetch& F, int H, int W, int64_t px, int64_t py, int64_t* ou,
                                           int64_t* ov) {
  int x0 = (int)(px >> 16), y0 = (int)(py >> 16);
  int64_t fx = px & 65535, fy = py & 65535;
  int x1 = x0 + 1 < W ? x0 + 1 : x0, y1 = y0 + 1 < H ? y0 + 1 : y0;
  int2 a = F(x0, y0), b = F(x1, y0);
  int2 c = F(x0, y1), d = F(x1, y1);
  int64_t gx = 65536 - fx, gy = 65536 - fy;
  int64_t r0u = (int64_t)a.x * gx + (int64_t)b.x * fx, r1u = (int64_t)c.x * gx + (int64_t)d.x * fx;
  int64_t r0v = (int64_t)a.y * gx + (int64_t)b.y * fx, r1v = (int64_t)c.y * gx + (int64_t)d.y * fx;
  *ou = (r0u * gy + r1u * fy + (1LL << 31)) >> 32;
  *ov = (r0v * gy + r1v * fy + (1LL << 31)) >> 32;
}

// g is the previous frame's value at the grid point (x, y) itself
template <typename Fetch>
__device__ __forceinline__ void sl_predict_g(const Fetch& F, int H, int W, int x, int y, int2 g, const SLConst& k,
                                             int dmax, int* pu, int* pv) {
  const int64_t XM = (int64_t)(W - 1) << 16, YM = (int64_t)(H - 1) << 16;
  const int64_t px = (int64_t)x << 16, py = (int64_t)y << 16;
  int64_t dx = sl_disp(g.x, k.cx, k.sx), dy = sl_disp(g.y, k.cy, k.sy);
  int64_t ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
  int64_t dinf = ax > ay ? ax : ay;
  int64_t lim = (int64_t)dmax << 16;
  int64_t qx, qy;
  if (dinf <= lim) {
    int64_t hx = clamp64(px - (dx >> 1), 0, XM), hy = clamp64(py - (dy >> 1), 0, YM);
    int64_t uh, vh;
    bilinear2f(F, H, W, hx, hy, &uh, &vh);
    qx = clamp64(px - sl_disp(uh, k.cx, k.sx), 0, XM);
    qy = clamp64(py - sl_disp(vh, k.cy, k.sy), 0, YM);
  } else {
    int n = 1;
    while (n < NMAX && (int64_t)n * lim < dinf) n++;
    qx = px;
    qy = py;
    for (int s = 0; s < n; s++) {
      int64_t us, vs;
      bilinear2f(F, H, W, qx, qy, &us, &vs);
      int64_t nx = qx - floor_div64(sl_disp(us, k.cx, k.sx), n);
      int64_t ny = qy - floor_div64(sl_disp(vs, k.cy, k.sy), n);
      qx = clamp64(nx, 0, XM);
      qy = clamp64(ny, 0, YM);
    }
  }
  int64_t ru, rv;
  bilinear2f(F, H, W, qx, qy, &ru, &rv);
  *pu = (int)ru;
  *pv = (int)rv;
}

template <typename Fetch>
__device__ __forceinline__ void sl_predict_f(const Fetch& F, int H, int W, int x, int y, const SLConst& k, int dmax,
                                             int* pu, int* pv) {
  sl_predict_g(F, H, W, x, y, F(x, y), k, dmax, pu, pv);
}

// the same reading every sample from the previous frame in global memory
__device__ __forceinline__ void sl_predict(const int2* __restrict__ prev, int H, int W, int x, int y,
                                           const SLConst& k, int dmax, int* pu, int* pv) {
  auto F = [&](int xx, int yy) { return prev[(size_t)yy * W + xx]; };
  sl_predict_f(F, H, W, x, y, k, dmax, pu, pv);
}

// Class table: 0 = 3-D Lorenzo; otherwise semi-Lagrangian with d_max cells.
__device__ __forceinline__ int class_dmax(int K, int cls) {
  if (cls == 0) return 0;
  if (K == 4) return cls == 1 ? 1 : (cls == 2 ? 2 : 4);
  return 2;
}

}  // namespace cpt
