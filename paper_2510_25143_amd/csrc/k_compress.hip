// k_compress.hip — the compression hot loop: per-block predictor choice and
// the per-vertex bound, prediction, quantization and write-back.
//
// Order (reproducible by construction): for every frame t, three colour
// phases; phase c processes every 16x16 block with (bx + by) mod 3 == c.
// Blocks of one colour share no face, so they run as independent
// workgroups.  Inside a block the vertices are taken in raster order; with
// the main-diagonal triangulation the raster predecessors of a vertex are
// exactly its neighbours on earlier anti-diagonals, so the workgroup sweeps
// the 31 anti-diagonals and processes each one in parallel.
//
// Per vertex (Alg. 3 and Alg. 4 of the paper): a vertex on a crossed face of
// the original field is stored losslessly; otherwise its bound is the
// minimum of eps' and the Alg. 2 bound of each of its (up to 36) faces,
// evaluated on the current values — reconstructed where already processed,
// original elsewhere.  22 of the 36 faces never touch a vertex of the same
// block processed before it; their bounds are computed for the whole block
// in parallel first.  The other 14 are computed during the sweep, one face
// per lane, sixteen lanes per vertex.
#include "cpt_device.hpp"
#include "launch.hpp"
#include "predict.hpp"

namespace cpt {

__constant__ FaceTable c_ft = make_face_table();

struct DynList {
  uint8_t idx[14];
  int n;
};
constexpr DynList make_dyn() {
  DynList D{};
  D.n = 0;
  FaceTable T = make_face_table();
  const uint8_t p1 = pack_off(-1, 0, 0), p2 = pack_off(0, -1, 0), p3 = pack_off(-1, -1, 0);
  for (int f = 0; f < T.n; f++) {
    uint8_t a = T.a[f], b = T.b[f];
    if (a == p1 || a == p2 || a == p3 || b == p1 || b == p2 || b == p3) D.idx[D.n++] = (uint8_t)f;
  }
  return D;
}
__constant__ DynList c_dyn = make_dyn();
static_assert(make_face_table().n == 36, "36 incident faces per interior vertex");
static_assert(make_dyn().n == 14, "14 faces meet a raster predecessor in the block");

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

template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* sh, Op op) {
  int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = op(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------ mode choice
// One workgroup per block of a decision frame.  Exhaustive trial: each
// candidate is micro-encoded over the block with the global bound eps'
// (Sec. VI-B): Lorenzo writes its reconstruction back to a candidate buffer
// (anti-diagonal sweep), semi-Lagrangian reads only the previous frame.  The
// rate score of each candidate uses the codes on the stride-2 subgrid.
__global__ __launch_bounds__(256) void k_modes(const int2* __restrict__ cur, const uint8_t* __restrict__ flags,
                                               FieldParams p, int t, size_t group_base,
                                               const int64_t* __restrict__ tlog,
                                               const uint16_t* __restrict__ selw, uint8_t* __restrict__ modes,
                                               float* __restrict__ feats) {
  __shared__ int2 C[TILE][TILE];
  __shared__ int2 P[TILE][TILE];
  __shared__ uint32_t hist[QSYM];
  __shared__ int64_t red[256];
  __shared__ int64_t R[4];
  __shared__ int sn, sL;
  __shared__ float fin[10];
  __shared__ float h1[64], h2[64], lg[4];

  const int tid = threadIdx.x, lx = tid & 15, ly = tid >> 4;
  const int bx = blockIdx.x, by = blockIdx.y;
  const int x0 = bx * TILE, y0 = by * TILE, x = x0 + lx, y = y0 + ly;
  const int H = p.H, W = p.W;
  const size_t HW = (size_t)H * W;
  const bool valid = x < W && y < H;
  const size_t gi = (size_t)y * W + x;
  const int2* cf = cur + (size_t)t * HW;
  const int2* pf = cur + (size_t)(t - 1) * HW;
  const int2 X = valid ? cf[gi] : make_int2(0, 0);
  const int2 Pv = valid ? pf[gi] : make_int2(0, 0);
  C[ly][lx] = X;
  P[ly][lx] = Pv;
  const SLConst slc{p.cx, p.sx, p.cy, p.sy};
  const int eps = p.eps;
  __syncthreads();

  // ---------------- block features (also the selector's input)
  int cls_learned = -1;
  if (feats != nullptr || p.predictor == 4) {
    int64_t s = eps > 1 ? eps : 1;
    int64_t S0 = 0, S1 = 0, S2 = 0, Dm = 0, Ds = 0, Sx = 0, Sy = 0, nf = 0, S6 = 0, S7 = 0, n = 0, m = 0;
    if (valid) {
      n = 1;
      S0 = (int64_t)iabs(X.x - Pv.x) + iabs(X.y - Pv.y);
      int lu = lorenzo_local(C, P, lx, ly, true, 0), lv = lorenzo_local(C, P, lx, ly, true, 1);
      int64_t r3 = (int64_t)iabs(X.x - lu) + iabs(X.y - lv);
      S1 = r3;
      if (lx + 1 < TILE && x + 1 < W) S2 += (int64_t)iabs(C[ly][lx + 1].x - X.x) + iabs(C[ly][lx + 1].y - X.y);
      if (ly + 1 < TILE && y + 1 < H) S2 += (int64_t)iabs(C[ly + 1][lx].x - X.x) + iabs(C[ly + 1][lx].y - X.y);
      const int64_t DCAP = (int64_t)1 << 40;
      int64_t dx = clamp64(sl_disp(Pv.x, p.cx, p.sx), -DCAP, DCAP);
      int64_t dy = clamp64(sl_disp(Pv.y, p.cy, p.sy), -DCAP, DCAP);
      int64_t ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
      int64_t d = ax > ay ? ax : ay;
      Dm = d;
      Ds = d;
      Sx = dx;
      Sy = dy;
      nf = flags[(size_t)t * HW + gi] ? 1 : 0;
      if ((lx & 3) == 0 && (ly & 3) == 0) {
        int pu, pv;
        sl_predict(pf, H, W, x, y, slc, 2, &pu, &pv);
        S6 = (int64_t)iabs(X.x - pu) + iabs(X.y - pv);
        S7 = r3;
        m = 1;
      }
    }
    auto add = [](int64_t a, int64_t b) { return a + b; };
    auto mx = [](int64_t a, int64_t b) { return a > b ? a : b; };
    S0 = block_reduce(S0, red, add);
    S1 = block_reduce(S1, red, add);
    S2 = block_reduce(S2, red, add);
    Dm = block_reduce(Dm, red, mx);
    Ds = block_reduce(Ds, red, add);
    Sx = block_reduce(Sx, red, add);
    Sy = block_reduce(Sy, red, add);
    nf = block_reduce(nf, red, add);
    S6 = block_reduce(S6, red, add);
    S7 = block_reduce(S7, red, add);
    n = block_reduce(n, red, add);
    m = block_reduce(m, red, add);
    if (tid == 0) {
      int64_t q[10] = {featq_num(S0, 2 * n * s), featq_num(S1, 2 * n * s), featq_num(S2, 2 * n * s),
                       featq_num(Dm, 65536),     featq_num(Ds, n * 65536),  featq_num(nf, n),
                       featq_num(S6, 2 * m * s), featq_num(S7, 2 * m * s),  featq_num(Sx, n * 65536),
                       featq_num(Sy, n * 65536)};
      for (int i = 0; i < 10; i++) fin[i] = (float)q[i] / 256.0f;
    }
    __syncthreads();
    size_t bi = group_base + (size_t)by * p.tx + bx;
    if (feats != nullptr && tid < 10) feats[bi * 10 + tid] = fin[tid];
    if (p.predictor == 4) {
      // 10-64-64-4 MLP, bf16 weights, fp32 fused multiply-add in input order
      if (tid < 64) {
        float a = bf16f(selw[640 + tid]);
        for (int i = 0; i < 10; i++) a = fmaf(bf16f(selw[tid * 10 + i]), fin[i], a);
        h1[tid] = a > 0.0f ? a : 0.0f;
      }
      __syncthreads();
      if (tid < 64) {
        float a = bf16f(selw[4800 + tid]);
        for (int i = 0; i < 64; i++) a = fmaf(bf16f(selw[704 + tid * 64 + i]), h1[i], a);
        h2[tid] = a > 0.0f ? a : 0.0f;
      }
      __syncthreads();
      if (tid < 4) {
        float a = bf16f(selw[5120 + tid]);
        for (int i = 0; i < 64; i++) a = fmaf(bf16f(selw[4864 + tid * 64 + i]), h2[i], a);
        lg[tid] = a;
      }
      __syncthreads();
      int best = 0;
      for (int c = 1; c < 4; c++)
        if (lg[c] > lg[best]) best = c;
      cls_learned = best;
    }
  }
  if (p.predictor == 4) {
    if (tid == 0) modes[group_base + (size_t)by * p.tx + bx] = (uint8_t)cls_learned;
    return;
  }

  // ---------------- exhaustive trial over the K candidates
  for (int cls = 0; cls < p.K; cls++) {
    for (int b = tid; b < QSYM; b += 256) hist[b] = 0;
    if (tid == 0) {
      sn = 0;
      sL = 0;
    }
    C[ly][lx] = X;
    __syncthreads();
    int qu = 0, qv = 0;
    if (cls == 0) {
      for (int d = 0; d < 2 * TILE - 1; d++) {
        if (valid && lx + ly == d) {
          int pu = lorenzo_local(C, P, lx, ly, true, 0), pv = lorenzo_local(C, P, lx, ly, true, 1);
          int ru, rv;
          qu = quantize(X.x, pu, eps, &ru);
          qv = quantize(X.y, pv, eps, &rv);
          C[ly][lx] = make_int2(ru, rv);
        }
        __syncthreads();
      }
    } else if (valid) {
      int pu, pv, ru, rv;
      sl_predict(pf, H, W, x, y, slc, class_dmax(p.K, cls), &pu, &pv);
      qu = quantize(X.x, pu, eps, &ru);
      qv = quantize(X.y, pv, eps, &rv);
    }
    if (valid && (lx & 1) == 0 && (ly & 1) == 0) {
      if (qu == 0) atomicAdd(&sL, 1);
      else {
        atomicAdd(&hist[qu], 1u);
        atomicAdd(&sn, 1);
      }
      if (qv == 0) atomicAdd(&sL, 1);
      else {
        atomicAdd(&hist[qv], 1u);
        atomicAdd(&sn, 1);
      }
    }
    __syncthreads();
    int64_t ts = 0;
    for (int b = tid; b < QSYM; b += 256) ts += tlog[hist[b]];
    ts = block_reduce(ts, red, [](int64_t a, int64_t b) { return a + b; });
    if (tid == 0) {
      int64_t n = sn, L = sL;
      int64_t h0 = n > 0 ? floor_div64(tlog[n] - ts, n) : 0;
      int64_t pen = (n + L) > 0 ? floor_div64((int64_t)16 * 65536 * L, n + L) : 0;
      int64_t lgK = p.K == 4 ? 2 : 1;
      int64_t meta = floor_div64(65536 * lgK, (int64_t)512 * p.bt);
      R[cls] = h0 + pen + meta;
    }
    __syncthreads();
  }
  if (tid == 0) {
    int best = 1;
    for (int c = 2; c < p.K; c++)
      if (R[c] < R[best]) best = c;
    int cls = 1000 * (R[0] - R[best]) > 3 * R[0] ? best : 0;
    modes[group_base + (size_t)by * p.tx + bx] = (uint8_t)cls;
  }
}

// --------------------------------------------------------------- the phase
__global__ __launch_bounds__(256) void k_phase(int2* __restrict__ cur, const uint8_t* __restrict__ flags,
                                               const uint8_t* __restrict__ modes, long long mode_base,
                                               FieldParams p, int t, int colour, uint8_t* __restrict__ xcode,
                                               uint32_t* __restrict__ qcode, int32_t* __restrict__ xi_dbg) {
  __shared__ int2 V[3][HALO][HALO];  // frames t-1, t, t+1 around the block
  __shared__ int XS[TILE][TILE];     // bound from the faces fixed for the whole sweep
  __shared__ int2 SLP[TILE][TILE];   // semi-Lagrangian predictions
  const int tid = threadIdx.x;
  const int by = blockIdx.y;
  const int b0 = ((colour - by) % 3 + 3) % 3;
  const int bx = b0 + 3 * (int)blockIdx.x;
  if (bx >= p.tx) return;
  const int H = p.H, W = p.W, T = p.T;
  const size_t HW = (size_t)H * W;
  const int x0 = bx * TILE, y0 = by * TILE;
  const int eps = p.eps;

  // ---- stage frames t-1, t, t+1 (block plus halo); the two corner cells
  // that belong to blocks of the same colour are never read and not loaded
  for (int i = tid; i < 3 * HALO * HALO; i += 256) {
    int f = i / (HALO * HALO), r = i - f * HALO * HALO;
    int hy = r / HALO, hx = r - hy * HALO;
    int gx = x0 - 1 + hx, gy = y0 - 1 + hy, tt = t - 1 + f;
    int2 v = make_int2(0, 0);
    bool corner = (hx == HALO - 1 && hy == 0) || (hx == 0 && hy == HALO - 1);
    if (!corner && gx >= 0 && gx < W && gy >= 0 && gy < H && tt >= 0 && tt < T)
      v = cur[(size_t)tt * HW + (size_t)gy * W + gx];
    V[f][hy][hx] = v;
  }
  int cls = 0;
  if (t >= 1) {
    if (p.predictor == 1) cls = 1;
    else if (mode_base >= 0) cls = modes[(size_t)mode_base + (size_t)by * p.tx + bx];
  }
  const int dmax = p.predictor == 1 ? 2 : class_dmax(p.K, cls);
  __syncthreads();

  // ---- faces whose other vertices stay fixed during the sweep
  {
    const int lx = tid & 15, ly = tid >> 4, x = x0 + lx, y = y0 + ly;
    int xi = 0;
    if (x < W && y < H) {
      const size_t gv = (size_t)t * HW + (size_t)y * W + x;
      if (!flags[gv]) {
        xi = eps;
        const int2 me = V[1][ly + 1][lx + 1];
        for (int f = 0; f < 36 && xi > 0; f++) {
          uint8_t a = c_ft.a[f], b = c_ft.b[f];
          int ax = off_dx(a), ay = off_dy(a), at = off_dt(a);
          int bxo = off_dx(b), byo = off_dy(b), bto = off_dt(b);
          if (x + ax < 0 || x + ax >= W || y + ay < 0 || y + ay >= H || t + at < 0 || t + at >= T) continue;
          if (x + bxo < 0 || x + bxo >= W || y + byo < 0 || y + byo >= H || t + bto < 0 || t + bto >= T) continue;
          bool da = at == 0 && ((ax == -1 && ay == 0 && lx > 0) || (ax == 0 && ay == -1 && ly > 0) ||
                                (ax == -1 && ay == -1 && lx > 0 && ly > 0));
          bool db = bto == 0 && ((bxo == -1 && byo == 0 && lx > 0) || (bxo == 0 && byo == -1 && ly > 0) ||
                                 (bxo == -1 && byo == -1 && lx > 0 && ly > 0));
          if (da || db) continue;
          int2 pa = V[1 + at][ly + 1 + ay][lx + 1 + ax];
          int2 pb = V[1 + bto][ly + 1 + byo][lx + 1 + bxo];
          xi = min(xi, face_bound(pa.x, pa.y, pb.x, pb.y, me.x, me.y, eps));
        }
      }
      if (cls != 0) {
        int pu, pv;
        sl_predict(cur + (size_t)(t - 1) * HW, H, W, x, y, SLConst{p.cx, p.sx, p.cy, p.sy}, dmax, &pu, &pv);
        SLP[ly][lx] = make_int2(pu, pv);
      }
    }
    XS[ly][lx] = xi;
  }
  __syncthreads();

  // ---- anti-diagonal sweep: row g of the block, dynamic face j
  const int g = tid >> 4, j = tid & 15;
  const int y = y0 + g;
  for (int d = 0; d < 2 * TILE - 1; d++) {
    const int lx = d - g, x = x0 + lx;
    const bool active = lx >= 0 && lx < TILE && x < W && y < H;
    int e = eps;
    size_t gv = 0;
    bool lossless = true;
    if (active) {
      gv = (size_t)t * HW + (size_t)y * W + x;
      lossless = flags[gv] != 0;
      if (!lossless && j < 14) {
        const int f = c_dyn.idx[j];
        uint8_t a = c_ft.a[f], b = c_ft.b[f];
        int ax = off_dx(a), ay = off_dy(a), at = off_dt(a);
        int bxo = off_dx(b), byo = off_dy(b), bto = off_dt(b);
        bool ok = !(x + ax < 0 || x + ax >= W || y + ay < 0 || y + ay >= H || t + at < 0 || t + at >= T) &&
                  !(x + bxo < 0 || x + bxo >= W || y + byo < 0 || y + byo >= H || t + bto < 0 || t + bto >= T);
        bool da = at == 0 && ((ax == -1 && ay == 0 && lx > 0) || (ax == 0 && ay == -1 && g > 0) ||
                              (ax == -1 && ay == -1 && lx > 0 && g > 0));
        bool db = bto == 0 && ((bxo == -1 && byo == 0 && lx > 0) || (bxo == 0 && byo == -1 && g > 0) ||
                               (bxo == -1 && byo == -1 && lx > 0 && g > 0));
        if (ok && (da || db)) {
          int2 me = V[1][g + 1][lx + 1];
          int2 pa = V[1 + at][g + 1 + ay][lx + 1 + ax];
          int2 pb = V[1 + bto][g + 1 + byo][lx + 1 + bxo];
          e = face_bound(pa.x, pa.y, pb.x, pb.y, me.x, me.y, eps);
        }
      }
    }
    e = min(e, __shfl_xor(e, 8, 16));
    e = min(e, __shfl_xor(e, 4, 16));
    e = min(e, __shfl_xor(e, 2, 16));
    e = min(e, __shfl_xor(e, 1, 16));
    if (active && j == 0) {
      int xi = lossless ? 0 : min(XS[g][lx], e);
      int code = xi_code(eps, xi);
      uint32_t qc = 0;
      if (code != XLOSSLESS) {
        int xt = eps >> code;
        int pu, pv;
        if (cls == 0) {
          pu = 0;
          pv = 0;
          // tile-local 3-D Lorenzo on the staged frames
          auto val = [&](int f, int i, int jj, int comp) -> int {
            if (i < 0 || jj < 0) return 0;
            int2 q = V[f][jj + 1][i + 1];
            return comp ? q.y : q.x;
          };
          for (int comp = 0; comp < 2; comp++) {
            int s = val(1, lx - 1, g, comp) + val(1, lx, g - 1, comp) - val(1, lx - 1, g - 1, comp);
            if (t > 0) s += val(0, lx, g, comp) - val(0, lx - 1, g, comp) - val(0, lx, g - 1, comp) +
                            val(0, lx - 1, g - 1, comp);
            if (comp) pv = s; else pu = s;
          }
        } else {
          pu = SLP[g][lx].x;
          pv = SLP[g][lx].y;
        }
        int2 me = V[1][g + 1][lx + 1];
        int ru, rv;
        int cu = quantize(me.x, pu, xt, &ru);
        int cvv = quantize(me.y, pv, xt, &rv);
        qc = (uint32_t)cu | ((uint32_t)cvv << 16);
        V[1][g + 1][lx + 1] = make_int2(ru, rv);
        cur[gv] = make_int2(ru, rv);
      }
      xcode[gv] = (uint8_t)code;
      qcode[gv] = qc;
      if (xi_dbg) xi_dbg[gv] = xi;
    }
    __syncthreads();
  }
}

// ============================================================ launchers
void launch_modes(const int2* cur, const uint8_t* flags, const FieldParams& p, int t, size_t group_base,
                  const int64_t* tlog, const uint16_t* selw, uint8_t* modes, float* feats, hipStream_t s) {
  dim3 grid(p.tx, p.ty);
  k_modes<<<grid, 256, 0, s>>>(cur, flags, p, t, group_base, tlog, selw, modes, feats);
}

void launch_phase(int2* cur, const uint8_t* flags, const uint8_t* modes, long long mode_base,
                  const FieldParams& p, int t, int colour, uint8_t* xcode, uint32_t* qcode, int32_t* xi_dbg,
                  hipStream_t s) {
  dim3 grid((p.tx + 2) / 3, p.ty);
  k_phase<<<grid, 256, 0, s>>>(cur, flags, modes, mode_base, p, t, colour, xcode, qcode, xi_dbg);
}

}  // namespace cpt
