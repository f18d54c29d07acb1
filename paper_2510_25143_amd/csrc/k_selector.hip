// k_selector.hip — training kernels of the learned predictor selector: a
// 10-64-64-4 ReLU network whose bf16 weights pick, per block, Lorenzo or
// semi-Lagrangian with d_max in {1, 2, 4} cells.  Inference runs inside the
// mode kernel (fp32 fused multiply-add in input order, bit-exact).
//
// Training: mean softmax cross-entropy over a minibatch.  The forward pass
// uses the fp32 master weights rounded to bf16 (what inference will see);
// activations and gradients are fp32.  Each workgroup of 64 threads (one per
// hidden unit) streams its share of the minibatch in a fixed order and keeps
// its partial gradient in registers; a second kernel sums the partials in
// workgroup order, so the result does not depend on scheduling.  Adam
// updates the master weights and refreshes the bf16 copy.
#include "cpt_device.hpp"
#include "launch.hpp"

namespace cpt {

constexpr int NF = 10, NH = 64, NC = 4;
constexpr int OW1 = 0, OB1 = 640, OW2 = 704, OB2 = 4800, OW3 = 4864, OB3 = 5120, NWT = 5124;

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(b);
}

// partial gradients of one workgroup over samples [lo, hi) of the index list
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ feats,
                                                 const int32_t* __restrict__ labels, const int32_t* __restrict__ idx,
                                                 int nbatch, int per_block, float inv_n, float* __restrict__ part,
                                                 float* __restrict__ loss_part) {
  __shared__ float W2s[NH][NH + 1];
  __shared__ float W3s[NC][NH];
  __shared__ float x[NF], h1[NH], h2[NH], g2[NH], g3[NC], lgt[NC];
  const int j = threadIdx.x;
  // bf16-rounded weights of this thread's unit
  float w1[NF];
  for (int i = 0; i < NF; i++) w1[i] = bf16_round(w[OW1 + j * NF + i]);
  const float b1 = bf16_round(w[OB1 + j]);
  const float b2 = bf16_round(w[OB2 + j]);
  for (int i = 0; i < NH; i++) W2s[j][i] = bf16_round(w[OW2 + j * NH + i]);
  for (int c = 0; c < NC; c++) W3s[c][j] = bf16_round(w[OW3 + c * NH + j]);
  const float b3 = j < NC ? bf16_round(w[OB3 + j]) : 0.0f;
  float gw1[NF], gb1 = 0.f, gw2[NH], gb2 = 0.f, gw3[NC], gb3 = 0.f;
  for (int i = 0; i < NF; i++) gw1[i] = 0.f;
  for (int i = 0; i < NH; i++) gw2[i] = 0.f;
  for (int c = 0; c < NC; c++) gw3[c] = 0.f;
  float lsum = 0.f;
  __syncthreads();
  const int lo = blockIdx.x * per_block, hi = min(lo + per_block, nbatch);
  for (int s = lo; s < hi; s++) {
    const int si = idx[s];
    if (j < NF) x[j] = feats[(size_t)si * NF + j];
    __syncthreads();
    float z1 = b1;
    for (int i = 0; i < NF; i++) z1 = fmaf(w1[i], x[i], z1);
    h1[j] = z1 > 0.f ? z1 : 0.f;
    __syncthreads();
    float z2 = b2;
    for (int i = 0; i < NH; i++) z2 = fmaf(W2s[j][i], h1[i], z2);
    h2[j] = z2 > 0.f ? z2 : 0.f;
    __syncthreads();
    if (j < NC) {
      float z3 = b3;
      for (int i = 0; i < NH; i++) z3 = fmaf(W3s[j][i], h2[i], z3);
      lgt[j] = z3;
    }
    __syncthreads();
    if (j == 0) {
      const int y = labels[si];
      float m = fmaxf(fmaxf(lgt[0], lgt[1]), fmaxf(lgt[2], lgt[3]));
      float e[NC], se = 0.f;
      for (int c = 0; c < NC; c++) {
        e[c] = expf(lgt[c] - m);
        se += e[c];
      }
      lsum += -(lgt[y] - m - logf(se));
      for (int c = 0; c < NC; c++) g3[c] = (e[c] / se - (c == y ? 1.f : 0.f)) * inv_n;
    }
    __syncthreads();
    // output layer
    for (int c = 0; c < NC; c++) gw3[c] = fmaf(g3[c], h2[j], gw3[c]);
    if (j < NC) gb3 += g3[j];
    float a = 0.f;
    for (int c = 0; c < NC; c++) a = fmaf(g3[c], W3s[c][j], a);
    const float gz2 = z2 > 0.f ? a : 0.f;
    g2[j] = gz2;
    gb2 += gz2;
    for (int i = 0; i < NH; i++) gw2[i] = fmaf(gz2, h1[i], gw2[i]);
    __syncthreads();
    float b = 0.f;
    for (int k = 0; k < NH; k++) b = fmaf(g2[k], W2s[k][j], b);
    const float gz1 = z1 > 0.f ? b : 0.f;
    gb1 += gz1;
    for (int i = 0; i < NF; i++) gw1[i] = fmaf(gz1, x[i], gw1[i]);
    __syncthreads();
  }
  float* P = part + (size_t)blockIdx.x * NWT;
  for (int i = 0; i < NF; i++) P[OW1 + j * NF + i] = gw1[i];
  P[OB1 + j] = gb1;
  for (int i = 0; i < NH; i++) P[OW2 + j * NH + i] = gw2[i];
  P[OB2 + j] = gb2;
  for (int c = 0; c < NC; c++) P[OW3 + c * NH + j] = gw3[c];
  if (j < NC) P[OB3 + j] = gb3;
  if (j == 0) loss_part[blockIdx.x] = lsum * inv_n;
}

// sum of the partials in workgroup order
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int nparts,
                                                    const float* __restrict__ loss_part, float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < NWT) {
    float s = 0.f;
    for (int b = 0; b < nparts; b++) s += part[(size_t)b * NWT + i];
    grad[i] = s;
  }
  if (i == 0) {
    float l = 0.f;
    for (int b = 0; b < nparts; b++) l += loss_part[b];
    *loss = l;
  }
}

// Adam step on the master weights; refreshes the bf16 copy
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, float lr, float b1, float b2, float eps,
                                              float c1, float c2, uint16_t* __restrict__ wbf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NWT) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wbf[i] = (uint16_t)(__float_as_uint(bf16_round(wi)) >> 16);
}

__global__ __launch_bounds__(256) void k_perm(int32_t* __restrict__ idx, int n, long long a, long long c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) idx[i] = (int32_t)(((long long)i * a + c) % n);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wbf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < NWT) wbf[i] = (uint16_t)(__float_as_uint(bf16_round(w[i])) >> 16);
}

// ============================================================ launchers
int selector_parts(int nbatch, int per_block) { return (nbatch + per_block - 1) / per_block; }

void launch_mlp_grad(const float* w, const float* feats, const int32_t* labels, const int32_t* idx, int nbatch,
                     int per_block, float inv_n, float* part, float* loss_part, float* grad, float* loss,
                     hipStream_t s) {
  const int nparts = selector_parts(nbatch, per_block);
  k_mlp_grad<<<nparts, 64, 0, s>>>(w, feats, labels, idx, nbatch, per_block, inv_n, part, loss_part);
  k_mlp_reduce<<<(NWT + 255) / 256, 256, 0, s>>>(part, nparts, loss_part, grad, loss);
}

void launch_adam(float* w, float* m, float* v, const float* g, float lr, float b1, float b2, float eps, float c1,
                 float c2, uint16_t* wbf, hipStream_t s) {
  k_adam<<<(NWT + 255) / 256, 256, 0, s>>>(w, m, v, g, lr, b1, b2, eps, c1, c2, wbf);
}

void launch_perm(int32_t* idx, int n, long long a, long long c, hipStream_t s) {
  if (n) k_perm<<<(n + 255) / 256, 256, 0, s>>>(idx, n, a, c);
}

void launch_to_bf16(const float* w, uint16_t* wbf, hipStream_t s) {
  k_to_bf16<<<(NWT + 255) / 256, 256, 0, s>>>(w, wbf);
}

}  // namespace cpt
