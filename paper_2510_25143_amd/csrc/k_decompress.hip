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

// Two waves per block: each lane prepares two vertices (v = lane + 128 k),
// lanes 0-31 of the first wave then sweep the Lorenzo anti-diagonals, and
// each lane writes its two vertices.  Every block of a frame is resident at
// once.  Global reads come in two batches, each with all its loads in flight:
// the per-vertex codes and the block rows' offsets with the previous frame,
// then the residual symbols (and, where the wave has any, the raw words)
// they point at.  Streams that failed a check are skipped.
constexpr int RC_THREADS = 128, RC_VPL = TILE * TILE / RC_THREADS;

__global__ __launch_bounds__(RC_THREADS) void k_reconstruct_b(DecDesc* __restrict__ D, const int* __restrict__ ord,
                                                              int ord0, const long long* __restrict__ pre, int m, int t,
                                                              const long long* __restrict__ mtab, DecodeBufs B) {
  __shared__ int C[2][TILE][TILE];       // reconstructed fixed-point values (u, v)
  __shared__ int P[2][HALO][HALO];       // previous frame around the block
  __shared__ int A[2][TILE][TILE];       // known value, or frame t-1 Lorenzo term plus q (2 xi~ + 1)
  __shared__ uint8_t KN[2][TILE][TILE];  // component already known (raw or semi-Lagrangian)
  const int j = find_field(pre, m, blockIdx.x);
  DecDesc& d = D[j == 0 ? ord0 : ord[j]];  // ord0 = ord[0]: one stream reads no table first
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
  const uint32_t* raw = d.sec[7];
  const long long nq = d.nq, nraw = d.nraw;
  uint32_t* err = &d.err;
  const long long mode_base = mtab[d.mtb + t];
  const int x0 = bx * TILE, y0 = by * TILE;
  const int2* prevf = t > 0 ? cur + (size_t)(t - 1) * HW : cur;

  // ---- read batch 1: codes, the offsets of the block's rows (segments), the
  // previous frame with a one-vertex halo
  constexpr int NH = HALO * HALO, KH = (NH + RC_THREADS - 1) / RC_THREADS;
  uint32_t vcode[RC_VPL], sqv[RC_VPL], srv[RC_VPL], vm = 0, hm = 0;
  int2 hp[KH];
#pragma unroll
  for (int k = 0; k < RC_VPL; k++) {
    const int v = lane + RC_THREADS * k, x = x0 + (v & 15), y = y0 + (v >> 4);
    const bool valid = (x < W) & (y < H);
    vm |= valid ? 1u << k : 0u;
    vcode[k] = xs[valid ? (size_t)t * HW + (size_t)y * W + x : 0];
    const long long sg = d.soff + (y < H ? ((long long)t * H + y) * p.tx + bx : 0);
    sqv[k] = B.sq[sg];
    srv[k] = B.sro[sg];
  }
#pragma unroll
  for (int k = 0; k < KH; k++) {
    const int i = lane + RC_THREADS * k, hy = i / HALO, hx = i - hy * HALO, x = x0 - 1 + hx, y = y0 - 1 + hy;
    const bool valid = (i < NH) & (t > 0) & (x >= 0) & (x < W) & (y >= 0) & (y < H);
    hm |= valid ? 1u << k : 0u;
    hp[k] = prevf[valid ? (size_t)y * W + x : 0];
  }
  const uint32_t qbase = B.sq[d.soff], rbase = B.sro[d.soff];
  int cls = 0;
  if (t >= 1) {
    if (p.predictor == 1) cls = 1;
    else if (mode_base >= 0) cls = B.modes[d.mbase + mode_base + (long long)by * p.tx + bx];
  }
  const int dmax = p.predictor == 1 ? 2 : class_dmax(p.K, cls);
#pragma unroll
  for (int k = 0; k < KH; k++) {
    const int i = lane + RC_THREADS * k;
    if (i < NH) {
      const int2 v = (hm >> k) & 1u ? hp[k] : make_int2(0, 0);
      (&P[0][0][0])[i] = v.x;
      (&P[1][0][0])[i] = v.y;
    }
  }

  // ---- read batch 2: the two residual symbols of every coded vertex, at its
  // segment's offset plus the coded vertices before it in the row (each
  // 16-lane DPP row holds one block row; index clamped into the stream)
  int vq[RC_VPL];
  uint32_t ridx[RC_VPL], rneed = 0;
#pragma unroll
  for (int k = 0; k < RC_VPL; k++) {
    if (!((vm >> k) & 1u)) vcode[k] = XLOSSLESS;
    const bool coded = ((vm >> k) & 1u) && vcode[k] != XLOSSLESS;
    const long long o = 2 * ((long long)(sqv[k] - qbase) + row16_exclusive(coded ? 1u : 0u));
    // the pair starts at an even position of an even-aligned array (nq is
    // even), so it is one 32-bit word
    const long long oc = nq >= 2 ? min(max(o, 0LL), nq - 2) : 0;
    const uint32_t qw = nq >= 2 ? *reinterpret_cast<const uint32_t*>(qs + oc) : 0u;
    vq[k] = coded ? (int)qw : 0;
  }
#pragma unroll
  for (int k = 0; k < RC_VPL; k++) {
    const bool valid = (vm >> k) & 1u;
    const uint32_t r = !valid ? 0u : vcode[k] == XLOSSLESS ? 2u : ((vq[k] & 0xFFFF) == 0) + (((uint32_t)vq[k] >> 16) == 0);
    ridx[k] = (srv[k] - rbase) + row16_exclusive(r);
    rneed |= r;
  }
  // ---- read batch 3 (only where the block has raw words): the two raw words a
  // vertex may use
  uint32_t rw0[RC_VPL] = {}, rw1[RC_VPL] = {};
  if (__builtin_amdgcn_readfirstlane(__ballot(rneed != 0) != 0ull ? 1 : 0) && nraw >= 1) {
#pragma unroll
    for (int k = 0; k < RC_VPL; k++) {
      rw0[k] = raw[min((long long)ridx[k], nraw - 1)];
      rw1[k] = raw[min((long long)ridx[k] + 1, nraw - 1)];
    }
  }
  __syncthreads();
  // frame t-1 from the staged halo where it covers the sample
  auto F = [&](int xx, int yy) {
    const int hx = xx - x0 + 1, hy = yy - y0 + 1;
    return (hx >= 0 && hx < HALO && hy >= 0 && hy < HALO) ? make_int2(P[0][hy][hx], P[1][hy][hx])
                                                          : prevf[(size_t)yy * W + xx];
  };

  // everything that does not depend on the block's own reconstruction
#pragma unroll
  for (int k = 0; k < RC_VPL; k++) {
    const int v = lane + RC_THREADS * k, lx = v & 15, ly = v >> 4;
    const int x = x0 + lx, y = y0 + ly;
    if (!((vm >> k) & 1u)) {
      vcode[k] = XLOSSLESS;
      continue;
    }
    const int code = (int)vcode[k];
    if (code == XLOSSLESS) vq[k] = 0;
    const int q[2] = {vq[k] & 0xFFFF, (int)((uint32_t)vq[k] >> 16)};
    int pr[2] = {0, 0};
    int64_t w = 0;
    if (code != XLOSSLESS) {
      w = 2 * (int64_t)(p.eps >> code) + 1;
      if (cls != 0) sl_predict_f(F, H, W, x, y, SLConst{p.cx, p.sx, p.cy, p.sy}, dmax, &pr[0], &pr[1]);
    }
    int used = 0;  // raw words taken so far by this vertex
    for (int c = 0; c < 2; c++) {
      if (code == XLOSSLESS || q[c] == 0) {
        const uint32_t b = used ? rw1[k] : rw0[k];
        used++;
        if (((b >> 23) & 0xFFu) == 0xFFu) atomicOr(err, 64u);
        const int val = to_fixed(__uint_as_float(b), p.k);
        // a stored original never reaches 2^24 on the field's grid; 2^25
        // and beyond (saturated by the conversion) is a corrupt stream
        if (val >= (1 << 25) || val <= -(1 << 25)) atomicOr(err, 128u);
        C[c][ly][lx] = val;
        A[c][ly][lx] = val;
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
          A[c][ly][lx] = (int)rv;
          KN[c][ly][lx] = 1;
        } else {
          // the part of the Lorenzo value that does not depend on this
          // frame's reconstruction; a magnitude of 2^30 or more (corrupt
          // stream) is saturated there, which still fails the range test
          int64_t a = (int)dq;
          if (t > 0)
            a += P[c][ly + 1][lx + 1] - (lx > 0 ? P[c][ly + 1][lx] : 0) - (ly > 0 ? P[c][ly][lx + 1] : 0) +
                 (lx > 0 && ly > 0 ? P[c][ly][lx] : 0);
          A[c][ly][lx] = (int)max(min(a, (int64_t)1 << 30), -((int64_t)1 << 30));
          KN[c][ly][lx] = 0;
        }
      }
    }
  }
  __syncthreads();

  // Lorenzo blocks: lanes 0-15 sweep the rows of u and lanes 16-31 the rows
  // of v along the anti-diagonals.  A lane keeps its last value (the left
  // neighbour of its next vertex); the row above arrives from the previous
  // lane of the same 16-lane DPP row by a row shift.  All 64 lanes of the
  // first wave step together (DPP reads need active source lanes).
  if (cls == 0 && __builtin_amdgcn_readfirstlane(lane >> 6) == 0) {
    const int c = (lane >> 4) & 1, row = lane & 15;
    const bool rowok = lane < 2 * TILE && y0 + row < H;
    const int cend = min(TILE, W - x0);
    int last = 0, upl = 0;
    for (int dd = 0; dd < 2 * TILE - 1; dd++) {
      const int col = dd - row;
      const int cc = min(max(col, 0), TILE - 1);
      const int a = A[c][row][cc];
      const bool kn = KN[c][row][cc] != 0;
      const int up = __builtin_amdgcn_update_dpp(0, last, 0x111, 0xF, 0xF, true);  // row_shr:1
      if (rowok && (unsigned)col < (unsigned)cend) {
        if (kn) {
          last = a;
        } else {
          const int64_t rv0 = (int64_t)(col > 0 ? last : 0) + (row > 0 ? up : 0) - (col > 0 && row > 0 ? upl : 0) + a;
          int64_t rv = rv0;
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
  }
  __syncthreads();
  // known raw components are restored bit-exactly; the rest are exact
  // multiples of 2^-k
#pragma unroll
  for (int k = 0; k < RC_VPL; k++) {
    const int v = lane + RC_THREADS * k, lx = v & 15, ly = v >> 4;
    const int x = x0 + lx, y = y0 + ly;
    if (!((vm >> k) & 1u)) continue;
    const size_t gv = (size_t)t * HW + (size_t)y * W + x;
    const int u = C[0][ly][lx], vv = C[1][ly][lx];
    cur[gv] = make_int2(u, vv);
    float fu, fv;
    if (vcode[k] == XLOSSLESS) {
      fu = __uint_as_float(rw0[k]);
      fv = __uint_as_float(rw1[k]);
    } else {
      const bool ru = (vq[k] & 0xFFFF) == 0;
      fu = ru ? __uint_as_float(rw0[k]) : from_fixed(u, p.k);
      fv = ((uint32_t)vq[k] >> 16) == 0 ? __uint_as_float(ru ? rw1[k] : rw0[k]) : from_fixed(vv, p.k);
    }
    field[gv] = fu;
    field[N + gv] = fv;
  }
}

// ============================================================ launchers
void launch_reconstruct_b(DecDesc* D, const int* ord, int ord0, const long long* pre, int m, long long nblocks,
                          int t, const long long* mtab, const DecodeBufs& B, hipStream_t s) {
  if (nblocks > 0) k_reconstruct_b<<<(unsigned)nblocks, RC_THREADS, 0, s>>>(D, ord, ord0, pre, m, t, mtab, B);
}

}  // namespace cpt
