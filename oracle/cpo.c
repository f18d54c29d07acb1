/*
 * cpo.c — CPU oracle for critical-point-trajectory-preserving lossy
 * compression of 2D time-varying vector fields (arXiv 2510.25143).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no source, header, table or generator with the HIP
 * library.  It is plain, single-threaded and slow on purpose: every step is
 * written the way the paper states it, so that a reader can check it by eye.
 *
 * Where the paper is silent or ambiguous, the reading taken is marked
 * READING and listed with its reason in the design notes of the repository.
 *
 * Paper map used in the citations below:
 *   Sec. III-A/B  piecewise-linear field, barycentric critical point (eq. def)
 *   Sec. III-C    space-time extrusion and the three-tetrahedron prism split
 *   Sec. III-E    face-level inside test (eq. inside-test)
 *   Sec. III-F    simulation of simplicity, Alg. 1
 *   Sec. III-G    error-bound derivation, Alg. 2
 *   Sec. IV-A     problem: pointwise bound and face invariance
 *   Sec. V        Alg. 3 (compression driver) and Alg. 4 (per-vertex bound)
 *   Sec. VI-A     semi-Lagrangian predictor (eqs. sl-dep, sl-sample, rk2-*,
 *                 substeps)
 *   Sec. VI-B     context-preserving micro-encoding and rate score
 *                 (eq. entropy and the rate estimate that follows it)
 */
#include "cpo.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---- format constants (READING: the paper prints none of these) ---- */
#define TILE 16          /* spatial block edge for blocking and mode choice */
/* R and the longest codeword are build-time constants so that the format
   study in tests/format_cost_study.py can measure other values; the stream
   records both and every build reads only its own. */
#ifndef CPO_QR
#define CPO_QR 512
#endif
#ifndef CPO_MAXLEN
#define CPO_MAXLEN 16
#endif
#define QR CPO_QR        /* residual quantization radius R */
#define QSYM (2 * QR)    /* residual-code alphabet; code 0 = unpredictable */
#define XSYM 25          /* bound-code alphabet; 24 = lossless */
#define XLOSSLESS 24
#define MAXLEN CPO_MAXLEN /* longest Huffman codeword */
#define CHUNK 1024       /* symbols per independently decodable chunk */
#define STRIDE 2         /* micro-encoding statistics subsample (Sec. VI-B) */
#define NMAX 32          /* maximum substeps, Sec. VI-A */
#define HDR_SLOTS 32
#define HDR_BYTES (8 * HDR_SLOTS)
#define MAGIC 0x31545043ull /* "CPT1" */
#define VERSION 1ull

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) q--;
  return q;
}
static int64_t iabs64(int64_t a) { return a < 0 ? -a : a; }
static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

/* ======================================================================
 * Fixed point.  Alg. 3 converts the field to integers before any test so
 * that simulation of simplicity works on exact values.  READING: the scale
 * is 2^k with k = 23 - e where max|x| = m 2^e (m in [0.5,1)), so every
 * original value fits 24 bits and every reconstructed value fits 25 bits.
 * The bound eps' = floor(eb_abs 2^k - 1/2): the half unit absorbs the
 * rounding of the conversion, so |x - x'| <= (eps' + 1/2) 2^-k <= eb_abs.
 * ==================================================================== */
int cpo_params(const float* field, int H, int W, int T, int eb_mode, double eb,
               int* k, double* eb_abs, int64_t* eps) {
  if (H < 2 || W < 2 || T < 1) return CPO_EINVAL;
  size_t n = 2 * (size_t)H * W * T;
  double mn = INFINITY, mx = -INFINITY, ma = 0.0;
  for (size_t i = 0; i < n; i++) {
    double x = field[i];
    if (!isfinite(x)) return CPO_EINVAL;
    if (x < mn) mn = x;
    if (x > mx) mx = x;
    if (fabs(x) > ma) ma = fabs(x);
  }
  if (ma >= ldexp(1.0, 100)) return CPO_EINVAL;
  int e = 0;
  if (ma > 0) frexp(ma, &e);
  int kk = 23 - e;
  if (kk > 120) kk = 120;
  double ea;
  if (eb_mode == 0) {
    if (!(eb > 0.0 && eb <= 0.5)) return CPO_EINVAL;
    ea = eb * (mx - mn);
  } else if (eb_mode == 1) {
    if (!(eb > 0.0) || !isfinite(eb)) return CPO_EINVAL;
    ea = eb;
  } else {
    return CPO_EINVAL;
  }
  double s = floor(ldexp(ea, kk) - 0.5);
  int64_t ep = 0;
  if (s > 0) ep = s >= 8388607.0 ? 8388607 : (int64_t)s;
  *k = kk;
  *eb_abs = ea;
  *eps = ep;
  return CPO_OK;
}

/* Values whose scaled magnitude leaves the int32 range (only a caller's k
   that does not fit the field, or a corrupt stream, gives one) saturate, so
   the conversion is defined for every finite input; callers reject such
   values before using them. */
void cpo_to_fixed(const float* x, size_t n, int k, int32_t* out) {
  for (size_t i = 0; i < n; i++) {
    double d = nearbyint(ldexp((double)x[i], k));
    out[i] = d >= 2147483647.0 ? INT32_MAX : (d <= -2147483648.0 ? INT32_MIN : (int32_t)d);
  }
}

/* 1 when every |x| 2^k stays below 2^24, the range the extraction needs
   (Sec. III-F works on the exact fixed-point values). */
static int fits_24(const float* x, size_t n, int k) {
  for (size_t i = 0; i < n; i++)
    if (!(fabs(ldexp((double)x[i], k)) < 16777216.0)) return 0;
  return 1;
}

/* ======================================================================
 * Simulation of simplicity (Sec. III-F).  READING: each vertex value is
 * perturbed symbolically, v by eps^(2^(2g)) and u by eps^(2^(2g+1)), with g
 * its global index (t H + y) W + x; the origin is not perturbed.  Expanding
 * det(p~, q~) for g_p < g_q in increasing powers of eps gives the terms
 *   u_p v_q - v_p u_q,  -u_q,  +v_q,  +u_p,  +1
 * and the sign of the edge is the sign of the first nonzero one.
 * ==================================================================== */
int cpo_sos_edge(int32_t up, int32_t vp, int32_t uq, int32_t vq) {
  int64_t d = (int64_t)up * vq - (int64_t)vp * uq;
  if (d != 0) return d > 0 ? 1 : -1;
  if (uq != 0) return uq < 0 ? 1 : -1;
  if (vq != 0) return vq > 0 ? 1 : -1;
  if (up != 0) return up > 0 ? 1 : -1;
  return 1;
}

/* Face-level test (Sec. III-E): for vertices a < b < c by global index the
   origin lies in the perturbed triangle iff det(a,b), det(b,c), det(c,a) share
   a strict sign; det(c,a) = -det(a,c).  The face's sign is that of det(a,b). */
static int face_test(const int32_t* U, const int32_t* V, size_t a, size_t b,
                     size_t c, int* sign) {
  int sab = cpo_sos_edge(U[a], V[a], U[b], V[b]);
  int sbc = cpo_sos_edge(U[b], V[b], U[c], V[c]);
  int sac = cpo_sos_edge(U[a], V[a], U[c], V[c]);
  *sign = sab;
  return sab == sbc && sbc == -sac;
}

/* Space-time faces (Sec. III-C).  Each quad is split by its main diagonal
   (READING; a single fixed diagonal gives the 36 incident faces per vertex
   that Alg. 4 names).  A prism over triangle a<b<c (spatial index order) is
   split into (a_t,b_t,c_t,c_t+1), (a_t,b_t,b_t+1,c_t+1),
   (a_t,a_t+1,b_t+1,c_t+1).  Every face is listed once, owned by its
   lowest-index vertex, in twelve types; vertex offsets are (dx,dy,dt) in
   increasing global index order. */
static const int FV[12][3][3] = {
    {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}}, /* 0  lower triangle, slice t */
    {{0, 0, 0}, {0, 1, 0}, {1, 1, 0}}, /* 1  upper triangle, slice t */
    {{0, 0, 0}, {1, 0, 0}, {1, 1, 1}}, /* 2  lower prism interior */
    {{0, 0, 0}, {1, 0, 1}, {1, 1, 1}}, /* 3  lower prism interior */
    {{0, 0, 0}, {0, 1, 0}, {1, 1, 1}}, /* 4  upper prism interior */
    {{0, 0, 0}, {0, 1, 1}, {1, 1, 1}}, /* 5  upper prism interior */
    {{0, 0, 0}, {1, 0, 0}, {1, 0, 1}}, /* 6  x-edge side */
    {{0, 0, 0}, {0, 0, 1}, {1, 0, 1}}, /* 7  x-edge side */
    {{0, 0, 0}, {0, 1, 0}, {0, 1, 1}}, /* 8  y-edge side */
    {{0, 0, 0}, {0, 0, 1}, {0, 1, 1}}, /* 9  y-edge side */
    {{0, 0, 0}, {1, 1, 0}, {1, 1, 1}}, /* 10 diagonal-edge side */
    {{0, 0, 0}, {0, 0, 1}, {1, 1, 1}}, /* 11 diagonal-edge side */
};

void cpo_face_vertices(int f, int* dx, int* dy, int* dt) {
  for (int i = 0; i < 3; i++) {
    dx[i] = FV[f][i][0];
    dy[i] = FV[f][i][1];
    dt[i] = FV[f][i][2];
  }
}

static int face_valid(int H, int W, int T, int x, int y, int t, int f) {
  for (int i = 0; i < 3; i++) {
    if (x + FV[f][i][0] >= W || y + FV[f][i][1] >= H || t + FV[f][i][2] >= T)
      return 0;
  }
  return x >= 0 && y >= 0 && t >= 0;
}

static size_t vid(int H, int W, int x, int y, int t) {
  return ((size_t)t * H + y) * W + x;
}

void cpo_face_masks(const int32_t* U, const int32_t* V, int H, int W, int T,
                    uint32_t* masks) {
  for (int t = 0; t < T; t++)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) {
        uint32_t m = 0;
        for (int f = 0; f < 12; f++) {
          if (!face_valid(H, W, T, x, y, t, f)) continue;
          size_t a = vid(H, W, x + FV[f][0][0], y + FV[f][0][1], t + FV[f][0][2]);
          size_t b = vid(H, W, x + FV[f][1][0], y + FV[f][1][1], t + FV[f][1][2]);
          size_t c = vid(H, W, x + FV[f][2][0], y + FV[f][2][1], t + FV[f][2][2]);
          int s;
          if (face_test(U, V, a, b, c, &s)) m |= (1u << f) | ((s > 0 ? 1u : 0u) << (12 + f));
        }
        masks[vid(H, W, x, y, t)] = m;
      }
}

int cpo_extract_fixed(const int32_t* U, const int32_t* V, int H, int W, int T,
                      uint64_t* codes, size_t cap, size_t* count) {
  size_t N = (size_t)H * W * T, cnt = 0;
  uint32_t* masks = (uint32_t*)malloc(N * sizeof(uint32_t));
  if (!masks) return CPO_ENOMEM;
  cpo_face_masks(U, V, H, W, T, masks);
  for (size_t g = 0; g < N; g++)
    for (int f = 0; f < 12; f++)
      if (masks[g] & (1u << f)) {
        if (cnt < cap && codes)
          codes[cnt] = (((uint64_t)g * 12 + f) << 1) | ((masks[g] >> (12 + f)) & 1u);
        cnt++;
      }
  free(masks);
  *count = cnt;
  return cnt > cap ? CPO_ECAPACITY : CPO_OK;
}

int cpo_extract(const float* field, int H, int W, int T, int k, uint64_t* codes,
                size_t cap, size_t* count) {
  if (H < 2 || W < 2 || T < 1) return CPO_EINVAL;
  size_t N = (size_t)H * W * T;
  if (!fits_24(field, 2 * N, k)) return CPO_EINVAL;
  int32_t* F = (int32_t*)malloc(2 * N * sizeof(int32_t));
  if (!F) return CPO_ENOMEM;
  cpo_to_fixed(field, 2 * N, k, F);
  int st = cpo_extract_fixed(F, F + N, H, W, T, codes, cap, count);
  free(F);
  return st;
}

/* The set C of Alg. 3: a vertex must be stored losslessly when any face that
   contains it is crossed in the original field (Alg. 4). */
void cpo_lossless_flags(const uint32_t* masks, int H, int W, int T, uint8_t* flags) {
  size_t N = (size_t)H * W * T;
  memset(flags, 0, N);
  for (int t = 0; t < T; t++)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) {
        uint32_t m = masks[vid(H, W, x, y, t)];
        for (int f = 0; f < 12; f++)
          if (m & (1u << f))
            for (int i = 0; i < 3; i++)
              flags[vid(H, W, x + FV[f][i][0], y + FV[f][i][1], t + FV[f][i][2])] = 1;
      }
}

/* The faces that contain vertex (x,y,t): their owners lie at offsets in
   {-1,0}^3.  nbr receives the two other vertices of each face. */
int cpo_incident_faces(int H, int W, int T, int x, int y, int t, int32_t* nbr) {
  int n = 0;
  for (int ot = -1; ot <= 0; ot++)
    for (int oy = -1; oy <= 0; oy++)
      for (int ox = -1; ox <= 0; ox++) {
        int X = x + ox, Y = y + oy, Tt = t + ot;
        for (int f = 0; f < 12; f++) {
          if (!face_valid(H, W, T, X, Y, Tt, f)) continue;
          int hit = -1;
          for (int i = 0; i < 3; i++)
            if (FV[f][i][0] == -ox && FV[f][i][1] == -oy && FV[f][i][2] == -ot) hit = i;
          if (hit < 0) continue;
          if (nbr) {
            int j = 0;
            for (int i = 0; i < 3; i++)
              if (i != hit)
                nbr[2 * n + j++] = (int32_t)vid(H, W, X + FV[f][i][0], Y + FV[f][i][1], Tt + FV[f][i][2]);
          }
          n++;
        }
      }
  return n;
}

/* ======================================================================
 * Alg. 2 (Sec. III-G): the largest perturbation of vertex 2 of a face that
 * keeps the signs of M, M0 and M1, hence the face's status.  READING: the
 * fractions are made strict and exact in integers, cand(N,D) =
 * floor((N-1)/D), so that eb*D < N; the same-sign relaxations use |u2|-1 and
 * |v2|-1 so the component cannot reach zero; the early returns of 0 come
 * before the relaxations, as written.
 * ==================================================================== */
static int64_t cand(int64_t N, int64_t D) {
  if (D == 0) return INT64_MAX;
  if (N == 0) return 0;
  return (N - 1) / D;
}
static int same_sign(int64_t a, int64_t b, int64_t c) {
  return (a > 0 && b > 0 && c > 0) || (a < 0 && b < 0 && c < 0);
}

int64_t cpo_alg2(int64_t u0, int64_t u1, int64_t u2, int64_t v0, int64_t v1,
                 int64_t v2) {
  int64_t M0 = u2 * v0 - u0 * v2;
  int64_t M1 = u1 * v2 - u2 * v1;
  int64_t M2 = u0 * v1 - u1 * v0;
  int64_t M = M0 + M1 + M2;
  if (M == 0) return 0;
  int64_t eb = cand(iabs64(M), iabs64(u1 - u0) + iabs64(v0 - v1));
  if (iabs64(u1) + iabs64(v1) != 0)
    eb = imin64(eb, cand(iabs64(M1), iabs64(u1) + iabs64(v1)));
  else
    return 0;
  if (iabs64(u0) + iabs64(v0) != 0)
    eb = imin64(eb, cand(iabs64(M0), iabs64(u0) + iabs64(v0)));
  else
    return 0;
  if (same_sign(u0, u1, u2)) eb = imax64(eb, iabs64(u2) - 1);
  if (same_sign(v0, v1, v2)) eb = imax64(eb, iabs64(v2) - 1);
  return eb;
}

/* Alg. 4: zero when the vertex touches a face of C, else the minimum of eps'
   and Alg. 2 over every incident face, evaluated on the current values
   (reconstructed where already processed, original elsewhere). */
int64_t cpo_vertex_bound(const int32_t* U, const int32_t* V, const uint8_t* flags,
                         int H, int W, int T, int x, int y, int t, int64_t eps) {
  size_t v = vid(H, W, x, y, t);
  if (flags[v]) return 0;
  int32_t nb[72];
  int nf = cpo_incident_faces(H, W, T, x, y, t, nb);
  int64_t xi = eps;
  for (int i = 0; i < nf; i++) {
    size_t a = (size_t)nb[2 * i], b = (size_t)nb[2 * i + 1];
    int64_t e = cpo_alg2(U[a], U[b], U[v], V[a], V[b], V[v]);
    if (e < xi) xi = e;
  }
  return xi;
}

/* READING: the per-vertex bound is quantized to eps' >> q, the smallest such
   power-of-two fraction not above xi; code 24 marks a lossless vertex. */
int32_t cpo_xi_code(int64_t eps, int64_t xi) {
  if (xi <= 0) return XLOSSLESS;
  int32_t q = 0;
  while ((eps >> q) > xi) q++;
  return q;
}

/* READING: residual quantization with bin width 2 xi~ + 1; |q| >= R makes
   the component unpredictable (stored raw). */
int32_t cpo_quantize(int64_t x, int64_t pred, int64_t xt, int64_t* recon) {
  int64_t w = 2 * xt + 1;
  int64_t q = floordiv(x - pred + xt, w);
  if (q >= QR || q <= -QR) {
    *recon = x;
    return 0;
  }
  *recon = pred + q * w;
  return (int32_t)(q + QR);
}

/* ======================================================================
 * Predictors.
 * First-order 3-D Lorenzo (Sec. VI): the seven causal neighbours of
 * (x,y,t).  READING: neighbours outside the spatial block, or before t=0,
 * count as zero, so every block predicts from its own values only.
 * ==================================================================== */
static int64_t lorenzo3(const int32_t* cur_t, const int32_t* prev, int W,
                        int x, int y, int x0, int y0) {
#define LV(P, xx, yy) (((P) == NULL || (xx) < x0 || (yy) < y0) ? 0 : (int64_t)(P)[(size_t)(yy) * W + (xx)])
  return LV(cur_t, x - 1, y) + LV(cur_t, x, y - 1) + LV(prev, x, y)
       - LV(cur_t, x - 1, y - 1) - LV(prev, x - 1, y) - LV(prev, x, y - 1)
       + LV(prev, x - 1, y - 1);
#undef LV
}

int64_t cpo_lorenzo3(const int32_t* cur_t, const int32_t* prev, int W, int x, int y,
                     int x0, int y0) {
  return lorenzo3(cur_t, prev, W, x, y, x0, y0);
}

/* Semi-Lagrangian predictor (Sec. VI-A) in Q16 cell units.  READING: the
   displacement of a fixed-point velocity u is floor(u c / 2^s), where c/2^s
   approximates dt/dx 2^(16-k) with c in [2^30, 2^31) (s at most 62; a zero
   factor is c = s = 0; 2^31 - 1 or more saturates to c = 2^31 - 1, s = 0);
   positions are clamped to the domain; bilinear sampling rounds half up. */
void cpo_sl_factor(double dt_dx, int k, int64_t* c, int64_t* s) {
  double f = ldexp(dt_dx, 16 - k);
  if (!(f > 0.0)) {
    *c = 0;
    *s = 0;
    return;
  }
  if (f >= 2147483647.0) {
    *c = 2147483647;
    *s = 0;
    return;
  }
  int e;
  frexp(f, &e);
  int sh = 31 - e;
  if (sh > 62) sh = 62;
  int64_t cc = (int64_t)nearbyint(ldexp(f, sh));
  if (cc >= 2147483648LL) {
    cc = 1073741824LL;
    sh -= 1;
  }
  if (cc == 0) sh = 0; /* a factor too small for 62 fraction bits: no displacement */
  *c = cc;
  *s = sh;
}

static int64_t clampi(int64_t a, int64_t lo, int64_t hi) {
  return a < lo ? lo : (a > hi ? hi : a);
}

int64_t cpo_bilinear(const int32_t* F, int H, int W, int64_t px, int64_t py) {
  int64_t x0 = px >> 16, y0 = py >> 16;
  int64_t fx = px & 65535, fy = py & 65535;
  int64_t x1 = x0 + 1 < W ? x0 + 1 : x0, y1 = y0 + 1 < H ? y0 + 1 : y0;
  int64_t a = F[y0 * W + x0], b = F[y0 * W + x1], c = F[y1 * W + x0], d = F[y1 * W + x1];
  int64_t s = a * (65536 - fx) * (65536 - fy) + b * fx * (65536 - fy)
            + c * (65536 - fx) * fy + d * fx * fy;
  return floordiv(s + (1LL << 31), 1LL << 32);
}

static int64_t disp(int64_t u, int64_t c, int64_t s) {
  return floordiv(u * c, (int64_t)1 << s);
}

void cpo_sl_predict(const int32_t* Up, const int32_t* Vp, int H, int W, int x,
                    int y, int64_t cx, int64_t sx, int64_t cy, int64_t sy,
                    int dmax, int nmax, int64_t* pu, int64_t* pv) {
  int64_t XM = (int64_t)(W - 1) << 16, YM = (int64_t)(H - 1) << 16;
  int64_t px = (int64_t)x << 16, py = (int64_t)y << 16;
  /* displacement estimate from the previous frame at the grid point */
  int64_t dx = disp(Up[(size_t)y * W + x], cx, sx);
  int64_t dy = disp(Vp[(size_t)y * W + x], cy, sy);
  int64_t dinf = imax64(iabs64(dx), iabs64(dy));
  int64_t lim = (int64_t)dmax << 16;
  int64_t qx, qy;
  if (dinf <= lim) {
    /* RK2 midpoint: half step, velocity there, full step */
    int64_t hx = clampi(px - floordiv(dx, 2), 0, XM);
    int64_t hy = clampi(py - floordiv(dy, 2), 0, YM);
    int64_t uh = cpo_bilinear(Up, H, W, hx, hy);
    int64_t vh = cpo_bilinear(Vp, H, W, hx, hy);
    qx = clampi(px - disp(uh, cx, sx), 0, XM);
    qy = clampi(py - disp(vh, cy, sy), 0, YM);
  } else {
    /* adaptive substepping: N = min(ceil(dinf/dmax), Nmax) Euler substeps */
    int64_t n = imin64((dinf + lim - 1) / lim, nmax);
    qx = px;
    qy = py;
    for (int64_t s = 0; s < n; s++) {
      int64_t us = cpo_bilinear(Up, H, W, qx, qy);
      int64_t vs = cpo_bilinear(Vp, H, W, qx, qy);
      int64_t nx = clampi(qx - floordiv(disp(us, cx, sx), n), 0, XM);
      int64_t ny = clampi(qy - floordiv(disp(vs, cy, sy), n), 0, YM);
      qx = nx;
      qy = ny;
    }
  }
  *pu = cpo_bilinear(Up, H, W, qx, qy);
  *pv = cpo_bilinear(Vp, H, W, qx, qy);
}

/* ======================================================================
 * Rate score of a candidate predictor on a block (Sec. VI-B).  READING: all
 * quantities in Q16 bits; T[h] = floor(h log2 h 2^16); the zero-order
 * entropy is floor((T[n] - sum T[h_k]) / n); the overflow penalty uses
 * lambda = 16 bits; the mode metadata is log2 K bits per block spread over
 * the block's 2 x 256 x mode_bt samples.
 * ==================================================================== */
int64_t cpo_tlog(int h) {
  if (h <= 1) return 0;
  return (int64_t)floor((double)h * log2((double)h) * 65536.0);
}

int64_t cpo_score(const int32_t* hist, int nbins, int n, int L, int K, int bt) {
  int64_t h0 = 0;
  if (n > 0) {
    int64_t s = cpo_tlog(n);
    for (int b = 0; b < nbins; b++)
      if (hist[b] > 0) s -= cpo_tlog(hist[b]);
    h0 = floordiv(s, n);
  }
  int64_t pen = (n + L) > 0 ? floordiv((int64_t)16 * 65536 * L, n + L) : 0;
  int64_t lg = K == 4 ? 2 : 1;
  int64_t meta = floordiv(65536 * lg, (int64_t)512 * bt);
  return h0 + pen + meta;
}

/* ======================================================================
 * Canonical Huffman code, lengths limited to MAXLEN by package-merge.
 * READING: leaves are ordered by (count, symbol); when a leaf and a package
 * weigh the same the leaf comes first.
 * ==================================================================== */
typedef struct {
  uint64_t w;
  int32_t sym;
} leaf_t;

static int leaf_cmp(const void* a, const void* b) {
  const leaf_t* x = (const leaf_t*)a;
  const leaf_t* y = (const leaf_t*)b;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return x->sym - y->sym;
}

int cpo_huffman_lengths(const uint64_t* counts, int nsym, int maxlen, uint8_t* lengths) {
  memset(lengths, 0, (size_t)nsym);
  leaf_t* lv = (leaf_t*)malloc(sizeof(leaf_t) * (size_t)(nsym > 0 ? nsym : 1));
  int n = 0;
  for (int s = 0; s < nsym; s++)
    if (counts[s] > 0) {
      lv[n].w = counts[s];
      lv[n].sym = s;
      n++;
    }
  if (n == 0) {
    free(lv);
    return CPO_OK;
  }
  if (n == 1) {
    lengths[lv[0].sym] = 1;
    free(lv);
    return CPO_OK;
  }
  if (maxlen < 1 || maxlen > 30 || n > (1 << maxlen)) {
    free(lv);
    return CPO_EINVAL;
  }
  qsort(lv, (size_t)n, sizeof(leaf_t), leaf_cmp);
  /* list[j] for j = 1..maxlen: weights and a leaf flag per item */
  int cap = 2 * n;
  uint64_t* lw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap * (maxlen + 1));
  uint8_t* lf = (uint8_t*)malloc((size_t)cap * (maxlen + 1));
  int* len = (int*)calloc((size_t)(maxlen + 1), sizeof(int));
  for (int i = 0; i < n; i++) {
    lw[1 * cap + i] = lv[i].w;
    lf[1 * cap + i] = 1;
  }
  len[1] = n;
  for (int j = 2; j <= maxlen; j++) {
    int np = len[j - 1] / 2, i = 0, p = 0, o = 0;
    while (i < n || p < np) {
      uint64_t pw = p < np ? lw[(j - 1) * cap + 2 * p] + lw[(j - 1) * cap + 2 * p + 1] : 0;
      if (i < n && (p >= np || lv[i].w <= pw)) {
        lw[j * cap + o] = lv[i].w;
        lf[j * cap + o] = 1;
        i++;
      } else {
        lw[j * cap + o] = pw;
        lf[j * cap + o] = 0;
        p++;
      }
      o++;
    }
    len[j] = o;
  }
  int* cl = (int*)calloc((size_t)n, sizeof(int));
  int m = 2 * n - 2;
  for (int j = maxlen; j >= 1; j--) {
    int l = 0;
    for (int i = 0; i < m && i < len[j]; i++) l += lf[j * cap + i];
    for (int r = 0; r < l; r++) cl[r]++;
    m = 2 * (m - l);
  }
  for (int r = 0; r < n; r++) lengths[lv[r].sym] = (uint8_t)cl[r];
  free(cl);
  free(len);
  free(lf);
  free(lw);
  free(lv);
  return CPO_OK;
}

/* canonical codewords: symbols ordered by (length, symbol) */
static void canonical_codes(const uint8_t* lengths, int nsym, uint32_t* codes);
void cpo_canonical_codes(const uint8_t* lengths, int nsym, uint32_t* codes) {
  memset(codes, 0, sizeof(uint32_t) * (size_t)nsym);
  canonical_codes(lengths, nsym, codes);
}
static void canonical_codes(const uint8_t* lengths, int nsym, uint32_t* codes) {
  uint32_t code = 0;
  int prev = 0, first = 1;
  for (int l = 1; l <= MAXLEN; l++)
    for (int s = 0; s < nsym; s++) {
      if (lengths[s] != l) continue;
      if (first) {
        code = 0;
        first = 0;
      } else {
        code = (code + 1) << (l - prev);
      }
      prev = l;
      codes[s] = code;
    }
}

/* ---------------------------------------------------------------- bytes */
typedef struct {
  uint8_t* p;
  size_t len, cap;
} buf_t;

static int buf_reserve(buf_t* b, size_t extra) {
  if (b->len + extra <= b->cap) return 0;
  size_t nc = b->cap ? b->cap : 1024;
  while (nc < b->len + extra) nc *= 2;
  uint8_t* q = (uint8_t*)realloc(b->p, nc);
  if (!q) return -1;
  b->p = q;
  b->cap = nc;
  return 0;
}
static int put_u32(buf_t* b, uint32_t v) {
  if (buf_reserve(b, 4)) return -1;
  for (int i = 0; i < 4; i++) b->p[b->len++] = (uint8_t)(v >> (8 * i));
  return 0;
}
static uint32_t get_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t get_u64(const uint8_t* p) {
  return (uint64_t)get_u32(p) | ((uint64_t)get_u32(p + 4) << 32);
}
static void set_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i));
}

/* Huffman-code nsym-alphabet symbols sym[0..n) into three sections:
   codebook (count, then symbol | length<<16 per used symbol), chunk table
   (bit count per CHUNK symbols) and the bitstream (MSB-first 32-bit words,
   every chunk starting on a word). */
static int huff_encode(const uint16_t* sym, size_t n, int nsym, buf_t* cb,
                       buf_t* ct, buf_t* bs) {
  uint64_t* cnt = (uint64_t*)calloc((size_t)nsym, sizeof(uint64_t));
  uint8_t* L = (uint8_t*)malloc((size_t)nsym);
  uint32_t* C = (uint32_t*)calloc((size_t)nsym, sizeof(uint32_t));
  for (size_t i = 0; i < n; i++) cnt[sym[i]]++;
  int st = cpo_huffman_lengths(cnt, nsym, MAXLEN, L);
  if (st) goto done;
  canonical_codes(L, nsym, C);
  uint32_t used = 0;
  for (int s = 0; s < nsym; s++) used += L[s] > 0;
  put_u32(cb, used);
  for (int s = 0; s < nsym; s++)
    if (L[s]) put_u32(cb, (uint32_t)s | ((uint32_t)L[s] << 16));
  size_t nch = (n + CHUNK - 1) / CHUNK;
  for (size_t c = 0; c < nch; c++) {
    size_t lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
    uint64_t bits = 0;
    for (size_t i = lo; i < hi; i++) bits += L[sym[i]];
    put_u32(ct, (uint32_t)bits);
    size_t words = (size_t)((bits + 31) / 32);
    if (buf_reserve(bs, 4 * words)) {
      st = CPO_ENOMEM;
      goto done;
    }
    uint32_t* w = (uint32_t*)calloc(words ? words : 1, sizeof(uint32_t));
    uint64_t p = 0;
    for (size_t i = lo; i < hi; i++) {
      int l = L[sym[i]];
      uint32_t code = C[sym[i]];
      for (int b = l - 1; b >= 0; b--) {
        uint32_t bit = (code >> b) & 1u;
        w[p / 32] |= bit << (31 - (p % 32));
        p++;
      }
    }
    for (size_t i = 0; i < words; i++) put_u32(bs, w[i]);
    free(w);
  }
done:
  free(cnt);
  free(L);
  free(C);
  return st;
}

/* Canonical decoding, one bit at a time.  Every check failure is CORRUPT. */
static int huff_decode(const uint8_t* cb, size_t cb_len, const uint8_t* ct,
                       size_t ct_len, const uint8_t* bs, size_t bs_len,
                       int nsym, size_t n, uint16_t* out) {
  if (cb_len < 4) return CPO_ECORRUPT;
  uint32_t used = get_u32(cb);
  if ((size_t)used > (size_t)nsym || cb_len != 4 + 4 * (size_t)used) return CPO_ECORRUPT;
  uint8_t* L = (uint8_t*)calloc((size_t)nsym, 1);
  uint32_t* C = (uint32_t*)calloc((size_t)nsym, sizeof(uint32_t));
  int st = CPO_OK;
  int prev = -1;
  uint64_t kraft = 0;
  for (uint32_t i = 0; i < used; i++) {
    uint32_t e = get_u32(cb + 4 + 4 * i);
    int s = (int)(e & 0xFFFF), l = (int)(e >> 16);
    if (s >= nsym || s <= prev || l < 1 || l > MAXLEN) {
      st = CPO_ECORRUPT;
      goto done;
    }
    prev = s;
    L[s] = (uint8_t)l;
    kraft += (uint64_t)1 << (MAXLEN - l);
  }
  if (kraft > ((uint64_t)1 << MAXLEN)) {
    st = CPO_ECORRUPT;
    goto done;
  }
  canonical_codes(L, nsym, C);
  size_t nch = (n + CHUNK - 1) / CHUNK;
  if (ct_len != 4 * nch) {
    st = CPO_ECORRUPT;
    goto done;
  }
  if (n > 0 && used == 0) {
    st = CPO_ECORRUPT;
    goto done;
  }
  size_t wofs = 0, nwords = bs_len / 4;
  if (bs_len % 4) {
    st = CPO_ECORRUPT;
    goto done;
  }
  for (size_t c = 0; c < nch; c++) {
    uint64_t bits = get_u32(ct + 4 * c);
    size_t words = (size_t)((bits + 31) / 32);
    if (wofs + words > nwords) {
      st = CPO_ECORRUPT;
      goto done;
    }
    size_t lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
    uint64_t p = 0;
    for (size_t i = lo; i < hi; i++) {
      uint32_t code = 0;
      int found = -1;
      for (int l = 1; l <= MAXLEN && found < 0; l++) {
        if (p >= bits) {
          st = CPO_ECORRUPT;
          goto done;
        }
        uint32_t wv = get_u32(bs + 4 * (wofs + p / 32));
        code = (code << 1) | ((wv >> (31 - (p % 32))) & 1u);
        p++;
        for (int s = 0; s < nsym; s++)
          if (L[s] == l && C[s] == code) {
            found = s;
            break;
          }
      }
      if (found < 0) {
        st = CPO_ECORRUPT;
        goto done;
      }
      out[i] = (uint16_t)found;
    }
    if (p != bits) {
      st = CPO_ECORRUPT;
      goto done;
    }
    wofs += words;
  }
  if (wofs != nwords) st = CPO_ECORRUPT;
done:
  free(L);
  free(C);
  return st;
}

/* ======================================================================
 * Learned predictor selector: block features and a 10-64-64-4 MLP with
 * bf16 weights and fp32 accumulation in a fixed order.
 * ==================================================================== */
static float bf16_to_f32(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float f;
  memcpy(&f, &b, 4);
  return f;
}
static float round_bf16(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  float f;
  memcpy(&f, &b, 4);
  return f;
}

enum { OW1 = 0, OB1 = 640, OW2 = 704, OB2 = 4800, OW3 = 4864, OB3 = 5120 };

int cpo_mlp_forward(const uint16_t* w, const float* x, float* logits) {
  float h1[CPO_HID], h2[CPO_HID];
  for (int j = 0; j < CPO_HID; j++) {
    float a = bf16_to_f32(w[OB1 + j]);
    for (int i = 0; i < CPO_NFEAT; i++) a = fmaf(bf16_to_f32(w[OW1 + j * CPO_NFEAT + i]), x[i], a);
    h1[j] = a > 0.0f ? a : 0.0f;
  }
  for (int j = 0; j < CPO_HID; j++) {
    float a = bf16_to_f32(w[OB2 + j]);
    for (int i = 0; i < CPO_HID; i++) a = fmaf(bf16_to_f32(w[OW2 + j * CPO_HID + i]), h1[i], a);
    h2[j] = a > 0.0f ? a : 0.0f;
  }
  int best = 0;
  for (int c = 0; c < CPO_NCLS; c++) {
    float a = bf16_to_f32(w[OB3 + c]);
    for (int i = 0; i < CPO_HID; i++) a = fmaf(bf16_to_f32(w[OW3 + c * CPO_HID + i]), h2[i], a);
    logits[c] = a;
    if (a > logits[best]) best = c;
  }
  return best;
}

/* Mean softmax cross-entropy and its gradient, in double.  The forward pass
   uses the weights rounded to bf16 when round != 0 (as the GPU trainer does);
   the gradient is taken with respect to those weights. */
static double mlp_loss_grad_impl(const float* wf, const float* x, const int32_t* lab,
                                 int n, int rnd, double* grad) {
  double* w = (double*)malloc(sizeof(double) * CPO_NW);
  for (int i = 0; i < CPO_NW; i++) w[i] = rnd ? (double)round_bf16(wf[i]) : (double)wf[i];
  memset(grad, 0, sizeof(double) * CPO_NW);
  double loss = 0;
  for (int s = 0; s < n; s++) {
    const float* xs = x + (size_t)s * CPO_NFEAT;
    double z1[CPO_HID], h1[CPO_HID], z2[CPO_HID], h2[CPO_HID], z3[CPO_NCLS], p[CPO_NCLS];
    for (int j = 0; j < CPO_HID; j++) {
      double a = w[OB1 + j];
      for (int i = 0; i < CPO_NFEAT; i++) a += w[OW1 + j * CPO_NFEAT + i] * xs[i];
      z1[j] = a;
      h1[j] = a > 0 ? a : 0;
    }
    for (int j = 0; j < CPO_HID; j++) {
      double a = w[OB2 + j];
      for (int i = 0; i < CPO_HID; i++) a += w[OW2 + j * CPO_HID + i] * h1[i];
      z2[j] = a;
      h2[j] = a > 0 ? a : 0;
    }
    double mx = -INFINITY;
    for (int c = 0; c < CPO_NCLS; c++) {
      double a = w[OB3 + c];
      for (int i = 0; i < CPO_HID; i++) a += w[OW3 + c * CPO_HID + i] * h2[i];
      z3[c] = a;
      if (a > mx) mx = a;
    }
    double se = 0;
    for (int c = 0; c < CPO_NCLS; c++) se += exp(z3[c] - mx);
    for (int c = 0; c < CPO_NCLS; c++) p[c] = exp(z3[c] - mx) / se;
    loss += -(z3[lab[s]] - mx - log(se));
    double g3[CPO_NCLS], g2[CPO_HID], g1[CPO_HID];
    for (int c = 0; c < CPO_NCLS; c++) g3[c] = (p[c] - (c == lab[s] ? 1.0 : 0.0)) / n;
    for (int c = 0; c < CPO_NCLS; c++) {
      grad[OB3 + c] += g3[c];
      for (int i = 0; i < CPO_HID; i++) grad[OW3 + c * CPO_HID + i] += g3[c] * h2[i];
    }
    for (int i = 0; i < CPO_HID; i++) {
      double a = 0;
      for (int c = 0; c < CPO_NCLS; c++) a += g3[c] * w[OW3 + c * CPO_HID + i];
      g2[i] = z2[i] > 0 ? a : 0;
    }
    for (int j = 0; j < CPO_HID; j++) {
      grad[OB2 + j] += g2[j];
      for (int i = 0; i < CPO_HID; i++) grad[OW2 + j * CPO_HID + i] += g2[j] * h1[i];
    }
    for (int i = 0; i < CPO_HID; i++) {
      double a = 0;
      for (int j = 0; j < CPO_HID; j++) a += g2[j] * w[OW2 + j * CPO_HID + i];
      g1[i] = z1[i] > 0 ? a : 0;
    }
    for (int j = 0; j < CPO_HID; j++) {
      grad[OB1 + j] += g1[j];
      for (int i = 0; i < CPO_NFEAT; i++) grad[OW1 + j * CPO_NFEAT + i] += g1[j] * xs[i];
    }
  }
  free(w);
  return loss / n;
}

double cpo_mlp_loss_grad(const float* w, const float* x, const int32_t* labels,
                         int n, double* grad) {
  return mlp_loss_grad_impl(w, x, labels, n, 1, grad);
}
double cpo_mlp_loss_grad_exact(const float* w, const float* x, const int32_t* labels,
                               int n, double* grad) {
  return mlp_loss_grad_impl(w, x, labels, n, 0, grad);
}

/* ======================================================================
 * The additional lossless stage after Huffman coding (Sec. V names a
 * general-purpose lossless coder after the Huffman stage; Sec. VII-B shows
 * the long zero runs it exploits).  READING: the paper fixes no format; the
 * stage here is zero-byte elision over the stream body in independent
 * 4096-byte blocks.  The most frequent symbol of each canonical code gets
 * the all-zero codeword, so runs of it become zero bytes.
 * Container: the 256-byte header unchanged but for slot 31 = ZBE_TAG; one
 * 32-bit entry per block of the body (the bytes after the header): the
 * block's encoded length in bytes, bit 31 set when the block is elided; then
 * the encoded blocks in order.  An elided block of n bytes is a mask of
 * ceil(n/8) bytes (bit i, least significant first, set when byte i is
 * nonzero), then its nonzero bytes in order, then zero bytes up to a
 * multiple of 4.  A block is elided exactly when that form is shorter than
 * n; otherwise it is stored as it is.
 * ==================================================================== */
#define ZBE_BLOCK 4096
#define ZBE_TAG 0x315A4245ull /* "EBZ1" */

static size_t zbe_nblocks(size_t body) { return (body + ZBE_BLOCK - 1) / ZBE_BLOCK; }
static size_t pad4(size_t n) { return (n + 3) & ~(size_t)3; }

size_t cpo_zbe_bound(size_t inner_len) {
  size_t body = inner_len > HDR_BYTES ? inner_len - HDR_BYTES : 0;
  return HDR_BYTES + 4 * zbe_nblocks(body) + body;
}

int cpo_zbe_encode(const uint8_t* in, size_t len, uint8_t* out, size_t cap, size_t* out_len) {
  /* the header must name the stream's own length and carry no tag yet */
  if (!in || len < HDR_BYTES || len % 4 || get_u64(in + 8 * 30) != len || get_u64(in + 8 * 31) != 0)
    return CPO_EINVAL;
  size_t body = len - HDR_BYTES, nb = zbe_nblocks(body);
  size_t total = HDR_BYTES + 4 * nb;
  for (size_t b = 0; b < nb; b++) {
    const uint8_t* p = in + HDR_BYTES + b * ZBE_BLOCK;
    size_t n = body - b * ZBE_BLOCK < ZBE_BLOCK ? body - b * ZBE_BLOCK : ZBE_BLOCK, nnz = 0;
    for (size_t i = 0; i < n; i++) nnz += p[i] != 0;
    size_t e = pad4((n + 7) / 8 + nnz);
    total += e < n ? e : n;
  }
  *out_len = total;
  if (!out || total > cap) return CPO_ECAPACITY;
  memcpy(out, in, HDR_BYTES);
  set_u64(out + 8 * 31, ZBE_TAG);
  uint8_t* tab = out + HDR_BYTES;
  size_t o = HDR_BYTES + 4 * nb;
  for (size_t b = 0; b < nb; b++) {
    const uint8_t* p = in + HDR_BYTES + b * ZBE_BLOCK;
    size_t n = body - b * ZBE_BLOCK < ZBE_BLOCK ? body - b * ZBE_BLOCK : ZBE_BLOCK, nnz = 0;
    for (size_t i = 0; i < n; i++) nnz += p[i] != 0;
    size_t m = (n + 7) / 8, e = pad4(m + nnz);
    uint32_t entry;
    if (e < n) {
      memset(out + o, 0, e);
      size_t w = o + m;
      for (size_t i = 0; i < n; i++)
        if (p[i]) {
          out[o + i / 8] |= (uint8_t)(1u << (i % 8));
          out[w++] = p[i];
        }
      entry = (uint32_t)e | 0x80000000u;
      o += e;
    } else {
      memcpy(out + o, p, n);
      entry = (uint32_t)n;
      o += n;
    }
    for (int i = 0; i < 4; i++) tab[4 * b + i] = (uint8_t)(entry >> (8 * i));
  }
  return CPO_OK;
}

/* The inverse; `out` receives the inner stream (header slot 31 back to 0).
   Every length, mask bit, stored byte and padding byte is checked: a
   container that the encoder above cannot have written is corrupt. */
int cpo_zbe_decode(const uint8_t* in, size_t len, uint8_t* out, size_t cap, size_t* out_len) {
  if (!in || len < HDR_BYTES) return CPO_ECORRUPT;
  if (get_u64(in + 8 * 31) != ZBE_TAG) return CPO_ECORRUPT;
  uint64_t inner = get_u64(in + 8 * 30);
  if (inner < HDR_BYTES || inner % 4 || inner > ((uint64_t)1 << 40)) return CPO_ECORRUPT;
  size_t body = (size_t)inner - HDR_BYTES, nb = zbe_nblocks(body);
  if (len < HDR_BYTES + 4 * nb) return CPO_ECORRUPT;
  *out_len = (size_t)inner;
  if (!out || inner > cap) return CPO_ECAPACITY;
  memcpy(out, in, HDR_BYTES);
  set_u64(out + 8 * 31, 0);
  size_t o = HDR_BYTES + 4 * nb;
  for (size_t b = 0; b < nb; b++) {
    uint32_t entry = get_u32(in + HDR_BYTES + 4 * b);
    size_t n = body - b * ZBE_BLOCK < ZBE_BLOCK ? body - b * ZBE_BLOCK : ZBE_BLOCK;
    size_t e = entry & 0x7FFFFFFFu;
    uint8_t* q = out + HDR_BYTES + b * ZBE_BLOCK;
    if (e > len - o) return CPO_ECORRUPT;
    if (!(entry & 0x80000000u)) {
      if (e != n) return CPO_ECORRUPT;
      memcpy(q, in + o, n);
    } else {
      size_t m = (n + 7) / 8, nnz = 0;
      if (e < m) return CPO_ECORRUPT;
      for (size_t i = 0; i < 8 * m; i++) {
        int bit = (in[o + i / 8] >> (i % 8)) & 1;
        if (bit && i >= n) return CPO_ECORRUPT;
        nnz += (size_t)bit;
      }
      if (pad4(m + nnz) != e || e >= n) return CPO_ECORRUPT;
      size_t r = o + m;
      for (size_t i = 0; i < n; i++) {
        if ((in[o + i / 8] >> (i % 8)) & 1) {
          if (in[r] == 0) return CPO_ECORRUPT;
          q[i] = in[r++];
        } else {
          q[i] = 0;
        }
      }
      for (size_t i = r; i < o + e; i++)
        if (in[i] != 0) return CPO_ECORRUPT;
    }
    o += e;
  }
  return o == len ? CPO_OK : CPO_ECORRUPT;
}

/* ======================================================================
 * Compression (Alg. 3 with Alg. 4), in the blocked order: for each frame,
 * three colour phases; in phase c every TILE x TILE block with
 * (bx + by) mod 3 == c is processed, its vertices in raster order.  Blocks
 * of one colour share no face, so their order does not matter.
 * ==================================================================== */
typedef struct {
  int H, W, T, k, predictor, bt, K, tx, ty;
  int64_t eps, cx, sx, cy, sy;
  const int32_t *U0, *V0; /* original fixed point */
  int32_t *U, *V;         /* current values */
  const uint8_t* flags;
  const uint16_t* selw;
} ctx_t;

static const int DMAX2[2] = {0, 2};
static const int DMAX4[4] = {0, 1, 2, 4};

static int class_dmax(const ctx_t* c, int cls) {
  if (c->K == 4) return DMAX4[cls];
  return DMAX2[cls ? 1 : 0];
}

/* mode groups: frames [g bt, (g+1) bt); decided at max(g bt, 1) when that
   frame lies inside the group */
static int group_decided(int g, int bt, int T) {
  int td = g * bt > 1 ? g * bt : 1;
  int end = (g + 1) * bt < T ? (g + 1) * bt : T;
  return td < end;
}
static int decided_before(int g, int bt, int T) {
  int n = 0;
  for (int i = 0; i < g; i++) n += group_decided(i, bt, T);
  return n;
}
static int n_decided(int bt, int T) {
  int G = (T + bt - 1) / bt;
  return decided_before(G, bt, T);
}

static void sl_pred(const ctx_t* c, int t, int x, int y, int dmax, int64_t* pu, int64_t* pv) {
  size_t HW = (size_t)c->H * c->W;
  cpo_sl_predict(c->U + (size_t)(t - 1) * HW, c->V + (size_t)(t - 1) * HW, c->H, c->W, x, y,
                 c->cx, c->sx, c->cy, c->sy, dmax, NMAX, pu, pv);
}

/* Context-preserving micro-encoding of one block under one candidate
   (Sec. VI-B): quantize with the global bound, write reconstructed values
   back to a candidate buffer, collect statistics on the stride-2 grid. */
static int64_t trial_score(const ctx_t* c, int t, int x0, int y0, int x1, int y1,
                           int cls, int32_t* SU, int32_t* SV, int32_t* hist) {
  size_t HW = (size_t)c->H * c->W;
  int W = c->W;
  memset(hist, 0, sizeof(int32_t) * QSYM);
  int n = 0, L = 0;
  for (int y = y0; y < y1; y++)
    for (int x = x0; x < x1; x++) {
      size_t o = (size_t)y * W + x;
      SU[o] = c->U0[(size_t)t * HW + o];
      SV[o] = c->V0[(size_t)t * HW + o];
    }
  for (int y = y0; y < y1; y++)
    for (int x = x0; x < x1; x++) {
      size_t o = (size_t)y * W + x;
      int64_t pu, pv, ru, rv;
      if (cls == 0) {
        pu = lorenzo3(SU, c->U + (size_t)(t - 1) * HW, W, x, y, x0, y0);
        pv = lorenzo3(SV, c->V + (size_t)(t - 1) * HW, W, x, y, x0, y0);
      } else {
        sl_pred(c, t, x, y, class_dmax(c, cls), &pu, &pv);
      }
      int32_t qu = cpo_quantize(SU[o], pu, c->eps, &ru);
      int32_t qv = cpo_quantize(SV[o], pv, c->eps, &rv);
      SU[o] = (int32_t)ru;
      SV[o] = (int32_t)rv;
      if (((x - x0) % STRIDE) == 0 && ((y - y0) % STRIDE) == 0) {
        if (qu == 0) L++; else { hist[qu]++; n++; }
        if (qv == 0) L++; else { hist[qv]++; n++; }
      }
    }
  return cpo_score(hist, QSYM, n, L, c->K, c->bt);
}

/* Features of a block at its decision frame, each a Q8 ratio of integers. */
static float featq(int64_t num, int64_t den) {
  if (den <= 0) return 0.0f;
  int64_t q = floordiv(num * 256, den);
  q = clampi(q, -65536, 65536);
  return (float)q / 256.0f;
}

static void block_features(const ctx_t* c, int t, int x0, int y0, int x1, int y1, float* f) {
  size_t HW = (size_t)c->H * c->W;
  int W = c->W;
  const int32_t *Ut = c->U0 + (size_t)t * HW, *Vt = c->V0 + (size_t)t * HW;
  const int32_t *Up = c->U + (size_t)(t - 1) * HW, *Vp = c->V + (size_t)(t - 1) * HW;
  int64_t s = c->eps > 1 ? c->eps : 1;
  int64_t n = 0, m = 0, S0 = 0, S1 = 0, S2 = 0, Dm = 0, Ds = 0, nf = 0, S6 = 0, S7 = 0, Sx = 0, Sy = 0;
  const int64_t DCAP = (int64_t)1 << 40;
  for (int y = y0; y < y1; y++)
    for (int x = x0; x < x1; x++) {
      size_t o = (size_t)y * W + x;
      n++;
      S0 += iabs64((int64_t)Ut[o] - Up[o]) + iabs64((int64_t)Vt[o] - Vp[o]);
      int64_t lu = lorenzo3(Ut, Up, W, x, y, x0, y0), lv = lorenzo3(Vt, Vp, W, x, y, x0, y0);
      int64_t r3 = iabs64(Ut[o] - lu) + iabs64(Vt[o] - lv);
      S1 += r3;
      if (x + 1 < x1) S2 += iabs64((int64_t)Ut[o + 1] - Ut[o]) + iabs64((int64_t)Vt[o + 1] - Vt[o]);
      if (y + 1 < y1) S2 += iabs64((int64_t)Ut[o + W] - Ut[o]) + iabs64((int64_t)Vt[o + W] - Vt[o]);
      int64_t dx = clampi(disp(Up[o], c->cx, c->sx), -DCAP, DCAP);
      int64_t dy = clampi(disp(Vp[o], c->cy, c->sy), -DCAP, DCAP);
      int64_t d = imax64(iabs64(dx), iabs64(dy));
      if (d > Dm) Dm = d;
      Ds += d;
      Sx += dx;
      Sy += dy;
      nf += c->flags[(size_t)t * HW + o] ? 1 : 0;
      if (((x - x0) % 4) == 0 && ((y - y0) % 4) == 0) {
        int64_t pu, pv;
        sl_pred(c, t, x, y, 2, &pu, &pv);
        S6 += iabs64(Ut[o] - pu) + iabs64(Vt[o] - pv);
        S7 += r3;
        m++;
      }
    }
  f[0] = featq(S0, 2 * n * s);
  f[1] = featq(S1, 2 * n * s);
  f[2] = featq(S2, 2 * n * s);
  f[3] = featq(Dm, 65536);
  f[4] = featq(Ds, n * 65536);
  f[5] = featq(nf, n);
  f[6] = featq(S6, 2 * m * s);
  f[7] = featq(S7, 2 * m * s);
  f[8] = featq(Sx, n * 65536);
  f[9] = featq(Sy, n * 65536);
}

/* Switching rule (Sec. VI-B): the best semi-Lagrangian candidate (lowest
   score, ties to the lower class) replaces Lorenzo only when it improves the
   score by more than 0.3 %. */
int cpo_choose(const int64_t* R, int K) {
  int best = 1;
  for (int k = 2; k < K; k++)
    if (R[k] < R[best]) best = k;
  return 1000 * (R[0] - R[best]) > 3 * R[0] ? best : 0;
}

/* scores (may be NULL) receives the K trial scores of the exhaustive choice */
static int decide_mode(const ctx_t* c, int t, int x0, int y0, int x1, int y1,
                       int32_t* SU, int32_t* SV, int32_t* hist, float* feat, int64_t* scores) {
  block_features(c, t, x0, y0, x1, y1, feat);
  if (c->predictor == 4) {
    float lg[CPO_NCLS];
    return cpo_mlp_forward(c->selw, feat, lg);
  }
  int64_t R[4] = {0, 0, 0, 0};
  for (int k = 0; k < c->K; k++) R[k] = trial_score(c, t, x0, y0, x1, y1, k, SU, SV, hist);
  if (scores) memcpy(scores, R, sizeof(int64_t) * (size_t)c->K);
  return cpo_choose(R, c->K);
}

/* The predictor class that the decision of Sec. VI-B gives block (bx, by)
   of a decision frame, and the block's features, from that frame's original
   values (Ut, Vt), the previous frame's current (reconstructed) values (Up,
   Vp) and the frame's lossless flags: the steps of compression, run on a
   two-frame copy.  Needs a predictor with a choice (2, 3 or 4); returns the
   class, or CPO_EINVAL / CPO_ENOMEM. */
static int block_mode_impl(const int32_t* Ut, const int32_t* Vt, const int32_t* Up,
                           const int32_t* Vp, const uint8_t* flags_t, int H, int W, int bx,
                           int by, const cpo_options* opt, int k, int64_t eps, float* feat,
                           int64_t* scores);

int cpo_block_mode(const int32_t* Ut, const int32_t* Vt, const int32_t* Up, const int32_t* Vp,
                   const uint8_t* flags_t, int H, int W, int bx, int by, const cpo_options* opt,
                   int k, int64_t eps, float* feat) {
  return block_mode_impl(Ut, Vt, Up, Vp, flags_t, H, W, bx, by, opt, k, eps, feat, NULL);
}

/* The same decision, also returning the K trial scores (Sec. VI-B rate
   estimate, Q16 bits per sample) of the exhaustive choice; predictor 2 or 3. */
int cpo_block_scores(const int32_t* Ut, const int32_t* Vt, const int32_t* Up, const int32_t* Vp,
                     const uint8_t* flags_t, int H, int W, int bx, int by, const cpo_options* opt,
                     int k, int64_t eps, int64_t* scores) {
  if (!opt || !scores || opt->predictor < 2 || opt->predictor > 3) return CPO_EINVAL;
  return block_mode_impl(Ut, Vt, Up, Vp, flags_t, H, W, bx, by, opt, k, eps, NULL, scores);
}

static int block_mode_impl(const int32_t* Ut, const int32_t* Vt, const int32_t* Up,
                           const int32_t* Vp, const uint8_t* flags_t, int H, int W, int bx,
                           int by, const cpo_options* opt, int k, int64_t eps, float* feat,
                           int64_t* scores) {
  if (!opt || opt->predictor < 2 || opt->predictor > 4 || opt->mode_bt < 1) return CPO_EINVAL;
  if (opt->predictor == 4 && !opt->selector_w) return CPO_EINVAL;
  ctx_t c;
  memset(&c, 0, sizeof(c));
  c.H = H;
  c.W = W;
  c.T = 2;
  c.k = k;
  c.eps = eps;
  c.predictor = opt->predictor;
  c.bt = opt->mode_bt;
  c.K = opt->predictor == 2 ? 2 : 4;
  c.tx = (W + TILE - 1) / TILE;
  c.ty = (H + TILE - 1) / TILE;
  c.selw = opt->selector_w;
  if (bx < 0 || by < 0 || bx >= c.tx || by >= c.ty) return CPO_EINVAL;
  cpo_sl_factor(opt->dt_dx, k, &c.cx, &c.sx);
  cpo_sl_factor(opt->dt_dy, k, &c.cy, &c.sy);
  size_t HW = (size_t)H * W;
  int32_t* F0 = (int32_t*)malloc(4 * HW * sizeof(int32_t));
  int32_t* F = (int32_t*)malloc(4 * HW * sizeof(int32_t));
  uint8_t* fl = (uint8_t*)calloc(2 * HW, 1);
  int32_t* SU = (int32_t*)malloc(HW * sizeof(int32_t));
  int32_t* SV = (int32_t*)malloc(HW * sizeof(int32_t));
  int32_t* hist = (int32_t*)malloc(QSYM * sizeof(int32_t));
  int r = CPO_ENOMEM;
  if (F0 && F && fl && SU && SV && hist) {
    /* frame 0 of the copy is the previous frame, frame 1 the decision frame */
    memcpy(F0, Up, HW * sizeof(int32_t));
    memcpy(F0 + HW, Ut, HW * sizeof(int32_t));
    memcpy(F0 + 2 * HW, Vp, HW * sizeof(int32_t));
    memcpy(F0 + 3 * HW, Vt, HW * sizeof(int32_t));
    memcpy(F, F0, 4 * HW * sizeof(int32_t));
    memcpy(fl + HW, flags_t, HW);
    c.U0 = F0;
    c.V0 = F0 + 2 * HW;
    c.U = F;
    c.V = F + 2 * HW;
    c.flags = fl;
    int x0 = bx * TILE, y0 = by * TILE;
    int x1 = x0 + TILE < W ? x0 + TILE : W, y1 = y0 + TILE < H ? y0 + TILE : H;
    float f[CPO_NFEAT];
    r = decide_mode(&c, 1, x0, y0, x1, y1, SU, SV, hist, f, scores);
    if (feat) memcpy(feat, f, sizeof(f));
  }
  free(F0);
  free(F);
  free(fl);
  free(SU);
  free(SV);
  free(hist);
  return r;
}

/* largest stream, plain or in the container of the lossless stage */
size_t cpo_compress_bound(int H, int W, int T) {
  size_t N = (size_t)H * W * T;
  size_t nch = (N + CHUNK - 1) / CHUNK, nq = 2 * N, nqch = (nq + CHUNK - 1) / CHUNK;
  size_t nd = (size_t)T * ((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE);
  return cpo_zbe_bound(HDR_BYTES + 4 * ((nd * 2 + 31) / 32) + (4 + 4 * XSYM) + 4 * nch +
                       4 * ((N * MAXLEN + 31) / 32 + nch) + (4 + 4 * QSYM) + 4 * nqch +
                       4 * ((nq * MAXLEN + 31) / 32 + nqch) + 8 * N);
}

int cpo_compress_ex(const float* field, int H, int W, int T, double eb,
                    const cpo_options* opt, uint8_t* out, size_t cap,
                    size_t* out_len, int32_t* xi_out, uint8_t* xcode_out,
                    uint32_t* qcode_out, uint8_t* modes_out, float* feats_out,
                    size_t* nblocks_out) {
  cpo_options dflt = {2, 1, 0, 0, 1.0, 1.0, NULL};
  if (!opt) opt = &dflt;
  if (opt->predictor < 0 || opt->predictor > 4 || opt->mode_bt < 1) return CPO_EINVAL;
  if (opt->backend < 0 || opt->backend > 1) return CPO_EINVAL;
  uint8_t* inner = NULL;
  if (opt->predictor == 4 && !opt->selector_w) return CPO_EINVAL;
  if (!(opt->dt_dx >= 0.0) || !(opt->dt_dy >= 0.0) || !isfinite(opt->dt_dx) || !isfinite(opt->dt_dy))
    return CPO_EINVAL;
  ctx_t c;
  memset(&c, 0, sizeof(c));
  double eb_abs;
  int st = cpo_params(field, H, W, T, opt->eb_mode, eb, &c.k, &eb_abs, &c.eps);
  if (st) return st;
  c.H = H;
  c.W = W;
  c.T = T;
  c.predictor = opt->predictor;
  c.bt = opt->mode_bt;
  c.K = opt->predictor == 2 ? 2 : (opt->predictor >= 3 ? 4 : 1);
  c.tx = (W + TILE - 1) / TILE;
  c.ty = (H + TILE - 1) / TILE;
  c.selw = opt->selector_w;
  cpo_sl_factor(opt->dt_dx, c.k, &c.cx, &c.sx);
  cpo_sl_factor(opt->dt_dy, c.k, &c.cy, &c.sy);
  size_t N = (size_t)H * W * T, HW = (size_t)H * W;
  int32_t* F0 = (int32_t*)malloc(2 * N * sizeof(int32_t));
  int32_t* F = (int32_t*)malloc(2 * N * sizeof(int32_t));
  uint32_t* masks = (uint32_t*)malloc(N * sizeof(uint32_t));
  uint8_t* flags = (uint8_t*)malloc(N);
  uint8_t* xcode = (uint8_t*)malloc(N);
  uint16_t* qu = (uint16_t*)calloc(N, sizeof(uint16_t));
  uint16_t* qv = (uint16_t*)calloc(N, sizeof(uint16_t));
  int32_t* SU = (int32_t*)malloc(HW * sizeof(int32_t));
  int32_t* SV = (int32_t*)malloc(HW * sizeof(int32_t));
  int32_t* hist = (int32_t*)malloc(QSYM * sizeof(int32_t));
  int nd_groups = n_decided(c.bt, T);
  size_t nblk = c.K > 1 ? (size_t)nd_groups * c.ty * c.tx : 0;
  uint8_t* modes = (uint8_t*)calloc(nblk ? nblk : 1, 1);
  uint16_t* qsym = NULL;
  uint16_t* xs = NULL;
  buf_t sec[8];
  memset(sec, 0, sizeof(sec));
  if (!F0 || !F || !masks || !flags || !xcode || !qu || !qv || !SU || !SV || !hist || !modes) {
    st = CPO_ENOMEM;
    goto done;
  }
  /* Alg. 3: fixed point, then the critical face set on the original field */
  cpo_to_fixed(field, 2 * N, c.k, F0);
  memcpy(F, F0, 2 * N * sizeof(int32_t));
  c.U0 = F0;
  c.V0 = F0 + N;
  c.U = F;
  c.V = F + N;
  cpo_face_masks(c.U0, c.V0, H, W, T, masks);
  cpo_lossless_flags(masks, H, W, T, flags);
  c.flags = flags;

  for (int t = 0; t < T; t++) {
    int g = t / c.bt;
    int decided = c.K > 1 && group_decided(g, c.bt, T);
    int td = g * c.bt > 1 ? g * c.bt : 1;
    for (int col = 0; col < 3; col++)
      for (int by = 0; by < c.ty; by++)
        for (int bx = 0; bx < c.tx; bx++) {
          if ((bx + by) % 3 != col) continue;
          int x0 = bx * TILE, y0 = by * TILE;
          int x1 = x0 + TILE < W ? x0 + TILE : W, y1 = y0 + TILE < H ? y0 + TILE : H;
          int cls = 0;
          if (t >= 1 && c.predictor == 1) cls = 1;
          if (t >= 1 && decided) {
            size_t bi = ((size_t)decided_before(g, c.bt, T) * c.ty + by) * c.tx + bx;
            if (t == td) {
              float feat[CPO_NFEAT];
              modes[bi] = (uint8_t)decide_mode(&c, t, x0, y0, x1, y1, SU, SV, hist, feat, NULL);
              if (feats_out) memcpy(feats_out + bi * CPO_NFEAT, feat, sizeof(feat));
            }
            cls = modes[bi];
          }
          for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
              size_t v = vid(H, W, x, y, t);
              int64_t xi = cpo_vertex_bound(c.U, c.V, flags, H, W, T, x, y, t, c.eps);
              int32_t code = cpo_xi_code(c.eps, xi);
              if (xi_out) xi_out[v] = (int32_t)xi;
              xcode[v] = (uint8_t)code;
              if (code == XLOSSLESS) continue; /* current value stays original */
              int64_t xt = c.eps >> code, pu, pv, ru, rv;
              if (cls == 0) {
                pu = lorenzo3(c.U + t * HW, t > 0 ? c.U + (t - 1) * HW : NULL, W, x, y, x0, y0);
                pv = lorenzo3(c.V + t * HW, t > 0 ? c.V + (t - 1) * HW : NULL, W, x, y, x0, y0);
              } else {
                sl_pred(&c, t, x, y, class_dmax(&c, cls), &pu, &pv);
              }
              qu[v] = (uint16_t)cpo_quantize(c.U0[v], pu, xt, &ru);
              qv[v] = (uint16_t)cpo_quantize(c.V0[v], pv, xt, &rv);
              c.U[v] = (int32_t)ru;
              c.V[v] = (int32_t)rv;
            }
        }
  }

  /* lossless_comp of Alg. 3: bound codes, residual codes, raw values */
  {
    size_t nq = 0, nraw = 0;
    for (size_t v = 0; v < N; v++) {
      if (xcode[v] == XLOSSLESS) nraw += 2;
      else { nq += 2; nraw += (qu[v] == 0) + (qv[v] == 0); }
    }
    xs = (uint16_t*)malloc((N ? N : 1) * sizeof(uint16_t));
    qsym = (uint16_t*)malloc((nq ? nq : 1) * sizeof(uint16_t));
    for (size_t v = 0; v < N; v++) xs[v] = xcode[v];
    size_t j = 0;
    for (size_t v = 0; v < N; v++)
      if (xcode[v] != XLOSSLESS) { qsym[j++] = qu[v]; qsym[j++] = qv[v]; }
    /* section 0: mode bits, LSB-first in 32-bit words */
    int mb = c.K == 4 ? 2 : (c.K == 2 ? 1 : 0);
    size_t nbits = nblk * (size_t)mb, nw = (nbits + 31) / 32;
    uint32_t* mw = (uint32_t*)calloc(nw ? nw : 1, sizeof(uint32_t));
    for (size_t b = 0; b < nblk; b++)
      for (int i = 0; i < mb; i++)
        if ((modes[b] >> i) & 1) mw[(b * mb + i) / 32] |= 1u << ((b * mb + i) % 32);
    for (size_t i = 0; i < nw; i++) put_u32(&sec[0], mw[i]);
    free(mw);
    st = huff_encode(xs, N, XSYM, &sec[1], &sec[2], &sec[3]);
    if (!st) st = huff_encode(qsym, nq, QSYM, &sec[4], &sec[5], &sec[6]);
    if (st) goto done;
    for (size_t v = 0; v < N; v++) {
      const float* fu = field + v;
      const float* fv = field + N + v;
      uint32_t bu, bv;
      memcpy(&bu, fu, 4);
      memcpy(&bv, fv, 4);
      if (xcode[v] == XLOSSLESS) { put_u32(&sec[7], bu); put_u32(&sec[7], bv); }
      else {
        if (qu[v] == 0) put_u32(&sec[7], bu);
        if (qv[v] == 0) put_u32(&sec[7], bv);
      }
    }
    size_t total = HDR_BYTES;
    for (int i = 0; i < 8; i++) total += sec[i].len;
    *out_len = total;
    uint8_t* dst = out;
    if (opt->backend == 1) {
      /* the Huffman stream is built aside, then the lossless stage writes out */
      inner = (uint8_t*)malloc(total);
      if (!inner) { st = CPO_ENOMEM; goto done; }
      dst = inner;
    } else if (total > cap || !out) {
      st = CPO_ECAPACITY;
      goto done;
    }
    uint8_t* h = dst;
    memset(h, 0, HDR_BYTES);
    uint64_t eb_bits;
    memcpy(&eb_bits, &eb_abs, 8);
    uint64_t slots[HDR_SLOTS] = {
        MAGIC | (VERSION << 32), (uint64_t)H, (uint64_t)W, (uint64_t)T,
        (uint64_t)(int64_t)c.k, eb_bits, (uint64_t)c.eps, QR, TILE,
        (uint64_t)c.predictor, (uint64_t)c.bt, (uint64_t)c.K,
        (uint64_t)c.cx, (uint64_t)c.sx, (uint64_t)c.cy, (uint64_t)c.sy,
        NMAX, CHUNK, MAXLEN, STRIDE,
        sec[0].len, sec[1].len, sec[2].len, sec[3].len,
        sec[4].len, sec[5].len, sec[6].len, sec[7].len,
        nq, nraw, total, 0};
    for (int i = 0; i < HDR_SLOTS; i++) set_u64(h + 8 * i, slots[i]);
    size_t o = HDR_BYTES;
    for (int i = 0; i < 8; i++) {
      if (sec[i].len) memcpy(dst + o, sec[i].p, sec[i].len);
      o += sec[i].len;
    }
    if (opt->backend == 1) {
      st = cpo_zbe_encode(inner, total, out, cap, out_len);
      if (st) goto done;
    }
  }
  if (xcode_out) memcpy(xcode_out, xcode, N);
  if (qcode_out)
    for (size_t v = 0; v < N; v++) qcode_out[v] = (uint32_t)qu[v] | ((uint32_t)qv[v] << 16);
  if (modes_out && nblk) memcpy(modes_out, modes, nblk);
  if (nblocks_out) *nblocks_out = nblk;
done:
  free(inner);
  for (int i = 0; i < 8; i++) free(sec[i].p);
  free(F0); free(F); free(masks); free(flags); free(xcode); free(qu); free(qv);
  free(SU); free(SV); free(hist); free(modes); free(qsym); free(xs);
  return st;
}

int cpo_compress(const float* field, int H, int W, int T, double eb,
                 const cpo_options* opt, uint8_t* out, size_t cap, size_t* out_len) {
  return cpo_compress_ex(field, H, W, T, eb, opt, out, cap, out_len, NULL, NULL,
                         NULL, NULL, NULL, NULL);
}

/* ======================================================================
 * Decompression: the inverse of the steps above.
 * ==================================================================== */
int cpo_stream_info(const uint8_t* b, size_t len, cpo_info* info) {
  if (!b || len < HDR_BYTES) return CPO_ECORRUPT;
  uint64_t s[HDR_SLOTS];
  for (int i = 0; i < HDR_SLOTS; i++) s[i] = get_u64(b + 8 * i);
  if (s[0] != (MAGIC | (VERSION << 32))) return CPO_ECORRUPT;
  if (s[1] < 2 || s[2] < 2 || s[3] < 1 || s[1] > (1u << 20) || s[2] > (1u << 20) || s[3] > (1u << 20))
    return CPO_ECORRUPT;
  if (s[7] != QR || s[8] != TILE || s[16] != NMAX || s[17] != CHUNK || s[18] != MAXLEN || s[19] != STRIDE)
    return CPO_ECORRUPT;
  int64_t k = (int64_t)s[4];
  if (k < -80 || k > 120) return CPO_ECORRUPT;
  if (s[6] > 8388607 || s[9] > 4 || s[10] < 1 || s[10] > 1024) return CPO_ECORRUPT;
  uint64_t K = s[9] == 2 ? 2 : (s[9] >= 3 ? 4 : 1);
  if (s[11] != K || s[13] > 62 || s[15] > 62 || s[12] > 2147483647u || s[14] > 2147483647u)
    return CPO_ECORRUPT;
  if (s[31] != 0 && s[31] != ZBE_TAG) return CPO_ECORRUPT;
  const int zbe = s[31] == ZBE_TAG;
  uint64_t total = HDR_BYTES;
  for (int i = 20; i < 28; i++) {
    if (s[i] % 4 || s[i] > ((uint64_t)1 << 40)) return CPO_ECORRUPT;
    total += s[i];
  }
  if (total != s[30]) return CPO_ECORRUPT;
  /* a plain stream holds every section; a container at least its table */
  if (zbe ? len < HDR_BYTES + 4 * zbe_nblocks(total - HDR_BYTES) : total > len) return CPO_ECORRUPT;
  info->H = (int32_t)s[1];
  info->W = (int32_t)s[2];
  info->T = (int32_t)s[3];
  info->k = (int32_t)k;
  memcpy(&info->eb_abs, &s[5], 8);
  info->eps = (int64_t)s[6];
  info->R = (int32_t)s[7];
  info->predictor = (int32_t)s[9];
  info->mode_bt = (int32_t)s[10];
  info->K = (int32_t)K;
  info->cx = (int64_t)s[12];
  info->sx = (int64_t)s[13];
  info->cy = (int64_t)s[14];
  info->sy = (int64_t)s[15];
  info->n_q = s[28];
  info->n_raw = s[29];
  info->total_len = s[30];
  info->backend = zbe;
  return CPO_OK;
}

/* Every fixed-point value a valid stream yields, stored or reconstructed,
   lies strictly inside (-2^25, 2^25); anything else marks a corrupt stream. */
static int fits_25(int64_t v) { return v < (1 << 25) && v > -(1 << 25); }

int cpo_decompress(const uint8_t* b, size_t len, float* field) {
  cpo_info in;
  int st = cpo_stream_info(b, len, &in);
  if (st) return st;
  if (in.backend) {
    uint8_t* inner = (uint8_t*)malloc(in.total_len);
    size_t il = 0;
    if (!inner) return CPO_ENOMEM;
    st = cpo_zbe_decode(b, len, inner, in.total_len, &il);
    if (!st) st = cpo_decompress(inner, il, field);
    free(inner);
    return st;
  }
  int H = in.H, W = in.W, T = in.T;
  size_t N = (size_t)H * W * T, HW = (size_t)H * W;
  uint64_t sl[8];
  size_t off[8];
  size_t o = HDR_BYTES;
  for (int i = 0; i < 8; i++) {
    sl[i] = get_u64(b + 8 * (20 + i));
    off[i] = o;
    o += sl[i];
  }
  ctx_t c;
  memset(&c, 0, sizeof(c));
  c.H = H; c.W = W; c.T = T; c.k = in.k; c.eps = in.eps; c.predictor = in.predictor;
  c.bt = in.mode_bt; c.K = in.K; c.cx = in.cx; c.sx = in.sx; c.cy = in.cy; c.sy = in.sy;
  c.tx = (W + TILE - 1) / TILE;
  c.ty = (H + TILE - 1) / TILE;
  int nd_groups = n_decided(c.bt, T);
  size_t nblk = c.K > 1 ? (size_t)nd_groups * c.ty * c.tx : 0;
  int mb = c.K == 4 ? 2 : (c.K == 2 ? 1 : 0);
  if (sl[0] != 4 * ((nblk * mb + 31) / 32)) return CPO_ECORRUPT;
  if (in.n_q > 2 * N || in.n_raw > 2 * N) return CPO_ECORRUPT;
  if (sl[7] != 4 * in.n_raw) return CPO_ECORRUPT;
  uint16_t* xs = (uint16_t*)malloc(N * sizeof(uint16_t));
  uint16_t* qs = (uint16_t*)malloc((in.n_q ? in.n_q : 1) * sizeof(uint16_t));
  int32_t* F = (int32_t*)malloc(2 * N * sizeof(int32_t));
  size_t* qofs = (size_t*)malloc(N * sizeof(size_t));
  size_t* rofs = (size_t*)malloc(N * sizeof(size_t));
  uint8_t* modes = (uint8_t*)calloc(nblk ? nblk : 1, 1);
  if (!xs || !qs || !F || !qofs || !rofs || !modes) { st = CPO_ENOMEM; goto done; }
  for (size_t i = 0; i < nblk; i++)
    for (int j = 0; j < mb; j++) {
      size_t bit = i * mb + j;
      uint32_t w = get_u32(b + off[0] + 4 * (bit / 32));
      modes[i] |= (uint8_t)(((w >> (bit % 32)) & 1u) << j);
    }
  for (size_t i = 0; i < nblk; i++)
    if (c.K == 2 && modes[i] > 1) { st = CPO_ECORRUPT; goto done; }
  st = huff_decode(b + off[1], sl[1], b + off[2], sl[2], b + off[3], sl[3], XSYM, N, xs);
  if (st) goto done;
  st = huff_decode(b + off[4], sl[4], b + off[5], sl[5], b + off[6], sl[6], QSYM, in.n_q, qs);
  if (st) goto done;
  {
    size_t nq = 0, nr = 0;
    for (size_t v = 0; v < N; v++) {
      if (xs[v] > XLOSSLESS) { st = CPO_ECORRUPT; goto done; }
      qofs[v] = nq;
      rofs[v] = nr;
      if (xs[v] == XLOSSLESS) nr += 2;
      else {
        if (nq + 2 > in.n_q) { st = CPO_ECORRUPT; goto done; }
        nr += (qs[nq] == 0) + (qs[nq + 1] == 0);
        nq += 2;
      }
      if (xs[v] != XLOSSLESS && (c.eps >> xs[v]) < 1) { st = CPO_ECORRUPT; goto done; }
    }
    if (nq != in.n_q || nr != in.n_raw) { st = CPO_ECORRUPT; goto done; }
  }
  c.U = F;
  c.V = F + N;
  for (int t = 0; t < T; t++) {
    int g = t / c.bt;
    int decided = c.K > 1 && group_decided(g, c.bt, T);
    for (int by = 0; by < c.ty; by++)
      for (int bx = 0; bx < c.tx; bx++) {
        int x0 = bx * TILE, y0 = by * TILE;
        int x1 = x0 + TILE < W ? x0 + TILE : W, y1 = y0 + TILE < H ? y0 + TILE : H;
        int cls = 0;
        if (t >= 1 && c.predictor == 1) cls = 1;
        if (t >= 1 && decided)
          cls = modes[((size_t)decided_before(g, c.bt, T) * c.ty + by) * c.tx + bx];
        for (int y = y0; y < y1; y++)
          for (int x = x0; x < x1; x++) {
            size_t v = vid(H, W, x, y, t);
            const uint8_t* raw = b + off[7] + 4 * rofs[v];
            float fu, fv;
            if (xs[v] == XLOSSLESS) {
              uint32_t a = get_u32(raw), bb = get_u32(raw + 4);
              memcpy(&fu, &a, 4);
              memcpy(&fv, &bb, 4);
              if (!isfinite(fu) || !isfinite(fv)) { st = CPO_ECORRUPT; goto done; }
              cpo_to_fixed(&fu, 1, c.k, &c.U[v]);
              cpo_to_fixed(&fv, 1, c.k, &c.V[v]);
              if (!fits_25(c.U[v]) || !fits_25(c.V[v])) { st = CPO_ECORRUPT; goto done; }
              field[v] = fu;
              field[N + v] = fv;
              continue;
            }
            int64_t xt = c.eps >> xs[v], pu, pv;
            if (cls == 0) {
              pu = lorenzo3(c.U + t * HW, t > 0 ? c.U + (t - 1) * HW : NULL, W, x, y, x0, y0);
              pv = lorenzo3(c.V + t * HW, t > 0 ? c.V + (t - 1) * HW : NULL, W, x, y, x0, y0);
            } else {
              sl_pred(&c, t, x, y, class_dmax(&c, cls), &pu, &pv);
            }
            int64_t pred[2] = {pu, pv};
            int32_t* plane[2] = {c.U, c.V};
            int ri = 0;
            for (int comp = 0; comp < 2; comp++) {
              uint16_t q = qs[qofs[v] + comp];
              float outv;
              if (q == 0) {
                uint32_t a = get_u32(raw + 4 * ri++);
                memcpy(&outv, &a, 4);
                if (!isfinite(outv)) { st = CPO_ECORRUPT; goto done; }
                cpo_to_fixed(&outv, 1, c.k, &plane[comp][v]);
                if (!fits_25(plane[comp][v])) { st = CPO_ECORRUPT; goto done; }
              } else {
                int64_t r = pred[comp] + (int64_t)((int)q - QR) * (2 * xt + 1);
                if (!fits_25(r)) { st = CPO_ECORRUPT; goto done; }
                plane[comp][v] = (int32_t)r;
                outv = (float)ldexp((double)r, -c.k);
              }
              field[(size_t)comp * N + v] = outv;
            }
          }
      }
  }
done:
  free(xs); free(qs); free(F); free(qofs); free(rofs); free(modes);
  return st;
}

/* ======================================================================
 * Verification (Sec. IV-A and the evaluation metrics): false cases per
 * slice faces (FC_t) and cross-slab faces (FC_s), max error and PSNR.
 * ==================================================================== */
int cpo_verify(const float* a, const float* bfield, int H, int W, int T, int k,
               uint64_t* fc_t, uint64_t* fc_s, double* max_err, double* psnr) {
  if (H < 2 || W < 2 || T < 1) return CPO_EINVAL;
  size_t N = (size_t)H * W * T;
  if (!fits_24(a, 2 * N, k) || !fits_24(bfield, 2 * N, k)) return CPO_EINVAL;
  int32_t* A = (int32_t*)malloc(2 * N * sizeof(int32_t));
  int32_t* B = (int32_t*)malloc(2 * N * sizeof(int32_t));
  uint32_t* ma = (uint32_t*)malloc(N * sizeof(uint32_t));
  uint32_t* mb = (uint32_t*)malloc(N * sizeof(uint32_t));
  if (!A || !B || !ma || !mb) { free(A); free(B); free(ma); free(mb); return CPO_ENOMEM; }
  cpo_to_fixed(a, 2 * N, k, A);
  cpo_to_fixed(bfield, 2 * N, k, B);
  cpo_face_masks(A, A + N, H, W, T, ma);
  cpo_face_masks(B, B + N, H, W, T, mb);
  uint64_t ft = 0, fs = 0;
  for (size_t v = 0; v < N; v++)
    for (int f = 0; f < 12; f++) {
      uint32_t ca = (ma[v] >> f) & 1, cb = (mb[v] >> f) & 1;
      uint32_t sa = (ma[v] >> (12 + f)) & 1, sb = (mb[v] >> (12 + f)) & 1;
      int bad = ca != cb || (ca && sa != sb);
      if (bad) { if (f < 2) ft++; else fs++; }
    }
  double me = 0, se = 0, mn = INFINITY, mx = -INFINITY;
  for (size_t i = 0; i < 2 * N; i++) {
    double d = fabs((double)a[i] - (double)bfield[i]);
    if (d > me) me = d;
    se += d * d;
    if (a[i] < mn) mn = a[i];
    if (a[i] > mx) mx = a[i];
  }
  double mse = se / (double)(2 * N);
  *fc_t = ft;
  *fc_s = fs;
  *max_err = me;
  *psnr = mse > 0 ? 20.0 * log10(mx - mn) - 10.0 * log10(mse) : INFINITY;
  free(A); free(B); free(ma); free(mb);
  return CPO_OK;
}

/* ======================================================================
 * Lemma 1 and the track count: every tetrahedron must have 0 or 2 crossed
 * faces; the two crossed faces of a tetrahedron are joined, and trajectories
 * are the connected components of crossed faces.
 * ==================================================================== */
static size_t uf_find(size_t* p, size_t a) {
  while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; }
  return a;
}

/* face index (owner*12 + type) of three vertices given as (x,y,t) */
static int64_t face_of(int H, int W, const int* X, const int* Y, const int* Tt) {
  int ord[3] = {0, 1, 2};
  size_t g[3];
  for (int i = 0; i < 3; i++) g[i] = vid(H, W, X[i], Y[i], Tt[i]);
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (g[ord[j]] < g[ord[i]]) { int tmp = ord[i]; ord[i] = ord[j]; ord[j] = tmp; }
  int o = ord[0];
  for (int f = 0; f < 12; f++) {
    int ok = 1;
    for (int i = 0; i < 3; i++) {
      int q = ord[i];
      if (X[q] - X[o] != FV[f][i][0] || Y[q] - Y[o] != FV[f][i][1] || Tt[q] - Tt[o] != FV[f][i][2]) ok = 0;
    }
    if (ok) return (int64_t)g[o] * 12 + f;
  }
  return -1;
}

int cpo_tracks(const float* field, int H, int W, int T, int k, uint64_t* bad_tets,
               uint64_t* n_tracks) {
  size_t N = (size_t)H * W * T;
  int32_t* F = (int32_t*)malloc(2 * N * sizeof(int32_t));
  uint32_t* m = (uint32_t*)malloc(N * sizeof(uint32_t));
  size_t* par = (size_t*)malloc(12 * N * sizeof(size_t));
  if (!F || !m || !par) { free(F); free(m); free(par); return CPO_ENOMEM; }
  cpo_to_fixed(field, 2 * N, k, F);
  cpo_face_masks(F, F + N, H, W, T, m);
  for (size_t i = 0; i < 12 * N; i++) par[i] = i;
  uint64_t bad = 0;
  /* triangles of each quad, vertices in spatial index order */
  static const int TRI[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
  for (int t = 0; t + 1 < T; t++)
    for (int y = 0; y + 1 < H; y++)
      for (int x = 0; x + 1 < W; x++)
        for (int tr = 0; tr < 2; tr++) {
          int ax = x + TRI[tr][0][0], ay = y + TRI[tr][0][1];
          int bx = x + TRI[tr][1][0], by = y + TRI[tr][1][1];
          int cx = x + TRI[tr][2][0], cy = y + TRI[tr][2][1];
          /* the three tetrahedra of the prism split, (x, y, t) per vertex */
          int tets[3][4][3] = {
              {{ax, ay, t}, {bx, by, t}, {cx, cy, t}, {cx, cy, t + 1}},
              {{ax, ay, t}, {bx, by, t}, {bx, by, t + 1}, {cx, cy, t + 1}},
              {{ax, ay, t}, {ax, ay, t + 1}, {bx, by, t + 1}, {cx, cy, t + 1}}};
          for (int q = 0; q < 3; q++) {
            int64_t crossed[4];
            int nc = 0;
            for (int skip = 0; skip < 4; skip++) {
              int X[3], Y[3], Tt[3], j = 0;
              for (int i = 0; i < 4; i++)
                if (i != skip) { X[j] = tets[q][i][0]; Y[j] = tets[q][i][1]; Tt[j] = tets[q][i][2]; j++; }
              int64_t fi = face_of(H, W, X, Y, Tt);
              if (fi < 0) { free(F); free(m); free(par); return CPO_EINVAL; }
              if (m[fi / 12] & (1u << (fi % 12))) crossed[nc++] = fi;
            }
            if (nc != 0 && nc != 2) bad++;
            if (nc == 2) {
              size_t ra = uf_find(par, (size_t)crossed[0]), rb = uf_find(par, (size_t)crossed[1]);
              if (ra != rb) par[ra] = rb;
            }
          }
        }
  uint64_t nt = 0;
  for (size_t g = 0; g < N; g++)
    for (int f = 0; f < 12; f++)
      if ((m[g] & (1u << f)) && uf_find(par, g * 12 + f) == g * 12 + f) nt++;
  *bad_tets = bad;
  *n_tracks = nt;
  free(F); free(m); free(par);
  return CPO_OK;
}
