/*
 * san_check.c — a driver that runs every entry point of the CPU oracle on
 * small synthetic fields and on corrupted streams, for a build with the
 * address and undefined-behaviour sanitizers (test infrastructure; built and
 * run by the test suite, never by the library).
 *
 * Fields: a few analytic swirls (values of the kind Sec. VII uses) plus a
 * deterministic hash noise, and small-integer fields full of ties.  Streams:
 * every predictor, plain and in the container of the zero-byte-elision
 * stage, then single-bit flips, truncations, and stored raw values replaced
 * by huge, tiny, negative-zero and non-finite floats; every call
 * must return without a sanitizer report (decoding may succeed or fail).
 * Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cpo.h"

static uint64_t st_hash(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static double noise(uint64_t i) { return (double)(st_hash(i) >> 11) / 9007199254740992.0 - 0.5; }

static void swirl_field(float* f, int H, int W, int T, int seed) {
  size_t N = (size_t)H * W * T;
  for (int t = 0; t < T; t++)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++) {
        double u = 0, v = 0;
        for (int k = 0; k < 3; k++) {
          double cx = W * (0.2 + 0.3 * k) + 0.31 * t, cy = H * (0.3 + 0.2 * k) - 0.17 * t;
          double dx = x - cx, dy = y - cy, r2 = dx * dx + dy * dy + 1e-9;
          double g = (k == 1 ? -1.5 : 1.0) * (1.0 - exp(-r2 / 9.0)) / r2;
          u -= dy * g;
          v += dx * g;
        }
        size_t i = ((size_t)t * H + y) * W + x;
        f[i] = (float)(u + 1e-3 * noise(i + 7919u * (uint64_t)seed));
        f[N + i] = (float)(v + 1e-3 * noise(i + N + 7919u * (uint64_t)seed));
      }
}

static void int_field(float* f, int H, int W, int T, int seed) {
  size_t N = (size_t)H * W * T;
  for (size_t i = 0; i < 2 * N; i++) f[i] = (float)((int)(st_hash(i * 31 + (uint64_t)seed) % 3) - 1);
}

static int failures = 0;
#define CHECK(c, msg)                                         \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "san_check: %s (line %d)\n", msg, __LINE__); \
      failures++;                                             \
    }                                                         \
  } while (0)

static uint64_t rd64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}

/* decode a (possibly corrupt) stream; any status is fine, a sanitizer
   report is not */
static void try_decode(const uint8_t* b, size_t len) {
  cpo_info in;
  if (cpo_stream_info(b, len, &in) != CPO_OK) return;
  size_t n = 2 * (size_t)in.H * in.W * in.T;
  if (n > ((size_t)1 << 26)) return;
  float* out = (float*)malloc(n * sizeof(float));
  if (!out) return;
  (void)cpo_decompress(b, len, out);
  free(out);
}

static void roundtrip(const float* f, int H, int W, int T, double eb, int pred, int bt,
                      const uint16_t* selw, int corrupt, int backend) {
  cpo_options o;
  memset(&o, 0, sizeof(o));
  o.backend = backend;
  o.predictor = pred;
  o.mode_bt = bt;
  o.dt_dx = 0.37;
  o.dt_dy = 0.29;
  o.selector_w = selw;
  size_t cap = cpo_compress_bound(H, W, T), len = 0;
  uint8_t* b = (uint8_t*)malloc(cap);
  float* g = (float*)malloc(2 * (size_t)H * W * T * sizeof(float));
  CHECK(b && g, "allocation");
  int st = cpo_compress(f, H, W, T, eb, &o, b, cap, &len);
  CHECK(st == CPO_OK, "compress");
  if (st == CPO_OK) {
    CHECK(cpo_decompress(b, len, g) == CPO_OK, "decompress");
    int k;
    double ea;
    int64_t eps;
    CHECK(cpo_params(f, H, W, T, 0, eb, &k, &ea, &eps) == CPO_OK, "params");
    uint64_t ft, fs;
    double me, ps;
    CHECK(cpo_verify(f, g, H, W, T, k, &ft, &fs, &me, &ps) == CPO_OK, "verify");
    CHECK(ft == 0 && fs == 0 && me <= ea, "guarantee");
    uint64_t bad, ntr;
    CHECK(cpo_tracks(g, H, W, T, k, &bad, &ntr) == CPO_OK && bad == 0, "tracks");
    size_t cnt = 0;
    int ex = cpo_extract(g, H, W, T, k, NULL, 0, &cnt);
    CHECK(ex == CPO_OK || ex == CPO_ECAPACITY, "extract count");
    if (corrupt) {
      uint8_t* c = (uint8_t*)malloc(len);
      const size_t step = 8 * len / 120 + 1;
      for (size_t bit = 0; bit < 8 * len; bit += step + (size_t)(st_hash(bit) % 7)) {
        memcpy(c, b, len);
        c[bit / 8] ^= (uint8_t)(1u << (bit % 8));
        try_decode(c, len);
      }
      for (size_t cut = 0; cut < len; cut += 1 + len / 23) try_decode(b, cut);
      /* stored raw values (the last section) replaced by hostile floats */
      size_t raw_off = 256;
      for (int i = 0; i < 7; i++) raw_off += (size_t)rd64(b + 8 * (20 + i));
      const uint32_t hostile[] = {0x7F7FFFFFu, 0xFF7FFFFFu, 0x7F800000u, 0x7FC00001u,
                                  0x80000000u, 0x00000001u, 0x4F000000u, 0xCF000001u};
      for (size_t o2 = raw_off; o2 + 4 <= len && o2 < raw_off + 64; o2 += 4)
        for (size_t h = 0; h < sizeof(hostile) / sizeof(hostile[0]); h++) {
          memcpy(c, b, len);
          memcpy(c + o2, &hostile[h], 4);
          try_decode(c, len);
        }
      free(c);
    }
  }
  free(b);
  free(g);
}

int main(void) {
  const int H = 23, W = 37, T = 4;
  size_t N = (size_t)H * W * T;
  float* f = (float*)malloc(2 * N * sizeof(float));
  uint16_t selw[5124];
  for (int i = 0; i < 5124; i++) selw[i] = (uint16_t)(0x3C00u + (st_hash((uint64_t)i) % 0x400u) - 0x200u);
  swirl_field(f, H, W, T, 1);
  const double ebs[3] = {1e-1, 1e-2, 1e-3};
  for (int pred = 0; pred <= 4; pred++)
    for (int e = 0; e < 3; e++)
      roundtrip(f, H, W, T, ebs[e], pred, pred >= 3 ? 2 : 1, selw, e == 1 && pred >= 2, e == 2 || pred == 3);
  int_field(f, H, W, T, 5);
  for (int pred = 0; pred <= 3; pred++) roundtrip(f, H, W, T, 0.25, pred, 1, selw, pred == 2, pred & 1);
  /* extraction and verification with a grid too fine for the values */
  size_t cnt;
  uint64_t ft, fs;
  double me, ps;
  CHECK(cpo_extract(f, H, W, T, 40, NULL, 0, &cnt) == CPO_EINVAL, "extract rejects a 2^24 overflow");
  CHECK(cpo_verify(f, f, H, W, T, 40, &ft, &fs, &me, &ps) == CPO_EINVAL, "verify rejects a 2^24 overflow");
  free(f);
  if (failures) {
    fprintf(stderr, "san_check: %d failures\n", failures);
    return 1;
  }
  printf("san_check ok\n");
  return 0;
}
