// api.cpp — C-ABI entry points of libcptraj: argument checks, the host-side
// parameter derivation, the per-device scratch arena, kernel orchestration
// and the stream layout.
//
// Stream layout (little-endian): a 256-byte header of 32 64-bit slots
// followed by eight sections, each a whole number of 32-bit words:
//   0 predictor classes of the decided blocks, bit-packed LSB-first
//   1 bound-code codebook      (count, then symbol | length << 16 per used symbol)
//   2 bound-code chunk table   (bits per 1024-symbol chunk)
//   3 bound-code bitstream     (MSB-first words, every chunk word-aligned)
//   4..6 the same three for the residual codes
//   7 raw float32 values of lossless vertices and unpredictable components
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cpt_device.hpp"
#include "cptraj.h"
#include "launch.hpp"

using namespace cpt;

namespace {

thread_local std::string g_err;

cpt_status fail(cpt_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(CPT_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int HDR_SLOTS = 32;
constexpr size_t HDR_BYTES = 8 * HDR_SLOTS;
constexpr uint64_t MAGIC = 0x31545043ull;  // "CPT1"
constexpr uint64_t VERSION = 1;
constexpr int STRIDE = 2;

// ------------------------------------------------------------ arena
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  uint64_t* host = nullptr;  // pinned staging for small readbacks
  int64_t* tlog = nullptr;   // entropy table floor(h log2 h 2^16)
  std::mutex mu;

  size_t off(size_t bytes) {
    size_t o = (used + 255) & ~(size_t)255;
    used = o + bytes;
    return o;
  }
};

std::mutex g_arena_mu;
std::vector<Arena*> g_arenas;

Arena* arena_for_device(cpt_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *st = fail(CPT_EHIP, "hipGetDevice failed");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_arena_mu);
  if ((int)g_arenas.size() <= dev) g_arenas.resize(dev + 1, nullptr);
  if (!g_arenas[dev]) {
    Arena* a = new Arena();
    if (hipHostMalloc((void**)&a->host, 4096, hipHostMallocDefault) != hipSuccess) {
      *st = fail(CPT_ENOMEM, "pinned staging allocation failed");
      delete a;
      return nullptr;
    }
    std::vector<int64_t> t(1025, 0);
    for (int h = 2; h <= 1024; h++) t[h] = (int64_t)std::floor((double)h * std::log2((double)h) * 65536.0);
    if (hipMalloc((void**)&a->tlog, t.size() * sizeof(int64_t)) != hipSuccess ||
        hipMemcpy(a->tlog, t.data(), t.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
      *st = fail(CPT_ENOMEM, "table allocation failed");
      return nullptr;
    }
    g_arenas[dev] = a;
  }
  *st = CPT_OK;
  return g_arenas[dev];
}

// Scratch layout for one field of N vertices.
struct Bufs {
  int2* cur;
  uint8_t *edges, *flags, *xcode, *modes;
  uint32_t *masks, *qcode, *nonll, *qofs, *rcnt, *rofs;
  uint16_t *qsym, *xs, *qs;
  uint32_t *xbits, *xwords, *xwofs, *qbits, *qwords, *qwofs, *part;
  uint32_t *tot, *xhist, *qhist, *used, *err, *xcb, *qcb, *xlut, *qlut;
  int* range;
  HuffTables *xt, *qt;
  unsigned long long* fc;
  double* cpart;
};

cpt_status carve(Arena& A, size_t N, size_t nblk, Bufs& b) {
  A.used = 0;
  size_t nchx = (N + CHUNK - 1) / CHUNK + 1, nchq = (2 * N + CHUNK - 1) / CHUNK + 1;
  struct Item {
    void** p;
    size_t bytes;
  };
  std::vector<Item> items = {
      {(void**)&b.cur, 8 * N},        {(void**)&b.edges, N},          {(void**)&b.flags, N},
      {(void**)&b.xcode, N},          {(void**)&b.modes, nblk + 1},   {(void**)&b.masks, 4 * N},
      {(void**)&b.qcode, 4 * N},      {(void**)&b.nonll, 4 * N},      {(void**)&b.qofs, 4 * N},
      {(void**)&b.rcnt, 4 * N},       {(void**)&b.rofs, 4 * N},       {(void**)&b.qsym, 4 * N},
      {(void**)&b.xs, 2 * N},         {(void**)&b.qs, 4 * N},         {(void**)&b.xbits, 4 * nchx},
      {(void**)&b.xwords, 4 * nchx},  {(void**)&b.xwofs, 4 * nchx},   {(void**)&b.qbits, 4 * nchq},
      {(void**)&b.qwords, 4 * nchq},  {(void**)&b.qwofs, 4 * nchq},
      {(void**)&b.part, 4 * (scan_partials_size(2 * N) + 16)},
      {(void**)&b.tot, 64},           {(void**)&b.xhist, 4 * 32},     {(void**)&b.qhist, 4 * QSYM},
      {(void**)&b.used, 16},          {(void**)&b.err, 16},           {(void**)&b.xcb, 4 * 32},
      {(void**)&b.qcb, 4 * (QSYM + 4)}, {(void**)&b.xlut, 4 << MAXLEN}, {(void**)&b.qlut, 4 << MAXLEN},
      {(void**)&b.range, 64},         {(void**)&b.xt, sizeof(HuffTables)}, {(void**)&b.qt, sizeof(HuffTables)},
      {(void**)&b.fc, 16},            {(void**)&b.cpart, 16 * (compare_partials(N) + 1)},
  };
  std::vector<size_t> offs;
  for (auto& it : items) offs.push_back(A.off(it.bytes));
  if (A.used > A.cap) {
    if (A.base) {
      if (hipDeviceSynchronize() != hipSuccess) return fail(CPT_EHIP, "synchronize before arena growth failed");
      (void)hipFree(A.base);
      A.base = nullptr;
      A.cap = 0;
    }
    size_t want = A.used + A.used / 8;
    if (hipMalloc((void**)&A.base, want) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CPT_ENOMEM, "scratch arena allocation of " + std::to_string(want) + " bytes failed");
    }
    A.cap = want;
  }
  for (size_t i = 0; i < items.size(); i++) *items[i].p = A.base + offs[i];
  return CPT_OK;
}

// ---------------------------------------------------- host-side derivations
// Fixed point 2^k with k = 23 - e for max|x| = m 2^e, m in [0.5, 1), capped at
// 120; eps' = floor(eb_abs 2^k - 1/2), at most 2^23 - 1.
cpt_status derive_params(double mn, double mx, double ma, int eb_mode, double eb, int* k, double* ea,
                         int64_t* eps) {
  if (ma >= std::ldexp(1.0, 100)) return fail(CPT_EINVAL, "field magnitude of 2^100 or more is not supported");
  int e = 0;
  if (ma > 0) std::frexp(ma, &e);
  int kk = 23 - e;
  if (kk > 120) kk = 120;
  double a;
  if (eb_mode == 0) {
    if (!(eb > 0.0 && eb <= 0.5)) return fail(CPT_EINVAL, "relative error bound must be in (0, 0.5]");
    a = eb * (mx - mn);
  } else if (eb_mode == 1) {
    if (!(eb > 0.0) || !std::isfinite(eb)) return fail(CPT_EINVAL, "absolute error bound must be positive");
    a = eb;
  } else {
    return fail(CPT_EINVAL, "eb_mode must be 0 or 1");
  }
  double s = std::floor(std::ldexp(a, kk) - 0.5);
  int64_t ep = 0;
  if (s > 0) ep = s >= 8388607.0 ? 8388607 : (int64_t)s;
  *k = kk;
  *ea = a;
  *eps = ep;
  return CPT_OK;
}

// displacement factor c / 2^s ~ dt_dx 2^(16-k), c < 2^31
void sl_factor(double dt_dx, int k, int64_t* c, int64_t* s) {
  double f = std::ldexp(dt_dx, 16 - k);
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
  std::frexp(f, &e);
  int sh = 31 - e;
  if (sh > 62) sh = 62;
  int64_t cc = (int64_t)std::nearbyint(std::ldexp(f, sh));
  if (cc >= 2147483648LL) {
    cc = 1073741824LL;
    sh -= 1;
  }
  *c = cc;
  *s = sh;
}

bool group_decided(int g, int bt, int T) {
  int td = g * bt > 1 ? g * bt : 1;
  int end = (g + 1) * bt < T ? (g + 1) * bt : T;
  return td < end;
}
int decided_before(int g, int bt, int T) {
  int n = 0;
  for (int i = 0; i < g; i++) n += group_decided(i, bt, T) ? 1 : 0;
  return n;
}

float key_to_float(int key) {
  int s = key >= 0 ? key : (key ^ 0x7FFFFFFF);
  float f;
  std::memcpy(&f, &s, 4);
  return f;
}

cpt_status check_dims(int H, int W, int T) {
  if (H < 2 || W < 2 || T < 1) return fail(CPT_EINVAL, "need H >= 2, W >= 2, T >= 1");
  if (H > 32768 || W > 32768) return fail(CPT_EINVAL, "H and W must be at most 32768");
  if ((double)H * W * T >= 2147483648.0) return fail(CPT_EINVAL, "H*W*T must be below 2^31");
  return CPT_OK;
}

struct Range {
  double mn, mx, ma;
};

cpt_status field_range(const float* f, size_t n, Bufs& b, Arena& A, hipStream_t s, Range* r) {
  launch_range(f, n, b.range, s);
  HIPCHK(hipMemcpyAsync(A.host, b.range, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int* h = (const int*)A.host;
  if (h[3]) return fail(CPT_EINVAL, "field contains NaN or Inf");
  r->mn = (double)key_to_float(h[0]);
  r->mx = (double)key_to_float(h[1]);
  float fa;
  std::memcpy(&fa, &h[2], 4);
  r->ma = (double)fa;
  return CPT_OK;
}

// ------------------------------------------------------- small kernels
struct Header {
  uint64_t s[HDR_SLOTS];
};

__global__ void k_write_header(Header h, uint8_t* out) {
  int i = threadIdx.x;
  if (i < HDR_SLOTS) {
    uint32_t* o = (uint32_t*)out;
    o[2 * i] = (uint32_t)(h.s[i] & 0xFFFFFFFFu);
    o[2 * i + 1] = (uint32_t)(h.s[i] >> 32);
  }
}

__global__ void k_pack_modes(const uint8_t* modes, size_t nblk, int mb, uint32_t* out, size_t nwords) {
  size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  uint32_t v = 0;
  for (int b = 0; b < 32; b++) {
    size_t bit = w * 32 + b;
    size_t blk = bit / mb;
    int k = (int)(bit % mb);
    if (blk < nblk && ((modes[blk] >> k) & 1)) v |= 1u << b;
  }
  out[w] = v;
}

__global__ void k_unpack_modes(const uint32_t* in, size_t nblk, int mb, int K, uint8_t* modes, uint32_t* err) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblk) return;
  uint32_t v = 0;
  for (int k = 0; k < mb; k++) {
    size_t bit = i * mb + k;
    v |= ((in[bit / 32] >> (bit % 32)) & 1u) << k;
  }
  if ((int)v >= K) atomicOr(err, 256u);
  modes[i] = (uint8_t)v;
}

unsigned nb256(size_t n) { return (unsigned)((n + 255) / 256); }

int mode_bits(int K) { return K == 4 ? 2 : (K == 2 ? 1 : 0); }

// ------------------------------------------------------------ kernel timing
// When enabled, launches of the main kernel families are bracketed by HIP
// events on the caller's stream; elapsed times are harvested after the
// call's final synchronisation.
enum { FAM_PHASE = 0, FAM_MODES = 1, FAM_RECON = 2, FAM_DECODE = 3, FAM_ENCODE = 4, FAM_EXTRACT = 5, NFAM = 6 };

struct Timing {
  bool on = false;
  std::mutex mu;
  std::vector<hipEvent_t> pool;
  struct Rec {
    int fam;
    hipEvent_t a, b;
    uint64_t units;
  };
  std::vector<Rec> pending;
  double ms[NFAM] = {0};
  uint64_t launches[NFAM] = {0}, units[NFAM] = {0};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void harvest() {
    for (auto& r : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.fam] += t;
        launches[r.fam] += 1;
        units[r.fam] += r.units;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
};
Timing g_tim;

struct TimeScope {
  int fam;
  uint64_t units;
  hipStream_t s;
  hipEvent_t a = nullptr;
  TimeScope(int f, uint64_t u, hipStream_t st) : fam(f), units(u), s(st) {
    if (!g_tim.on) return;
    std::lock_guard<std::mutex> lk(g_tim.mu);
    a = g_tim.get();
    (void)hipEventRecord(a, s);
  }
  ~TimeScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_tim.mu);
    hipEvent_t b = g_tim.get();
    (void)hipEventRecord(b, s);
    g_tim.pending.push_back({fam, a, b, units});
  }
};

void harvest_timing() {
  if (!g_tim.on) return;
  std::lock_guard<std::mutex> lk(g_tim.mu);
  g_tim.harvest();
}

// vertices of colour c in one frame
uint64_t colour_vertices(int H, int W, int c) {
  int tx = (W + TILE - 1) / TILE, ty = (H + TILE - 1) / TILE;
  uint64_t n = 0;
  for (int by = 0; by < ty; by++)
    for (int bx = 0; bx < tx; bx++)
      if ((bx + by) % 3 == c) n += (uint64_t)std::min(TILE, W - bx * TILE) * std::min(TILE, H - by * TILE);
  return n;
}

// ------------------------------------------------------------ compress
cpt_status compress_impl(const float* field, int H, int W, int T, double eb, const cpt_options* opt_in,
                         uint8_t* out, size_t cap, size_t* out_len, int32_t* xi_dbg, uint8_t* xcode_dbg,
                         uint32_t* qcode_dbg, uint8_t* modes_dbg, float* feats_dbg, size_t* nblocks,
                         hipStream_t s) {
  if (!field || !out_len) return fail(CPT_EINVAL, "null field or out_len");
  cpt_status st = check_dims(H, W, T);
  if (st) return st;
  cpt_options opt{sizeof(cpt_options), 0, CPT_PRED_MIX2, 1, 1.0, 1.0, nullptr};
  if (opt_in) {
    if (opt_in->struct_size != sizeof(cpt_options)) return fail(CPT_EINVAL, "cpt_options.struct_size mismatch");
    opt = *opt_in;
  }
  if (opt.predictor < 0 || opt.predictor > 4) return fail(CPT_EINVAL, "unknown predictor");
  if (opt.mode_bt < 1 || opt.mode_bt > 1024) return fail(CPT_EINVAL, "mode_bt must be in 1..1024");
  if (opt.predictor == CPT_PRED_LEARNED && !opt.selector_w) return fail(CPT_EINVAL, "learned predictor needs selector_w");
  if (!(opt.dt_dx >= 0.0) || !(opt.dt_dy >= 0.0) || !std::isfinite(opt.dt_dx) || !std::isfinite(opt.dt_dy))
    return fail(CPT_EINVAL, "dt_dx and dt_dy must be finite and non-negative");
  if (out && ((uintptr_t)out & 3)) return fail(CPT_EINVAL, "out must be 4-byte aligned");

  const size_t N = (size_t)H * W * T;
  const int tx = (W + TILE - 1) / TILE, ty = (H + TILE - 1) / TILE;
  const int K = opt.predictor == 2 ? 2 : (opt.predictor >= 3 ? 4 : 1);
  const int bt = opt.mode_bt;
  const int G = (T + bt - 1) / bt;
  const size_t ndec = K > 1 ? (size_t)decided_before(G, bt, T) : 0;
  const size_t nblk = ndec * (size_t)tx * ty;

  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  Bufs b;
  st = carve(A, N, nblk, b);
  if (st) return st;

  Range r;
  st = field_range(field, 2 * N, b, A, s, &r);
  if (st) return st;
  FieldParams p;
  double eb_abs;
  int64_t eps;
  st = derive_params(r.mn, r.mx, r.ma, opt.eb_mode, eb, &p.k, &eb_abs, &eps);
  if (st) return st;
  p.H = H;
  p.W = W;
  p.T = T;
  p.eps = (int)eps;
  p.tx = tx;
  p.ty = ty;
  p.predictor = opt.predictor;
  p.K = K;
  p.bt = bt;
  sl_factor(opt.dt_dx, p.k, &p.cx, &p.sx);
  sl_factor(opt.dt_dy, p.k, &p.cy, &p.sy);

  // Alg. 3: fixed point, crossed faces of the original field, lossless flags
  launch_convert(field, N, p.k, b.cur, s);
  {
    TimeScope ts(FAM_EXTRACT, N, s);
    launch_masks(b.cur, H, W, T, b.edges, b.masks, s);
  }
  launch_flags(b.masks, H, W, T, b.flags, s);

  uint64_t cv[3] = {colour_vertices(H, W, 0), colour_vertices(H, W, 1), colour_vertices(H, W, 2)};
  for (int t = 0; t < T; t++) {
    int g = t / bt;
    bool dec = K > 1 && group_decided(g, bt, T);
    int td = g * bt > 1 ? g * bt : 1;
    size_t gbase = dec ? (size_t)decided_before(g, bt, T) * tx * ty : 0;
    if (dec && t == td) {
      TimeScope ts(FAM_MODES, (uint64_t)H * W, s);
      launch_modes(b.cur, b.flags, p, t, gbase, A.tlog, opt.selector_w, b.modes, feats_dbg, s);
    }
    long long mbase = (dec && t >= 1) ? (long long)gbase : -1;
    for (int c = 0; c < 3; c++) {
      TimeScope ts(FAM_PHASE, cv[c], s);
      launch_phase(b.cur, b.flags, b.modes, mbase, p, t, c, b.xcode, b.qcode, xi_dbg, s);
    }
  }

  // lossless_comp of Alg. 3: Huffman codes of both code streams, raw values
  launch_hist(b.xcode, b.qcode, N, b.xhist, b.qhist, nullptr, nullptr, s);
  launch_codebooks(b.xhist, b.qhist, b.xt, b.qt, b.xcb, b.qcb, b.used, s);
  launch_raw_count(b.xcode, b.qcode, N, b.rcnt, b.nonll, s);
  launch_scan(b.nonll, N, b.qofs, b.part, b.tot + 0, s);
  launch_scan(b.rcnt, N, b.rofs, b.part, b.tot + 1, s);
  HIPCHK(hipMemcpyAsync(A.host, b.tot, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(A.host + 1, b.used, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint32_t* h32 = (const uint32_t*)A.host;
  const size_t n_nonll = h32[0], n_raw = h32[1], used_x = h32[2], used_q = h32[3];
  const size_t nq = 2 * n_nonll;
  const size_t nchx = (N + CHUNK - 1) / CHUNK, nchq = (nq + CHUNK - 1) / CHUNK;
  launch_gather_q(b.xcode, b.qcode, b.qofs, N, b.qsym, s);
  launch_chunk_bits_x(b.xcode, N, b.xt, b.xbits, b.xwords, s);
  launch_chunk_bits_q(b.qsym, nq, b.qt, b.qbits, b.qwords, s);
  launch_scan(b.xwords, nchx, b.xwofs, b.part, b.tot + 2, s);
  launch_scan(b.qwords, nchq, b.qwofs, b.part, b.tot + 3, s);
  HIPCHK(hipMemcpyAsync(A.host, b.tot + 2, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const size_t words_x = h32[0], words_q = h32[1];

  const int mb = mode_bits(K);
  const size_t mwords = (nblk * mb + 31) / 32;
  uint64_t sec[8] = {4 * mwords,  4 * (1 + used_x), 4 * nchx, 4 * words_x,
                     4 * (1 + used_q), 4 * nchq,    4 * words_q, 4 * n_raw};
  size_t off[8], total = HDR_BYTES;
  for (int i = 0; i < 8; i++) {
    off[i] = total;
    total += sec[i];
  }
  *out_len = total;
  if (nblocks) *nblocks = nblk;
  if (!out || total > cap) {
    HIPCHK(hipStreamSynchronize(s));
    return fail(CPT_ECAPACITY, "output capacity " + std::to_string(cap) + " below stream length " +
                                   std::to_string(total));
  }
  if (mwords) k_pack_modes<<<nb256(mwords), 256, 0, s>>>(b.modes, nblk, mb, (uint32_t*)(out + off[0]), mwords);
  HIPCHK(hipMemcpyAsync(out + off[1], b.xcb, sec[1], hipMemcpyDeviceToDevice, s));
  if (sec[2]) HIPCHK(hipMemcpyAsync(out + off[2], b.xbits, sec[2], hipMemcpyDeviceToDevice, s));
  {
    TimeScope ts(FAM_ENCODE, N, s);
    launch_encode_x(b.xcode, N, b.xt, b.xwofs, (uint32_t*)(out + off[3]), s);
  }
  HIPCHK(hipMemcpyAsync(out + off[4], b.qcb, sec[4], hipMemcpyDeviceToDevice, s));
  if (sec[5]) HIPCHK(hipMemcpyAsync(out + off[5], b.qbits, sec[5], hipMemcpyDeviceToDevice, s));
  {
    TimeScope ts(FAM_ENCODE, nq, s);
    launch_encode_q(b.qsym, nq, b.qt, b.qwofs, (uint32_t*)(out + off[6]), s);
  }
  launch_raw(field, b.xcode, b.qcode, b.rofs, N, (uint32_t*)(out + off[7]), s);
  Header hd;
  uint64_t ebits;
  std::memcpy(&ebits, &eb_abs, 8);
  uint64_t slots[HDR_SLOTS] = {MAGIC | (VERSION << 32), (uint64_t)H, (uint64_t)W, (uint64_t)T,
                               (uint64_t)(int64_t)p.k, ebits, (uint64_t)eps, (uint64_t)QR, (uint64_t)TILE,
                               (uint64_t)p.predictor, (uint64_t)bt, (uint64_t)K, (uint64_t)p.cx, (uint64_t)p.sx,
                               (uint64_t)p.cy, (uint64_t)p.sy, (uint64_t)NMAX, (uint64_t)CHUNK, (uint64_t)MAXLEN,
                               (uint64_t)STRIDE, sec[0], sec[1], sec[2], sec[3], sec[4], sec[5], sec[6], sec[7],
                               nq, n_raw, total, 0};
  std::memcpy(hd.s, slots, sizeof(slots));
  k_write_header<<<1, 64, 0, s>>>(hd, out);
  if (xcode_dbg) HIPCHK(hipMemcpyAsync(xcode_dbg, b.xcode, N, hipMemcpyDeviceToDevice, s));
  if (qcode_dbg) HIPCHK(hipMemcpyAsync(qcode_dbg, b.qcode, 4 * N, hipMemcpyDeviceToDevice, s));
  if (modes_dbg && nblk) HIPCHK(hipMemcpyAsync(modes_dbg, b.modes, nblk, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  harvest_timing();
  return CPT_OK;
}

// ----------------------------------------------------------- stream info
uint64_t rd64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
  return v;
}

struct Parsed {
  cpt_info info;
  int64_t cx, sx, cy, sy;
  uint64_t sec[8];
};

cpt_status parse_header(const uint8_t* h, size_t len, Parsed* P) {
  if (len < HDR_BYTES) return fail(CPT_ECORRUPT, "stream shorter than its header");
  uint64_t s[HDR_SLOTS];
  for (int i = 0; i < HDR_SLOTS; i++) s[i] = rd64(h + 8 * i);
  if (s[0] != (MAGIC | (VERSION << 32))) return fail(CPT_ECORRUPT, "bad magic or version");
  if (s[1] < 2 || s[2] < 2 || s[3] < 1 || s[1] > 32768 || s[2] > 32768 || s[3] > (1u << 20))
    return fail(CPT_ECORRUPT, "bad dimensions");
  if ((double)s[1] * (double)s[2] * (double)s[3] >= 2147483648.0) return fail(CPT_ECORRUPT, "too many vertices");
  if (s[7] != (uint64_t)QR || s[8] != (uint64_t)TILE || s[16] != (uint64_t)NMAX || s[17] != (uint64_t)CHUNK ||
      s[18] != (uint64_t)MAXLEN || s[19] != (uint64_t)STRIDE)
    return fail(CPT_ECORRUPT, "unsupported format constants");
  int64_t k = (int64_t)s[4];
  if (k < -80 || k > 120) return fail(CPT_ECORRUPT, "bad exponent");
  if (s[6] > 8388607 || s[9] > 4 || s[10] < 1 || s[10] > 1024) return fail(CPT_ECORRUPT, "bad parameters");
  uint64_t K = s[9] == 2 ? 2 : (s[9] >= 3 ? 4 : 1);
  if (s[11] != K || s[13] > 62 || s[15] > 62 || s[12] > 2147483647u || s[14] > 2147483647u)
    return fail(CPT_ECORRUPT, "bad predictor parameters");
  uint64_t total = HDR_BYTES;
  for (int i = 0; i < 8; i++) {
    if (s[20 + i] % 4 || s[20 + i] > len) return fail(CPT_ECORRUPT, "bad section length");
    total += s[20 + i];
    P->sec[i] = s[20 + i];
  }
  if (total != s[30] || total > len) return fail(CPT_ECORRUPT, "section lengths do not add up");
  cpt_info& I = P->info;
  I.H = (int32_t)s[1];
  I.W = (int32_t)s[2];
  I.T = (int32_t)s[3];
  I.k = (int32_t)k;
  std::memcpy(&I.eb_abs, &s[5], 8);
  I.eps = (int64_t)s[6];
  I.predictor = (int32_t)s[9];
  I.mode_bt = (int32_t)s[10];
  I.K = (int32_t)K;
  I.R = (int32_t)s[7];
  I.n_q = s[28];
  I.n_raw = s[29];
  I.total_len = s[30];
  P->cx = (int64_t)s[12];
  P->sx = (int64_t)s[13];
  P->cy = (int64_t)s[14];
  P->sy = (int64_t)s[15];
  return CPT_OK;
}

// ---------------------------------------------------------- decompress
cpt_status decompress_impl(const uint8_t* bytes, size_t len, float* field, hipStream_t s) {
  if (!bytes || !field) return fail(CPT_EINVAL, "null pointer");
  if ((uintptr_t)bytes & 3) return fail(CPT_EINVAL, "stream must be 4-byte aligned");
  if (len < HDR_BYTES) return fail(CPT_ECORRUPT, "stream shorter than its header");
  cpt_status st;
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  HIPCHK(hipMemcpyAsync(A.host, bytes, HDR_BYTES, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  Parsed P;
  st = parse_header((const uint8_t*)A.host, len, &P);
  if (st) return st;
  const cpt_info& I = P.info;
  const int H = I.H, W = I.W, T = I.T;
  const size_t N = (size_t)H * W * T;
  const int tx = (W + TILE - 1) / TILE, ty = (H + TILE - 1) / TILE;
  const int bt = I.mode_bt, K = I.K;
  const int G = (T + bt - 1) / bt;
  const size_t ndec = K > 1 ? (size_t)decided_before(G, bt, T) : 0;
  const size_t nblk = ndec * (size_t)tx * ty;
  const int mb = mode_bits(K);
  const size_t nq = I.n_q, n_raw = I.n_raw;
  const size_t nchx = (N + CHUNK - 1) / CHUNK, nchq = (nq + CHUNK - 1) / CHUNK;
  if (P.sec[0] != 4 * ((nblk * mb + 31) / 32)) return fail(CPT_ECORRUPT, "mode section size");
  if (nq > 2 * N || n_raw > 2 * N || (nq & 1)) return fail(CPT_ECORRUPT, "symbol counts");
  if (P.sec[7] != 4 * n_raw) return fail(CPT_ECORRUPT, "raw section size");
  if (P.sec[2] != 4 * nchx || P.sec[5] != 4 * nchq) return fail(CPT_ECORRUPT, "chunk table size");
  if (P.sec[1] < 4 || P.sec[4] < 4) return fail(CPT_ECORRUPT, "codebook size");
  Bufs b;
  st = carve(A, N, nblk, b);
  if (st) return st;
  size_t off[8], o = HDR_BYTES;
  for (int i = 0; i < 8; i++) {
    off[i] = o;
    o += P.sec[i];
  }
  const uint32_t* w = (const uint32_t*)bytes;
  auto sec32 = [&](int i) { return w + off[i] / 4; };
  launch_zero_u32(b.err, 4, s);
  if (nblk) k_unpack_modes<<<nb256(nblk), 256, 0, s>>>(sec32(0), nblk, mb, K, b.modes, b.err);
  launch_build_lut(sec32(1), P.sec[1] / 4, XSYM, b.xlut, b.err, s);
  launch_build_lut(sec32(4), P.sec[4] / 4, QSYM, b.qlut, b.err, s);
  launch_words_from_bits(sec32(2), nchx, b.xwords, s);
  launch_scan(b.xwords, nchx, b.xwofs, b.part, b.tot + 0, s);
  {
    TimeScope ts(FAM_DECODE, N, s);
    launch_decode(b.xlut, sec32(2), b.xwofs, sec32(3), P.sec[3] / 4, N, XSYM, b.xs, b.err, s);
  }
  launch_dec_nonll(b.xs, N, b.nonll, s);
  launch_scan(b.nonll, N, b.qofs, b.part, b.tot + 1, s);
  launch_words_from_bits(sec32(5), nchq, b.qwords, s);
  launch_scan(b.qwords, nchq, b.qwofs, b.part, b.tot + 2, s);
  {
    TimeScope ts(FAM_DECODE, nq, s);
    launch_decode(b.qlut, sec32(5), b.qwofs, sec32(6), P.sec[6] / 4, nq, QSYM, b.qs, b.err, s);
  }
  launch_dec_counts(b.xs, b.qs, b.qofs, N, nq, (int)I.eps, b.rcnt, b.err, s);
  launch_scan(b.rcnt, N, b.rofs, b.part, b.tot + 3, s);
  HIPCHK(hipMemcpyAsync(A.host, b.tot, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(A.host + 2, b.err, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint32_t* h32 = (const uint32_t*)A.host;
  if (h32[4]) return fail(CPT_ECORRUPT, "stream failed a device check (code " + std::to_string(h32[4]) + ")");
  if (h32[0] != P.sec[3] / 4 || h32[2] != P.sec[6] / 4) return fail(CPT_ECORRUPT, "bitstream sizes");
  if (2 * (size_t)h32[1] != nq || h32[3] != n_raw) return fail(CPT_ECORRUPT, "symbol counts do not match");
  FieldParams p;
  p.H = H;
  p.W = W;
  p.T = T;
  p.k = I.k;
  p.eps = (int)I.eps;
  p.tx = tx;
  p.ty = ty;
  p.predictor = I.predictor;
  p.K = K;
  p.bt = bt;
  p.cx = P.cx;
  p.sx = P.sx;
  p.cy = P.cy;
  p.sy = P.sy;
  for (int t = 0; t < T; t++) {
    int g = t / bt;
    bool dec = K > 1 && group_decided(g, bt, T);
    long long mbase = (dec && t >= 1) ? (long long)decided_before(g, bt, T) * tx * ty : -1;
    TimeScope ts(FAM_RECON, (uint64_t)H * W, s);
    launch_reconstruct(b.cur, field, b.xs, b.qs, b.qofs, sec32(7), b.rofs, b.modes, mbase, p, t, b.err, s);
  }
  HIPCHK(hipMemcpyAsync(A.host, b.err, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  harvest_timing();
  if (h32[0]) return fail(CPT_ECORRUPT, "reconstruction failed a check (code " + std::to_string(h32[0]) + ")");
  return CPT_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* cpt_last_error(void) { return g_err.c_str(); }

// selector training scratch (grow-only, per process)
namespace {
struct TrainBufs {
  float *m = nullptr, *v = nullptr, *grad = nullptr, *part = nullptr, *lpart = nullptr, *loss = nullptr;
  int32_t* idx = nullptr;
  size_t parts_cap = 0, n_cap = 0;
};
TrainBufs g_tb;
std::mutex g_tb_mu;
constexpr int SEL_NW = 5124;
constexpr int SEL_PER_BLOCK = 16;

cpt_status train_bufs(int n, int batch) {
  size_t parts = (size_t)selector_parts(std::max(n, batch), SEL_PER_BLOCK);
  if (!g_tb.m) {
    if (hipMalloc((void**)&g_tb.m, SEL_NW * 4) != hipSuccess || hipMalloc((void**)&g_tb.v, SEL_NW * 4) != hipSuccess ||
        hipMalloc((void**)&g_tb.grad, SEL_NW * 4) != hipSuccess || hipMalloc((void**)&g_tb.loss, 16) != hipSuccess)
      return fail(CPT_ENOMEM, "selector buffers");
  }
  if (parts > g_tb.parts_cap) {
    if (g_tb.part) (void)hipFree(g_tb.part);
    if (g_tb.lpart) (void)hipFree(g_tb.lpart);
    if (hipMalloc((void**)&g_tb.part, parts * SEL_NW * 4) != hipSuccess ||
        hipMalloc((void**)&g_tb.lpart, parts * 4) != hipSuccess)
      return fail(CPT_ENOMEM, "selector partial buffers");
    g_tb.parts_cap = parts;
  }
  if ((size_t)n > g_tb.n_cap) {
    if (g_tb.idx) (void)hipFree(g_tb.idx);
    if (hipMalloc((void**)&g_tb.idx, (size_t)n * 4) != hipSuccess) return fail(CPT_ENOMEM, "selector index buffer");
    g_tb.n_cap = n;
  }
  return CPT_OK;
}

long long gcd_ll(long long a, long long b) {
  while (b) {
    long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}
}  // namespace

cpt_status cpt_selector_grad(const float* w, const float* feats, const int32_t* labels, int n, float* grad,
                             float* loss, void* stream) {
  if (!w || !feats || !labels || !grad || !loss || n <= 0) return fail(CPT_EINVAL, "bad selector_grad arguments");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_tb_mu);
  cpt_status st = train_bufs(n, n);
  if (st) return st;
  launch_perm(g_tb.idx, n, 1, 0, s);
  launch_mlp_grad(w, feats, labels, g_tb.idx, n, SEL_PER_BLOCK, 1.0f / (float)n, g_tb.part, g_tb.lpart, grad,
                  g_tb.loss, s);
  HIPCHK(hipMemcpyAsync(loss, g_tb.loss, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return CPT_OK;
}

cpt_status cpt_selector_train(const float* feats, const int32_t* labels, int n, float* w, uint16_t* w_bf16,
                              const cpt_train_options* opt_in, float* final_loss, void* stream) {
  if (!feats || !labels || !w || !w_bf16 || n <= 0) return fail(CPT_EINVAL, "bad selector_train arguments");
  cpt_train_options opt{sizeof(cpt_train_options), 20, 1024, 2e-3f, 0};
  if (opt_in) {
    if (opt_in->struct_size != sizeof(cpt_train_options)) return fail(CPT_EINVAL, "cpt_train_options.struct_size");
    opt = *opt_in;
  }
  if (opt.epochs < 0 || opt.batch < 1 || !(opt.lr > 0.f)) return fail(CPT_EINVAL, "bad training options");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_tb_mu);
  const int batch = std::min(opt.batch, n);
  cpt_status st = train_bufs(n, batch);
  if (st) return st;
  HIPCHK(hipMemsetAsync(g_tb.m, 0, SEL_NW * 4, s));
  HIPCHK(hipMemsetAsync(g_tb.v, 0, SEL_NW * 4, s));
  // per-epoch sample order i -> (a i + c) mod n with gcd(a, n) = 1
  long long a = 2654435761LL % n;
  if (a == 0) a = 1;
  while (gcd_ll(a, n) != 1) a++;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double p1 = 1.0, p2 = 1.0;
  uint64_t state = opt.seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  for (int e = 0; e < opt.epochs; e++) {
    state ^= state >> 33;
    state *= 0xFF51AFD7ED558CCDull;
    state ^= state >> 33;
    launch_perm(g_tb.idx, n, a, (long long)(state % (uint64_t)n), s);
    for (int b0 = 0; b0 + batch <= n; b0 += batch) {
      launch_mlp_grad(w, feats, labels, g_tb.idx + b0, batch, SEL_PER_BLOCK, 1.0f / (float)batch, g_tb.part,
                      g_tb.lpart, g_tb.grad, g_tb.loss, s);
      p1 *= b1;
      p2 *= b2;
      launch_adam(w, g_tb.m, g_tb.v, g_tb.grad, opt.lr, b1, b2, eps, (float)(1.0 - p1), (float)(1.0 - p2), w_bf16, s);
    }
  }
  launch_to_bf16(w, w_bf16, s);
  if (final_loss) {
    launch_perm(g_tb.idx, n, 1, 0, s);
    launch_mlp_grad(w, feats, labels, g_tb.idx, n, SEL_PER_BLOCK, 1.0f / (float)n, g_tb.part, g_tb.lpart, g_tb.grad,
                    g_tb.loss, s);
    HIPCHK(hipMemcpyAsync(final_loss, g_tb.loss, 4, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return CPT_OK;
}

cpt_status cpt_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tim.mu);
  g_tim.on = on != 0;
  for (int i = 0; i < NFAM; i++) {
    g_tim.ms[i] = 0;
    g_tim.launches[i] = 0;
    g_tim.units[i] = 0;
  }
  return CPT_OK;
}

cpt_status cpt_timing_read(int family, double* total_ms, uint64_t* launches, uint64_t* units) {
  if (family < 0 || family >= NFAM || !total_ms || !launches || !units) return fail(CPT_EINVAL, "bad timing query");
  std::lock_guard<std::mutex> lk(g_tim.mu);
  *total_ms = g_tim.ms[family];
  *launches = g_tim.launches[family];
  *units = g_tim.units[family];
  return CPT_OK;
}

cpt_status cpt_compress_bound(int H, int W, int T, size_t* max_bytes) {
  if (!max_bytes) return fail(CPT_EINVAL, "null max_bytes");
  cpt_status st = check_dims(H, W, T);
  if (st) return st;
  size_t N = (size_t)H * W * T;
  size_t nchx = (N + CHUNK - 1) / CHUNK, nq = 2 * N, nchq = (nq + CHUNK - 1) / CHUNK;
  size_t nd = (size_t)T * ((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE);
  *max_bytes = HDR_BYTES + 4 * ((nd * 2 + 31) / 32) + (4 + 4 * XSYM) + 4 * nchx +
               4 * ((N * MAXLEN + 31) / 32 + nchx) + (4 + 4 * QSYM) + 4 * nchq +
               4 * ((nq * MAXLEN + 31) / 32 + nchq) + 8 * N;
  return CPT_OK;
}

cpt_status cpt_compress(const float* field, int H, int W, int T, double eb, const cpt_options* opt, uint8_t* out,
                        size_t cap, size_t* out_len, void* stream) {
  try {
    return compress_impl(field, H, W, T, eb, opt, out, cap, out_len, nullptr, nullptr, nullptr, nullptr, nullptr,
                         nullptr, (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_compress_debug(const float* field, int H, int W, int T, double eb, const cpt_options* opt,
                              uint8_t* out, size_t cap, size_t* out_len, int32_t* xi, uint8_t* xcode,
                              uint32_t* qcode, uint8_t* modes, float* feats, size_t* nblocks, void* stream) {
  try {
    return compress_impl(field, H, W, T, eb, opt, out, cap, out_len, xi, xcode, qcode, modes, feats, nblocks,
                         (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_stream_info(const uint8_t* bytes, size_t len, cpt_info* info) {
  if (!bytes || !info) return fail(CPT_EINVAL, "null pointer");
  Parsed P;
  cpt_status st = parse_header(bytes, len, &P);
  if (st) return st;
  *info = P.info;
  return CPT_OK;
}

cpt_status cpt_decompress(const uint8_t* bytes, size_t len, float* field, void* stream) {
  try {
    return decompress_impl(bytes, len, field, (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_field_params(const float* field, int H, int W, int T, int eb_mode, double eb, int* k,
                            double* eb_abs, int64_t* eps, void* stream) {
  if (!field || !k || !eb_abs || !eps) return fail(CPT_EINVAL, "null pointer");
  cpt_status st = check_dims(H, W, T);
  if (st) return st;
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  std::lock_guard<std::mutex> lk(Ap->mu);
  Bufs b;
  st = carve(*Ap, 1, 0, b);
  if (st) return st;
  Range r;
  st = field_range(field, 2 * (size_t)H * W * T, b, *Ap, (hipStream_t)stream, &r);
  if (st) return st;
  return derive_params(r.mn, r.mx, r.ma, eb_mode, eb, k, eb_abs, eps);
}

cpt_status cpt_extract_trajectories(const float* field, int H, int W, int T, int k, uint64_t* codes, size_t cap,
                                    size_t* count, void* stream) {
  if (!field || !count) return fail(CPT_EINVAL, "null pointer");
  cpt_status st = check_dims(H, W, T);
  if (st) return st;
  if (k < -80 || k > 120) return fail(CPT_EINVAL, "k must be in -80..120");
  hipStream_t s = (hipStream_t)stream;
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  const size_t N = (size_t)H * W * T;
  Bufs b;
  st = carve(A, N, 0, b);
  if (st) return st;
  Range r;
  st = field_range(field, 2 * N, b, A, s, &r);
  if (st) return st;
  if (std::ldexp(r.ma, k) >= 16777216.0) return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
  launch_convert(field, N, k, b.cur, s);
  launch_masks(b.cur, H, W, T, b.edges, b.masks, s);
  launch_count_faces(b.masks, N, b.nonll, s);
  launch_scan(b.nonll, N, b.qofs, b.part, b.tot, s);
  HIPCHK(hipMemcpyAsync(A.host, b.tot, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  size_t total = *(const uint32_t*)A.host;
  *count = total;
  if (total > cap || (total && !codes)) return fail(CPT_ECAPACITY, "codes capacity below " + std::to_string(total));
  launch_write_codes(b.masks, b.qofs, N, codes, cap, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return CPT_OK;
}

cpt_status cpt_verify(const float* a, const float* bf, int H, int W, int T, int k, cpt_verify_result* res,
                      void* stream) {
  if (!a || !bf || !res) return fail(CPT_EINVAL, "null pointer");
  cpt_status st = check_dims(H, W, T);
  if (st) return st;
  if (k < -80 || k > 120) return fail(CPT_EINVAL, "k must be in -80..120");
  hipStream_t s = (hipStream_t)stream;
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  const size_t N = (size_t)H * W * T;
  Bufs b;
  st = carve(A, N, 0, b);
  if (st) return st;
  Range ra, rb;
  st = field_range(a, 2 * N, b, A, s, &ra);
  if (st) return st;
  st = field_range(bf, 2 * N, b, A, s, &rb);
  if (st) return st;
  if (std::ldexp(std::max(ra.ma, rb.ma), k) >= 16777216.0) return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
  launch_convert(a, N, k, b.cur, s);
  launch_masks(b.cur, H, W, T, b.edges, b.masks, s);
  launch_convert(bf, N, k, b.cur, s);
  launch_masks(b.cur, H, W, T, b.edges, b.qcode, s);
  launch_compare(b.masks, b.qcode, a, bf, N, b.fc, b.cpart, s);
  size_t np = compare_partials(N);
  std::vector<double> part(2 * np);
  HIPCHK(hipMemcpyAsync(part.data(), b.cpart, 16 * np, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(A.host, b.fc, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double me = 0, se = 0;
  for (size_t i = 0; i < np; i++) {
    me = std::max(me, part[2 * i]);
    se += part[2 * i + 1];
  }
  res->fc_t = A.host[0];
  res->fc_s = A.host[1];
  res->max_err = me;
  double mse = se / (double)(2 * N);
  res->psnr = mse > 0 ? 20.0 * std::log10(ra.mx - ra.mn) - 10.0 * std::log10(mse) : INFINITY;
  return CPT_OK;
}

}  // extern "C"
