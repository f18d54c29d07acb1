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

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.hpp"
#include "cpt_device.hpp"
#include "cptraj.h"
#include "launch.hpp"

using namespace cpt;

namespace {

thread_local std::string g_err;
thread_local bool g_capturing = false;  // inside a graph capture: no timing events

cpt_status fail(cpt_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(CPT_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ arena
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
};

struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  uint64_t* host = nullptr;  // pinned staging for small readbacks
  int64_t* tlog = nullptr;   // entropy table floor(h log2 h 2^16)
  char* stage = nullptr;     // pinned staging for batch descriptors and tables
  size_t stage_cap = 0;
  hipStream_t lib = nullptr;  // library stream for graph replays and the persistent schedule
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<GraphEntry> graphs;  // most recent last
  std::mutex mu;

  void drop_graphs() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }

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
struct Bufs {  // scratch of the extraction, verification and parameter calls
  uint32_t *masks, *masks2, *nonll, *qofs, *part, *tot;
  int* range;
  unsigned long long* fc;
  double* cpart;
};

cpt_status reserve(Arena& A);

cpt_status carve(Arena& A, size_t N, Bufs& b) {
  A.used = 0;
  struct Item {
    void** p;
    size_t bytes;
  };
  std::vector<Item> items = {
      {(void**)&b.masks, 4 * N},
      {(void**)&b.masks2, 4 * N},     {(void**)&b.nonll, 4 * N},      {(void**)&b.qofs, 4 * N},
      {(void**)&b.part, 4 * (scan_partials_size(N) + 16)},            {(void**)&b.tot, 64},
      {(void**)&b.range, 64},         {(void**)&b.fc, 16},            {(void**)&b.cpart, 16 * (compare_partials(N) + 1)},
  };
  std::vector<size_t> offs;
  for (auto& it : items) offs.push_back(A.off(it.bytes));
  cpt_status st = reserve(A);
  if (st) return st;
  for (size_t i = 0; i < items.size(); i++) *items[i].p = A.base + offs[i];
  return CPT_OK;
}

// grows the arena to A.used bytes (every earlier carve is invalidated)
cpt_status reserve(Arena& A) {
  if (A.used > A.cap) {
    if (A.base) {
      if (hipDeviceSynchronize() != hipSuccess) return fail(CPT_EHIP, "synchronize before arena growth failed");
      A.drop_graphs();
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
  return CPT_OK;
}

// Largest Huffman stream of a field, and the most blocks of its body
size_t huffman_bound(int H, int W, int T) {
  const size_t N = (size_t)H * W * T;
  const size_t nchx = (N + CHUNK - 1) / CHUNK, nq = 2 * N, nchq = (nq + CHUNK - 1) / CHUNK;
  const size_t nd = (size_t)T * ((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE);
  return HDR_BYTES + 4 * ((nd * 2 + 31) / 32) + (4 + 4 * XSYM) + 4 * nchx + 4 * ((N * MAXLEN + 31) / 32 + nchx) +
         (4 + 4 * QSYM) + 4 * nchq + 4 * ((nq * MAXLEN + 31) / 32 + nchq) + 8 * N;
}
size_t zbe_blocks(size_t inner_len) { return (inner_len - HDR_BYTES + ZBE_BLOCK - 1) / ZBE_BLOCK; }

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
unsigned nb256(size_t n) { return (unsigned)((n + 255) / 256); }

int mode_bits(int K) { return K == 4 ? 2 : (K == 2 ? 1 : 0); }

// ------------------------------------------------------------ kernel timing
// When enabled, launches of the main kernel families are bracketed by HIP
// events on the caller's stream; elapsed times are harvested after the
// call's final synchronisation.
enum { FAM_PHASE = 0, FAM_MODES = 1, FAM_RECON = 2, FAM_DECODE = 3, FAM_ENCODE = 4, FAM_EXTRACT = 5, NFAM = 6 };

struct Timing {
  bool on = false;
  int period = 1;              // bracket every period-th launch of a family
  uint64_t seen[NFAM] = {0};  // launches of each family since enabling
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
    // timing only: no system-scope fence, so a bracketed launch costs no
    // cache writeback and invalidation of its own
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
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
    if (!g_tim.on || g_capturing) return;
    std::lock_guard<std::mutex> lk(g_tim.mu);
    if (g_tim.seen[fam]++ % (uint64_t)g_tim.period != 0) return;
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
// Everything about a batch that depends only on the dimensions and options.
// The launch order lists the fields by decreasing T (ties by index), so the
// fields still running at frame t are a prefix of it.
struct Plan {
  int n = 0;
  cpt_options opt{};
  int K = 1, maxT = 0;
  std::vector<FieldDesc> D;
  std::vector<int> ord;
  std::vector<long long> rpre, gpre, hpre, cxpre, cqpre, fpre;  // natural order
  std::vector<long long> zpre, ioff;  // lossless stage: most blocks per field, Huffman stream scratch offsets
  long long ZB = 0, IB = 0;
  std::vector<long long> mpre, ppre;                      // launch order
  std::vector<int> m_at, mstate_at, gidx_at;              // per frame
  std::vector<uint64_t> hw_at, cv_at;                     // vertices per frame / per phase
  long long Ntot = 0, CX = 0, CQ = 0, NB = 0, Rtot = 0;
  std::string key;
  // persistent schedule
  int group = 0;
  std::vector<SchedSeg> seg;
  std::vector<long long> sstart;
  long long nitems = 0;
};

cpt_status check_options(const cpt_options* opt_in, double eb, cpt_options* opt) {
  *opt = cpt_options{sizeof(cpt_options), 0, CPT_PRED_MIX2, 1, 1.0, 1.0, nullptr, 0};
  if (opt_in) {
    // the struct as declared, or as it was before the backend field
    constexpr size_t before_backend = offsetof(cpt_options, backend);
    if (opt_in->struct_size == sizeof(cpt_options)) {
      *opt = *opt_in;
    } else if (opt_in->struct_size >= before_backend && opt_in->struct_size < sizeof(cpt_options)) {
      std::memcpy(opt, opt_in, before_backend);
      opt->backend = 0;
    } else {
      return fail(CPT_EINVAL, "cpt_options.struct_size mismatch");
    }
    opt->struct_size = sizeof(cpt_options);
  }
  if (opt->backend < 0 || opt->backend > 1) return fail(CPT_EINVAL, "backend must be 0 or 1");
  if (opt->predictor < 0 || opt->predictor > 4) return fail(CPT_EINVAL, "unknown predictor");
  if (opt->mode_bt < 1 || opt->mode_bt > 1024) return fail(CPT_EINVAL, "mode_bt must be in 1..1024");
  if (opt->predictor == CPT_PRED_LEARNED && !opt->selector_w)
    return fail(CPT_EINVAL, "learned predictor needs selector_w");
  if (opt->predictor == CPT_PRED_LEARNED && ((uintptr_t)opt->selector_w & 15))
    return fail(CPT_EINVAL, "selector_w must be 16-byte aligned");
  if (!(opt->dt_dx >= 0.0) || !(opt->dt_dy >= 0.0) || !std::isfinite(opt->dt_dx) || !std::isfinite(opt->dt_dy))
    return fail(CPT_EINVAL, "dt_dx and dt_dy must be finite and non-negative");
  if (opt->eb_mode == 0) {
    if (!(eb > 0.0 && eb <= 0.5)) return fail(CPT_EINVAL, "relative error bound must be in (0, 0.5]");
  } else if (opt->eb_mode == 1) {
    if (!(eb > 0.0) || !std::isfinite(eb)) return fail(CPT_EINVAL, "absolute error bound must be positive");
  } else {
    return fail(CPT_EINVAL, "eb_mode must be 0 or 1");
  }
  return CPT_OK;
}

cpt_status make_plan(int n, const int32_t* HWT, const cpt_options& opt, double eb, Plan& P) {
  if (n < 1 || n > 65536) return fail(CPT_EINVAL, "batch size must be in 1..65536");
  if (!HWT) return fail(CPT_EINVAL, "null HWT");
  P.n = n;
  P.opt = opt;
  P.K = opt.predictor == 2 ? 2 : (opt.predictor >= 3 ? 4 : 1);
  const int K = P.K, bt = opt.mode_bt, mb = mode_bits(K);
  P.D.assign(n, FieldDesc{});
  for (auto* v : {&P.rpre, &P.gpre, &P.hpre, &P.cxpre, &P.cqpre, &P.fpre, &P.mpre, &P.ppre, &P.zpre, &P.ioff})
    v->assign(n + 1, 0);
  P.key = std::to_string(n) + ":" + std::to_string(opt.predictor) + ":" + std::to_string(bt) + ":" +
          std::to_string(opt.backend);
  for (int i = 0; i < n; i++) {
    const int H = HWT[3 * i], W = HWT[3 * i + 1], T = HWT[3 * i + 2];
    cpt_status st = check_dims(H, W, T);
    if (st) return fail(st, "field " + std::to_string(i) + ": " + g_err);
    FieldDesc& d = P.D[i];
    d.H = H;
    d.W = W;
    d.T = T;
    d.tx = (W + TILE - 1) / TILE;
    d.ty = (H + TILE - 1) / TILE;
    const long long N = (long long)H * W * T;
    const int G = (T + bt - 1) / bt;
    d.ndec = K > 1 ? decided_before(G, bt, T) : 0;
    d.N = N;
    d.voff = P.Ntot;
    d.ro = P.Rtot;
    d.cxb = P.CX;
    d.cqb = P.CQ;
    d.mbase = P.NB;
    d.nchx = (N + CHUNK - 1) / CHUNK;
    const long long nblk = (long long)d.ndec * d.tx * d.ty;
    d.mwords = (nblk * mb + 31) / 32;
    d.eb_mode = opt.eb_mode;
    d.predictor = opt.predictor;
    d.K = K;
    d.bt = bt;
    d.eb = eb;
    d.dt_dx = opt.dt_dx;
    d.dt_dy = opt.dt_dy;
    const long long ncq = (2 * N + CHUNK - 1) / CHUNK;
    P.Ntot += N;
    P.Rtot += (N + 15) / 16;
    P.CX += d.nchx;
    P.CQ += ncq;
    P.NB += nblk;
    P.rpre[i + 1] = P.rpre[i] + (2 * N + RANGE_SPAN_FLOATS - 1) / RANGE_SPAN_FLOATS;
    P.gpre[i + 1] = P.gpre[i] + (N + HIST_WG_VERTICES - 1) / HIST_WG_VERTICES;
    P.hpre[i + 1] = P.hpre[i] + (N + HIST_SPAN_VERTICES - 1) / HIST_SPAN_VERTICES;
    P.cxpre[i + 1] = P.cxpre[i] + d.nchx;
    P.cqpre[i + 1] = P.cqpre[i] + ncq;
    if (opt.backend == 1) {
      const size_t hb = huffman_bound(H, W, T);
      d.zbase = P.zpre[i];
      P.zpre[i + 1] = P.zpre[i] + (long long)zbe_blocks(hb);
      P.ioff[i + 1] = P.ioff[i] + (long long)((hb + 255) & ~(size_t)255);
    } else {
      P.zpre[i + 1] = P.zpre[i];
      P.ioff[i + 1] = P.ioff[i];
    }
    P.maxT = std::max(P.maxT, T);
    P.key += ":" + std::to_string(H) + "x" + std::to_string(W) + "x" + std::to_string(T);
  }
  for (auto v : {P.rpre.back(), P.gpre.back(), P.hpre.back(), P.cxpre.back(), P.cqpre.back(), P.zpre.back()})
    if (v >= 2147483647LL) return fail(CPT_EINVAL, "batch too large for one launch");
  P.ZB = P.zpre.back();
  P.IB = P.ioff.back();
  P.ord.resize(n);
  for (int i = 0; i < n; i++) P.ord[i] = i;
  std::stable_sort(P.ord.begin(), P.ord.end(), [&](int a, int b) { return P.D[a].T > P.D[b].T; });
  for (int j = 0; j < n; j++) {
    const FieldDesc& d = P.D[P.ord[j]];
    P.mpre[j + 1] = P.mpre[j] + (long long)d.tx * d.ty;
    P.ppre[j + 1] = P.ppre[j] + (long long)phase_cols(d.tx) * d.ty;
  }
  if (P.mpre.back() >= 2147483647LL || P.ppre.back() >= 2147483647LL)
    return fail(CPT_EINVAL, "batch too large for one launch");
  const int T0 = P.maxT;
  P.m_at.assign(T0, 0);
  P.mstate_at.assign(T0, MODES_NONE);
  P.gidx_at.assign(T0, 0);
  P.hw_at.assign(T0, 0);
  P.cv_at.assign(3 * (size_t)T0, 0);
  int m = n;
  for (int t = 0; t < T0; t++) {
    while (m > 0 && P.D[P.ord[m - 1]].T <= t) m--;
    P.m_at[t] = m;
    // the predictor groups depend on t and bt only for the fields that
    // reach frame t; checked field by field
    int ms = MODES_NONE, gi = 0;
    for (int j = 0; j < m; j++) {
      const FieldDesc& d = P.D[P.ord[j]];
      int msj = MODES_NONE, gij = 0;
      if (K > 1 && t >= 1) {
        const int g = t / bt;
        if (group_decided(g, bt, d.T)) {
          const int td = g * bt > 1 ? g * bt : 1;
          msj = t == td ? MODES_DECIDE : MODES_READ;
          gij = decided_before(g, bt, d.T);
        }
      }
      if (j == 0) {
        ms = msj;
        gi = gij;
      } else if (ms != msj || gi != gij) {
        return fail(CPT_EHIP, "internal: predictor groups differ between fields of one frame");
      }
      P.hw_at[t] += (uint64_t)d.H * d.W;
      for (int c = 0; c < 3; c++) P.cv_at[3 * t + c] += colour_vertices(d.H, d.W, c);
    }
    P.mstate_at[t] = ms;
    P.gidx_at[t] = gi;
  }
  return CPT_OK;
}

cpt_status build_schedule(Plan& P, int group) {
  if (P.group == group && !P.seg.empty()) return CPT_OK;
  P.group = group;
  P.seg.clear();
  P.sstart.assign(1, 0);
  std::vector<long long> items(P.n), nb(P.n);
  for (int f = 0; f < P.n; f++) {
    nb[f] = (long long)phase_cols(P.D[f].tx) * P.D[f].ty;
    items[f] = (nb[f] + group - 1) / group;
  }
  for (int r = 0; r < 3 * P.maxT; r++) {
    const int t = r / 3, c = r % 3;
    for (int j = 0; j < P.m_at[t]; j++) {
      const int f = P.ord[j];
      const long long need = (long long)r * items[f];
      if (need >= 4294967295LL) return fail(CPT_EINVAL, "field too large for the persistent schedule");
      SchedSeg sg{f, t, c, P.mstate_at[t], P.gidx_at[t], (int)nb[f], (unsigned)need, 0};
      P.seg.push_back(sg);
      P.sstart.push_back(P.sstart.back() + items[f]);
    }
  }
  P.nitems = P.sstart.back();
  if (P.nitems >= 2147483647LL) return fail(CPT_EINVAL, "batch too large for the persistent schedule");
  return CPT_OK;
}

// Scratch of a batch.  The tables block (descriptors, launch order, prefix
// tables, schedule) is contiguous and uploaded in one copy.
struct BatchBufs {
  FieldDesc* D;
  int* ord;
  long long *rpre, *gpre, *hpre, *cxpre, *cqpre, *fpre, *mpre, *ppre, *sstart;
  SchedSeg* seg;
  size_t tables_bytes;
  uint8_t* inner;           // Huffman streams ahead of the lossless stage
  uint32_t *ztab, *zlen;    // per block: table entry, encoded length
  long long* zoff;          // per block: offset in its container's payload
  unsigned *done, *ctl;
  int4* range;
  int2* cur;
  uint8_t *flags, *xcode, *modes;
  uint32_t* qcode;
  EntropyBufs E;
};

template <typename T>
size_t vec_bytes(const std::vector<T>& v) {
  return v.size() * sizeof(T);
}

cpt_status carve_batch(Arena& A, const Plan& P, BatchBufs& b) {
  A.used = 0;
  const int n = P.n;
  const size_t N = (size_t)P.Ntot, CX = (size_t)P.CX, CQ = (size_t)P.CQ, R = (size_t)P.Rtot;
  struct Item {
    void** p;
    size_t bytes;
  };
  std::vector<Item> tables = {
      {(void**)&b.D, sizeof(FieldDesc) * n}, {(void**)&b.ord, 4 * (size_t)n},
      {(void**)&b.rpre, vec_bytes(P.rpre)},   {(void**)&b.gpre, vec_bytes(P.gpre)},
      {(void**)&b.hpre, vec_bytes(P.hpre)},   {(void**)&b.cxpre, vec_bytes(P.cxpre)},
      {(void**)&b.cqpre, vec_bytes(P.cqpre)}, {(void**)&b.fpre, vec_bytes(P.fpre)},
      {(void**)&b.mpre, vec_bytes(P.mpre)},
      {(void**)&b.ppre, vec_bytes(P.ppre)},   {(void**)&b.sstart, 8 * (P.sstart.size() + 1)},
      {(void**)&b.seg, sizeof(SchedSeg) * (P.seg.size() + 1)},
  };
  std::vector<Item> rest = {
      {(void**)&b.done, 4 * (size_t)n + 64},   {(void**)&b.ctl, 64},
      {(void**)&b.range, 16 * (size_t)RANGE_SLOTS * RANGE_SLOT_STRIDE * n},       {(void**)&b.cur, 8 * N},
      {(void**)&b.flags, N},                    {(void**)&b.xcode, N},
      {(void**)&b.modes, (size_t)P.NB + 1},     {(void**)&b.qcode, 4 * N},
      {(void**)&b.E.sn, 4 * R + 16},            {(void**)&b.E.sq, 4 * R + 16},
      {(void**)&b.E.sr, 4 * R + 16},            {(void**)&b.E.sro, 4 * R + 16},
      {(void**)&b.E.qsym, 2 * CQ * CHUNK},      {(void**)&b.E.xbits, 4 * CX},
      {(void**)&b.E.xwords, 4 * CX},            {(void**)&b.E.xwofs, 4 * CX},
      {(void**)&b.E.qbits, 4 * CQ},             {(void**)&b.E.qwords, 4 * CQ},
      {(void**)&b.E.qwofs, 4 * CQ},             {(void**)&b.E.part, 4 * (scan_partials_size(N) + 16)},
      {(void**)&b.E.xhist, 128 * (size_t)HIST_SLOTS * n},    {(void**)&b.E.qhist, 4 * (size_t)QSYM * HIST_SLOTS * n},
      {(void**)&b.E.xcb, 128 * (size_t)n},      {(void**)&b.E.qcb, 4 * (size_t)(QSYM + 4) * n},
      {(void**)&b.E.used, 8 * (size_t)n},       {(void**)&b.E.xt, sizeof(HuffTables) * n},
      {(void**)&b.E.qt, sizeof(HuffTables) * n},
      {(void**)&b.inner, (size_t)P.IB + 16},    {(void**)&b.ztab, 4 * (size_t)P.ZB + 16},
      {(void**)&b.zlen, 4 * (size_t)P.ZB + 16}, {(void**)&b.zoff, 8 * (size_t)P.ZB + 16},
  };
  std::vector<size_t> offs;
  size_t t0 = 0;
  for (size_t i = 0; i < tables.size(); i++) {
    size_t o = A.off(tables[i].bytes);
    if (i == 0) t0 = o;
    offs.push_back(o);
  }
  b.tables_bytes = A.used - t0;
  for (auto& it : rest) offs.push_back(A.off(it.bytes));
  cpt_status st = reserve(A);
  if (st) return st;
  size_t k = 0;
  for (auto& it : tables) *it.p = A.base + offs[k++];
  for (auto& it : rest) *it.p = A.base + offs[k++];
  return CPT_OK;
}

cpt_status reserve_stage(Arena& A, size_t bytes) {
  if (bytes <= A.stage_cap) return CPT_OK;
  if (A.stage) (void)hipHostFree(A.stage);
  A.stage = nullptr;
  A.stage_cap = 0;
  size_t want = bytes + bytes / 4 + 4096;
  if (hipHostMalloc((void**)&A.stage, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CPT_ENOMEM, "pinned staging allocation failed");
  }
  A.stage_cap = want;
  return CPT_OK;
}

// copy the host tables into the staging buffer at the offsets of b
void stage_tables(const Plan& P, const BatchBufs& b, char* stage) {
  const char* base = (const char*)b.D;
  auto put = [&](const void* dev, const void* src, size_t bytes) {
    if (bytes) std::memcpy(stage + ((const char*)dev - base), src, bytes);
  };
  put(b.D, P.D.data(), sizeof(FieldDesc) * P.n);
  put(b.ord, P.ord.data(), 4 * (size_t)P.n);
  put(b.rpre, P.rpre.data(), vec_bytes(P.rpre));
  put(b.gpre, P.gpre.data(), vec_bytes(P.gpre));
  put(b.hpre, P.hpre.data(), vec_bytes(P.hpre));
  put(b.cxpre, P.cxpre.data(), vec_bytes(P.cxpre));
  put(b.cqpre, P.cqpre.data(), vec_bytes(P.cqpre));
  put(b.fpre, P.fpre.data(), vec_bytes(P.fpre));
  put(b.mpre, P.mpre.data(), vec_bytes(P.mpre));
  put(b.ppre, P.ppre.data(), vec_bytes(P.ppre));
  put(b.sstart, P.sstart.data(), vec_bytes(P.sstart));
  put(b.seg, P.seg.data(), vec_bytes(P.seg));
}

struct ExecChoice {
  int schedule = CPT_SCHED_LAUNCH, group = 1, grid = 0;
  bool graph = false;
  int ftile = 0;  // tile shape of the field pass (FP_SHAPE_TW / FP_SHAPE_TH)
  int pblocks = 2;  // blocks per workgroup of the per-phase launches (1 or 2)
};

// the field pass's workgroups per field for tile shape `shape`
cpt_status set_fieldpass_shape(Plan& P, int shape) {
  const long long tw = FP_SHAPE_TW[shape], th = FP_SHAPE_TH[shape];
  P.fpre.assign(P.n + 1, 0);
  for (int i = 0; i < P.n; i++)
    P.fpre[i + 1] = P.fpre[i] + ((P.D[i].W + tw - 1) / tw) * ((P.D[i].H + th - 1) / th);
  if (P.fpre.back() >= 2147483647LL) return fail(CPT_EINVAL, "batch too large for one launch");
  return CPT_OK;
}

std::mutex g_tune_mu;
std::map<std::string, ExecChoice> g_tuned;

// The whole device pipeline of a batch, enqueued on s without any host
// synchronisation.
void enqueue_compress(const Plan& P, const BatchBufs& b, const ExecChoice& ex, const Arena& A, hipStream_t s) {
  const int n = P.n;
  BatchView B{b.D, b.ord, P.ord[0], b.cur, b.flags, b.xcode, b.qcode, b.modes, A.tlog, P.opt.selector_w};
  // Alg. 3: fixed point, crossed faces of the original field, lossless flags
  {
    TimeScope ts(FAM_EXTRACT, (uint64_t)P.Ntot, s);
    launch_fieldpass_b(b.D, n, b.rpre, P.rpre.back(), b.fpre, P.fpre.back(), b.range, b.cur, b.flags, ex.ftile, s);
  }
  if (ex.schedule == CPT_SCHED_PERSISTENT) {
    launch_zero_u32(b.done, (size_t)n, s);
    launch_zero_u32(b.ctl, 16, s);
    TimeScope ts(FAM_PHASE, (uint64_t)P.Ntot, s);
    launch_persist(B, b.seg, b.sstart, (int)P.seg.size(), P.nitems, ex.group, ex.grid, b.done, b.ctl, s);
  } else {
    for (int t = 0; t < P.maxT; t++) {
      const int m = P.m_at[t], gi = P.gidx_at[t];
      int ms = P.mstate_at[t];
      if (ex.schedule == CPT_SCHED_LAUNCH && ms == MODES_DECIDE) {
        TimeScope ts(FAM_MODES, P.hw_at[t], s);
        launch_modes_b(B, b.mpre, m, P.mpre[m], t, gi, s);
        ms = MODES_READ;
      }
      for (int c = 0; c < 3; c++) {
        TimeScope ts(FAM_PHASE, P.cv_at[3 * t + c], s);
        launch_phase_b(B, b.ppre, m, P.ppre[m], t, c, ms, gi, ex.schedule == CPT_SCHED_FUSED, ex.pblocks, s);
      }
    }
  }
  // lossless_comp of Alg. 3: Huffman codes of both code streams, raw values
  launch_codes_b(b.D, n, B, b.E, b.hpre, P.hpre.back(), b.gpre, P.gpre.back(), P.Rtot, s);
  launch_chunks_b(b.D, n, B, b.E, b.cxpre, P.CX, b.cqpre, P.CQ, s);
  {
    TimeScope ts(FAM_ENCODE, (uint64_t)P.Ntot, s);
    launch_assemble_b(b.D, n, B, b.E, b.cxpre, P.CX, b.cqpre, P.CQ, b.hpre, P.hpre.back(), s);
  }
  // the additional lossless stage (Sec. V) into the caller's outputs
  if (P.opt.backend == 1) launch_zbe_b(b.D, n, P.ZB, b.ztab, b.zlen, b.zoff, s);
}

cpt_status library_stream(Arena& A) {
  if (A.lib) return CPT_OK;
  HIPCHK(hipStreamCreateWithFlags(&A.lib, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&A.ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&A.ev[1], hipEventDisableTiming));
  return CPT_OK;
}

// replays (capturing first if needed) the pipeline as a graph on the
// library stream, ordered after and before the work on s
cpt_status run_graph(const Plan& P, const BatchBufs& b, const ExecChoice& ex, Arena& A, hipStream_t s) {
  cpt_status st = library_stream(A);
  if (st) return st;
  char tag[160];
  std::snprintf(tag, sizeof(tag), "|%d:%d:%d:%d:%d|%p:%zu|%p:%p", ex.schedule, ex.group, ex.grid, ex.ftile, ex.pblocks,
                (void*)A.base, A.cap, (const void*)P.opt.selector_w, (void*)A.tlog);
  const std::string key = P.key + tag;
  hipGraphExec_t exec = nullptr;
  for (size_t i = 0; i < A.graphs.size(); i++)
    if (A.graphs[i].key == key) {
      GraphEntry e = A.graphs[i];
      A.graphs.erase(A.graphs.begin() + i);
      A.graphs.push_back(e);
      exec = e.exec;
      break;
    }
  if (!exec) {
    HIPCHK(hipStreamBeginCapture(A.lib, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    enqueue_compress(P, b, ex, A, A.lib);
    g_capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e1 = hipStreamEndCapture(A.lib, &g);
    if (e1 != hipSuccess || !g) return fail(CPT_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e1));
    hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(CPT_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e2));
    if (A.graphs.size() >= 8) {
      (void)hipGraphExecDestroy(A.graphs.front().exec);
      A.graphs.erase(A.graphs.begin());
    }
    A.graphs.push_back({key, exec});
  }
  HIPCHK(hipEventRecord(A.ev[0], s));
  HIPCHK(hipStreamWaitEvent(A.lib, A.ev[0], 0));
  HIPCHK(hipGraphLaunch(exec, A.lib));
  HIPCHK(hipEventRecord(A.ev[1], A.lib));
  HIPCHK(hipStreamWaitEvent(s, A.ev[1], 0));
  return CPT_OK;
}

struct Debug {
  int32_t* xi = nullptr;
  uint8_t* xcode = nullptr;
  uint32_t* qcode = nullptr;
  uint8_t* modes = nullptr;
  float* feats = nullptr;
  size_t* nblocks = nullptr;
};

ExecChoice resolve_exec(const cpt_exec_options* ex, const Plan& P) {
  ExecChoice c;
  int sched = CPT_SCHED_AUTO;
  if (ex) {
    sched = ex->schedule;
    c.group = ex->group > 0 ? ex->group : 1;
    c.grid = ex->grid;
    c.graph = ex->use_graph != 0;
    // a struct without a field (an earlier layout) means its default
    if (ex->struct_size >= offsetof(cpt_exec_options, field_tile) + sizeof(int32_t)) c.ftile = ex->field_tile;
    if (ex->struct_size >= offsetof(cpt_exec_options, phase_blocks) + sizeof(int32_t) && ex->phase_blocks != 0)
      c.pblocks = ex->phase_blocks;
  }
  if (sched == CPT_SCHED_AUTO) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(P.key);
    if (it != g_tuned.end()) {
      c.schedule = it->second.schedule;
      c.group = it->second.group;
      c.grid = it->second.grid;
      c.graph = c.graph || it->second.graph;
      c.ftile = it->second.ftile;
      c.pblocks = it->second.pblocks;
    } else {
      c.schedule = CPT_SCHED_LAUNCH;
    }
  } else {
    c.schedule = sched;
  }
  return c;
}

const char* reason_text(int r) {
  switch (r) {
    case REASON_NONFINITE: return "field contains NaN or Inf";
    case REASON_MAGNITUDE: return "field magnitude of 2^100 or more is not supported";
    case REASON_CAPACITY: return "output capacity below the stream length";
    default: return "failed";
  }
}

// Compress n fields; lens / status are host arrays.  With dbg (n == 1) the
// internals are copied out as well.
cpt_status compress_batch_impl(int n, const float* const* fields, const int32_t* HWT, double eb,
                               const cpt_options* opt_in, const cpt_exec_options* ex_in, uint8_t* const* outs,
                               const size_t* caps, size_t* lens, int32_t* status, const Debug* dbg, hipStream_t s,
                               const ExecChoice* forced = nullptr) {
  if (!fields || !outs || !caps || !lens) return fail(CPT_EINVAL, "null argument");
  if (ex_in && ex_in->struct_size != sizeof(cpt_exec_options) &&
      ex_in->struct_size != offsetof(cpt_exec_options, phase_blocks) &&
      ex_in->struct_size != offsetof(cpt_exec_options, field_tile))
    return fail(CPT_EINVAL, "cpt_exec_options.struct_size mismatch");
  if (ex_in && ex_in->struct_size >= offsetof(cpt_exec_options, phase_blocks) &&
      (ex_in->field_tile < 0 || ex_in->field_tile >= FP_SHAPES))
    return fail(CPT_EINVAL, "field_tile must be 0, 1 or 2");
  if (ex_in && ex_in->struct_size == sizeof(cpt_exec_options) && (ex_in->phase_blocks < 0 || ex_in->phase_blocks > 2))
    return fail(CPT_EINVAL, "phase_blocks must be 0, 1 or 2");
  cpt_options opt;
  cpt_status st = check_options(opt_in, eb, &opt);
  if (st) return st;
  Plan P;
  st = make_plan(n, HWT, opt, eb, P);
  if (st) return st;
  for (int i = 0; i < n; i++) {
    if (!fields[i]) return fail(CPT_EINVAL, "field " + std::to_string(i) + ": null pointer");
    if (outs[i] && ((uintptr_t)outs[i] & 3)) return fail(CPT_EINVAL, "out must be 4-byte aligned");
    P.D[i].field = fields[i];
    P.D[i].out = outs[i];
    P.D[i].cap = (long long)std::min(caps[i], (size_t)1 << 62);
  }
  if (dbg && n == 1) {
    P.D[0].xi_dbg = dbg->xi;
    P.D[0].feats_dbg = dbg->feats;
  }
  ExecChoice ex = forced ? *forced : resolve_exec(ex_in, P);
  if (ex.schedule < CPT_SCHED_LAUNCH || ex.schedule > CPT_SCHED_PERSISTENT) return fail(CPT_EINVAL, "unknown schedule");
  if (ex.group < 1 || ex.group > 64) return fail(CPT_EINVAL, "group must be in 1..64");
  if (ex.grid < 0) return fail(CPT_EINVAL, "grid must be 0 (as many workgroups as fit at once) or positive");
  if (ex.ftile < 0 || ex.ftile >= FP_SHAPES) return fail(CPT_EINVAL, "field_tile must be 0, 1 or 2");
  if (ex.pblocks < 1 || ex.pblocks > 2) return fail(CPT_EINVAL, "phase_blocks must be 0, 1 or 2");
  st = set_fieldpass_shape(P, ex.ftile);
  if (st) return st;
  if (ex.schedule == CPT_SCHED_PERSISTENT)
    return fail(CPT_EUNSUPPORTED, "the persistent schedule is disabled: its launch did not complete on the device");
  if (ex.schedule == CPT_SCHED_PERSISTENT) {
    // never a launch without workgroups: 0 asks for every workgroup that
    // fits on the device at once, and more than one per item is pointless
    if (ex.grid == 0) ex.grid = persist_grid();
    if (ex.grid <= 0) return fail(CPT_EHIP, "occupancy query for the persistent kernel failed");
    st = build_schedule(P, ex.group);
    if (st) return st;
    ex.grid = (int)std::min<long long>(ex.grid, std::max<long long>(P.nitems, 1));
  }
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  BatchBufs b;
  st = carve_batch(A, P, b);
  if (st) return st;
  if (P.opt.backend == 1)
    for (int i = 0; i < n; i++) {
      // the Huffman stream goes to library scratch, the container to the caller
      FieldDesc& d = P.D[i];
      d.zout = d.out;
      d.zcap = d.cap;
      d.out = b.inner + P.ioff[i];
      d.cap = P.ioff[i + 1] - P.ioff[i];
    }
  const size_t rb_off = (b.tables_bytes + 255) & ~(size_t)255;
  const size_t rb_bytes = sizeof(FieldDesc) * n + 64;
  st = reserve_stage(A, rb_off + rb_bytes);
  if (st) return st;
  stage_tables(P, b, A.stage);
  HIPCHK(hipMemcpyAsync(b.D, A.stage, b.tables_bytes, hipMemcpyHostToDevice, s));
  if (ex.graph) {
    st = run_graph(P, b, ex, A, s);
    if (st) return st;
  } else {
    enqueue_compress(P, b, ex, A, s);
  }
  if (dbg && n == 1) {
    const size_t N = (size_t)P.Ntot;
    if (dbg->xcode) HIPCHK(hipMemcpyAsync(dbg->xcode, b.xcode, N, hipMemcpyDeviceToDevice, s));
    if (dbg->qcode) HIPCHK(hipMemcpyAsync(dbg->qcode, b.qcode, 4 * N, hipMemcpyDeviceToDevice, s));
    if (dbg->modes && P.NB) HIPCHK(hipMemcpyAsync(dbg->modes, b.modes, (size_t)P.NB, hipMemcpyDeviceToDevice, s));
    if (dbg->nblocks) *dbg->nblocks = (size_t)P.NB;
  }
  char* rb = A.stage + rb_off;
  HIPCHK(hipMemcpyAsync(rb, b.D, sizeof(FieldDesc) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(rb + sizeof(FieldDesc) * n, b.ctl, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  harvest_timing();
  const FieldDesc* Dh = (const FieldDesc*)rb;
  const uint32_t* ctl = (const uint32_t*)(rb + sizeof(FieldDesc) * n);
  if (ex.schedule == CPT_SCHED_PERSISTENT && ctl[1])
    return fail(CPT_EHIP, "persistent schedule gave up waiting for a stage (spin budget exhausted)");
  cpt_status first = CPT_OK;
  for (int i = 0; i < n; i++) {
    lens[i] = (size_t)Dh[i].len;
    if (status) status[i] = Dh[i].status;
    if (Dh[i].status && first == CPT_OK) {
      first = (cpt_status)Dh[i].status;
      std::string m = reason_text(Dh[i].reason);
      if (Dh[i].reason == REASON_CAPACITY)
        m = "output capacity " + std::to_string(caps[i]) + " below stream length " + std::to_string(Dh[i].len);
      g_err = n > 1 ? "field " + std::to_string(i) + ": " + m : m;
    }
  }
  return first;
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
  if (s[0] != (STREAM_MAGIC | (STREAM_VERSION << 32))) return fail(CPT_ECORRUPT, "bad magic or version");
  if (s[1] < 2 || s[2] < 2 || s[3] < 1 || s[1] > 32768 || s[2] > 32768 || s[3] > (1u << 20))
    return fail(CPT_ECORRUPT, "bad dimensions");
  if ((double)s[1] * (double)s[2] * (double)s[3] >= 2147483648.0) return fail(CPT_ECORRUPT, "too many vertices");
  if (s[7] != (uint64_t)QR || s[8] != (uint64_t)TILE || s[16] != (uint64_t)NMAX || s[17] != (uint64_t)CHUNK ||
      s[18] != (uint64_t)MAXLEN || s[19] != (uint64_t)SL_STRIDE)
    return fail(CPT_ECORRUPT, "unsupported format constants");
  int64_t k = (int64_t)s[4];
  if (k < -80 || k > 120) return fail(CPT_ECORRUPT, "bad exponent");
  if (s[6] > 8388607 || s[9] > 4 || s[10] < 1 || s[10] > 1024) return fail(CPT_ECORRUPT, "bad parameters");
  uint64_t K = s[9] == 2 ? 2 : (s[9] >= 3 ? 4 : 1);
  if (s[11] != K || s[13] > 62 || s[15] > 62 || s[12] > 2147483647u || s[14] > 2147483647u)
    return fail(CPT_ECORRUPT, "bad predictor parameters");
  if (s[31] != 0 && s[31] != ZBE_TAG) return fail(CPT_ECORRUPT, "bad container tag");
  const bool zbe = s[31] == ZBE_TAG;
  uint64_t total = HDR_BYTES;
  for (int i = 0; i < 8; i++) {
    if (s[20 + i] % 4 || s[20 + i] > ((uint64_t)1 << 40)) return fail(CPT_ECORRUPT, "bad section length");
    total += s[20 + i];
    P->sec[i] = s[20 + i];
  }
  if (total != s[30]) return fail(CPT_ECORRUPT, "section lengths do not add up");
  // a plain stream holds every section, a container at least its block table
  if (zbe ? len < HDR_BYTES + 4 * zbe_blocks(total) : total > len)
    return fail(CPT_ECORRUPT, "stream shorter than its sections");
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
  I.backend = zbe ? 1 : 0;
  I.pad = 0;
  P->cx = (int64_t)s[12];
  P->sx = (int64_t)s[13];
  P->cy = (int64_t)s[14];
  P->sy = (int64_t)s[15];
  return CPT_OK;
}

// ---------------------------------------------------------- decompress
__global__ void k_gather_headers(const uint8_t* const* __restrict__ ptrs, int n, uint32_t* __restrict__ out) {
  const int f = blockIdx.x, i = threadIdx.x;
  if (f < n && i < (int)(HDR_BYTES / 4)) out[(size_t)f * (HDR_BYTES / 4) + i] = ((const uint32_t*)ptrs[f])[i];
}

// Host plan of a batched decompression, from the parsed headers of the
// streams that pass the header checks.
struct DPlan {
  int n = 0, maxT = 0;
  std::vector<DecDesc> D;
  std::vector<int> ord;
  std::vector<long long> mpre, cxpre, cqpre, dxpre, dqpre, spre, rpre, mtab;
  std::vector<long long> upre, ioff;  // containers: blocks per stream, scratch offsets of their expansions
  std::vector<int> m_at;
  long long Ntot = 0, CX = 0, CQ = 0, QS = 0, NB = 0, Stot = 0, ZB = 0, IB = 0;
};

struct DBufs {
  DecDesc* D;
  int* ord;
  long long *mpre, *cxpre, *cqpre, *dxpre, *dqpre, *spre, *rpre, *mtab, *upre;
  size_t tables_bytes;
  uint8_t* inner;   // expansions of the containers
  long long* uoff;  // per container block: its offset in the container's payload
  DecodeBufs B;
};

cpt_status carve_dec(Arena& A, const DPlan& P, DBufs& b) {
  A.used = 0;
  const int n = P.n;
  const size_t N = (size_t)P.Ntot, CX = (size_t)P.CX, CQ = (size_t)P.CQ, S = (size_t)P.Stot;
  struct Item {
    void** p;
    size_t bytes;
  };
  std::vector<Item> tables = {
      {(void**)&b.D, sizeof(DecDesc) * n},  {(void**)&b.ord, 4 * (size_t)n},
      {(void**)&b.mpre, vec_bytes(P.mpre)}, {(void**)&b.cxpre, vec_bytes(P.cxpre)},
      {(void**)&b.cqpre, vec_bytes(P.cqpre)}, {(void**)&b.dxpre, vec_bytes(P.dxpre)},
      {(void**)&b.dqpre, vec_bytes(P.dqpre)}, {(void**)&b.spre, vec_bytes(P.spre)},
      {(void**)&b.rpre, vec_bytes(P.rpre)}, {(void**)&b.mtab, vec_bytes(P.mtab)},
      {(void**)&b.upre, vec_bytes(P.upre)},
  };
  std::vector<Item> rest = {
      {(void**)&b.B.lut, 8 * (size_t)n * LUT_WORDS}, {(void**)&b.B.xw, 4 * CX + 16},
      {(void**)&b.B.xwofs, 4 * CX + 16},                  {(void**)&b.B.qw, 4 * CQ + 16},
      {(void**)&b.B.qwofs, 4 * CQ + 16},                  {(void**)&b.B.xs, 2 * N},
      {(void**)&b.B.qs, 2 * (size_t)P.QS + 16},           {(void**)&b.B.sn, 4 * S + 16},
      {(void**)&b.B.sq, 4 * S + 16},                      {(void**)&b.B.sr, 4 * S + 16},
      {(void**)&b.B.sro, 4 * S + 16},                     {(void**)&b.B.modes, (size_t)P.NB + 16},
      {(void**)&b.B.cur, 8 * N},
      {(void**)&b.B.part, 4 * (scan_partials_size(std::max(S, std::max(CX, CQ))) + 16)},
      {(void**)&b.inner, (size_t)P.IB + 16},
      {(void**)&b.uoff, 8 * (size_t)P.ZB + 16},
  };
  std::vector<size_t> offs;
  size_t t0 = 0;
  for (size_t i = 0; i < tables.size(); i++) {
    size_t o = A.off(tables[i].bytes);
    if (i == 0) t0 = o;
    offs.push_back(o);
  }
  b.tables_bytes = A.used - t0;
  for (auto& it : rest) offs.push_back(A.off(it.bytes));
  cpt_status st = reserve(A);
  if (st) return st;
  size_t k = 0;
  for (auto& it : tables) *it.p = A.base + offs[k++];
  for (auto& it : rest) *it.p = A.base + offs[k++];
  return CPT_OK;
}

// Decompress n streams; status (host, n) receives each stream's outcome.
// Every stream's outcome into status (host, may be NULL); the first failure,
// if any, is returned with its message.
cpt_status report_streams(int n, const std::vector<int32_t>& st_f, const std::vector<std::string>& why,
                          int32_t* status) {
  cpt_status first = CPT_OK;
  for (int i = 0; i < n; i++) {
    if (status) status[i] = st_f[i];
    if (st_f[i] && first == CPT_OK) {
      first = (cpt_status)st_f[i];
      g_err = n > 1 ? "stream " + std::to_string(i) + ": " + why[i] : why[i];
    }
  }
  return first;
}

cpt_status decompress_batch_impl(int n, const uint8_t* const* streams, const size_t* lens, float* const* fields,
                                 const size_t* caps, int32_t* status, hipStream_t s) {
  if (n < 1 || n > 65536) return fail(CPT_EINVAL, "batch size must be in 1..65536");
  if (!streams || !lens || !fields || !caps) return fail(CPT_EINVAL, "null pointer");
  std::vector<int32_t> st_f(n, CPT_OK);
  std::vector<std::string> why(n);
  int safe = -1;  // first stream long enough for a header
  for (int i = 0; i < n; i++) {
    if (!streams[i] || !fields[i]) return fail(CPT_EINVAL, "stream " + std::to_string(i) + ": null pointer");
    if ((uintptr_t)streams[i] & 3) return fail(CPT_EINVAL, "stream must be 4-byte aligned");
    if (lens[i] < HDR_BYTES) {
      st_f[i] = CPT_ECORRUPT;
      why[i] = "stream shorter than its header";
    } else if (safe < 0) {
      safe = i;
    }
  }
  // nothing to read: no device work and no staging at all
  if (safe < 0) return report_streams(n, st_f, why, status);
  cpt_status st;
  Arena* Ap = arena_for_device(&st);
  if (!Ap) return st;
  Arena& A = *Ap;
  std::lock_guard<std::mutex> lk(A.mu);
  // ---- headers: one gather, one copy (streams too short for a header read
  // the header of one that is not; their status is already set)
  {
    A.used = 0;
    const size_t po = A.off(8 * (size_t)n), ho = A.off(HDR_BYTES * (size_t)n);
    st = reserve(A);
    if (st) return st;
    st = reserve_stage(A, HDR_BYTES * (size_t)n + 8 * (size_t)n + 256);
    if (st) return st;
    std::vector<const uint8_t*> ptrs(n);
    for (int i = 0; i < n; i++) ptrs[i] = st_f[i] ? streams[safe] : streams[i];
    std::memcpy(A.stage, ptrs.data(), 8 * (size_t)n);
    HIPCHK(hipMemcpyAsync(A.base + po, A.stage, 8 * (size_t)n, hipMemcpyHostToDevice, s));
    k_gather_headers<<<n, 64, 0, s>>>((const uint8_t* const*)(A.base + po), n, (uint32_t*)(A.base + ho));
    HIPCHK(hipMemcpyAsync(A.stage, A.base + ho, HDR_BYTES * (size_t)n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  std::vector<uint8_t> hdr((const uint8_t*)A.stage, (const uint8_t*)A.stage + HDR_BYTES * (size_t)n);
  // ---- plan
  DPlan P;
  std::vector<int> live;
  for (int i = 0; i < n; i++) {
    if (st_f[i]) continue;
    Parsed Q;
    cpt_status ps = parse_header(hdr.data() + HDR_BYTES * (size_t)i, lens[i], &Q);
    if (ps) {
      st_f[i] = ps;
      why[i] = g_err;
      continue;
    }
    const cpt_info& I = Q.info;
    const int H = I.H, W = I.W, T = I.T, bt = I.mode_bt, K = I.K;
    const long long N = (long long)H * W * T;
    if ((unsigned long long)(2 * N) > (unsigned long long)caps[i]) {
      st_f[i] = CPT_ECAPACITY;
      why[i] = "output holds " + std::to_string(caps[i]) + " floats, the stream needs " + std::to_string(2 * N);
      continue;
    }
    const int tx = (W + TILE - 1) / TILE, ty = (H + TILE - 1) / TILE;
    const int G = (T + bt - 1) / bt;
    const long long ndec = K > 1 ? decided_before(G, bt, T) : 0;
    const long long nblk = ndec * tx * ty;
    const int mb = mode_bits(K);
    const long long nq = (long long)I.n_q, nraw = (long long)I.n_raw;
    const long long nchx = (N + CHUNK - 1) / CHUNK, nchq = (nq + CHUNK - 1) / CHUNK;
    std::string bad;
    if ((long long)Q.sec[0] != 4 * ((nblk * mb + 31) / 32)) bad = "mode section size";
    else if (nq > 2 * N || nraw > 2 * N || (nq & 1)) bad = "symbol counts";
    else if ((long long)Q.sec[7] != 4 * nraw) bad = "raw section size";
    else if ((long long)Q.sec[2] != 4 * nchx || (long long)Q.sec[5] != 4 * nchq) bad = "chunk table size";
    else if (Q.sec[1] < 4 || Q.sec[4] < 4) bad = "codebook size";
    if (!bad.empty()) {
      st_f[i] = CPT_ECORRUPT;
      why[i] = bad;
      continue;
    }
    DecDesc d{};
    d.p.H = H;
    d.p.W = W;
    d.p.T = T;
    d.p.k = I.k;
    d.p.eps = (int)I.eps;
    d.p.tx = tx;
    d.p.ty = ty;
    d.p.predictor = I.predictor;
    d.p.K = K;
    d.p.bt = bt;
    d.p.cx = Q.cx;
    d.p.sx = Q.sx;
    d.p.cy = Q.cy;
    d.p.sy = Q.sy;
    d.N = N;
    d.nq = nq;
    d.nraw = nraw;
    d.nchx = nchx;
    d.nchq = nchq;
    d.nblk = nblk;
    d.mb = mb;
    size_t o = HDR_BYTES;
    for (int k = 0; k < 8; k++) {
      d.sec[k] = (const uint32_t*)(streams[i] + o);
      d.secw[k] = (long long)(Q.sec[k] / 4);
      o += Q.sec[k];
    }
    d.out = fields[i];
    if (I.backend) {
      // sections are found in the container's expansion (pointers set once
      // the scratch is carved); offsets relative to its start for now
      d.zin = streams[i];
      d.zlen = (long long)lens[i];
      d.ilen = (long long)I.total_len;
      d.nzb = (long long)zbe_blocks(I.total_len);
      d.zbb = P.ZB;
      P.ZB += d.nzb;
    }
    P.ioff.push_back(P.IB);
    if (I.backend) P.IB += (long long)((I.total_len + 255) & ~(uint64_t)255);
    d.voff = P.Ntot;
    d.soff = P.Stot;
    d.nseg = (long long)T * H * tx;
    d.cxb = P.CX;
    d.cqb = P.CQ;
    d.qsb = P.QS;
    d.mbase = P.NB;
    d.mtb = (long long)P.mtab.size();
    for (int t = 0; t < T; t++) {
      long long mo = -1;
      if (K > 1 && t >= 1) {
        const int g = t / bt;
        if (group_decided(g, bt, T)) mo = (long long)decided_before(g, bt, T) * tx * ty;
      }
      P.mtab.push_back(mo);
    }
    P.Ntot += N;
    P.Stot += d.nseg;
    P.CX += nchx;
    P.CQ += nchq;
    P.QS += nq;
    P.NB += nblk;
    P.maxT = std::max(P.maxT, T);
    P.D.push_back(d);
    live.push_back(i);
  }
  const int m = (int)P.D.size();
  P.n = m;
  if (m > 0) {
    for (auto* v : {&P.mpre, &P.cxpre, &P.cqpre, &P.dxpre, &P.dqpre, &P.spre, &P.rpre, &P.upre}) v->assign(m + 1, 0);
    for (int j = 0; j < m; j++) {
      const DecDesc& d = P.D[j];
      P.upre[j + 1] = P.upre[j] + d.nzb;
      P.mpre[j + 1] = P.mpre[j] + (d.nblk + 255) / 256;
      P.cxpre[j + 1] = P.cxpre[j] + d.nchx;
      P.cqpre[j + 1] = P.cqpre[j] + d.nchq;
      P.dxpre[j + 1] = P.dxpre[j] + (d.nchx + 255) / 256;
      P.dqpre[j + 1] = P.dqpre[j] + (d.nchq + 255) / 256;
      P.spre[j + 1] = P.spre[j] + (d.nseg + 255) / 256;
    }
    P.ord.resize(m);
    for (int j = 0; j < m; j++) P.ord[j] = j;
    std::stable_sort(P.ord.begin(), P.ord.end(), [&](int a, int b) { return P.D[a].p.T > P.D[b].p.T; });
    for (int j = 0; j < m; j++) {
      const DecDesc& d = P.D[P.ord[j]];
      P.rpre[j + 1] = P.rpre[j] + (long long)d.p.tx * d.p.ty;
    }
    P.m_at.assign(P.maxT, 0);
    int mm = m;
    for (int t = 0; t < P.maxT; t++) {
      while (mm > 0 && P.D[P.ord[mm - 1]].p.T <= t) mm--;
      P.m_at[t] = mm;
    }
    for (auto v : {P.mpre.back(), P.dxpre.back() + P.dqpre.back(), P.spre.back(), P.rpre.back()})
      if (v >= 2147483647LL) return fail(CPT_EINVAL, "batch too large for one launch");
    if (P.upre.back() >= 2147483647LL) return fail(CPT_EINVAL, "batch too large for one launch");
    DBufs b;
    st = carve_dec(A, P, b);
    if (st) return st;
    for (int j = 0; j < m; j++) {
      DecDesc& d = P.D[j];
      if (!d.nzb) continue;
      // the container's sections are read from its expansion
      d.inner = b.inner + P.ioff[j];
      const uint8_t* base0 = (const uint8_t*)d.sec[0] - HDR_BYTES;
      for (int k = 0; k < 8; k++) d.sec[k] = (const uint32_t*)(d.inner + ((const uint8_t*)d.sec[k] - base0));
    }
    const size_t rb_off = (b.tables_bytes + 255) & ~(size_t)255;
    st = reserve_stage(A, rb_off + sizeof(DecDesc) * m + 64);
    if (st) return st;
    {
      const char* base = (const char*)b.D;
      auto put = [&](const void* dev, const void* src, size_t bytes) {
        if (bytes) std::memcpy(A.stage + ((const char*)dev - base), src, bytes);
      };
      put(b.D, P.D.data(), sizeof(DecDesc) * m);
      put(b.ord, P.ord.data(), 4 * (size_t)m);
      put(b.mpre, P.mpre.data(), vec_bytes(P.mpre));
      put(b.cxpre, P.cxpre.data(), vec_bytes(P.cxpre));
      put(b.cqpre, P.cqpre.data(), vec_bytes(P.cqpre));
      put(b.dxpre, P.dxpre.data(), vec_bytes(P.dxpre));
      put(b.dqpre, P.dqpre.data(), vec_bytes(P.dqpre));
      put(b.spre, P.spre.data(), vec_bytes(P.spre));
      put(b.rpre, P.rpre.data(), vec_bytes(P.rpre));
      put(b.mtab, P.mtab.data(), vec_bytes(P.mtab));
      put(b.upre, P.upre.data(), vec_bytes(P.upre));
    }
    HIPCHK(hipMemcpyAsync(b.D, A.stage, b.tables_bytes, hipMemcpyHostToDevice, s));
    // containers of the lossless stage are expanded first
    if (P.ZB > 0) launch_unzbe_b(b.D, m, b.upre, P.ZB, b.uoff, s);
    launch_decode_front_b(b.D, m, b.B, b.mpre, P.mpre.back(), b.cxpre, P.CX, b.cqpre, P.CQ, s);
    {
      TimeScope ts(FAM_DECODE, (uint64_t)(P.Ntot + P.QS), s);
      launch_decode_b(b.D, m, b.B, b.dxpre, P.dxpre.back(), b.dqpre, P.dqpre.back(), b.spre, P.spre.back(), P.Stot,
                      P.CX, P.CQ, s);
    }
    for (int t = 0; t < P.maxT; t++) {
      const int mt = P.m_at[t];
      uint64_t units = 0;
      for (int j = 0; j < mt; j++) units += (uint64_t)P.D[P.ord[j]].p.H * P.D[P.ord[j]].p.W;
      TimeScope ts(FAM_RECON, units, s);
      launch_reconstruct_b(b.D, b.ord, P.ord[0], b.rpre, mt, P.rpre[mt], t, b.mtab, b.B, s);
    }
    char* rb = A.stage + rb_off;
    HIPCHK(hipMemcpyAsync(rb, b.D, sizeof(DecDesc) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    harvest_timing();
    const DecDesc* Dh = (const DecDesc*)rb;
    for (int j = 0; j < m; j++) {
      const int i = live[j];
      if (Dh[j].status || Dh[j].err) {
        st_f[i] = CPT_ECORRUPT;
        why[i] = "stream failed a device check (code " + std::to_string(Dh[j].err) + ")";
      }
    }
  }
  return report_streams(n, st_f, why, status);
}

}  // namespace

// ================================================ allocation-free check
// cpt_verify_noalloc keeps every intermediate array of the check in one fixed
// device array that the library's code object holds on each GPU from load
// until the process ends.  The array's name is only a host-side stand-in:
// host code uses the device address taken once per device with
// hipGetSymbolAddress, never the name itself.
static __device__ __align__(256) unsigned char scratch[CPT_VERIFY_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mu;  // one call at a time per process: every call shares the array
unsigned char* g_na_ptr[NA_MAX_DEVICES] = {nullptr};

// Byte offsets of the check's arrays inside the scratch array for N vertices:
// range records of both fields (2 x 16 B), the false-case counters and the
// reduced error sums (4 x 8 B), fixed-point values, edge signs, both face
// masks and the per-workgroup error partials.
struct NaLayout {
  size_t range, res, masks, masks2, part, end;
};
constexpr size_t na_up(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr NaLayout na_layout(size_t N) {
  auto up = na_up;
  NaLayout L{};
  L.range = 0;
  L.res = 256;
  L.masks = 512;
  L.masks2 = L.masks + up(4 * N);
  L.part = L.masks2 + up(4 * N);
  L.end = L.part + up(16 * ((N + 255) / 256));  // compare_partials(N) workgroup partials
  return L;
}
static_assert(na_layout(CPT_VERIFY_NOALLOC_MAX_VERTICES).end <= CPT_VERIFY_NOALLOC_SCRATCH_BYTES &&
                  na_layout(CPT_VERIFY_NOALLOC_MAX_VERTICES + 1ull).end > CPT_VERIFY_NOALLOC_SCRATCH_BYTES,
              "the vertex limit is the largest field whose arrays fit the scratch array");

// the per-workgroup error partials of k_compare reduced in index order, as
// the host does for cpt_verify: max |a - b| and the sum of squares
__global__ void k_na_sum_partials(const double* __restrict__ part, size_t np, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double me = 0.0, se = 0.0;
  for (size_t i = 0; i < np; i++) {
    me = std::max(me, part[2 * i]);
    se += part[2 * i + 1];
  }
  out[0] = me;
  out[1] = se;
}

// the calling device's scratch address, looked up on its first call there
cpt_status na_scratch(unsigned char** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CPT_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= NA_MAX_DEVICES) return fail(CPT_EUNSUPPORTED, "device index beyond the supported 64");
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CPT_EHIP, std::string("hipGetSymbolAddress of the check's scratch array failed: ") +
                                hipGetErrorString(e));
    g_na_ptr[dev] = (unsigned char*)p;
  }
  *ptr = g_na_ptr[dev];
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
  g_tim.on = on > 0;
  g_tim.period = on > 0 ? on : 1;
  for (int i = 0; i < NFAM; i++) {
    g_tim.seen[i] = 0;
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
  // a container adds one table entry per block to a Huffman stream's bytes
  const size_t hb = huffman_bound(H, W, T);
  *max_bytes = hb + 4 * zbe_blocks(hb);
  return CPT_OK;
}

cpt_status cpt_compress(const float* field, int H, int W, int T, double eb, const cpt_options* opt, uint8_t* out,
                        size_t cap, size_t* out_len, void* stream) {
  try {
    if (!out_len) return fail(CPT_EINVAL, "null out_len");
    const int32_t hwt[3] = {H, W, T};
    return compress_batch_impl(1, &field, hwt, eb, opt, nullptr, &out, &cap, out_len, nullptr, nullptr,
                               (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_compress_debug(const float* field, int H, int W, int T, double eb, const cpt_options* opt,
                              uint8_t* out, size_t cap, size_t* out_len, int32_t* xi, uint8_t* xcode,
                              uint32_t* qcode, uint8_t* modes, float* feats, size_t* nblocks, void* stream) {
  try {
    if (!out_len) return fail(CPT_EINVAL, "null out_len");
    const int32_t hwt[3] = {H, W, T};
    Debug dbg;
    dbg.xi = xi;
    dbg.xcode = xcode;
    dbg.qcode = qcode;
    dbg.modes = modes;
    dbg.feats = feats;
    dbg.nblocks = nblocks;
    return compress_batch_impl(1, &field, hwt, eb, opt, nullptr, &out, &cap, out_len, nullptr, &dbg,
                               (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_compress_batch(int n, const float* const* fields, const int32_t* HWT, double eb,
                              const cpt_options* opt, const cpt_exec_options* ex, uint8_t* const* outs,
                              const size_t* caps, size_t* lens, int32_t* status, void* stream) {
  try {
    return compress_batch_impl(n, fields, HWT, eb, opt, ex, outs, caps, lens, status, nullptr, (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_autotune_batch(int n, const float* const* fields, const int32_t* HWT, double eb,
                              const cpt_options* opt_in, uint8_t* const* outs, const size_t* caps, int reps,
                              cpt_exec_options* best, double* ms, void* stream) {
  try {
    if (!best || reps < 1 || n < 1) return fail(CPT_EINVAL, "bad autotune arguments");
    hipStream_t s = (hipStream_t)stream;
    cpt_options opt;
    cpt_status st = check_options(opt_in, eb, &opt);
    if (st) return st;
    Plan P;
    st = make_plan(n, HWT, opt, eb, P);
    if (st) return st;
    // four schedules with the default field tile and phase workgroup, then
    // the fastest of them with the other field tiles, then the fastest so
    // far with one block per phase workgroup (filled in as they are timed)
    ExecChoice cand[CPT_TUNE_CANDIDATES] = {{CPT_SCHED_LAUNCH, 1, 0, false, 0, 2},
                                            {CPT_SCHED_FUSED, 1, 0, false, 0, 2},
                                            {CPT_SCHED_LAUNCH, 1, 0, true, 0, 2},
                                            {CPT_SCHED_FUSED, 1, 0, true, 0, 2}};
    static_assert(CPT_TUNE_CANDIDATES == 4 + FP_SHAPES - 1 + 1, "schedules, field tiles, phase workgroup");
    std::vector<size_t> lens(n), ref;
    std::vector<unsigned long long> dig(n), refdig;
    // the digests of the candidates' streams (the tuner is not a hot path:
    // one small allocation for its n digests) and the timing events,
    // released on every way out
    struct TuneRes {
      unsigned long long* ddig = nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      ~TuneRes() {
        if (ddig) (void)hipFree(ddig);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
      }
    } R;
    HIPCHK(hipMalloc((void**)&R.ddig, 8 * (size_t)n));
    HIPCHK(hipEventCreate(&R.e0));
    HIPCHK(hipEventCreate(&R.e1));
    unsigned long long* ddig = R.ddig;
    hipEvent_t e0 = R.e0, e1 = R.e1;
    int bi = -1;
    double bms = 0;
    for (int c = 0; c < CPT_TUNE_CANDIDATES; c++) {
      if (c >= 4 && c < 4 + FP_SHAPES - 1) {
        cand[c] = cand[bi];
        cand[c].ftile = c - 3;
      } else if (c == 4 + FP_SHAPES - 1) {
        cand[c] = cand[bi];
        cand[c].pblocks = 1;
      }
      st = compress_batch_impl(n, fields, HWT, eb, &opt, nullptr, outs, caps, lens.data(), nullptr, nullptr, s,
                               &cand[c]);
      if (st) break;
      if (ref.empty()) ref = lens;
      if (lens != ref) {
        st = fail(CPT_EHIP, "internal: schedules disagree on stream lengths");
        break;
      }
      // every candidate must write the same bytes, not only as many
      launch_hash_streams(n, outs, lens.data(), ddig, s);
      if (hipMemcpyAsync(dig.data(), ddig, 8 * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        st = fail(CPT_EHIP, "stream digest readback failed");
        break;
      }
      if (refdig.empty()) refdig = dig;
      if (dig != refdig) {
        st = fail(CPT_EHIP, "internal: schedules disagree on stream bytes");
        break;
      }
      float tot = 0.f;
      for (int r = 0; r < reps && !st; r++) {
        (void)hipEventRecord(e0, s);
        st = compress_batch_impl(n, fields, HWT, eb, &opt, nullptr, outs, caps, lens.data(), nullptr, nullptr, s,
                                 &cand[c]);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        tot += t;
      }
      if (st) break;
      const double m = tot / reps;
      if (ms) ms[c] = m;
      if (bi < 0 || m < bms) {
        bi = c;
        bms = m;
      }
    }
    if (st) return st;
    ExecChoice b = cand[bi];
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[P.key] = b;
    }
    *best = cpt_exec_options{sizeof(cpt_exec_options), b.schedule, b.group, b.grid, b.graph ? 1 : 0, b.ftile, b.pblocks};
    return CPT_OK;
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

cpt_status cpt_decompress(const uint8_t* bytes, size_t len, float* field, size_t field_cap, void* stream) {
  try {
    if (!bytes || !field) return fail(CPT_EINVAL, "null pointer");
    return decompress_batch_impl(1, &bytes, &len, &field, &field_cap, nullptr, (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_decompress_batch(int n, const uint8_t* const* streams, const size_t* lens, float* const* fields,
                                const size_t* field_caps, int32_t* status, void* stream) {
  try {
    return decompress_batch_impl(n, streams, lens, fields, field_caps, status, (hipStream_t)stream);
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

cpt_status cpt_field_params(const float* field, int H, int W, int T, int eb_mode, double eb, int* k,
                            double* eb_abs, int64_t* eps, void* stream) {
  try {
    if (!field || !k || !eb_abs || !eps) return fail(CPT_EINVAL, "null pointer");
    const cpt_options o{sizeof(cpt_options), eb_mode, CPT_PRED_MIX2, 1, 1.0, 1.0, nullptr};
    cpt_options opt;
    cpt_status st = check_options(&o, eb, &opt);
    if (st) return st;
    const int32_t hwt[3] = {H, W, T};
    Plan P;
    st = make_plan(1, hwt, opt, eb, P);
    if (st) return st;
    P.D[0].field = field;
    hipStream_t s = (hipStream_t)stream;
    Arena* Ap = arena_for_device(&st);
    if (!Ap) return st;
    Arena& A = *Ap;
    std::lock_guard<std::mutex> lk(A.mu);
    // the compressor's own range and parameter kernels, on one field
    A.used = 0;
    const size_t od = A.off(sizeof(FieldDesc)), orp = A.off(vec_bytes(P.rpre)),
                 org = A.off(16 * (size_t)RANGE_SLOTS * RANGE_SLOT_STRIDE);
    st = reserve(A);
    if (st) return st;
    st = reserve_stage(A, sizeof(FieldDesc) + vec_bytes(P.rpre) + 64);
    if (st) return st;
    std::memcpy(A.stage, P.D.data(), sizeof(FieldDesc));
    std::memcpy(A.stage + sizeof(FieldDesc), P.rpre.data(), vec_bytes(P.rpre));
    FieldDesc* D = (FieldDesc*)(A.base + od);
    const long long* rpre = (const long long*)(A.base + orp);
    HIPCHK(hipMemcpyAsync(D, A.stage, sizeof(FieldDesc), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(A.base + orp, A.stage + sizeof(FieldDesc), vec_bytes(P.rpre), hipMemcpyHostToDevice, s));
    launch_params_b(D, 1, rpre, P.rpre[1], (int4*)(A.base + org), s);
    HIPCHK(hipMemcpyAsync(A.stage, D, sizeof(FieldDesc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    const FieldDesc* Dh = (const FieldDesc*)A.stage;
    if (Dh->status) return fail(CPT_EINVAL, reason_text(Dh->reason));
    *k = Dh->p.k;
    *eb_abs = Dh->eb_abs;
    *eps = Dh->p.eps;
    return CPT_OK;
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
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
  st = carve(A, N, b);
  if (st) return st;
  Range r;
  st = field_range(field, 2 * N, b, A, s, &r);
  if (st) return st;
  if (std::ldexp(r.ma, k) >= 16777216.0) return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
  launch_maskpass(field, H, W, T, k, b.masks, s);
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

cpt_status cpt_tracks(const float* field, int H, int W, int T, int k, uint64_t* bad_tets, uint64_t* n_tracks,
                      void* stream) {
  try {
    if (!field || !bad_tets || !n_tracks) return fail(CPT_EINVAL, "null pointer");
    cpt_status st = check_dims(H, W, T);
    if (st) return st;
    if (k < -80 || k > 120) return fail(CPT_EINVAL, "k must be in -80..120");
    hipStream_t s = (hipStream_t)stream;
    Arena* Ap = arena_for_device(&st);
    if (!Ap) return st;
    Arena& A = *Ap;
    std::lock_guard<std::mutex> lk(A.mu);
    const size_t N = (size_t)H * W * T;
    // pass 1: how many crossed faces
    Bufs b;
    st = carve(A, N, b);
    if (st) return st;
    Range r;
    st = field_range(field, 2 * N, b, A, s, &r);
    if (st) return st;
    if (std::ldexp(r.ma, k) >= 16777216.0) return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
    launch_maskpass(field, H, W, T, k, b.masks, s);
    launch_count_faces(b.masks, N, b.nonll, s);
    launch_scan(b.nonll, N, b.qofs, b.part, b.tot, s);
    HIPCHK(hipMemcpyAsync(A.host, b.tot, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const size_t M = *(const uint32_t*)A.host;
    if (M >= 2147483647u) return fail(CPT_EUNSUPPORTED, "2^31 or more crossed faces");
    // pass 2: the same masks and offsets with room for the union-find
    st = carve(A, N, b);
    if (st) return st;
    const size_t op = A.off(4 * M + 4), ot = A.off(16);
    st = reserve(A);
    if (st) return st;
    st = carve(A, N, b);  // the arena may have moved: carve again, same offsets
    if (st) return st;
    (void)A.off(4 * M + 4);
    (void)A.off(16);
    int* parent = (int*)(A.base + op);
    unsigned long long* ctr = (unsigned long long*)(A.base + ot);
    launch_maskpass(field, H, W, T, k, b.masks, s);
    launch_count_faces(b.masks, N, b.nonll, s);
    launch_scan(b.nonll, N, b.qofs, b.part, b.tot, s);
    launch_tracks(b.masks, b.qofs, H, W, T, (long long)M, parent, ctr, s);
    HIPCHK(hipMemcpyAsync(A.host, ctr, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    *bad_tets = A.host[0];
    *n_tracks = A.host[1];
    return CPT_OK;
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
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
  st = carve(A, N, b);
  if (st) return st;
  Range ra, rb;
  st = field_range(a, 2 * N, b, A, s, &ra);
  if (st) return st;
  st = field_range(bf, 2 * N, b, A, s, &rb);
  if (st) return st;
  if (std::ldexp(std::max(ra.ma, rb.ma), k) >= 16777216.0) return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
  launch_maskpass(a, H, W, T, k, b.masks, s);
  launch_maskpass(bf, H, W, T, k, b.masks2, s);
  launch_compare(b.masks, b.masks2, a, bf, N, b.fc, b.cpart, s);
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

cpt_status cpt_verify_noalloc(const float* a, const float* bf, int H, int W, int T, int k,
                              cpt_verify_result* res, void* stream) {
  try {
    if (!a || !bf || !res) return fail(CPT_EINVAL, "null pointer");
    cpt_status st = check_dims(H, W, T);
    if (st) return st;
    if (k < -80 || k > 120) return fail(CPT_EINVAL, "k must be in -80..120");
    const size_t N = (size_t)H * W * T;
    const NaLayout L = na_layout(N);
    if (L.end > CPT_VERIFY_NOALLOC_SCRATCH_BYTES)
      return fail(CPT_EUNSUPPORTED, "the allocation-free check holds at most " +
                                        std::to_string(CPT_VERIFY_NOALLOC_MAX_VERTICES) + " vertices; this field has " +
                                        std::to_string(N));
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_na_mu);
    unsigned char* base = nullptr;
    st = na_scratch(&base);
    if (st) return st;
    int* ra = (int*)(base + L.range);
    int* rb = ra + 4;
    unsigned long long* fc = (unsigned long long*)(base + L.res);
    double* sums = (double*)(base + L.res + 16);
    uint32_t* ma = (uint32_t*)(base + L.masks);
    uint32_t* mb = (uint32_t*)(base + L.masks2);
    double* part = (double*)(base + L.part);
    // value ranges of both fields (each record is cleared by its own kernel)
    launch_range(a, 2 * N, ra, s);
    launch_range(bf, 2 * N, rb, s);
    int hr[8];  // pageable host memory: no pinned staging is allocated
    HIPCHK(hipMemcpyAsync(hr, ra, sizeof(hr), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hr[3] || hr[7]) return fail(CPT_EINVAL, "field contains NaN or Inf");
    float fa, fb;
    std::memcpy(&fa, &hr[2], 4);
    std::memcpy(&fb, &hr[6], 4);
    if (std::ldexp(std::max((double)fa, (double)fb), k) >= 16777216.0)
      return fail(CPT_EINVAL, "max|x| 2^k must be below 2^24");
    // crossed faces of both fields, then the comparison (counters cleared by
    // a kernel inside launch_compare)
    launch_maskpass(a, H, W, T, k, ma, s);
    launch_maskpass(bf, H, W, T, k, mb, s);
    launch_compare(ma, mb, a, bf, N, fc, part, s);
    k_na_sum_partials<<<1, 64, 0, s>>>(part, compare_partials(N), sums);
    uint64_t hres[4];
    HIPCHK(hipMemcpyAsync(hres, fc, sizeof(hres), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    double me, se;
    std::memcpy(&me, &hres[2], 8);
    std::memcpy(&se, &hres[3], 8);
    res->fc_t = hres[0];
    res->fc_s = hres[1];
    res->max_err = me;
    const double mn = (double)key_to_float(hr[0]), mx = (double)key_to_float(hr[1]);
    const double mse = se / (double)(2 * N);
    res->psnr = mse > 0 ? 20.0 * std::log10(mx - mn) - 10.0 * std::log10(mse) : INFINITY;
    return CPT_OK;
  } catch (...) {
    return fail(CPT_EHIP, "unexpected exception");
  }
}

}  // extern "C"
