// batch.hpp — per-field descriptors for the device-driven compression path.
//
// Compression of one field or of many fields of uneven sizes runs the same
// kernels: every launch covers all fields that take part in it, every
// workgroup finds its field in a prefix table of per-field workgroup counts,
// and every data-dependent quantity (fixed-point exponent, bound, stream
// layout, lengths) lives in device memory.  The host only enqueues work, so
// a whole batch can be captured into one HIP graph and replayed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace cpt {

// per-field status (the cpt_status values) and failure reasons
enum { STATUS_OK = 0, STATUS_EINVAL = -1, STATUS_ECAPACITY = -4 };
enum { REASON_NONE = 0, REASON_NONFINITE = 1, REASON_MAGNITUDE = 2, REASON_CAPACITY = 3 };

// stream format: a header of 32 little-endian 64-bit slots, then 8 sections
constexpr int HDR_SLOTS = 32;
constexpr size_t HDR_BYTES = 8 * HDR_SLOTS;
constexpr uint64_t STREAM_MAGIC = 0x31545043ull;  // "CPT1"
constexpr uint64_t STREAM_VERSION = 1;
constexpr int SL_STRIDE = 2;  // stride of the rate-estimate subgrid
// lossless stage after Huffman coding: zero-byte elision in blocks of the body
constexpr int ZBE_BLOCK = 4096;
constexpr uint64_t ZBE_TAG = 0x315A4245ull;  // header slot 31 of a container ("EBZ1")

struct FieldDesc {
  // fixed by the dimensions and the call (host)
  int H, W, T, tx, ty;
  int ndec;              // decided predictor groups
  long long N;           // vertices
  long long voff;        // first vertex in the concatenated vertex arrays
  long long ro;          // first run of 16 vertices in the concatenated run arrays
  long long cxb;         // first bound-code chunk in the concatenated chunk arrays
  long long cqb;         // first residual-code chunk (room for 2N symbols)
  long long mbase;       // first predictor block in the concatenated mode array
  long long nchx;        // bound-code chunks
  long long mwords;      // words of the predictor-class section
  const float* field;    // input (2,T,H,W)
  uint8_t* out;          // output stream
  long long cap;         // its capacity in bytes
  int32_t* xi_dbg;       // optional per-vertex bounds
  float* feats_dbg;      // optional per-block features
  // with the lossless stage: out / cap above are the Huffman stream in
  // library scratch, zout / zcap the caller's container output
  uint8_t* zout;
  long long zcap;
  long long zbase;       // first block in the concatenated block tables
  long long ilen;        // Huffman stream length once the container is laid out
  int eb_mode, predictor, K, bt;
  double eb, dt_dx, dt_dy;
  // derived on the device
  FieldParams p;
  double eb_abs;
  int status, reason;
  long long len;         // stream length (also when it does not fit)
  long long sec[8];      // section lengths in bytes
  long long off[8];      // section offsets in bytes
  long long nq, nraw, nchq;
};

// What the kernels of one launch see: the descriptors, the order in which
// the launch visits the fields, and the concatenated scratch arrays.
struct BatchView {
  FieldDesc* D;
  const int* ord;
  int ord0;  // ord[0], so that a launch over one field reads no table first
  int2* cur;
  uint8_t* flags;
  uint8_t* xcode;
  uint32_t* qcode;
  uint8_t* modes;
  const int64_t* tlog;
  const uint16_t* selw;
};

// Predictor classes available to a phase of frame t.
enum { MODES_NONE = 0, MODES_READ = 1, MODES_DECIDE = 2 };

// One stage (frame t, colour c) of one field in the persistent schedule.
struct SchedSeg {
  int f, t, c, mstate, gidx, nb;
  unsigned need;  // items of the field that finish before this stage may start
  int pad;
};

// index j with pre[j] <= e < pre[j + 1], for pre[0] = 0 <= e < pre[n]
__device__ __forceinline__ int find_field(const long long* pre, int n, long long e) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// column-padded colour-phase grid of a field: (tx + 2) / 3 workgroups per row
__host__ __device__ __forceinline__ int phase_cols(int tx) { return (tx + 2) / 3; }

// launchers (k_field.hip)
constexpr long long RANGE_SPAN_FLOATS = 256 * 256;
// range slots per field (int4 each, RANGE_SLOT_STRIDE int4 apart)
constexpr int RANGE_SLOTS = 32, RANGE_SLOT_STRIDE = 8;
// range, parameters, then conversion, edges, faces and flags fused in one
// time-marching kernel over 32x16 tiles (rpre: range workgroups per field,
// fpre: tiles per field)
// range and parameters only (k, eps', displacement factors into D[f].p)
void launch_params_b(FieldDesc* D, int n, const long long* rpre, long long rblocks, int4* range, hipStream_t s);
void launch_fieldpass_b(FieldDesc* D, int n, const long long* rpre, long long rblocks, const long long* fpre,
                        long long fblocks, int4* range, int2* cur, uint8_t* flags, int shape, hipStream_t s);
// tile shapes of the fused field pass (an execution choice: same output)
constexpr int FP_SHAPES = 3;
constexpr int FP_SHAPE_TW[FP_SHAPES] = {32, 64, 16};
constexpr int FP_SHAPE_TH[FP_SHAPES] = {16, 8, 32};

// launchers (k_entropy.hip); gpre: HIST_WG-vertex histogram workgroups per
// field, hpre: HIST_SPAN-vertex workgroups, cxpre / cqpre: bound-code /
// residual-code chunk capacity per field
constexpr long long HIST_SPAN_VERTICES = 256 * 16;
constexpr long long HIST_WG_VERTICES = 4 * HIST_SPAN_VERTICES;
constexpr int HIST_SLOTS = 8;  // partial histograms per field and alphabet
struct EntropyBufs {
  uint32_t *xhist, *qhist, *xcb, *qcb, *used;
  HuffTables *xt, *qt;
  // per run of 16 consecutive vertices of a field: residual-coded vertices
  // and their exclusive prefix, raw words and their exclusive prefix
  uint32_t *sn, *sq, *sr, *sro;
  uint16_t* qsym;
  uint32_t *xbits, *xwords, *xwofs, *qbits, *qwords, *qwofs;
  uint32_t* part;
};
void launch_codes_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* hpre,
                    long long hblocks, const long long* gpre, long long gblocks, long long Rtot, hipStream_t s);
void launch_chunks_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* cxpre,
                     long long cxtot, const long long* cqpre, long long cqtot, hipStream_t s);
void launch_assemble_b(FieldDesc* D, int n, const BatchView& B, const EntropyBufs& E, const long long* cxpre,
                       long long cxtot, const long long* cqpre, long long cqtot, const long long* hpre,
                       long long hblocks, hipStream_t s);

// ------------------------------------------------------- batched decoding
// Per-stream descriptor of a batched decompression: header values and
// section pointers (host), scratch offsets, and the device's verdict.
struct DecDesc {
  FieldParams p;            // dimensions and predictor parameters from the header
  long long N;              // vertices
  long long voff;           // first vertex in the concatenated per-vertex arrays
  long long nq, nraw;       // residual symbols and raw values (header)
  long long nchx, nchq;     // chunks of both code streams
  long long cxb, cqb;       // first chunk in the concatenated chunk arrays
  long long qsb;            // first residual symbol in the concatenated symbol array
  long long mbase, nblk;    // predictor classes: first and count
  long long mtb;            // first entry of the stream in the per-frame class-offset table
  long long soff, nseg;     // block rows (segments): first in the concatenated segment arrays, count
  int mb;                   // bits per predictor class
  const uint32_t* sec[8];   // the stream's sections (device)
  long long secw[8];        // their lengths in words
  float* out;               // decompressed field (2, T, H, W)
  // a container of the lossless stage: its bytes, length and blocks, the
  // first of them in the concatenated block offsets, and the scratch copy of
  // the Huffman stream it expands to (ilen bytes); nzb = 0 for a plain stream
  const uint8_t* zin;
  long long zlen, nzb, zbb, ilen;
  uint8_t* inner;
  uint32_t err;             // device error bits
  int status;               // 0 ok, else a cpt_status
};

// A segment is one block row: the vertices x in [16 bx, min(16 bx + 16, W))
// of row y of frame t, segment index (t H + y) tx + bx.  Segments follow
// the vertex order, so per-segment prefix sums of residual-coded vertices
// and raw words locate every vertex's symbols and raw words.
struct DecodeBufs {
  uint32_t* lut;            // two decoding tables of LUT_WORDS words per stream
  uint32_t *xw, *xwofs, *qw, *qwofs;  // chunk words and their prefix sums
  uint16_t *xs, *qs;        // decoded symbols
  uint32_t *sn, *sq;        // per segment: residual-coded vertices, their exclusive prefix
  uint32_t *sr, *sro;       // per segment: raw words, their exclusive prefix
  uint8_t* modes;
  int2* cur;
  uint32_t* part;
};

// k_entropy.hip: headers and tables (before decoding), decoding, offsets
void launch_decode_front_b(DecDesc* D, int n, const DecodeBufs& B, const long long* mpre, long long mblocks,
                           const long long* cxpre, long long cxtot, const long long* cqpre, long long cqtot,
                           hipStream_t s);
// spre: workgroups of 256 segments per stream; Stot: all segments
void launch_decode_b(DecDesc* D, int n, const DecodeBufs& B, const long long* dxpre, long long dxblocks,
                     const long long* dqpre, long long dqblocks, const long long* spre, long long sblocks,
                     long long Stot, long long CX, long long CQ, hipStream_t s);
// k_backend.hip: the lossless stage (zero-byte elision).  zblocks: the
// fields' most blocks together (from their Huffman streams' bounds), the
// size of the per-block tables; D[f].zbase: a field's first entry
void launch_zbe_b(FieldDesc* D, int n, long long zblocks, uint32_t* ztab, uint32_t* zlen, long long* zoff,
                  hipStream_t s);
// its inverse into each container's scratch copy (upre: blocks per stream)
void launch_unzbe_b(DecDesc* D, int n, const long long* upre, long long ublocks, long long* uoff, hipStream_t s);
// digests of n device byte strings (host arrays of pointers and lengths) into h[n]
void launch_hash_streams(int n, const uint8_t* const* p, const size_t* len, unsigned long long* h, hipStream_t s);

// k_decompress.hip: reconstruction of frame t of the first m streams of the
// launch order (pre: blocks per stream)
// mtab[mtb + t]: offset of frame t's predictor classes in the stream's
// class array, or -1 when frame t has none
void launch_reconstruct_b(DecDesc* D, const int* ord, int ord0, const long long* pre, int m, long long nblocks,
                          int t, const long long* mtab, const DecodeBufs& B, hipStream_t s);

// launchers (k_compress.hip)
void launch_modes_b(const BatchView& B, const long long* pre, int m, long long nblocks, int t, int gidx,
                    hipStream_t s);
// nb: blocks per workgroup without the fused predictor choice (1 or 2)
void launch_phase_b(const BatchView& B, const long long* pre, int m, long long nblocks, int t, int c,
                    int mstate, int gidx, bool fused, int nb, hipStream_t s);
// workgroups of the persistent kernel that fit on the current device at once
int persist_grid();
void launch_persist(const BatchView& B, const SchedSeg* seg, const long long* sstart, int nseg, long long nitems,
                    int group, int grid, unsigned* done, unsigned* ctl, hipStream_t s);

}  // namespace cpt
