/*
 * cptraj.h — C ABI of libcptraj, an MI355X (gfx950) implementation of
 * error-bounded lossy compression of 2D time-varying vector fields that
 * preserves every critical-point trajectory, after "Time-Varying Vector
 * Field Compression with Preserved Critical Point Trajectories"
 * (arXiv 2510.25143).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Fields are float32 arrays of shape (2, T, H, W): the u plane then the v
 *   plane, each [t][y][x] with x fastest.  The mesh is the regular grid split
 *   along each quad's main diagonal, extruded in time and cut into three
 *   tetrahedra per prism (Sec. III-C).
 * - Pointers marked "device" are HIP device pointers; "host" are host
 *   pointers.  The caller owns and allocates every buffer; the library never
 *   frees caller memory.  The library keeps a grow-only scratch arena per
 *   device for its intermediate arrays (allocated on first use, reused).
 * - `stream` is a hipStream_t passed as void*.  Work is ordered on it.  Calls
 *   that return a length or count to the host synchronise the stream before
 *   returning that value; output data is complete once the stream is
 *   synchronised.
 * - Every entry point returns a cpt_status; on failure cpt_last_error()
 *   gives a message (thread-local).  No C++ exception crosses the ABI.
 * - Supported sizes: 2 <= H, W <= 32768, 1 <= T, H*W*T < 2^31.
 */
#ifndef CPTRAJ_H
#define CPTRAJ_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPT_OK = 0,
  CPT_EINVAL = -1,       /* bad argument, non-finite input, unsupported size */
  CPT_ENOMEM = -2,       /* device allocation failed */
  CPT_ECORRUPT = -3,     /* stream fails a consistency check */
  CPT_ECAPACITY = -4,    /* output buffer too small; needed size reported */
  CPT_EHIP = -5,         /* HIP runtime error (message in cpt_last_error) */
  CPT_EUNSUPPORTED = -6  /* valid request the library does not handle */
} cpt_status;

/* Predictor choice (Sec. VI).  CPT_PRED_MIX2 is the paper's mixture of
 * predictors: per block and frame, Lorenzo or semi-Lagrangian (d_max = 2
 * cells) chosen by the rate estimate of Sec. VI-B.  MIX4 adds the
 * semi-Lagrangian backtrace step as a choice (d_max 1, 2 or 4 cells).
 * LEARNED picks among the same four classes with the selector network. */
typedef enum {
  CPT_PRED_LORENZO = 0,
  CPT_PRED_SL = 1,
  CPT_PRED_MIX2 = 2,
  CPT_PRED_MIX4 = 3,
  CPT_PRED_LEARNED = 4
} cpt_predictor;

typedef struct {
  uint32_t struct_size;   /* sizeof(cpt_options) */
  int32_t eb_mode;        /* 0: eb relative to max-min over both components
                             (default), 1: eb absolute */
  int32_t predictor;      /* cpt_predictor, default CPT_PRED_MIX2 */
  int32_t mode_bt;        /* frames per predictor block (>= 1, default 1) */
  double dt_dx, dt_dy;    /* time step over grid spacing for the
                             semi-Lagrangian backtrace (default 1.0) */
  const uint16_t* selector_w; /* device, bf16 selector weights (5124 values,
                                 16-byte aligned, else CPT_EINVAL) when
                                 predictor == CPT_PRED_LEARNED */
  int32_t backend;        /* lossless stage after Huffman coding (Sec. V):
                             0 none (default), 1 zero-byte elision of the
                             stream body in 4096-byte blocks.  A caller
                             passing the size of the struct without this
                             field gets 0. */
} cpt_options;

/* Parameters stored in a stream's header. */
typedef struct {
  int32_t H, W, T;
  int32_t k;          /* fixed-point exponent: x_fp = rint(x * 2^k) */
  double eb_abs;      /* absolute bound in field units */
  int64_t eps;        /* bound eps' in fixed-point units */
  int32_t predictor, mode_bt, K, R;
  uint64_t total_len, n_q, n_raw;  /* total_len: bytes of the Huffman stream */
  int32_t backend;    /* 1: the stream is a container of the lossless stage */
  int32_t pad;
} cpt_info;

/* Outcome of comparing two fields on the same fixed-point grid. */
typedef struct {
  uint64_t fc_t;      /* faces in time slices whose status or sign changed */
  uint64_t fc_s;      /* space-time faces across slabs that changed */
  double max_err;     /* max |a - b| over both components */
  double psnr;        /* 20 log10(range(a)) - 10 log10(MSE) */
} cpt_verify_result;

/* Largest stream cpt_compress can produce for these dimensions, with or
 * without the lossless stage. */
cpt_status cpt_compress_bound(int H, int W, int T, size_t* max_bytes);

/*
 * Compress a field (Alg. 3 with Alg. 4 and the predictors of Sec. VI; the
 * guarantees are those of Sec. IV-A: |x - x'| <= eb_abs pointwise, and every
 * space-time face keeps its crossed status and sign).
 *   field   device, (2,T,H,W) float32, all finite
 *   eb      error bound (relative in (0, 0.5], or absolute > 0)
 *   opt     host, may be NULL for defaults
 *   out     device, capacity `cap` bytes, 4-byte aligned
 *   out_len host, receives the stream length (also on CPT_ECAPACITY)
 * Synchronises `stream`.  The stream is bit-identical to the reference CPU
 * implementation's for the same input and options.
 */
cpt_status cpt_compress(const float* field, int H, int W, int T, double eb, const cpt_options* opt,
                        uint8_t* out, size_t cap, size_t* out_len, void* stream);

/* Same as cpt_compress, also writing per-vertex and per-block internals
 * (device buffers; any may be NULL): xi [N] int32 bound before quantization
 * (0 when lossless), xcode [N] bound code (24 = lossless), qcode [N] residual
 * codes u | v << 16, modes [nblocks] predictor class per block, feats
 * [nblocks][10] selector features; *nblocks receives the block count. */
cpt_status cpt_compress_debug(const float* field, int H, int W, int T, double eb, const cpt_options* opt,
                              uint8_t* out, size_t cap, size_t* out_len, int32_t* xi, uint8_t* xcode,
                              uint32_t* qcode, uint8_t* modes, float* feats, size_t* nblocks, void* stream);

/* ---- Batches of independent fields and execution control ----
 * A batch runs the compressor of cpt_compress over n fields of any sizes in
 * one device pipeline: every launch covers all fields that take part in it,
 * and nothing returns to the host before the final lengths.  The order of
 * work inside a field is the one of Sec. V (frame by frame, three colour
 * phases of 16x16 blocks per frame), so every stream is bit-identical to the
 * one cpt_compress writes for that field alone, whatever the schedule.
 * Schedules only change how that work is launched: */
typedef enum {
  CPT_SCHED_AUTO = 0,       /* the choice cpt_autotune_batch made for this
                               batch shape, else CPT_SCHED_LAUNCH */
  CPT_SCHED_LAUNCH = 1,     /* per frame: a predictor-choice launch, then
                               one launch per colour phase */
  CPT_SCHED_FUSED = 2,      /* per frame and colour: one launch that also
                               chooses the predictor class of its blocks */
  CPT_SCHED_PERSISTENT = 3  /* one persistent launch for all phases of all
                               fields: workgroups take numbered work items
                               (groups of blocks of one phase of one field)
                               and wait on per-field stage counters.
                               Disabled: its launch did not complete on the
                               device; returns CPT_EUNSUPPORTED */
} cpt_schedule;

typedef struct {
  uint32_t struct_size;  /* sizeof(cpt_exec_options) */
  int32_t schedule;      /* cpt_schedule (default CPT_SCHED_AUTO) */
  int32_t group;         /* persistent schedule: blocks per work item
                            (1..64; 0 means 1) */
  int32_t grid;          /* persistent schedule: workgroups of the launch
                            (0: as many as fit on the device at once,
                            capped at the number of work items) */
  int32_t use_graph;     /* 1: record the call's device work as a HIP graph
                            on first use and replay it on later calls with
                            the same shapes, options and schedule */
  int32_t field_tile;    /* tile of the fused field pass: 0 = 32x16,
                            1 = 64x8, 2 = 16x32 vertices (the output does not
                            depend on it; CPT_SCHED_AUTO takes the tuned
                            one).  A struct_size that ends before this field
                            (the earlier layout) means 0. */
  int32_t phase_blocks;  /* 16x16 blocks per workgroup of the per-phase
                            launches (CPT_SCHED_LAUNCH): 1 or 2, 0 meaning
                            2; the fused schedule always takes one.  The
                            output does not depend on it; CPT_SCHED_AUTO
                            takes the tuned one.  A struct_size that ends
                            before this field means 0. */
} cpt_exec_options;

/*
 * Compress n fields (1 <= n <= 65536) with shared eb and options.
 *   fields  host array of n device pointers, field i of shape
 *           (2, HWT[3i+2], HWT[3i], HWT[3i+1]) float32
 *   HWT     host, 3n int32: H, W, T of each field (limits as cpt_compress)
 *   ex      host, may be NULL for defaults
 *   outs    host array of n device pointers (4-byte aligned), capacities
 *           caps[i] bytes (host array)
 *   lens    host, n: stream lengths (also when a stream did not fit)
 *   status  host, n (may be NULL): per-field cpt_status
 * Returns CPT_OK when every field succeeded, else the status of the first
 * field that failed (message names it).  Fields that fail (non-finite
 * values, magnitude, capacity) leave the others unaffected.  Synchronises
 * `stream`.  Graph replays run on a library stream ordered after and
 * before `stream` by events.
 */
cpt_status cpt_compress_batch(int n, const float* const* fields, const int32_t* HWT, double eb,
                              const cpt_options* opt, const cpt_exec_options* ex, uint8_t* const* outs,
                              const size_t* caps, size_t* lens, int32_t* status, void* stream);

/* Number of execution choices cpt_autotune_batch times, in this order:
 * LAUNCH, FUSED, LAUNCH replayed as a graph, FUSED replayed as a graph (all
 * with field tile 0 and two blocks per phase workgroup), then the fastest of
 * those four with field tiles 1 and 2, then the fastest so far with one
 * block per phase workgroup. */
#define CPT_TUNE_CANDIDATES 7

/*
 * Time every candidate execution choice on this batch (arguments as for
 * cpt_compress_batch; the outputs are written), `reps` timed runs each after
 * one warm-up, and remember the fastest for CPT_SCHED_AUTO calls with the
 * same shapes and options (process-wide; graph replay is used when it won
 * or when the call asks for it).  best (host) receives it; ms
 * (host, CPT_TUNE_CANDIDATES entries, may be NULL) the mean device time per
 * run of each candidate.  Only execution parameters are tuned; all
 * candidates write identical streams.  Synchronises `stream`.
 */
cpt_status cpt_autotune_batch(int n, const float* const* fields, const int32_t* HWT, double eb,
                              const cpt_options* opt, uint8_t* const* outs, const size_t* caps, int reps,
                              cpt_exec_options* best, double* ms, void* stream);

/*
 * Decompress n streams (1 <= n <= 65536) in one device pipeline, as
 * cpt_decompress does for each: streams (host array of device pointers,
 * 4-byte aligned) of lens[i] bytes (host) into fields (host array of device
 * pointers, each (2,T,H,W) float32 as its header says, holding at least
 * field_caps[i] floats (host array)).  Streams may differ in size, predictor
 * and block height.  status (host, n, may be NULL) receives each stream's
 * outcome: CPT_ECORRUPT for a corrupt stream, CPT_ECAPACITY when its field
 * needs more than field_caps[i] floats (nothing is written to it); either
 * leaves the others unaffected.  Returns CPT_OK when every stream succeeded,
 * else the first failure.  Synchronises `stream` twice (after reading the
 * headers, and at the end); when no stream is long enough for a header it
 * returns CPT_ECORRUPT without any device work.
 */
cpt_status cpt_decompress_batch(int n, const uint8_t* const* streams, const size_t* lens, float* const* fields,
                                const size_t* field_caps, int32_t* status, void* stream);

/* Parse a stream header (host bytes, at least 256). */
cpt_status cpt_stream_info(const uint8_t* bytes, size_t len, cpt_info* info);

/*
 * The decompressor D of Sec. IV-A: reverse the entropy coding and the
 * predictions of Sec. VI (Lorenzo, semi-Lagrangian, in the processing order
 * the compressor used) and return the reconstructed field, within eb_abs of
 * the original at every vertex and with every space-time face's critical
 * status and sign unchanged.
 *   bytes      device, the stream (4-byte aligned), len bytes
 *   field      device, (2,T,H,W) float32 as given by cpt_stream_info
 *   field_cap  floats the caller allocated at `field`; CPT_ECAPACITY (and
 *              nothing written) when it is below 2 T H W
 * Any inconsistency gives CPT_ECORRUPT without out-of-bounds access, and the
 * output is then undefined.  Synchronises `stream`.
 */
cpt_status cpt_decompress(const uint8_t* bytes, size_t len, float* field, size_t field_cap, void* stream);

/*
 * Critical-point trajectory pieces (Sec. III-E/F): the crossed space-time
 * faces of the field on the fixed-point grid 2^k, under simulation of
 * simplicity, as sorted codes ((g * 12 + type) << 1) | (sign > 0) where g =
 * (t H + y) W + x is the face's owner vertex and type 0..11 its face type.
 *   codes  device, capacity `cap` entries; count receives the number found
 *          (also on CPT_ECAPACITY, when nothing is written)
 * Requires max|x| 2^k < 2^24.  Synchronises `stream`.
 */
cpt_status cpt_extract_trajectories(const float* field, int H, int W, int T, int k, uint64_t* codes, size_t cap,
                                    size_t* count, void* stream);

/* Critical-point trajectories of a field (device, (2,T,H,W) float32) on the
 * grid 2^k (Sec. IV-B): the crossed faces of cpt_extract_trajectories
 * joined through the tetrahedra of the prism split (two crossed faces of one
 * tetrahedron belong to one trajectory) into connected components.
 *   bad_tets  host, receives the tetrahedra with a crossed-face count other
 *             than 0 or 2 (Lemma 1 makes it 0)
 *   n_tracks  host, receives the number of components (#Traj of Sec. VII-A)
 * Requires max|x| 2^k < 2^24.  Synchronises `stream`. */
cpt_status cpt_tracks(const float* field, int H, int W, int T, int k, uint64_t* bad_tets, uint64_t* n_tracks,
                      void* stream);

/* The check of Sec. IV-A with the metrics of Sec. VII-A: both fields
 * (device, (2,T,H,W) float32) converted to the grid 2^k, their crossed faces
 * and signs extracted as cpt_extract_trajectories does, and every face whose
 * crossed status or sign differs counted as a false case, in time slices
 * (face types 0-1: FC_t) or across slabs (types 2-11: FC_s); also the
 * largest |a - b| and PSNR = 20 log10(max a - min a) - 10 log10(MSE) over
 * both components.  Requires max|x| 2^k < 2^24 for both fields, else
 * CPT_EINVAL.  Synchronises `stream`. */
cpt_status cpt_verify(const float* a, const float* b, int H, int W, int T, int k, cpt_verify_result* res,
                      void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the check
 * of cpt_verify, same arguments and results bit for bit, without any device
 * or pinned allocation.  Its intermediate arrays (both face masks and the
 * error partials: about 8.06 bytes per vertex) live
 * in one fixed array of CPT_VERIFY_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on from load until the process ends, so fields
 * of more than CPT_VERIFY_NOALLOC_MAX_VERTICES vertices (H W T) are refused
 * with CPT_EUNSUPPORTED before any device work.  Every call on one GPU
 * shares that array: overlapping calls would race, so the library runs one
 * call at a time per process (a lock held until the call has synchronised
 * its stream).  Synchronises `stream` twice. */
#define CPT_VERIFY_NOALLOC_SCRATCH_BYTES (128u << 20)
#define CPT_VERIFY_NOALLOC_MAX_VERTICES 16647040u
cpt_status cpt_verify_noalloc(const float* a, const float* b, int H, int W, int T, int k, cpt_verify_result* res,
                              void* stream);

/* Fixed-point exponent k and bound eps' the compressor derives for a field
 * (device) and bound; synchronises `stream`. */
cpt_status cpt_field_params(const float* field, int H, int W, int T, int eb_mode, double eb, int* k,
                            double* eb_abs, int64_t* eps, void* stream);

/* ---- Learned predictor selector (training on the device) ----
 * Network: 10 inputs (the block features written by cpt_compress_debug),
 * ReLU hidden layers of 64 and 64, 4 outputs (Lorenzo, semi-Lagrangian with
 * d_max 1, 2, 4 cells).  Weight layout (5124 values): W1[64][10], b1[64],
 * W2[64][64], b2[64], W3[4][64], b3[4].  Inference (in cpt_compress with
 * CPT_PRED_LEARNED) uses the bf16 copy with fp32 fused multiply-add in input
 * order and picks the first largest logit. */
typedef struct {
  uint32_t struct_size;  /* sizeof(cpt_train_options) */
  int32_t epochs;        /* passes over the data (default 20) */
  int32_t batch;         /* minibatch size (default 1024) */
  float lr;              /* Adam step size (default 2e-3) */
  uint64_t seed;         /* sample-order seed */
} cpt_train_options;

/* Mean softmax cross-entropy of the network with fp32 master weights `w`
 * (device, rounded to bf16 for the forward pass) over n samples (device:
 * feats [n][10] float32, labels [n] int32 in 0..3), and its gradient with
 * respect to the rounded weights (device grad [5124]); loss is a host
 * float.  Deterministic.  Synchronises `stream`. */
cpt_status cpt_selector_grad(const float* w, const float* feats, const int32_t* labels, int n, float* grad,
                             float* loss, void* stream);

/* Adam training of the network on n samples (device arrays as above).  `w`
 * (device, 5124 float32) holds the initial weights and receives the trained
 * master weights; `w_bf16` (device, 5124) receives their bf16 rounding.
 * final_loss (host, may be NULL) receives the full-data loss after training.
 * Deterministic for a given seed.  Synchronises `stream`. */
cpt_status cpt_selector_train(const float* feats, const int32_t* labels, int n, float* w, uint16_t* w_bf16,
                              const cpt_train_options* opt, float* final_loss, void* stream);

/* Kernel timing for benchmarks.  cpt_timing_enable(n) with n >= 1 resets
 * the counters and brackets every n-th launch of each of the main kernel
 * families with HIP events on the stream it is launched on (0 disables;
 * every bracket adds a gap of several microseconds between kernels, so a
 * period above 1 keeps the timed work close to an untimed run).
 * cpt_timing_read returns the accumulated device time, the number of
 * bracketed launches and the work units (vertices or symbols) they covered.
 * Families: 0 per-vertex bound/predict/quantize phase, 1 predictor choice,
 * 2 frame reconstruction, 3 Huffman decoding, 4 Huffman encoding, 5 face
 * extraction.  Process-wide; not for concurrent callers. */
cpt_status cpt_timing_enable(int on);
cpt_status cpt_timing_read(int family, double* total_ms, uint64_t* launches, uint64_t* units);

/* Message of the last failure on this thread. */
const char* cpt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
