/*
 * cpo.h — interface of the CPU oracle (test infrastructure only).
 *
 * The oracle is a plain, slow, single-threaded C implementation of the
 * critical-point-trajectory-preserving compressor of "Time-Varying Vector
 * Field Compression with Preserved Critical Point Trajectories"
 * (arXiv 2510.25143).  It exists to check the HIP library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source with the HIP library and includes none of its headers.
 *
 * All arrays are host memory.  Fields are float32 laid out (2,T,H,W):
 * the u plane, then the v plane, each [t][y][x] with x fastest.
 */
#ifndef CPO_H
#define CPO_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CPO_OK = 0, CPO_EINVAL = -1, CPO_ENOMEM = -2, CPO_ECORRUPT = -3,
       CPO_ECAPACITY = -4 };

typedef struct {
  int32_t predictor;   /* 0 Lorenzo only, 1 semi-Lagrangian only,
                          2 mixture K=2, 3 mixture K=4 (exhaustive),
                          4 mixture K=4 chosen by the learned selector */
  int32_t mode_bt;     /* frames per mode block (>= 1) */
  int32_t eb_mode;     /* 0: eb relative to the value range, 1: absolute */
  int32_t backend;     /* 0: Huffman stream, 1: zero-byte elision after it */
  double dt_dx, dt_dy; /* time step over grid spacing (cells per unit velocity) */
  const uint16_t* selector_w; /* bf16 MLP weights (predictor 4), host */
} cpo_options;

typedef struct {
  int32_t H, W, T, k;
  double eb_abs;
  int64_t eps;
  int32_t predictor, mode_bt, K, R;
  int64_t cx, sx, cy, sy;
  uint64_t total_len, n_q, n_raw;  /* total_len: bytes of the Huffman stream */
  int32_t backend;                 /* 1: the stream is a zero-byte-elision container */
  int32_t pad;
} cpo_info;

/* Fixed-point parameters (scale 2^k, bound eps' in fixed-point units). */
int cpo_params(const float* field, int H, int W, int T, int eb_mode, double eb,
               int* k, double* eb_abs, int64_t* eps);
/* Exact float -> fixed conversion rint(x * 2^k); n values. */
void cpo_to_fixed(const float* x, size_t n, int k, int32_t* out);

/* Edge sign under simulation of simplicity for an edge whose first vertex
   has the lower global index. */
int cpo_sos_edge(int32_t up, int32_t vp, int32_t uq, int32_t vq);

/* Face masks from fixed-point planes U, V ([T][H][W] each): per owner
   vertex, bit f (0..11) = face type f crossed, bit 12+f = its sign is +. */
void cpo_face_masks(const int32_t* U, const int32_t* V, int H, int W, int T,
                    uint32_t* masks);
/* Sorted face codes ((g*12+type)<<1 | sign) of the crossed faces. */
int cpo_extract_fixed(const int32_t* U, const int32_t* V, int H, int W, int T,
                      uint64_t* codes, size_t cap, size_t* count);
int cpo_extract(const float* field, int H, int W, int T, int k,
                uint64_t* codes, size_t cap, size_t* count);
/* Vertex offsets of face type f relative to its owner: dx,dy,dt of 3 vertices
   in increasing global index order. */
void cpo_face_vertices(int f, int* dx, int* dy, int* dt);
/* 1 where a vertex lies on a crossed face. */
void cpo_lossless_flags(const uint32_t* masks, int H, int W, int T, uint8_t* flags);
/* Number of faces incident to vertex (x,y,t). */
int cpo_incident_faces(int H, int W, int T, int x, int y, int t,
                       int32_t* nbr /* [36][2] vertex indices, may be NULL */);

/* Error-bound derivation for perturbing vertex 2 of a face (exact integers). */
int64_t cpo_alg2(int64_t u0, int64_t u1, int64_t u2, int64_t v0, int64_t v1,
                 int64_t v2);

/* Semi-Lagrangian prediction of both components at grid point (x,y) from
   previous-frame planes Up, Vp ([H][W]). */
void cpo_sl_predict(const int32_t* Up, const int32_t* Vp, int H, int W,
                    int x, int y, int64_t cx, int64_t sx, int64_t cy,
                    int64_t sy, int dmax, int nmax, int64_t* pu, int64_t* pv);
void cpo_sl_factor(double dt_dx, int k, int64_t* c, int64_t* s);
int64_t cpo_bilinear(const int32_t* F, int H, int W, int64_t px, int64_t py);

/* Tile-local first-order 3-D Lorenzo prediction; cur_t and prev are planes
   ([H][W], prev NULL at t = 0); values left of x0 or above y0 count as 0. */
int64_t cpo_lorenzo3(const int32_t* cur_t, const int32_t* prev, int W, int x,
                     int y, int x0, int y0);
/* Mode choice from the candidate scores R[0..K) (0 = Lorenzo). */
int cpo_choose(const int64_t* R, int K);

/* Residual quantizer: returns code (0 = unpredictable), writes recon. */
int32_t cpo_quantize(int64_t x, int64_t pred, int64_t xt, int64_t* recon);
/* Error-bound code: smallest q with (eps>>q) <= xi, 24 for xi == 0. */
int32_t cpo_xi_code(int64_t eps, int64_t xi);
/* Alg. 4 bound of vertex (x,y,t) on the current values U, V ([T][H][W]:
   reconstructed where already processed, original elsewhere) with the
   lossless flags; 0 for a flagged vertex. */
int64_t cpo_vertex_bound(const int32_t* U, const int32_t* V, const uint8_t* flags,
                         int H, int W, int T, int x, int y, int t, int64_t eps);

/* Entropy-score table entry floor(h log2 h 2^16) and block score. */
int64_t cpo_tlog(int h);
int64_t cpo_score(const int32_t* hist_counts, int nbins, int n, int L,
                  int K, int bt);

/* Length-limited Huffman code lengths by package-merge. */
int cpo_huffman_lengths(const uint64_t* counts, int nsym, int maxlen,
                        uint8_t* lengths);

/* Selector features (10 per block) and MLP. */
enum { CPO_NFEAT = 10, CPO_HID = 64, CPO_NCLS = 4,
       CPO_NW = 64 * 10 + 64 + 64 * 64 + 64 + 4 * 64 + 4 };
int cpo_mlp_forward(const uint16_t* w_bf16, const float* x, float* logits);
/* Cross-entropy loss gradient in double for fp32 weights (master copy);
   x [n][10], labels [n]; grad [CPO_NW]; returns mean loss. */
double cpo_mlp_loss_grad(const float* w, const float* x, const int32_t* labels,
                         int n, double* grad);
/* Same loss and gradient without bf16 rounding (for finite differences). */
double cpo_mlp_loss_grad_exact(const float* w, const float* x,
                               const int32_t* labels, int n, double* grad);

/* Compression.  Debug outputs (any may be NULL): xi [N] per-vertex bound,
   xcode [N], qcode [N] (u | v<<16), modes [nblocks], feats [nblocks][10]. */
int cpo_compress_ex(const float* field, int H, int W, int T, double eb,
                    const cpo_options* opt, uint8_t* out, size_t cap,
                    size_t* out_len, int32_t* xi, uint8_t* xcode,
                    uint32_t* qcode, uint8_t* modes, float* feats,
                    size_t* nblocks);
int cpo_compress(const float* field, int H, int W, int T, double eb,
                 const cpo_options* opt, uint8_t* out, size_t cap,
                 size_t* out_len);
/* Predictor class of block (bx,by) at a decision frame (Sec. VI-B) from the
   frame's original planes Ut, Vt, the previous frame's current planes Up, Vp
   and the frame's lossless flags ([H][W] each); feat [10] may be NULL.
   Returns the class or a negative status. */
int cpo_block_mode(const int32_t* Ut, const int32_t* Vt, const int32_t* Up,
                   const int32_t* Vp, const uint8_t* flags_t, int H, int W,
                   int bx, int by, const cpo_options* opt, int k, int64_t eps,
                   float* feat);
/* The same decision's K trial scores (Q16 bits per sample, Sec. VI-B) for
   predictor 2 or 3, into scores [K]; returns the class or a negative status. */
int cpo_block_scores(const int32_t* Ut, const int32_t* Vt, const int32_t* Up,
                     const int32_t* Vp, const uint8_t* flags_t, int H, int W,
                     int bx, int by, const cpo_options* opt, int k, int64_t eps,
                     int64_t* scores);
/* Canonical codewords of a code with the given lengths (0 = unused):
   symbols ordered by (length, symbol), each codeword the previous one plus
   one, shifted left by the length difference. */
void cpo_canonical_codes(const uint8_t* lengths, int nsym, uint32_t* codes);
size_t cpo_compress_bound(int H, int W, int T);
/* The lossless stage after Huffman coding: zero-byte elision of a stream's
   body in 4096-byte blocks (encode: ECAPACITY with the needed size in
   out_len when cap is short; decode: the inner stream back). */
size_t cpo_zbe_bound(size_t inner_len);
int cpo_zbe_encode(const uint8_t* in, size_t len, uint8_t* out, size_t cap, size_t* out_len);
int cpo_zbe_decode(const uint8_t* in, size_t len, uint8_t* out, size_t cap, size_t* out_len);
int cpo_stream_info(const uint8_t* bytes, size_t len, cpo_info* info);
int cpo_decompress(const uint8_t* bytes, size_t len, float* field);

/* Comparison of two fields on the same fixed-point grid 2^k (both need
   |x| 2^k < 2^24, else CPO_EINVAL). */
int cpo_verify(const float* a, const float* b, int H, int W, int T, int k,
               uint64_t* fc_t, uint64_t* fc_s, double* max_err, double* psnr);
/* Lemma-1 check and trajectory count over the tetrahedra. */
int cpo_tracks(const float* field, int H, int W, int T, int k,
               uint64_t* bad_tets, uint64_t* n_tracks);

#ifdef __cplusplus
}
#endif
#endif
