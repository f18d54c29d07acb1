// launch.hpp — host-side launchers of the libcptraj kernels (one per kernel
// family), called by the C-ABI entry points in api.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cpt {

// Per-field parameters of the compressor, fixed for one stream.
struct FieldParams {
  int H, W, T, k;
  int eps;          // eps' in fixed-point units
  int tx, ty;       // blocks per row / column
  int predictor;    // 0 Lorenzo, 1 semi-Lagrangian, 2 mix K=2, 3 mix K=4, 4 learned K=4
  int K;            // mode classes (1, 2 or 4)
  int bt;           // frames per mode block
  int64_t cx, sx, cy, sy;  // semi-Lagrangian displacement factors
};

// k_field.hip
void launch_range(const float* x, size_t n, int* r, hipStream_t s);
// the face masks of a float field on the grid 2^k in one time-marching pass
void launch_maskpass(const float* f, int H, int W, int T, int k, uint32_t* masks, hipStream_t s);
size_t scan_partials_size(size_t n);
void launch_scan(const uint32_t* in, size_t n, uint32_t* out, uint32_t* part, uint32_t* total, hipStream_t s);
void launch_count_faces(const uint32_t* masks, size_t N, uint32_t* cnt, hipStream_t s);
void launch_write_codes(const uint32_t* masks, const uint32_t* ofs, size_t N, uint64_t* codes, size_t cap,
                        hipStream_t s);
size_t compare_partials(size_t N);
void launch_compare(const uint32_t* ma, const uint32_t* mb, const float* a, const float* b, size_t N,
                    unsigned long long* fc, double* part, hipStream_t s);

// k_tracks.hip: Lemma-1 violations (ctr[0]) and trajectories (ctr[1]) from
// the face masks and the exclusive prefix sums of the per-vertex crossed-face
// counts (M crossed faces in all); parent: M ints
void launch_tracks(const uint32_t* masks, const uint32_t* ofs, int H, int W, int T, long long M, int* parent,
                   unsigned long long* ctr, hipStream_t s);

// k_entropy.hip
struct HuffTables {
  uint32_t code[1024];
  uint8_t len[1024];
};
void launch_zero_u32(uint32_t* p, size_t n, hipStream_t s);
// k_selector.hip
int selector_parts(int nbatch, int per_block);
void launch_mlp_grad(const float* w, const float* feats, const int32_t* labels, const int32_t* idx, int nbatch,
                     int per_block, float inv_n, float* part, float* loss_part, float* grad, float* loss,
                     hipStream_t s);
void launch_adam(float* w, float* m, float* v, const float* g, float lr, float b1, float b2, float eps, float c1,
                 float c2, uint16_t* wbf, hipStream_t s);
void launch_perm(int32_t* idx, int n, long long a, long long c, hipStream_t s);
void launch_to_bf16(const float* w, uint16_t* wbf, hipStream_t s);

}  // namespace cpt
