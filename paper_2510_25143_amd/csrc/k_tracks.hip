// k_tracks.hip — critical-point trajectories as connected components of
// crossed faces (Sec. IV-B: under simulation of simplicity every tetrahedron
// has zero or two crossed faces, Lemma 1, so the crossed faces chain into
// trajectories, and Theorem 2 makes them equal before and after
// compression when every face keeps its status).
//
// Each space-time cell (x, y, t), x < W-1, y < H-1, t < T-1, holds the two
// triangles of the main-diagonal split, each extruded to a prism of three
// tetrahedra (Sec. III-C); a face is named by its owner (its vertex of
// smallest global index (t H + y) W + x) and its type (the offsets of its
// other vertices from the owner, as the extraction numbers them).  One
// thread per cell counts the crossed faces of its six tetrahedra: a count
// other than 0 or 2 is a Lemma-1 violation; for a count of 2 the two faces
// are united in a lock-free union-find over the crossed faces, numbered in
// (owner, type) order: a face's number is the exclusive prefix sum of the
// crossed-face counts of the vertices before its owner plus its rank among
// its owner's crossed faces.  Trajectories are the roots that remain.
#include "cpt_device.hpp"
#include "launch.hpp"

namespace cpt {

namespace {

struct TetFaces {
  int8_t dx[6][4], dy[6][4], dt[6][4], type[6][4];
};

constexpr bool same_vertex(const int* a, const int* b) { return a[0] == b[0] && a[1] == b[1] && a[2] == b[2]; }

// the face type whose vertex offsets (from its owner) are the set v[0..2]
constexpr int face_type_of(const int (*v)[3]) {
  for (int f = 0; f < 12; f++) {
    int hits = 0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) hits += same_vertex(v[i], FTYPE[f][j]) ? 1 : 0;
    if (hits == 3) return f;
  }
  return -1;
}

constexpr TetFaces make_tet_faces() {
  TetFaces R{};
  // triangles (x, y offsets) with vertices in increasing spatial index
  const int tri[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
  // the three tetrahedra of a prism over a < b < c: (vertex, time) pairs
  const int tet[3][4][2] = {{{0, 0}, {1, 0}, {2, 0}, {2, 1}},
                            {{0, 0}, {1, 0}, {1, 1}, {2, 1}},
                            {{0, 0}, {0, 1}, {1, 1}, {2, 1}}};
  for (int tr = 0; tr < 2; tr++)
    for (int q = 0; q < 3; q++) {
      const int k = 3 * tr + q;
      int v[4][3] = {};
      for (int i = 0; i < 4; i++) {
        v[i][0] = tri[tr][tet[q][i][0]][0];
        v[i][1] = tri[tr][tet[q][i][0]][1];
        v[i][2] = tet[q][i][1];
      }
      for (int s = 0; s < 4; s++) {  // the face opposite vertex s
        int f[3][3] = {};
        int n = 0;
        for (int i = 0; i < 4; i++)
          if (i != s) {
            f[n][0] = v[i][0];
            f[n][1] = v[i][1];
            f[n][2] = v[i][2];
            n++;
          }
        // owner: smallest (t, y, x); offsets of the face from it
        int o = 0;
        for (int i = 1; i < 3; i++)
          if (f[i][2] < f[o][2] || (f[i][2] == f[o][2] && (f[i][1] < f[o][1] || (f[i][1] == f[o][1] && f[i][0] < f[o][0]))))
            o = i;
        int rel[3][3] = {};
        for (int i = 0; i < 3; i++) {
          rel[i][0] = f[i][0] - f[o][0];
          rel[i][1] = f[i][1] - f[o][1];
          rel[i][2] = f[i][2] - f[o][2];
        }
        R.dx[k][s] = (int8_t)f[o][0];
        R.dy[k][s] = (int8_t)f[o][1];
        R.dt[k][s] = (int8_t)f[o][2];
        R.type[k][s] = (int8_t)face_type_of(rel);
      }
    }
  return R;
}

constexpr bool tet_faces_typed() {
  TetFaces R = make_tet_faces();
  for (int k = 0; k < 6; k++)
    for (int s = 0; s < 4; s++)
      if (R.type[k][s] < 0) return false;
  return true;
}
static_assert(tet_faces_typed(), "every face of the prism split is one of the twelve face types");

__constant__ TetFaces c_tet = make_tet_faces();

__device__ __forceinline__ int ld_parent(const int* p, int i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of i; parents only ever point to smaller indices, so the walk ends
__device__ int uf_find(int* p, int i) {
  for (;;) {
    const int q = ld_parent(p, i);
    if (q == i) return i;
    const int r = ld_parent(p, q);
    if (r != q) __hip_atomic_store(p + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // halve the path
    i = r;
  }
}

// hook the larger root under the smaller until both share one root
__device__ void uf_unite(int* p, int a, int b) {
  for (;;) {
    a = uf_find(p, a);
    b = uf_find(p, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    int expected = b;
    if (__hip_atomic_compare_exchange_strong(p + b, &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

}  // namespace

__global__ __launch_bounds__(256) void k_uf_init(int* __restrict__ parent, long long M) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) parent[i] = (int)i;
}

__global__ __launch_bounds__(256) void k_tet_pairs(const uint32_t* __restrict__ masks, int H, int W, int T,
                                                   const uint32_t* __restrict__ ofs, int* __restrict__ parent,
                                                   unsigned long long* __restrict__ ctr) {
  const long long cells = (long long)(W - 1) * (H - 1) * (T - 1);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned nbad = 0;
  if (i < cells) {
    const int x = (int)(i % (W - 1));
    const long long r = i / (W - 1);
    const int y = (int)(r % (H - 1)), t = (int)(r / (H - 1));
    // every face of the cell's tetrahedra is owned by one of its eight
    // corners: load their masks once, and leave when none has a crossed face
    const size_t HW = (size_t)H * W, g0 = ((size_t)t * H + y) * W + x;
    uint32_t m[8];
    uint32_t any = 0;
#pragma unroll
    for (int o = 0; o < 8; o++) {
      m[o] = masks[g0 + (size_t)(o >> 2) * HW + (size_t)((o >> 1) & 1) * W + (o & 1)];
      any |= m[o];
    }
    if (any & 0xFFFu) {
#pragma unroll
      for (int k = 0; k < 6; k++) {
        int fa = 0, fb = 0;
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const int o = c_tet.dt[k][s] * 4 + c_tet.dy[k][s] * 2 + c_tet.dx[k][s];
          const int type = c_tet.type[k][s];
          if ((m[o] >> type) & 1u) {
            const size_t g = g0 + (size_t)c_tet.dt[k][s] * HW + (size_t)c_tet.dy[k][s] * W + c_tet.dx[k][s];
            const int face = (int)(ofs[g] + (uint32_t)__popc(m[o] & ((1u << type) - 1u)));
            if (cnt == 0) fa = face; else fb = face;
            cnt++;
          }
        }
        if (cnt != 0 && cnt != 2) nbad++;
        if (cnt == 2) uf_unite(parent, fa, fb);
      }
    }
  }
  if (nbad) atomicAdd(&ctr[0], (unsigned long long)nbad);
}

__global__ __launch_bounds__(256) void k_uf_roots(const int* __restrict__ parent, long long M,
                                                  unsigned long long* __restrict__ ctr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long b = __ballot(i < M && parent[i] == (int)i);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(&ctr[1], (unsigned long long)__popcll(b));
}

__global__ void k_zero_ctr(unsigned long long* ctr) {
  if (threadIdx.x < 2) ctr[threadIdx.x] = 0;
}

void launch_tracks(const uint32_t* masks, const uint32_t* ofs, int H, int W, int T, long long M, int* parent,
                   unsigned long long* ctr, hipStream_t s) {
  k_zero_ctr<<<1, 64, 0, s>>>(ctr);
  const long long cells = (long long)(W - 1) * (H - 1) * (T - 1);
  if (M > 0) k_uf_init<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(parent, M);
  // without crossed faces no tetrahedron has two, so the union is never reached
  if (cells > 0) k_tet_pairs<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(masks, H, W, T, ofs, parent, ctr);
  if (M > 0) k_uf_roots<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(parent, M, ctr);
}

}  // namespace cpt
