// k_backend.hip — the lossless stage after Huffman coding (Sec. V: a
// general-purpose lossless coder follows the Huffman stage; Sec. VII-B: the
// zero runs it removes): zero-byte elision of the stream body in independent
// 4096-byte blocks, and its inverse.
//
// Container: the 256-byte header of the Huffman stream with slot 31 set to
// ZBE_TAG; one 32-bit entry per 4096-byte block of the body (the bytes after
// the header): the block's encoded length in bytes, bit 31 set when the
// block is elided; then the encoded blocks.  An elided block of n bytes is a
// mask of ceil(n / 8) bytes (bit i, least significant first, marks a nonzero
// byte i), the nonzero bytes in order, and zero bytes up to a multiple of 4;
// a block is elided exactly when that is shorter than n.
//
// A workgroup of 256 threads works one block at a time, 16 bytes per
// thread: a pass that counts nonzero bytes and decides, a per-field pass
// that lays the blocks out, and a pass that builds each encoded block in
// LDS and stores it with 32-bit writes.  Decoding mirrors it and checks every length, mask bit,
// stored byte and padding byte, so that no read leaves the container.
#include <algorithm>

#include "batch.hpp"
#include "cpt_device.hpp"

namespace cpt {

namespace {

// nonzero bytes of a 32-bit word, as a 4-bit mask (bit j: byte j)
__device__ __forceinline__ uint32_t nz_bytes(uint32_t v) {
  return (v & 0xFFu ? 1u : 0u) | (v & 0xFF00u ? 2u : 0u) | (v & 0xFF0000u ? 4u : 0u) | (v & 0xFF000000u ? 8u : 0u);
}

__device__ __forceinline__ long long pad4(long long n) { return (n + 3) & ~3ll; }

// this thread's 16 bytes of a block of nbytes (a multiple of 4), zero past it
__device__ __forceinline__ uint4 load16(const uint8_t* p, int tid, int nbytes) {
  const int o = 16 * tid;
  if (o + 16 <= nbytes) return *(const uint4*)(p + o);
  const uint32_t* w = (const uint32_t*)(p + o);
  uint4 r = make_uint4(0, 0, 0, 0);
  if (o + 4 <= nbytes) r.x = w[0];
  if (o + 8 <= nbytes) r.y = w[1];
  if (o + 12 <= nbytes) r.z = w[2];
  return r;
}

__device__ __forceinline__ uint32_t mask16(uint4 v) {
  return nz_bytes(v.x) | (nz_bytes(v.y) << 4) | (nz_bytes(v.z) << 8) | (nz_bytes(v.w) << 12);
}

// exclusive prefix of v over the workgroup's 256 threads (total in *sum)
template <typename T>
__device__ __forceinline__ T wg_exclusive(T v, T* sh, T* sum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  T x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  T base = 0;
  for (int i = 0; i < w; i++) base += sh[i];
  if (sum) *sum = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + x - v;
}

}  // namespace

// ------------------------------------------------------------------ encode
// The grid is fixed (the number of blocks is known only on the device):
// workgroup w takes blocks w, w + grid, ... of every field in turn.
__global__ __launch_bounds__(256) void k_zbe_count_b(const FieldDesc* __restrict__ D, int n,
                                                     uint32_t* __restrict__ ztab, uint32_t* __restrict__ zlen) {
  __shared__ int sh[4];
  for (int f = 0; f < n; f++) {
    const FieldDesc& d = D[f];
    if (d.status) continue;
    const long long body = d.len - (long long)HDR_BYTES;
    const long long nb = (body + ZBE_BLOCK - 1) / ZBE_BLOCK;
    for (long long b = blockIdx.x; b < nb; b += gridDim.x) {
      const int nbytes = (int)min((long long)ZBE_BLOCK, body - b * ZBE_BLOCK);
      const uint4 v = load16(d.out + HDR_BYTES + b * ZBE_BLOCK, threadIdx.x, nbytes);
      int tot = 0;
      (void)wg_exclusive<int>(__popc(mask16(v)), sh, &tot);
      if (threadIdx.x == 0) {
        const long long e = pad4((nbytes + 7) / 8 + tot);
        const bool elide = e < nbytes;
        ztab[d.zbase + b] = elide ? ((uint32_t)e | 0x80000000u) : (uint32_t)nbytes;
        zlen[d.zbase + b] = elide ? (uint32_t)e : (uint32_t)nbytes;
      }
    }
  }
}

// one workgroup per field: block offsets, container length, capacity check,
// header (slot 31 = tag) and block table
__global__ __launch_bounds__(256) void k_zbe_layout_b(FieldDesc* __restrict__ D, const uint32_t* __restrict__ ztab,
                                                      const uint32_t* __restrict__ zlen,
                                                      long long* __restrict__ zoff) {
  __shared__ long long sh[4];
  __shared__ int ok;
  FieldDesc& d = D[blockIdx.x];
  if (d.status) return;
  const int tid = threadIdx.x;
  const long long inner = d.len, body = inner - (long long)HDR_BYTES;
  const long long nb = (body + ZBE_BLOCK - 1) / ZBE_BLOCK;
  const long long per = (nb + 255) / 256, lo = min(nb, per * tid), hi = min(nb, lo + per);
  long long s = 0;
  for (long long i = lo; i < hi; i++) s += zlen[d.zbase + i];
  long long total = 0;
  long long run = wg_exclusive<long long>(s, sh, &total);
  for (long long i = lo; i < hi; i++) {
    zoff[d.zbase + i] = run;
    run += zlen[d.zbase + i];
  }
  const long long clen = (long long)HDR_BYTES + 4 * nb + total;
  if (tid == 0) {
    ok = d.zout != nullptr && clen <= d.zcap;
    d.ilen = inner;
    d.len = clen;
    if (!ok) {
      d.status = STATUS_ECAPACITY;
      d.reason = REASON_CAPACITY;
    }
  }
  __syncthreads();
  if (!ok) return;
  const uint32_t* h = (const uint32_t*)d.out;
  uint32_t* o = (uint32_t*)d.zout;
  if (tid < (int)(HDR_BYTES / 4))
    o[tid] = tid == 62 ? (uint32_t)(ZBE_TAG & 0xFFFFFFFFu) : (tid == 63 ? (uint32_t)(ZBE_TAG >> 32) : h[tid]);
  for (long long i = tid; i < nb; i += 256) o[HDR_BYTES / 4 + i] = ztab[d.zbase + i];
}

__device__ __forceinline__ void zbe_write_block(const FieldDesc& d, long long b, long long nb, long long body,
                                                const uint32_t* __restrict__ ztab, const long long* __restrict__ zoff,
                                                int* sh, uint8_t* enc) {
  const int tid = threadIdx.x;
  const int nbytes = (int)min((long long)ZBE_BLOCK, body - b * ZBE_BLOCK);
  const uint32_t entry = ztab[d.zbase + b];
  uint32_t* dst = (uint32_t*)(d.zout + HDR_BYTES + 4 * nb + zoff[d.zbase + b]);
  const uint4 v = load16(d.out + HDR_BYTES + b * ZBE_BLOCK, tid, nbytes);
  if (!(entry >> 31)) {  // stored
    const int o = 4 * tid;
    if (16 * tid < nbytes) dst[o] = v.x;
    if (16 * tid + 4 < nbytes) dst[o + 1] = v.y;
    if (16 * tid + 8 < nbytes) dst[o + 2] = v.z;
    if (16 * tid + 12 < nbytes) dst[o + 3] = v.w;
    return;
  }
  const int e = (int)(entry & 0x7FFFFFFFu), m = (nbytes + 7) / 8;
  const uint32_t mk = mask16(v);
  int nnz = 0;
  int pos = wg_exclusive<int>(__popc(mk), sh, &nnz);
  if (2 * tid < m) enc[2 * tid] = (uint8_t)(mk & 0xFFu);
  if (2 * tid + 1 < m) enc[2 * tid + 1] = (uint8_t)(mk >> 8);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 16; j++)
    if ((mk >> j) & 1u) enc[m + pos++] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
  if (tid == 0)
    for (int i = m + nnz; i < e; i++) enc[i] = 0;
  __syncthreads();
  const uint32_t* e32 = (const uint32_t*)enc;
  for (int i = tid; i < e / 4; i += 256) dst[i] = e32[i];
  __syncthreads();  // enc is reused by the workgroup's next block
}

__global__ __launch_bounds__(256) void k_zbe_write_b(const FieldDesc* __restrict__ D, int n,
                                                     const uint32_t* __restrict__ ztab,
                                                     const long long* __restrict__ zoff) {
  __shared__ int sh[4];
  __shared__ __align__(16) uint8_t enc[ZBE_BLOCK];
  for (int f = 0; f < n; f++) {
    const FieldDesc& d = D[f];
    if (d.status) continue;
    const long long body = d.ilen - (long long)HDR_BYTES;
    const long long nb = (body + ZBE_BLOCK - 1) / ZBE_BLOCK;
    for (long long b = blockIdx.x; b < nb; b += gridDim.x) zbe_write_block(d, b, nb, body, ztab, zoff, sh, enc);
  }
}

// ------------------------------------------------------------------ decode
// one workgroup per container: block offsets (and the check that the table
// adds up to the container), and the inner header with slot 31 cleared
__global__ __launch_bounds__(256) void k_unzbe_scan_b(DecDesc* __restrict__ D, int n, long long* __restrict__ uoff) {
  __shared__ long long sh[4];
  DecDesc& d = D[blockIdx.x];
  if (d.nzb == 0) return;
  const int tid = threadIdx.x;
  const long long nb = d.nzb;
  const uint32_t* tab = (const uint32_t*)(d.zin + HDR_BYTES);
  const long long per = (nb + 255) / 256, lo = min(nb, per * tid), hi = min(nb, lo + per);
  long long s = 0;
  uint32_t odd = 0;  // every encoded length is a whole number of words
  for (long long i = lo; i < hi; i++) {
    s += tab[i] & 0x7FFFFFFFu;
    odd |= tab[i] & 3u;
  }
  long long total = 0;
  long long run = wg_exclusive<long long>(s, sh, &total);
  for (long long i = lo; i < hi; i++) {
    uoff[d.zbb + i] = run;
    run += tab[i] & 0x7FFFFFFFu;
  }
  if (odd) atomicOr(&d.err, 512u);
  if (tid == 0 && (long long)HDR_BYTES + 4 * nb + total != d.zlen) atomicOr(&d.err, 512u);
  const uint32_t* h = (const uint32_t*)d.zin;
  uint32_t* o = (uint32_t*)d.inner;
  if (tid < (int)(HDR_BYTES / 4)) o[tid] = tid >= 62 ? 0u : h[tid];
}

// one workgroup per block of every container (upre[j]: blocks of the
// containers before j)
__global__ __launch_bounds__(256) void k_unzbe_block_b(DecDesc* __restrict__ D, const long long* __restrict__ upre,
                                                       int n, const long long* __restrict__ uoff) {
  __shared__ int sh[4];
  __shared__ int bad;
  const int j = find_field(upre, n, blockIdx.x);
  DecDesc& d = D[j];
  const long long b = (long long)blockIdx.x - upre[j];
  // a table that does not add up to the container, or has a length that is
  // not a whole number of words, stops every block of it here
  if (b >= d.nzb || (d.err & 512u)) return;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  const long long body = d.ilen - (long long)HDR_BYTES;
  const int nbytes = (int)min((long long)ZBE_BLOCK, body - b * ZBE_BLOCK);
  const uint32_t entry = ((const uint32_t*)(d.zin + HDR_BYTES))[b];
  const int e = (int)(entry & 0x7FFFFFFFu);
  const uint8_t* src = d.zin + HDR_BYTES + 4 * d.nzb + uoff[d.zbb + b];
  uint32_t* out = (uint32_t*)(d.inner + HDR_BYTES + b * ZBE_BLOCK);
  __syncthreads();
  if (!(entry >> 31)) {  // stored: exactly the block's bytes
    if (e != nbytes) {
      if (tid == 0) atomicOr(&d.err, 512u);
      return;
    }
    const uint32_t* s32 = (const uint32_t*)src;
    for (int i = tid; i < nbytes / 4; i += 256) out[i] = s32[i];
    return;
  }
  const int m = (nbytes + 7) / 8;
  if (e < m || e >= nbytes) {
    if (tid == 0) atomicOr(&d.err, 512u);
    return;
  }
  uint32_t mk = (2 * tid < m ? src[2 * tid] : 0u) | (2 * tid + 1 < m ? (uint32_t)src[2 * tid + 1] << 8 : 0u);
  const int o = 16 * tid;
  const uint32_t past = o >= nbytes ? 0xFFFFu : (o + 16 > nbytes ? (0xFFFFu << (nbytes - o)) & 0xFFFFu : 0u);
  if (mk & past) bad = 1;  // a mask bit past the block
  mk &= ~past;
  int nnz = 0;
  int pos = wg_exclusive<int>(__popc(mk), sh, &nnz);
  if (pad4(m + nnz) != e) bad = 1;
  uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
  for (int jb = 0; jb < 16; jb++)
    if ((mk >> jb) & 1u) {
      const uint32_t byte = pos < e - m ? src[m + pos] : 0u;
      if (byte == 0) bad = 1;  // a stored byte must be nonzero
      w[jb >> 2] |= byte << (8 * (jb & 3));
      pos++;
    }
  if (tid == 0)
    for (int i = m + nnz; i < e; i++)
      if (src[i] != 0) bad = 1;  // padding
  if (o < nbytes) out[4 * tid] = w[0];
  if (o + 4 < nbytes) out[4 * tid + 1] = w[1];
  if (o + 8 < nbytes) out[4 * tid + 2] = w[2];
  if (o + 12 < nbytes) out[4 * tid + 3] = w[3];
  __syncthreads();
  if (tid == 0 && bad) atomicOr(&d.err, 512u);
}

// ============================================================ stream hash
// A position-sensitive 64-bit digest of a byte string for comparing the
// outputs of execution choices: the sum modulo 2^64 of splitmix64 (Steele,
// Lea and Flood's generator finaliser, constants as published) of
// (word index << 32 | word), over its little-endian 32-bit words (the last
// one zero-padded).  Addition commutes, so the atomics give one result.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_hash_clear(unsigned long long* h, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_hash_bytes(const uint8_t* __restrict__ p, size_t len,
                                                    unsigned long long* __restrict__ h) {
  const size_t nw = (len + 3) / 4;
  uint64_t acc = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t w = 0;
    for (int b = 0; b < 4; b++)
      if (4 * i + b < len) w |= (uint32_t)p[4 * i + b] << (8 * b);
    acc += splitmix64(((uint64_t)i << 32) | w);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(h, (unsigned long long)acc);
}

// ================================================================ launchers
void launch_hash_streams(int n, const uint8_t* const* p, const size_t* len, unsigned long long* h, hipStream_t s) {
  k_hash_clear<<<(n + 255) / 256, 256, 0, s>>>(h, n);
  for (int i = 0; i < n; i++) {
    const size_t nw = (len[i] + 3) / 4;
    const unsigned grid = (unsigned)std::min<size_t>((nw + 255) / 256, 1024);
    if (grid > 0) k_hash_bytes<<<grid, 256, 0, s>>>(p[i], len[i], h + i);
  }
}


void launch_zbe_b(FieldDesc* D, int n, long long zblocks, uint32_t* ztab, uint32_t* zlen, long long* zoff,
                  hipStream_t s) {
  const unsigned grid = (unsigned)std::min<long long>(zblocks, 4096);
  if (grid > 0) k_zbe_count_b<<<grid, 256, 0, s>>>(D, n, ztab, zlen);
  k_zbe_layout_b<<<n, 256, 0, s>>>(D, ztab, zlen, zoff);
  if (grid > 0) k_zbe_write_b<<<grid, 256, 0, s>>>(D, n, ztab, zoff);
}

void launch_unzbe_b(DecDesc* D, int n, const long long* upre, long long ublocks, long long* uoff, hipStream_t s) {
  k_unzbe_scan_b<<<n, 256, 0, s>>>(D, n, uoff);
  if (ublocks > 0) k_unzbe_block_b<<<(unsigned)ublocks, 256, 0, s>>>(D, upre, n, uoff);
}

}  // namespace cpt
