// Network construction kernels.
//  - fixed-probability rows (classifier connectivity): row i tests every
//    target j with one Bernoulli draw keyed (seed, CONN, proj; 0, i, j, 0);
//    a block owns a row and compacts hits in ascending j with ballots.
//  - pairwise-Bernoulli Gaussian rows (topographic map, Tab. B): same, with the
//    threshold looked up by squared torus distance.
//  - DEEP R bitfield init (Sec. 2.1.2, Fig. 2A).
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int BUILD_NT = 256;

// exclusive ordered offset of a flag within the block, and the block total
__device__ __forceinline__ int block_scan_flag(bool f, int* s_wave, int* total) {
  uint64_t m = ballot(f);
  int lane = lane_id(), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  int pre = __popcll(m & lanemask_lt());
  if (lane == 0) s_wave[w] = __popcll(m);
  __syncthreads();
  int base = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    int c = s_wave[i];
    base += (i < w) ? c : 0;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + pre;
}

__device__ __forceinline__ int torus_d2(int L, int i, int j) {
  int dx = abs(i % L - j % L), dy = abs(i / L - j / L);
  dx = min(dx, L - dx);
  dy = min(dy, L - dy);
  return dx * dx + dy * dy;
}

__global__ void __launch_bounds__(BUILD_NT) k_rows(uint64_t seed, ProjDev P, uint64_t T_const,
                                                   const uint64_t* T_d2, int L, double sigma,
                                                   float g_init, int gauss, int fill) {
  __shared__ int s_wave[BUILD_NT / WAVE];
  const int i = blockIdx.x;
  int count = 0;
  for (int j0 = 0; j0 < P.n_post; j0 += BUILD_NT) {
    int j = j0 + (int)threadIdx.x;
    bool hit = false;
    if (j < P.n_post && !(P.recurrent && j == i)) {
      uint64_t T = gauss ? T_d2[torus_d2(L, i, j)] : T_const;
      hit = (uint64_t)draw_u32(seed, TAG_CONN, P.proj_id, 0, i, j, 0) < T;
    }
    int tot;
    int off = block_scan_flag(hit, s_wave, &tot);
    if (fill && hit && count + off < P.cap) {
      int64_t s = (int64_t)i * P.cap + count + off;
      P.ind[s] = j;
      P.w[s] = gauss ? g_init : (float)(sigma * draw_normal(seed, TAG_WINIT, P.proj_id, 0, i, j, 0));
    }
    count += tot;
  }
  if (threadIdx.x == 0) P.len[i] = fill ? min(count, P.cap) : count;
}

void launch_fixed_rows(hipStream_t s, uint64_t seed, const ProjDev& P, uint64_t T, double sigma, bool fill) {
  hipLaunchKernelGGL(k_rows, dim3(P.n_pre), dim3(BUILD_NT), 0, s, seed, P, T, (const uint64_t*)nullptr, 0,
                     sigma, 0.0f, 0, (int)fill);
}

void launch_gauss_rows(hipStream_t s, uint64_t seed, const ProjDev& P, int L, const uint64_t* T_d2,
                       float g_init, bool fill) {
  hipLaunchKernelGGL(k_rows, dim3(P.n_pre), dim3(BUILD_NT), 0, s, seed, P, (uint64_t)0, T_d2, L, 0.0, g_init,
                     1, (int)fill);
}

__global__ void k_dense_init(uint64_t seed, int proj_id, int rows, int cols, double sigma, float* W) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)rows * cols) return;
  int k = (int)(q / cols), j = (int)(q % cols);
  W[q] = (float)(sigma * draw_normal(seed, TAG_WINIT, proj_id, 0, k, j, 0));
}

void launch_dense_init(hipStream_t s, uint64_t seed, int proj_id, int rows, int cols, double sigma, float* W) {
  int64_t n = (int64_t)rows * cols;
  hipLaunchKernelGGL(k_dense_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, proj_id, rows,
                     cols, sigma, W);
}

// one thread per bitfield word: conn cleared, sign bits random (top draw bit)
__global__ void k_sign_random(uint64_t seed, ProjDev P) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)P.n_pre * P.words) return;
  int i = (int)(q / P.words), wd = (int)(q % P.words);
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    int j = wd * 32 + b;
    if (j >= P.n_post) break;
    bits |= (draw_u32(seed, TAG_SIGN, P.proj_id, 0, i, j, 0) >> 31) << b;
  }
  P.sign[q] = bits;
  P.conn[q] = 0u;
}

// existing synapses: set the connectivity bit, sign bit = weight < 0
__global__ void k_bits_from_rows(ProjDev P) {
  const int i = blockIdx.x;
  const int n = P.len[i];
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    int64_t s = (int64_t)i * P.cap + k;
    int j = P.ind[s];
    uint32_t mask = 1u << (j & 31);
    int64_t wd = (int64_t)i * P.words + (j >> 5);
    atomicOr(&P.conn[wd], mask);
    if (P.w[s] < 0.0f) atomicOr(&P.sign[wd], mask);
    else atomicAnd(&P.sign[wd], ~mask);
  }
}

void launch_deepr_bits_init(hipStream_t s, uint64_t seed, const ProjDev& P) {
  int64_t n = (int64_t)P.n_pre * P.words;
  hipLaunchKernelGGL(k_sign_random, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, P);
  hipLaunchKernelGGL(k_bits_from_rows, dim3(P.n_pre), dim3(256), 0, s, P);
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n16; q += stride)
    p[q] = make_uint4(0, 0, 0, 0);
}
__global__ void k_fill_zero_bytes(uint8_t* p, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = 0;
}

// zero-fill kernel (kept out of hipMemsetAsync so the sequence stays graph-safe)
void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  if (bytes == 0) return;
  size_t n16 = bytes / 16, rem = bytes % 16;
  if (n16) {
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16);
  }
  if (rem)
    hipLaunchKernelGGL(k_fill_zero_bytes, dim3(1), dim3(16), 0, s, (uint8_t*)p + n16 * 16, rem);
}

// Zero several ranges: blockIdx.y picks the range, x strides over its words.
__global__ void __launch_bounds__(256) k_fill_zero_ranges(const ZeroRange* __restrict__ R) {
  const ZeroRange r = R[blockIdx.y];
  uint32_t* p = (uint32_t*)r.p;
  const unsigned long long n = r.bytes / 4;
  for (unsigned long long q = (unsigned long long)blockIdx.x * 256 + threadIdx.x; q < n;
       q += (unsigned long long)gridDim.x * 256)
    p[q] = 0u;
}

void launch_fill_zero_ranges(hipStream_t s, const ZeroRange* ranges, int n, unsigned long long max_bytes) {
  if (n <= 0 || max_bytes == 0) return;
  unsigned long long bx = (max_bytes / 4 + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_fill_zero_ranges, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, s, ranges);
}

__global__ void k_advance_counts(uint64_t* step, uint64_t steps, uint32_t* updates, uint32_t n_upd) {
  if (threadIdx.x == 0) {
    *step += steps;
    *updates += n_upd;
  }
}

void launch_advance_counts(hipStream_t s, uint64_t* step, uint64_t steps, uint32_t* updates, uint32_t n_upd) {
  hipLaunchKernelGGL(k_advance_counts, dim3(1), dim3(64), 0, s, step, steps, updates, n_upd);
}

__global__ void k_copy(uint4* __restrict__ d, const uint4* __restrict__ s, size_t n16) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n16; q += stride) d[q] = s[q];
}

void launch_copy(hipStream_t s, void* dst, const void* src, size_t bytes) {
  size_t n16 = bytes / 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
}

}  // namespace rs
