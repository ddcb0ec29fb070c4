// DEEP R rewiring (paper Sec. 2.1.2, Fig. 2), entirely on the device.
//  k_deepr_elim:   one wave per row.  Synapses whose weight sign differs from
//                  the sign bit of their potential connection are removed
//                  (weight exactly zero never is), their connectivity bits
//                  cleared, the row compacted and the dormant count recorded.
//                  Whole records move: index, weight, Adam moments, gradient
//                  and the per-instance eligibility traces.
//  k_deepr_distribute: one workgroup.  The dormant counts are summed and the
//                  activations spread uniformly over rows; activations that
//                  land on a row without room are redrawn in further rounds.
//                  (The paper does this summing/spreading on the host; doing
//                  it on the device keeps the training loop free of host
//                  round trips.)
//  k_deepr_form:   one wave per row with activations.  Lane 0 draws targets
//                  whose connectivity bit is clear (and that are not the row
//                  itself in recurrent projections), sets the bits and appends
//                  synapses; the wave zeroes their records.
#include <mutex>

#include "rs_compact.hpp"
#include "rs_kernels.hpp"

namespace rs {

__device__ __forceinline__ void elim_body(const ProjDev& P, const int B, long long* stats, const int i) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* holes = (int*)smem;
  int* tail = holes + P.cap;
  uint8_t* remf = (uint8_t*)(tail + P.cap);
  const int lane = lane_id();
  const int n = P.len[i];
  const int64_t base = (int64_t)i * P.cap;
  // 256 slots at a time: their indices and weights loaded together
  // (unconditionally: lanes past the row's end read its last slot again),
  // then their sign words, then the tests; two memory round trips per 256
  // slots instead of two per 64
  constexpr int EU = 4;
  const int64_t wbase = (int64_t)i * P.words;
  for (int k0 = 0; k0 < n; k0 += EU * WAVE) {
    int jj[EU];
    float ww[EU];
    uint32_t sw[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int64_t q = base + min(k0 + u * WAVE + lane, n - 1);
      jj[u] = P.ind[q];
      ww[u] = P.w[q];
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) sw[u] = P.sign[wbase + (jj[u] >> 5)];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int k = k0 + u * WAVE + lane;
      if (k < n) {
        const int j = jj[u];
        const bool neg = (sw[u] >> (j & 31)) & 1u;
        const bool rem = (ww[u] > 0.0f && neg) || (ww[u] < 0.0f && !neg);
        remf[k] = rem;
        if (rem) atomicAnd(&P.conn[wbase + (j >> 5)], ~(1u << (j & 31)));
      }
    }
  }
  __syncthreads();
  int n2;
  const int pairs = wave_compaction_plan(n, remf, holes, tail, &n2);
  for (int q = lane; q < pairs; q += WAVE) {
    const int64_t d = base + holes[q], s = base + tail[q];
    P.ind[d] = P.ind[s];
    P.w[d] = P.w[s];
    P.m[d] = P.m[s];
    P.v[d] = P.v[s];
    P.G[d] = P.G[s];
  }
  if (P.ebar) {
    const int R = P.erec;
    for (int q = 0; q < pairs; ++q) {
      const int64_t d = base + holes[q], s = base + tail[q];
      for (int c = lane; c < R; c += WAVE) P.ebar[d * R + c] = P.ebar[s * R + c];
      if (P.eps)
        for (int c = lane; c < B; c += WAVE) P.eps[d * B + c] = P.eps[s * B + c];
    }
  }
  if (lane == 0) {
    P.len[i] = n2;
    P.dormant[i] = n - n2;
    if (n > n2) atomicAdd((unsigned long long*)&stats[0], (unsigned long long)(n - n2));
  }
}
__global__ void __launch_bounds__(WAVE) k_deepr_elim(ProjDev P, int B, long long* stats) {
  elim_body(P, B, stats, blockIdx.x);
}

constexpr int DIST_NT = 1024;

__device__ __forceinline__ int block_sum_i(int v, int* s_red) {
  v = wave_sum_i(v);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) s_red[w] = v;
  __syncthreads();
  int t = 0;
  for (int q = 0; q < DIST_NT / WAVE; ++q) t += s_red[q];
  __syncthreads();
  return t;
}

__device__ __forceinline__ void distribute_body(const uint64_t seed, const ProjDev& P, const uint64_t step,
                                                long long* stats) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* cnt = (int*)smem;           // [n_pre]
  int* asg = cnt + P.n_pre;        // [n_pre]
  __shared__ int s_red[DIST_NT / WAVE];
  const int tid = threadIdx.x;
  int limit = P.n_post - (P.recurrent ? 1 : 0);
  limit = limit < P.cap ? limit : P.cap;
  int d = 0;
  for (int r = tid; r < P.n_pre; r += DIST_NT) {
    d += P.dormant[r];
    asg[r] = 0;
  }
  int pending = block_sum_i(d, s_red);
  for (int round = 0; pending > 0 && round < MAX_ROUNDS; ++round) {
    for (int r = tid; r < P.n_pre; r += DIST_NT) cnt[r] = 0;
    __syncthreads();
    for (int a = tid; a < pending; a += DIST_NT) {
      const uint32_t u = draw_u32(seed, TAG_DR_ROW, P.proj_id, step, (uint64_t)a, (uint64_t)round, 0);
      atomicAdd(&cnt[below(u, (uint32_t)P.n_pre)], 1);
    }
    __syncthreads();
    int rej = 0;
    for (int r = tid; r < P.n_pre; r += DIST_NT) {
      int room = limit - P.len[r] - asg[r];
      room = room > 0 ? room : 0;
      const int acc = cnt[r] < room ? cnt[r] : room;
      asg[r] += acc;
      rej += cnt[r] - acc;
    }
    pending = block_sum_i(rej, s_red);
  }
  if (pending > 0 && tid == 0) {  // deterministic fallback: lowest rows with room first
    for (int r = 0; r < P.n_pre && pending > 0; ++r) {
      const int room = limit - P.len[r] - asg[r];
      if (room <= 0) continue;
      const int take = pending < room ? pending : room;
      asg[r] += take;
      pending -= take;
    }
  }
  __syncthreads();
  int placed = 0;
  for (int r = tid; r < P.n_pre; r += DIST_NT) {
    P.assigned[r] = asg[r];
    placed += asg[r];
  }
  placed = block_sum_i(placed, s_red);
  if (tid == 0) {
    atomicAdd((unsigned long long*)&stats[2], (unsigned long long)placed);
    if (pending > 0) atomicAdd((unsigned long long*)&stats[3], (unsigned long long)pending);
  }
}
__global__ void __launch_bounds__(DIST_NT) k_deepr_distribute(uint64_t seed, ProjDev P, uint64_t step,
                                                              long long* stats) {
  distribute_body(seed, P, step, stats);
}

__device__ __forceinline__ void form_body(const uint64_t seed, const ProjDev& P, const int B, const uint64_t step,
                                          long long* stats, const int r) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* newj = (int*)smem;  // [cap]
  const int lane = lane_id();
  const int na = P.assigned[r];
  if (na == 0) return;
  const int n0 = P.len[r];
  __shared__ int s_found;
  __shared__ int s_cand[WAVE];  // first candidate target of each of the next 64 activations
  // Activations take their targets in order (each sees the targets taken
  // before it), so lane 0 decides them one by one; the draws of their first
  // candidates do not depend on that order and are made by all lanes at once.
  uint32_t* row = P.conn + (int64_t)r * P.words;
  int found = 0;
  bool stop = false;
  for (int k0 = 0; k0 < na; k0 += WAVE) {
    if (k0 + lane < na)
      s_cand[lane] = (int)below(draw_u32(seed, TAG_DR_TGT, P.proj_id, step, r, k0 + lane, 0), (uint32_t)P.n_post);
    __syncthreads();
    if (lane == 0 && !stop) {
      const int k1 = min(na, k0 + WAVE);
      for (int k = k0; k < k1; ++k) {
        int j = -1;
        for (int t = 0; t < MAX_TRIES; ++t) {
          const int c = t == 0 ? s_cand[k - k0]
                               : (int)below(draw_u32(seed, TAG_DR_TGT, P.proj_id, step, r, k, t), (uint32_t)P.n_post);
          if (!((row[c >> 5] >> (c & 31)) & 1u) && !(P.recurrent && c == r)) { j = c; break; }
        }
        if (j < 0) {
          const int start = (int)below(draw_u32(seed, TAG_DR_TGT, P.proj_id, step, r, k, MAX_TRIES),
                                       (uint32_t)P.n_post);
          for (int dd = 0; dd < P.n_post; ++dd) {
            const int c = (start + dd) % P.n_post;
            if (!((row[c >> 5] >> (c & 31)) & 1u) && !(P.recurrent && c == r)) { j = c; break; }
          }
        }
        if (j < 0) {  // no free target: bitfield inconsistent with the row
          stop = true;
          break;
        }
        row[j >> 5] |= 1u << (j & 31);
        newj[k] = j;
        ++found;
      }
    }
    __syncthreads();  // s_cand is rewritten for the next 64
  }
  if (lane == 0) s_found = found;
  __syncthreads();
  const int nf = s_found;
  const int64_t base = (int64_t)r * P.cap + n0;
  for (int k = lane; k < nf; k += WAVE) {
    P.ind[base + k] = newj[k];
    P.w[base + k] = 0.0f;
    P.m[base + k] = 0.0f;
    P.v[base + k] = 0.0f;
    P.G[base + k] = 0.0f;
  }
  if (P.ebar) {
    const int R = P.erec;
    for (int k = 0; k < nf; ++k) {
      for (int c = lane; c < R; c += WAVE) P.ebar[(base + k) * R + c] = 0.0f;
      if (P.eps)
        for (int c = lane; c < B; c += WAVE) P.eps[(base + k) * B + c] = 0.0f;
    }
  }
  if (lane == 0) {
    P.len[r] = n0 + nf;
    if (nf) atomicAdd((unsigned long long*)&stats[1], (unsigned long long)nf);
  }
}
__global__ void __launch_bounds__(WAVE) k_deepr_form(uint64_t seed, ProjDev P, int B, uint64_t step,
                                                     long long* stats) {
  form_body(seed, P, B, step, stats, blockIdx.x);
}

// DEEP R of several projections (of several networks) in one launch per
// phase.  Elimination and formation: workgroup g takes row work[g].y of
// projection work[g].x; distribution: one workgroup per projection.  The
// random step is D.step plus the device step count where the launch replays.
__device__ __forceinline__ uint64_t deepr_step(const DeeprArgs& d) {
  return d.step + (d.step_base ? *d.step_base : 0ull);
}
__global__ void __launch_bounds__(WAVE) k_deepr_elim_multi(const DeeprArgs* __restrict__ D,
                                                           const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const DeeprArgs d = D[w.x];
  elim_body(d.P, d.B, d.stats, w.y);
}
__global__ void __launch_bounds__(DIST_NT) k_deepr_distribute_multi(const DeeprArgs* __restrict__ D) {
  const DeeprArgs d = D[blockIdx.x];
  distribute_body(d.seed, d.P, deepr_step(d), d.stats);
}
__global__ void __launch_bounds__(WAVE) k_deepr_form_multi(const DeeprArgs* __restrict__ D,
                                                           const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const DeeprArgs d = D[w.x];
  form_body(d.seed, d.P, d.B, deepr_step(d), d.stats, w.y);
}

void deepr_attrs() {
  static std::once_flag once;
  std::call_once(once, [] {
    allow_dynamic_lds((const void*)k_deepr_distribute, 128 * 1024);
    allow_dynamic_lds((const void*)k_deepr_distribute_multi, 128 * 1024);
  });
}

void launch_deepr(hipStream_t s, uint64_t seed, const ProjDev& P, int B, uint64_t step, long long* stats) {
  deepr_attrs();
  const size_t sm_elim = (size_t)P.cap * 9 + 16;
  hipLaunchKernelGGL(k_deepr_elim, dim3(P.n_pre), dim3(WAVE), sm_elim, s, P, B, stats);
  hipLaunchKernelGGL(k_deepr_distribute, dim3(1), dim3(DIST_NT), (size_t)P.n_pre * 8, s, seed, P, step, stats);
  hipLaunchKernelGGL(k_deepr_form, dim3(P.n_pre), dim3(WAVE), (size_t)P.cap * 4 + 16, s, seed, P, B, step,
                     stats);
}

}  // namespace rs

namespace rs {
void launch_deepr_multi(hipStream_t s, const DeeprArgs* D, int n_proj, const int2* rows, int n_rows, int max_cap,
                        int max_pre) {
  deepr_attrs();
  if (n_proj <= 0) return;
  hipLaunchKernelGGL(k_deepr_elim_multi, dim3(n_rows), dim3(WAVE), (size_t)max_cap * 9 + 16, s, D, rows);
  hipLaunchKernelGGL(k_deepr_distribute_multi, dim3(n_proj), dim3(DIST_NT), (size_t)max_pre * 8, s, D);
  hipLaunchKernelGGL(k_deepr_form_multi, dim3(n_rows), dim3(WAVE), (size_t)max_cap * 4 + 16, s, D, rows);
}
}  // namespace rs
