// Topographic-map rewiring (paper Sec. 2.1.3, Fig. 3; Tab. B and G).
//  k_topo_distribute: one workgroup spreads the N_attempts attempts uniformly,
//                     with replacement, over presynaptic rows and lists the
//                     rows that received any (host code in the paper).
//  k_topo_rewire:     one wave per listed row.  The row's bitfield section is
//                     staged in LDS; lane 0 sets k distinct random candidate
//                     bits; lanes test every existing synapse against its
//                     target bit and eliminate with the weight-dependent
//                     probability (draw keyed by the synapse's slot before any
//                     removal); the row is compacted; lane 0 then visits the
//                     remaining candidates in ascending target order and forms
//                     synapses with the distance-dependent probability while
//                     the row has room.  All bits end cleared.
#include <algorithm>
#include <mutex>

#include "rs_compact.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int TD_NT = 1024;

__global__ void __launch_bounds__(TD_NT) k_topo_distribute(uint64_t seed, TopoDev t, uint64_t step) {
  if (step == STEP_FROM_DEVICE) step = *t.step_dev;
  extern __shared__ __align__(16) unsigned char smem[];
  int* k = (int*)smem;  // [n_pre]
  __shared__ int s_n;
  const int tid = threadIdx.x, n_pre = t.P.n_pre;
  for (int r = tid; r < n_pre; r += TD_NT) k[r] = 0;
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int a = tid; a < t.n_attempts; a += TD_NT)
    atomicAdd(&k[below(draw_u32(seed, TAG_TP_ROW, t.P.proj_id, step, (uint64_t)a, 0, 0), (uint32_t)n_pre)], 1);
  __syncthreads();
  for (int r = tid; r < n_pre; r += TD_NT) {
    t.kcount[r] = k[r];
    if (k[r] > 0) t.rowlist[atomicAdd(&s_n, 1)] = r;
  }
  __syncthreads();
  if (tid == 0) *t.nrows = s_n;
}

__device__ __forceinline__ int torus_d2_t(int L, int i, int j) {
  int dx = abs(i % L - j % L), dy = abs(i / L - j / L);
  dx = min(dx, L - dx);
  dy = min(dy, L - dy);
  return dx * dx + dy * dy;
}

// Column view of an attached simulation: column j holds col_len[j] slot
// indices at col_ent[j*col_cap ...]; -1 marks a removed synapse.  Entries of
// one row are only ever touched by the wave rewiring that row, and appends
// take their place by an atomic, so concurrent rows do not conflict.
__device__ void col_rename(const TopoDev& t, int j, int from, int to) {
  int* col = t.col_ent + (int64_t)j * t.col_cap;
  const int n = min(t.col_len[j], t.col_cap);
  for (int k = 0; k < n; ++k)
    if (col[k] == from) {
      col[k] = to;
      return;
    }
}
__device__ void col_append(const TopoDev& t, int j, int slot) {
  const int pos = atomicAdd(&t.col_len[j], 1);
  if (pos >= 0 && pos < t.col_cap) t.col_ent[(int64_t)j * t.col_cap + pos] = slot;
  else *t.col_dirty = 1;  // full column: the next simulation launch rebuilds the view
}

// Rewire row r, which received kr attempts, as one wave.  smem holds the
// row's bitfield section, kr candidates and the compaction plan.
__device__ void topo_rewire_row(uint64_t seed, const TopoDev& t, uint64_t step, int r, int kr,
                                unsigned char* smem) {
  const ProjDev& P = t.P;
  uint32_t* bits = (uint32_t*)smem;          // [words]
  int* cand = (int*)(bits + P.words);        // [n_attempts]
  int* holes = cand + t.n_attempts;          // [cap]
  int* tail = holes + P.cap;                 // [cap]
  uint8_t* remf = (uint8_t*)(tail + P.cap);  // [cap]
  const int lane = lane_id();
  kr = min(kr, P.n_post);
  __shared__ int s_kr;
  if (lane == 0) s_kr = kr;
  uint32_t* gbits = t.bits + (int64_t)r * P.words;
  for (int w = lane; w < P.words; w += WAVE) bits[w] = gbits[w];
  __syncthreads();
  // candidate targets without replacement
  if (lane == 0) {
    for (int c = 0; c < kr; ++c) {
      int j = -1;
      for (int tr = 0; tr < MAX_TRIES; ++tr) {
        const int x = (int)below(draw_u32(seed, TAG_TP_TGT, P.proj_id, step, r, c, tr), (uint32_t)P.n_post);
        if (!((bits[x >> 5] >> (x & 31)) & 1u)) { j = x; break; }
      }
      if (j < 0) {
        const int start = (int)below(draw_u32(seed, TAG_TP_TGT, P.proj_id, step, r, c, MAX_TRIES),
                                     (uint32_t)P.n_post);
        for (int d = 0; d < P.n_post; ++d) {
          const int x = (start + d) % P.n_post;
          if (!((bits[x >> 5] >> (x & 31)) & 1u)) { j = x; break; }
        }
      }
      if (j < 0) { s_kr = c; break; }
      bits[j >> 5] |= 1u << (j & 31);
      cand[c] = j;
    }
  }
  __syncthreads();
  kr = s_kr;
  // elimination attempts on existing synapses that are candidates
  const int n = P.len[r];
  const int64_t base = (int64_t)r * P.cap;
  for (int s = lane; s < n; s += WAVE) {
    const int j = P.ind[base + s];
    bool rem = false;
    if ((bits[j >> 5] >> (j & 31)) & 1u) {
      const uint64_t T = P.w[base + s] < t.g_theta ? t.T_dep : t.T_pot;
      rem = (uint64_t)draw_u32(seed, TAG_TP_ELIM, P.proj_id, step, r, s, 0) < T;
      atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    remf[s] = rem;
  }
  __syncthreads();
  // the simulation's column view: removed synapses leave a tombstone
  if (t.col_len)
    for (int s = lane; s < n; s += WAVE)
      if (remf[s]) col_rename(t, P.ind[base + s], (int)(base + s), -1);
  __syncthreads();
  int n2;
  const int pairs = wave_compaction_plan(n, remf, holes, tail, &n2);
  for (int p = lane; p < pairs; p += WAVE) {
    const int64_t d = base + holes[p], s = base + tail[p];
    const int j = P.ind[s];
    P.ind[d] = j;
    P.w[d] = P.w[s];
    if (t.col_len) col_rename(t, j, (int)s, (int)d);  // moved synapses keep their entry
  }
  __syncthreads();
  // formation attempts on the remaining candidates, ascending target order
  if (lane == 0) {
    for (int a = 1; a < kr; ++a) {
      const int x = cand[a];
      int b = a - 1;
      while (b >= 0 && cand[b] > x) { cand[b + 1] = cand[b]; --b; }
      cand[b + 1] = x;
    }
    int len = n2;
    long long formed = 0, blocked = 0;
    for (int c = 0; c < kr; ++c) {
      const int j = cand[c];
      if (!((bits[j >> 5] >> (j & 31)) & 1u)) continue;
      bits[j >> 5] &= ~(1u << (j & 31));
      const uint64_t T = t.T_d2[torus_d2_t(t.L, r, j)];
      if ((uint64_t)draw_u32(seed, TAG_TP_FORM, P.proj_id, step, r, j, 0) < T) {
        if (len < P.cap) {
          P.ind[base + len] = j;
          P.w[base + len] = t.g_new;
          if (t.col_len) col_append(t, j, (int)(base + len));
          ++len;
          ++formed;
        } else {
          ++blocked;
        }
      }
    }
    P.len[r] = len;
    if (t.col_dirty && !t.col_len && (n > n2 || formed)) *t.col_dirty = 1;
    if (n > n2) atomicAdd((unsigned long long*)&t.stats[0], (unsigned long long)(n - n2));
    if (formed) atomicAdd((unsigned long long*)&t.stats[1], (unsigned long long)formed);
    if (blocked) atomicAdd((unsigned long long*)&t.stats[2], (unsigned long long)blocked);
  }
  __syncthreads();
  for (int w = lane; w < P.words; w += WAVE) gbits[w] = bits[w];
}

// Two launches: the row list from k_topo_distribute, one wave per listed row.
__global__ void __launch_bounds__(WAVE) k_topo_rewire(uint64_t seed, TopoDev t, uint64_t step) {
  if (step == STEP_FROM_DEVICE) step = *t.step_dev;
  extern __shared__ __align__(16) unsigned char smem[];
  const int q = blockIdx.x;
  if (q >= *t.nrows) return;
  const int r = t.rowlist[q];
  topo_rewire_row(seed, t, step, r, t.kcount[r], smem);
}

// One launch (up to TOPO_FUSED_MAX attempts): wave a draws the row of every
// attempt itself and rewires row rows[a] if a is the first attempt on it,
// with the row's attempt count as k.  Same rows, counts and draws as the
// two-launch form.
constexpr int TOPO_FUSED_MAX = 2048;
__global__ void __launch_bounds__(WAVE) k_topo_rewire_fused(uint64_t seed, TopoDev t, uint64_t step) {
  if (step == STEP_FROM_DEVICE) step = *t.step_dev;
  extern __shared__ __align__(16) unsigned char smem[];
  int* rows = (int*)smem;  // [n_attempts]
  const int a = blockIdx.x, lane = lane_id(), na = t.n_attempts;
  for (int i = lane; i < na; i += WAVE)
    rows[i] = (int)below(draw_u32(seed, TAG_TP_ROW, t.P.proj_id, step, (uint64_t)i, 0, 0), (uint32_t)t.P.n_pre);
  __syncthreads();
  const int r = rows[a];
  bool earlier = false;
  int cnt = 0;
  for (int i = lane; i < na; i += WAVE)
    if (rows[i] == r) {
      ++cnt;
      earlier |= i < a;
    }
  if (ballot(earlier)) return;  // another wave owns the row
  const int kr = wave_sum_i(cnt);
  topo_rewire_row(seed, t, step, r, kr, smem + (((size_t)na * 4 + 15) & ~(size_t)15));
}

// Both projections of a map with a lateral projection in one launch: waves
// below a.n_attempts rewire projection a exactly as k_topo_rewire_fused
// does, the rest projection b.
__device__ __forceinline__ void rewire_attempt(uint64_t seed, const TopoDev& t, uint64_t step, int at) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* rows = (int*)smem;  // [n_attempts]
  const int lane = lane_id(), na = t.n_attempts;
  for (int i = lane; i < na; i += WAVE)
    rows[i] = (int)below(draw_u32(seed, TAG_TP_ROW, t.P.proj_id, step, (uint64_t)i, 0, 0), (uint32_t)t.P.n_pre);
  __syncthreads();
  const int r = rows[at];
  bool earlier = false;
  int cnt = 0;
  for (int i = lane; i < na; i += WAVE)
    if (rows[i] == r) {
      ++cnt;
      earlier |= i < at;
    }
  if (ballot(earlier)) return;  // another wave owns the row
  const int kr = wave_sum_i(cnt);
  topo_rewire_row(seed, t, step, r, kr, smem + (((size_t)na * 4 + 15) & ~(size_t)15));
}
__global__ void __launch_bounds__(WAVE) k_topo_rewire_fused_pair(uint64_t seed, TopoDev a, TopoDev b,
                                                                 uint64_t step) {
  if (step == STEP_FROM_DEVICE) step = *a.step_dev;
  // one inlined body per projection, each reading its own kernel argument
  if ((int)blockIdx.x < a.n_attempts) rewire_attempt(seed, a, step, (int)blockIdx.x);
  else rewire_attempt(seed, b, step, (int)blockIdx.x - a.n_attempts);
}

static size_t fused_lds(const TopoDev& t) {
  return (((size_t)t.n_attempts * 4 + 15) & ~(size_t)15) + (size_t)t.P.words * 4 + (size_t)t.n_attempts * 4 +
         (size_t)t.P.cap * 9 + 16;
}

void launch_topo_rewire_pair(hipStream_t s, uint64_t seed, const TopoDev& a, const TopoDev& b, uint64_t step) {
  const bool fa = a.n_attempts > 0 && a.n_attempts <= TOPO_FUSED_MAX;
  const bool fb = b.n_attempts > 0 && b.n_attempts <= TOPO_FUSED_MAX;
  if (!fa || !fb) {
    launch_topo_rewire(s, seed, a, step);
    launch_topo_rewire(s, seed, b, step);
    return;
  }
  topo_rewire_attrs();
  const size_t lds = std::max(fused_lds(a), fused_lds(b));
  hipLaunchKernelGGL(k_topo_rewire_fused_pair, dim3(a.n_attempts + b.n_attempts), dim3(WAVE), lds, s, seed, a, b,
                     step);
}

void topo_rewire_attrs() {
  static std::once_flag once;
  std::call_once(once, [] { allow_dynamic_lds((const void*)k_topo_distribute, 128 * 1024); });
}

void launch_topo_rewire(hipStream_t s, uint64_t seed, const TopoDev& t, uint64_t step) {
  topo_rewire_attrs();
  const size_t sm = (size_t)t.P.words * 4 + (size_t)t.n_attempts * 4 + (size_t)t.P.cap * 9 + 16;
  if (t.n_attempts > 0 && t.n_attempts <= TOPO_FUSED_MAX) {
    const size_t rows = ((size_t)t.n_attempts * 4 + 15) & ~(size_t)15;
    hipLaunchKernelGGL(k_topo_rewire_fused, dim3(t.n_attempts), dim3(WAVE), rows + sm, s, seed, t, step);
    return;
  }
  hipLaunchKernelGGL(k_topo_distribute, dim3(1), dim3(TD_NT), (size_t)t.P.n_pre * 4, s, seed, t, step);
  if (t.n_attempts == 0) return;
  hipLaunchKernelGGL(k_topo_rewire, dim3(t.n_attempts), dim3(WAVE), sm, s, seed, t, step);
}

}  // namespace rs
