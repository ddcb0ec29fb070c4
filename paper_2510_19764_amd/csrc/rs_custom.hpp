// Custom connectivity updates on ragged rows (paper, Sec. 2.1): a rule's row
// update runs in parallel over the rows of a projection; within it the
// synapses of the row are visited (for_each_synapse), any of them may be
// removed (remove_synapse, with the ragged rule: the row's last synapse moves
// into the freed slot), and new synapses are appended (add_synapse, with the
// variables a rule does not set starting at zero).  A rule's host update runs
// on the host between row updates (the paper's host_update_code).
//
// A rule is a struct with these device members, all called by every lane of
// the row's wave:
//   bool active(const RowCtx&)        the row takes part (false: untouched)
//   void begin(RowCtx&)               row-local preparation (LDS: ctx.smem)
//   Visit visit(const RowCtx&, const Syn&)   one synapse; lanes in parallel
//   void removed(const RowCtx&, const Syn&)  each synapse finally removed
//   void add(RowCtx&, Adder&)         appends, lane 0 only (ctx.lane == 0)
//   void end(const RowCtx&, int removed, int added)   lane 0 only
// and `static constexpr size_t smem_bytes(const ProjDev&)` for its LDS.
//
// Semantics, fixed so that rows run in parallel and a row's lanes too:
//   - visit() sees every synapse the row held when its update began, with its
//     slot at that time; its decisions must not depend on each other (a rule
//     keys any random draw by that slot), which makes the result equal to the
//     sequential loop with swap-removal and re-examination;
//   - a Visit with stop set ends the iteration after it: only synapses in
//     slots up to the first stopping one (ascending) count as visited, and
//     only they can be removed;
//   - removal then compacts the row canonically (the sequential rule's
//     closed form), moving every record: index, weight, optimiser state,
//     gradient and the eligibility traces of all batch instances;
//   - add() appends after the removals, in call order, while the row has room.
#pragma once
#include "rs_compact.hpp"
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {
namespace custom {

struct RowCtx {
  const ProjDev& P;
  int id_pre;             // the row
  int n;                  // synapses the row held when the update began
  int lane;
  uint64_t seed, step;
  unsigned char* smem;    // the rule's LDS
  __device__ uint32_t rng(uint32_t tag, uint64_t c2, uint64_t c3 = 0) const {
    return draw_u32(seed, tag, P.proj_id, step, (uint64_t)id_pre, c2, c3);
  }
};

struct Syn {
  int slot;       // slot when the row's update began
  int id_post;    // target
  float w;        // weight
};

struct Visit {
  bool remove = false;
  bool stop = false;
};

// Appends synapses for lane 0; the wave writes their records afterwards.
struct Adder {
  int* tgt;
  float* w;
  int room;
  int count = 0;
  __device__ bool add_synapse(int id_post, float weight) {
    if (count >= room) return false;
    tgt[count] = id_post;
    w[count] = weight;
    ++count;
    return true;
  }
};

// LDS of the row machinery: holes, tail (int[cap]), removal flags
// (u8[cap]), new targets and weights (int, float [cap]), then the rule's.
__host__ __device__ inline size_t row_smem_base(int cap) {
  return (((size_t)cap * 4 * 4 + (size_t)cap + 16) + 15) & ~(size_t)15;
}

template <class Rule>
__global__ void __launch_bounds__(WAVE) k_row_update(ProjDev P, Rule rule, uint64_t seed, uint64_t step, int B,
                                                      long long* stats) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* holes = (int*)smem;
  int* tail = holes + P.cap;
  int* newj = tail + P.cap;
  float* neww = (float*)(newj + P.cap);
  uint8_t* remf = (uint8_t*)(neww + P.cap);
  __shared__ int s_stop, s_added;
  const int r = blockIdx.x, lane = lane_id();
  RowCtx ctx{P, r, P.len[r], lane, seed, step, smem + row_smem_base(P.cap)};
  if (!rule.active(ctx)) return;
  if (lane == 0) s_stop = ctx.n;
  rule.begin(ctx);
  __syncthreads();
  const int n = ctx.n;
  const int64_t base = (int64_t)r * P.cap;
  // for_each_synapse: every lane visits its slots
  for (int k = lane; k < n; k += WAVE) {
    const Syn s{k, P.ind[base + k], P.w[base + k]};
    const Visit v = rule.visit(ctx, s);
    remf[k] = v.remove;
    if (v.stop) atomicMin(&s_stop, k);
  }
  __syncthreads();
  const int stop = s_stop;
  for (int k = lane; k < n; k += WAVE) {
    if (k > stop) remf[k] = 0;
    if (remf[k]) rule.removed(ctx, Syn{k, P.ind[base + k], P.w[base + k]});
  }
  __syncthreads();
  int n2;
  const int pairs = wave_compaction_plan(n, remf, holes, tail, &n2);
  for (int q = lane; q < pairs; q += WAVE) {
    const int64_t d = base + holes[q], s = base + tail[q];
    P.ind[d] = P.ind[s];
    P.w[d] = P.w[s];
    if (P.m) P.m[d] = P.m[s];
    if (P.v) P.v[d] = P.v[s];
    if (P.G) P.G[d] = P.G[s];
  }
  if (P.ebar)
    for (int q = 0; q < pairs; ++q) {
      const int64_t d = base + holes[q], s = base + tail[q];
      for (int c = lane; c < P.erec; c += WAVE) P.ebar[d * P.erec + c] = P.ebar[s * P.erec + c];
      if (P.eps)
        for (int c = lane; c < B; c += WAVE) P.eps[d * B + c] = P.eps[s * B + c];
    }
  __syncthreads();
  // add_synapse: lane 0 runs the rule's appends
  if (lane == 0) {
    Adder ad{newj, neww, P.cap - n2};
    rule.add(ctx, ad);
    s_added = ad.count;
    rule.end(ctx, n - n2, ad.count);
  }
  __syncthreads();
  const int na = s_added;
  for (int k = lane; k < na; k += WAVE) {
    const int64_t s = base + n2 + k;
    P.ind[s] = newj[k];
    P.w[s] = neww[k];
    if (P.m) P.m[s] = 0.0f;
    if (P.v) P.v[s] = 0.0f;
    if (P.G) P.G[s] = 0.0f;
  }
  if (P.ebar)
    for (int k = 0; k < na; ++k) {
      const int64_t s = base + n2 + k;
      for (int c = lane; c < P.erec; c += WAVE) P.ebar[s * P.erec + c] = 0.0f;
      if (P.eps)
        for (int c = lane; c < B; c += WAVE) P.eps[s * B + c] = 0.0f;
    }
  if (lane == 0) {
    P.len[r] = n2 + na;
    if (n > n2) atomicAdd((unsigned long long*)&stats[0], (unsigned long long)(n - n2));
    if (na) atomicAdd((unsigned long long*)&stats[1], (unsigned long long)na);
  }
}

// Run a rule's row update over every row of P (stats: int64[2], removed and
// added, incremented).
template <class Rule>
void launch_row_update(hipStream_t s, const ProjDev& P, const Rule& rule, uint64_t seed, uint64_t step, int B,
                       long long* stats) {
  const size_t sm = row_smem_base(P.cap) + Rule::smem_bytes(P);
  hipLaunchKernelGGL(k_row_update<Rule>, dim3(P.n_pre), dim3(WAVE), sm, s, P, rule, seed, step, B, stats);
}

}  // namespace custom
}  // namespace rs
