// Topographic-map simulation (topographic-map model, Tab. A-F, H): a Poisson
// source sheet drives an L x L sheet of conductance-based LIF neurons through
// one ragged projection with all-to-all additive STDP.
//
// k_topo_sim is one workgroup of 1024 threads that runs up to a whole
// rewiring interval of steps without leaving the kernel: per step the work is a
// few thousand neurons and a handful of spikes, so a launch or a grid barrier
// per phase would cost more than the phase.  Target-neuron state lives in
// registers and the STDP traces in LDS for the launch, and both go back to HBM
// at its end; rows stay in global memory (L2-resident, the rewiring kernels
// edit them between launches).
//
// One step t (the order of the model readings):
//   A  decay the STDP traces x (source) and y (target) by exp(-h/tau); done
//      for the first step of a launch only, the others take it at the end of
//      phase C of the step before (y then also takes the step's spikes, and
//      potentiation reads x through 1/exp(-h/tau_+)), which saves a barrier
//   B  deliver the spikes drawn at t-1 (delay t_d = h): one wave per spiking
//      source, a lane per synapse adds its weight to the target's conductance
//      (64-bit fixed point in LDS, so the sum does not depend on the order of
//      arrival) and depresses the weight by A_- y_target; x_source += 1
//      Meanwhile the upper half of the workgroup draws the source's spikes of
//      step t, eight channels per generator call, into a second list; each
//      drawing thread keeps its channels' thresholds in registers and looks
//      them up again only when the stimulus moves
//   C  each thread owns up to four target neurons, whose V, g, refractory
//      count and spike count stay in registers for the launch: exponential
//      Euler with the synaptic current held over the step, threshold, reset,
//      refractory count, g decay; spiking targets are listed
//   D  potentiation: one wave per spiking target walks its column (the
//      synapses onto it) and adds A_+ x_source, clipped to g_max
// The column view (slot indices grouped by target, one padded column per
// target) is kept up to date by the rewiring kernels, which know every slot
// they remove, move or fill; it is rebuilt from the rows at the start of a
// launch only after the build, a restore of rows or a full column.  Launched from a recorded graph, the kernel
// takes its first step from device memory (STEP_FROM_DEVICE) and every launch
// writes the step count it reached back.
#include <mutex>

#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int TS_NT = 1024;
constexpr int TS_MAX_N = 4096;
constexpr int TS_PER = TS_MAX_N / TS_NT;  // target neurons owned by each thread
static_assert(TS_MAX_N / 8 <= TS_NT / 2, "the upper half of the workgroup draws every source group");
static_assert((TS_NT / 2) % WAVE == 0, "drawing threads form whole waves");
static_assert(TS_MAX_N / 32 <= TS_NT, "one thread per word of source spike bits");

// acc (int64), y, x (float), two source lists, the target list and the
// column lengths (int)
size_t topo_sim_lds_bytes(int N) {
  return (size_t)N * (8 + 4 + 4 + 4 + 4 + 4 + 4);
}

bool topo_sim_fits(int N) { return N >= 1 && N <= TS_MAX_N; }

// Add the wall-clock ticks since `prev` to `acc` and restart from now.
__device__ __forceinline__ void phase_mark(long long& acc, long long& prev) {
  const long long now = (long long)wall_clock64();
  acc += now - prev;
  prev = now;
}

__device__ __forceinline__ int axis_dist(int L, int a, int b) {
  const int d = abs(a - b);
  return min(d, L - d);
}

// Rebuild the column view from the rows: column j lists at col_ent[j*col_cap]
// the slot indices i*cap+s of the col_len[j] synapses onto j (the LDS copy
// clen holds the lengths).  Needed only after the build, a restore of rows or
// a full column; otherwise the rewiring kernels edit the view in place.  A row
// holds each target at most once, so no column exceeds N = col_cap entries.
__device__ void topo_columns(const ProjDev& P, const TopoSimDev& sd, int* clen) {
  const int N = sd.N, tid = threadIdx.x;
  for (int j = tid; j < N; j += TS_NT) clen[j] = 0;
  __syncthreads();
  for (int i = tid; i < N; i += TS_NT) {
    const int n = P.len[i];
    const int64_t base = (int64_t)i * P.cap;
    for (int s = 0; s < n; ++s) {
      const int j = P.ind[base + s];
      const int pos = atomicAdd(&clen[j], 1);
      if (pos < sd.col_cap) sd.col_ent[(int64_t)j * sd.col_cap + pos] = (int)(base + s);
    }
  }
  __syncthreads();
  for (int j = tid; j < N; j += TS_NT) sd.col_len[j] = clen[j];
}

// TIMED: the phase timers are compiled in (a separate instance, so that the
// untimed kernel carries none of their registers or branches).
template <bool TIMED>
__global__ void __launch_bounds__(TS_NT) k_topo_sim(uint64_t seed, ProjDev P, TopoSimDev sd, uint64_t t0,
                                                    int n_steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (t0 == STEP_FROM_DEVICE) t0 = *sd.step_dev;
  // optional phase timers (Fig. 10 split): thread 0 reads the device wall clock
  const bool tm = TIMED && threadIdx.x == 0;
  long long tprev = tm ? (long long)wall_clock64() : 0, tk[TOPO_PHASES] = {0, 0, 0, 0};
  const int N = sd.N, tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  long long* acc = (long long*)smem;          // [N] delivered conductance, fixed point
  float* y = (float*)(acc + N);               // [N] target trace
  float* x = y + N;                           // [N] source trace
  int* pre0 = (int*)(x + N);                  // [N] source lists: this step's deliveries and
  int* pre1 = pre0 + N;                       // [N]   the next step's, alternating
  int* post = pre1 + N;                       // [N] targets that spiked this step
  int* clen = post + N;                       // [N] column lengths
  __shared__ int s_npre[2], s_npost;
  __shared__ int s_stim[3];

  // Every load of the launch's starting state is issued before any of it is
  // used, so the prologue costs one memory round trip (two with a rebuild).
  const int dirty = *sd.col_dirty;  // uniform: one value read by every thread
  float Vr[TS_PER], gr[TS_PER], xr[TS_PER], yr[TS_PER];  // target neurons j = tid + m*TS_NT
  int refr[TS_PER];
  uint32_t cnt[TS_PER];
#pragma unroll
  for (int m = 0; m < TS_PER; ++m) {
    const int j = tid + m * TS_NT;
    const bool ok = j < N;
    Vr[m] = ok ? sd.V[j] : 0.f;
    gr[m] = ok ? sd.g[j] : 0.f;
    refr[m] = ok ? sd.ref[j] : 0;
    cnt[m] = ok ? sd.count[j] : 0u;
    xr[m] = ok ? sd.x[j] : 0.f;
    yr[m] = ok ? sd.y[j] : 0.f;
  }
  const int words = (N + 31) / 32;  // <= TS_NT
  uint32_t zw = tid < words ? sd.zin[tid] : 0u;  // spikes drawn at the step before t0
  const int L = sd.L, Ls = sd.stim_L, cap = P.cap, ngrp = (N + 7) / 8;  // ngrp <= TS_NT / 2
  if (tid < 3) {  // stimulus position of t0's epoch
    const uint32_t u = draw_u32(seed, TAG_STIM, 0, t0 / (uint64_t)sd.stim_steps, (uint64_t)tid, 0, 0);
    s_stim[tid] = tid < 2 ? (int)below(u, (uint32_t)Ls) : (int)(u & 1u);
  }
  if (tid == 0) {
    s_npre[0] = 0;
    s_npre[1] = 0;
  }
  if (dirty) {
    topo_columns(P, sd, clen);
    if (tid == 0) *sd.col_dirty = 0;
  } else {
    for (int j = tid; j < N; j += TS_NT) clen[j] = min(sd.col_len[j], sd.col_cap);
  }
  // ---- A of the first step: trace decay.  Later steps decay their traces at
  // the end of the step before (phase C).
#pragma unroll
  for (int m = 0; m < TS_PER; ++m) {
    const int j = tid + m * TS_NT;
    if (j < N) {
      acc[j] = 0;
      x[j] = xr[m] * sd.dx;
      y[j] = yr[m] * sd.dy;
    }
  }
  __syncthreads();
  while (zw) {
    const int b = __builtin_ctz(zw);
    zw &= zw - 1;
    pre0[atomicAdd(&s_npre[0], 1)] = tid * 32 + b;
  }
  uint64_t thr[8];  // this thread's source thresholds for the current stimulus epoch
  __syncthreads();
  if (tm) phase_mark(tk[3], tprev);
  for (int k = 0; k < n_steps; ++k) {
    const uint64_t t = t0 + (uint64_t)k;
    const int cb = k & 1, nb = cb ^ 1;
    if (tid == 0) s_npost = 0;  // D of the step before read it before the barrier
    // ---- B: delivery with depression, one wave per spiking source from wave 0
    // up; every slot of the padded row is loaded together with the row length.
    // Meanwhile the upper half of the workgroup draws this step's source spikes,
    // eight channels per generator call, into the other list.
    const int npre = s_npre[cb];
    int* cur = cb ? pre1 : pre0;
    int* nxt = cb ? pre0 : pre1;
    for (int q = wv; q < npre; q += TS_NT / WAVE) {
      const int i = cur[q];
      const int64_t base = (int64_t)i * cap;
      const int n = P.len[i];
      for (int s = lane; s < cap; s += WAVE) {
        const int j = P.ind[base + s];
        const float w = P.w[base + s];
        if (s < n) {
          atomicAdd((unsigned long long*)&acc[j], (unsigned long long)__double2ll_rn((double)w * FIX_SCALE));
          if (sd.stdp) P.w[base + s] = fmaxf(0.f, w - sd.A_minus * y[j]);
        }
      }
      if (lane == 0) x[i] += 1.f;
    }
    const bool last = k == n_steps - 1;
    if (tid >= TS_NT / 2) {  // whole waves: TS_NT / 2 is a multiple of the wave size
      const int c = tid - TS_NT / 2;
      uint32_t byte = 0;
      if (c < ngrp) {
        if (k == 0 || t % (uint64_t)sd.stim_steps == 0) {
          const int cx = s_stim[0], cy = s_stim[1], orient = s_stim[2];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int i = 8 * c + b;
            thr[b] = 0;  // channels beyond the sheet never fire
            if (i < N) {
              const int dxs = axis_dist(Ls, (i % L) % Ls, cx), dys = axis_dist(Ls, (i / L) % Ls, cy);
              const int d2 = sd.stim_kind ? (orient ? dys * dys : dxs * dxs) : dxs * dxs + dys * dys;
              thr[b] = sd.T_in[d2];
            }
          }
        }
        const U64x4 o = philox(seed, (uint64_t)TAG_TP_INPUT, t, (uint64_t)c, 0, 0);
        const uint64_t wd[4] = {o.x0, o.x1, o.x2, o.x3};
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint32_t u = (b & 1) ? (uint32_t)wd[b >> 1] : (uint32_t)(wd[b >> 1] >> 32);
          if ((uint64_t)u < thr[b]) {
            byte |= 1u << b;
            nxt[atomicAdd(&s_npre[nb], 1)] = 8 * c + b;
          }
        }
      }
      if (last) {
        // four consecutive threads hold one 32-bit word of source bits
        uint32_t wbits = byte << (8 * (lane & 3));
        wbits |= __shfl_xor(wbits, 1, WAVE);
        wbits |= __shfl_xor(wbits, 2, WAVE);
        if ((lane & 3) == 0 && c < ngrp) sd.zin[c >> 2] = wbits;
      }
    }
    __syncthreads();
    if (tm) phase_mark(tk[0], tprev);
    // ---- C: neurons (registers)
#pragma unroll
    for (int m = 0; m < TS_PER; ++m) {
      const int j = tid + m * TS_NT;
      bool z = false;
      if (j < N) {
        const float gj = gr[m] + (float)((double)acc[j] * FIX_INV);
        acc[j] = 0;
        float v = Vr[m];
        if (refr[m] > 0) {
          refr[m] -= 1;
          v = sd.V_reset;
        } else {
          const float I = gj * (sd.E_exc - v);
          const float RI = sd.R * I;
          v = sd.V_rest + RI + (v - sd.V_rest - RI) * sd.em;
          if (v >= sd.V_th) {
            z = true;
            v = sd.V_reset;
            refr[m] = sd.ref_steps;
            cnt[m] += 1u;
            post[atomicAdd(&s_npost, 1)] = j;
          }
        }
        Vr[m] = v;
        gr[m] = gj * sd.es;
        // traces: y += z now (potentiation does not read y), and both traces
        // take the next step's decay, except after a launch's last step
        const float yz = y[j] + (z ? 1.f : 0.f);
        y[j] = last ? yz : yz * sd.dy;
        if (!last) x[j] *= sd.dx;
      }
      if (last && m * TS_NT < N) {
        const uint64_t mz = ballot(z);
        const int w0 = (m * TS_NT + wv * WAVE) >> 5, words = (N + 31) / 32;
        if (lane == 0 && w0 < words) sd.zout[w0] = (uint32_t)mz;
        if (lane == 0 && w0 + 1 < words) sd.zout[w0 + 1] = (uint32_t)(mz >> 32);
      }
    }
    if (tid == 0) s_npre[cb] = 0;  // the list step k+1 draws into; read at the start of B
    __syncthreads();
    if (tm) phase_mark(tk[1], tprev);
    // ---- D: potentiation along the columns of spiking targets.  x already
    // carries the next step's decay unless this is the launch's last step.
    const int npost = s_npost;
    const float xs = last ? 1.f : sd.inv_dx;
    if (sd.stdp) {
      for (int q = wv; q < npost; q += TS_NT / WAVE) {
        const int j = post[q];
        const int* col = sd.col_ent + (int64_t)j * sd.col_cap;
        for (int e = lane; e < clen[j]; e += WAVE) {
          const int slot = col[e];
          if (slot < 0) continue;  // removed by a rewire
          const float w = P.w[slot] + sd.A_plus * (x[slot / cap] * xs);
          P.w[slot] = fminf(w, sd.g_max);
        }
      }
    }
    // stimulus position of the next step's epoch
    if (tid < 3 && !last && (t + 1) % (uint64_t)sd.stim_steps == 0) {
      const uint32_t u = draw_u32(seed, TAG_STIM, 0, (t + 1) / (uint64_t)sd.stim_steps, (uint64_t)tid, 0, 0);
      s_stim[tid] = tid < 2 ? (int)below(u, (uint32_t)Ls) : (int)(u & 1u);
    }
    __syncthreads();
    if (tm) phase_mark(tk[2], tprev);
  }
#pragma unroll
  for (int m = 0; m < TS_PER; ++m) {
    const int j = tid + m * TS_NT;
    if (j < N) {
      sd.V[j] = Vr[m];
      sd.g[j] = gr[m];
      sd.ref[j] = refr[m];
      sd.count[j] = cnt[m];
    }
  }
  for (int j = tid; j < N; j += TS_NT) {
    sd.y[j] = y[j];
    sd.x[j] = x[j];
  }
  if (tid == 0) *sd.step_dev = t0 + (uint64_t)n_steps;
  if (tm)
    for (int q = 0; q < TOPO_PHASES; ++q) atomicAdd(&sd.ticks[q], (unsigned long long)tk[q]);
}

void topo_sim_attrs() {
  static std::once_flag once;
  std::call_once(once, [] {
    allow_dynamic_lds((const void*)k_topo_sim<false>, 160 * 1024);
    allow_dynamic_lds((const void*)k_topo_sim<true>, 160 * 1024);
  });
}

void launch_topo_sim(hipStream_t s, uint64_t seed, const ProjDev& P, const TopoSimDev& sd, uint64_t t0,
                     int n_steps) {
  topo_sim_attrs();
  if (sd.ticks)
    hipLaunchKernelGGL(k_topo_sim<true>, dim3(1), dim3(TS_NT), topo_sim_lds_bytes(sd.N), s, seed, P, sd, t0,
                       n_steps);
  else
    hipLaunchKernelGGL(k_topo_sim<false>, dim3(1), dim3(TS_NT), topo_sim_lds_bytes(sd.N), s, seed, P, sd, t0,
                       n_steps);
}

}  // namespace rs
