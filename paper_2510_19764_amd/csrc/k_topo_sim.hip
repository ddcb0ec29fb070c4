// Topographic-map simulation (topographic-map model, Tab. A-F, H): a Poisson
// source sheet drives an L x L sheet of conductance-based LIF neurons through
// one ragged projection with all-to-all additive STDP.
//
// k_topo_sim is one workgroup of 1024 threads that runs up to a whole
// rewiring interval of steps without leaving the kernel: per step the work is a
// few thousand neurons and a handful of spikes, so a launch or a grid barrier
// per phase would cost more than the phase.  Neuron and trace state lives in
// LDS for the launch and goes back to HBM at its end; rows stay in global
// memory (L2-resident, the rewiring kernels edit them between launches).
//
// One step t (the order of the model readings):
//   A  decay the STDP traces x (source) and y (target) by exp(-h/tau)
//   B  deliver the spikes drawn at t-1 (delay t_d = h): one wave per spiking
//      source, a lane per synapse adds its weight to the target's conductance
//      (64-bit fixed point in LDS, so the sum does not depend on the order of
//      arrival) and depresses the weight by A_- y_target; x_source += 1
//   C  each thread owns target neurons: exponential Euler with the synaptic
//      current held over the step, threshold, reset, refractory count, g decay;
//      spiking targets are listed.  The same threads draw this step's input
//      spikes for their source neurons and list them for step t+1
//   D  potentiation: one wave per spiking target walks its column (the
//      synapses onto it) and adds A_+ x_source, clipped to g_max; y += 1
// The column view (slot indices grouped by target) is rebuilt at the start of
// a launch only when the rows changed since the last build (the rewiring
// kernels raise a flag), so an interval in which no synapse was formed or
// eliminated skips the remap.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int TS_NT = 1024;
constexpr int TS_MAX_N = 4096;

size_t topo_sim_lds_bytes(int N) {
  // V, g, y, x (float), ref (int), acc (int64), pre list, post list (int)
  return (size_t)N * (4 * 4 + 4 + 8 + 4 + 4);
}

bool topo_sim_fits(int N) { return N >= 1 && N <= TS_MAX_N; }

__device__ __forceinline__ int axis_dist(int L, int a, int b) {
  const int d = abs(a - b);
  return min(d, L - d);
}

// Rebuild the column view: col_off[j]..col_off[j+1] lists the slots i*cap+s
// whose target is j.  cnt and cur are LDS scratch of N ints each.
__device__ void topo_columns(const ProjDev& P, const TopoSimDev& sd, int* cnt, int* cur, int* part) {
  const int N = sd.N, tid = threadIdx.x;
  for (int j = tid; j < N; j += TS_NT) cnt[j] = 0;
  __syncthreads();
  for (int i = tid; i < N; i += TS_NT) {
    const int n = P.len[i];
    const int* ind = P.ind + (int64_t)i * P.cap;
    for (int s = 0; s < n; ++s) atomicAdd(&cnt[ind[s]], 1);
  }
  __syncthreads();
  // exclusive scan of cnt: each thread sums a contiguous chunk, then a
  // Hillis-Steele scan over the 1024 chunk sums
  const int per = (N + TS_NT - 1) / TS_NT, lo = min(tid * per, N), hi = min(lo + per, N);
  int sum = 0;
  for (int j = lo; j < hi; ++j) sum += cnt[j];
  part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < TS_NT; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - sum;
  for (int j = lo; j < hi; ++j) {
    sd.col_off[j] = run;
    cur[j] = run;
    run += cnt[j];
  }
  if (tid == TS_NT - 1) sd.col_off[N] = part[TS_NT - 1];
  __syncthreads();
  for (int i = tid; i < N; i += TS_NT) {
    const int n = P.len[i];
    const int64_t base = (int64_t)i * P.cap;
    for (int s = 0; s < n; ++s) sd.col_ent[atomicAdd(&cur[P.ind[base + s]], 1)] = (int)(base + s);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(TS_NT) k_topo_sim(uint64_t seed, ProjDev P, TopoSimDev sd, uint64_t t0,
                                                    int n_steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = sd.N, tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  long long* acc = (long long*)smem;          // [N]
  float* V = (float*)(acc + N);               // [N]
  float* g = V + N;                           // [N]
  float* y = g + N;                           // [N]
  float* x = y + N;                           // [N]
  int* ref = (int*)(x + N);                   // [N]
  int* pre = ref + N;                         // [N] sources to deliver (B), then next step's (C)
  int* post = pre + N;                        // [N] targets that spiked this step
  __shared__ int part[TS_NT];
  __shared__ int s_npre[2], s_npost;
  __shared__ int s_stim[3];

  if (*sd.col_dirty) {  // uniform: one value read by every thread
    topo_columns(P, sd, (int*)acc, (int*)acc + N, part);
    if (tid == 0) *sd.col_dirty = 0;
  }
  for (int j = tid; j < N; j += TS_NT) {
    acc[j] = 0;
    V[j] = sd.V[j];
    g[j] = sd.g[j];
    y[j] = sd.y[j];
    x[j] = sd.x[j];
    ref[j] = sd.ref[j];
  }
  if (tid == 0) {
    s_npre[0] = 0;
    s_npre[1] = 0;
  }
  __syncthreads();
  // spikes drawn at the step before t0 (a bit per source)
  for (int w = tid; w < (N + 31) / 32; w += TS_NT) {
    uint32_t m = sd.zin[w];
    while (m) {
      const int b = __builtin_ctz(m);
      m &= m - 1;
      pre[atomicAdd(&s_npre[0], 1)] = w * 32 + b;
    }
  }

  const int L = sd.L;
  for (int k = 0; k < n_steps; ++k) {
    const uint64_t t = t0 + (uint64_t)k;
    const int cb = k & 1, nb = cb ^ 1;
    // ---- A: trace decay; stimulus position for this step's epoch
    for (int j = tid; j < N; j += TS_NT) {
      x[j] *= sd.dx;
      y[j] *= sd.dy;
    }
    if (tid < 3 && (k == 0 || t % (uint64_t)sd.stim_steps == 0)) {
      const uint64_t e = t / (uint64_t)sd.stim_steps;
      const uint32_t u = draw_u32(seed, TAG_STIM, 0, e, (uint64_t)tid, 0, 0);
      s_stim[tid] = tid < 2 ? (int)below(u, (uint32_t)L) : (int)(u & 1u);
    }
    if (tid == 0) {
      s_npre[nb] = 0;
      s_npost = 0;
    }
    __syncthreads();
    // ---- B: delivery with depression, one wave per spiking source
    const int npre = s_npre[cb];
    for (int q = wv; q < npre; q += TS_NT / WAVE) {
      const int i = pre[q];
      const int n = P.len[i];
      const int64_t base = (int64_t)i * P.cap;
      for (int s = lane; s < n; s += WAVE) {
        const int j = P.ind[base + s];
        const float w = P.w[base + s];
        atomicAdd((unsigned long long*)&acc[j], (unsigned long long)__double2ll_rn((double)w * FIX_SCALE));
        if (sd.stdp) P.w[base + s] = fmaxf(0.f, w - sd.A_minus * y[j]);
      }
      if (lane == 0) x[i] += 1.f;
    }
    __syncthreads();
    // ---- C: neurons, then this step's input draws
    const bool last = k == n_steps - 1;
    const int cx = s_stim[0], cy = s_stim[1], orient = s_stim[2];
    for (int j0 = 0; j0 < N; j0 += TS_NT) {
      const int j = j0 + tid;
      bool z = false, zi = false;
      if (j < N) {
        float gj = g[j] + (float)((double)acc[j] * FIX_INV);
        acc[j] = 0;
        float v = V[j];
        if (ref[j] > 0) {
          ref[j] -= 1;
          v = sd.V_reset;
        } else {
          const float I = gj * (sd.E_exc - v);
          const float RI = sd.R * I;
          v = sd.V_rest + RI + (v - sd.V_rest - RI) * sd.em;
          if (v >= sd.V_th) {
            z = true;
            v = sd.V_reset;
            ref[j] = sd.ref_steps;
            sd.count[j] += 1u;
            post[atomicAdd(&s_npost, 1)] = j;
          }
        }
        V[j] = v;
        g[j] = gj * sd.es;
        // input neuron j of the source sheet
        const int dxs = axis_dist(L, j % L, cx), dys = axis_dist(L, j / L, cy);
        const int d2 = sd.stim_kind ? (orient ? dys * dys : dxs * dxs) : dxs * dxs + dys * dys;
        const uint32_t u = draw_u32(seed, TAG_INPUT, 0, t, 0, (uint64_t)j, 0);
        zi = (uint64_t)u < sd.T_in[d2];
        if (zi) pre[atomicAdd(&s_npre[nb], 1)] = j;  // the list of step t was consumed in B
      }
      if (last) {
        const uint64_t mz = ballot(z), mi = ballot(zi);
        const int w0 = (j0 + wv * WAVE) >> 5;
        const int words = (N + 31) / 32;
        if (lane == 0 && w0 < words) {
          sd.zout[w0] = (uint32_t)mz;
          sd.zin[w0] = (uint32_t)mi;
        }
        if (lane == 0 && w0 + 1 < words) {
          sd.zout[w0 + 1] = (uint32_t)(mz >> 32);
          sd.zin[w0 + 1] = (uint32_t)(mi >> 32);
        }
      }
    }
    __syncthreads();
    // ---- D: potentiation along the columns of spiking targets
    const int npost = s_npost;
    if (sd.stdp) {
      for (int q = wv; q < npost; q += TS_NT / WAVE) {
        const int j = post[q];
        const int e0 = sd.col_off[j], e1 = sd.col_off[j + 1];
        for (int e = e0 + lane; e < e1; e += WAVE) {
          const int slot = sd.col_ent[e];
          const float w = P.w[slot] + sd.A_plus * x[slot / P.cap];
          P.w[slot] = fminf(w, sd.g_max);
        }
      }
    }
    for (int q = tid; q < npost; q += TS_NT) y[post[q]] += 1.f;
    __syncthreads();
  }
  for (int j = tid; j < N; j += TS_NT) {
    sd.V[j] = V[j];
    sd.g[j] = g[j];
    sd.y[j] = y[j];
    sd.x[j] = x[j];
    sd.ref[j] = ref[j];
  }
}

void launch_topo_sim(hipStream_t s, uint64_t seed, const ProjDev& P, const TopoSimDev& sd, uint64_t t0,
                     int n_steps) {
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)k_topo_sim, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_topo_sim, dim3(1), dim3(TS_NT), topo_sim_lds_bytes(sd.N), s, seed, P, sd, t0, n_steps);
}

}  // namespace rs
