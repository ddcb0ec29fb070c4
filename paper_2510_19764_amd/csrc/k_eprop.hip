// Per-timestep kernels of the e-prop classifier (paper, recurrent classifier
// section; eligibility traces eq. eprop_elig_1/2 and eprop_elig_lif).
//
// k_fwd: one workgroup per batch instance b.  Spikes and surrogate derivatives
//   from the state at the start of the step, ordered spike compaction with
//   ballots, propagation of input and recurrent spikes through the ragged rows
//   (one wave per spiking row, lanes over its slots, accumulation into LDS),
//   neuron update with subtractive reset, presynaptic traces, leaky readout,
//   softmax error and learning signal L_j = sum_k W_out[k][j] delta_k.
//   Input currents are accumulated as 64-bit fixed point (2^-36 resolution) so
//   the sum does not depend on the order of the LDS atomics.
// k_eprop_*: per-synapse eligibility traces over every batch instance and the
//   batch-summed gradient G_ji += sum_b L_j ebar_ji; workgroups past the rows
//   accumulate the readout delta rule.  State is laid out batch-innermost
//   ([slot][B], [neuron][B]) so a wave reads 64 consecutive instances.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int FWD_NT = 1024;
constexpr int FWD_MAX_ITEMS = 8;  // n_rec <= FWD_NT * FWD_MAX_ITEMS

__device__ __forceinline__ int block_scan_flag_fwd(bool f, int* s_wave, int* total) {
  uint64_t m = ballot(f);
  int lane = lane_id(), w = threadIdx.x / WAVE;
  constexpr int nw = FWD_NT / WAVE;
  int pre = __popcll(m & lanemask_lt());
  if (lane == 0) s_wave[w] = __popcll(m);
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < nw; ++i) {
    int c = s_wave[i];
    base += (i < w) ? c : 0;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + pre;
}

__global__ void __launch_bounds__(FWD_NT) k_fwd(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  long long* acc = (long long*)smem;                        // [n_rec]
  int* zlist = (int*)(acc + a.n_rec);                       // [n_rec]
  uint32_t* xflags = (uint32_t*)(zlist + a.n_rec);          // [(n_in+31)/32]
  const int xwords = (a.n_in + 31) >> 5;
  float* ylds = (float*)(xflags + xwords);                  // [n_out]
  float* dlds = ylds + a.n_out;                             // [n_out]
  __shared__ int s_wave[FWD_NT / WAVE];
  __shared__ unsigned long long s_events;

  const int b = blockIdx.x, tid = threadIdx.x, B = a.B;
  const int lane = lane_id(), wv = tid / WAVE;
  const int items = (a.n_rec + FWD_NT - 1) / FWD_NT;

  for (int q = tid; q < xwords; q += FWD_NT) xflags[q] = 0u;
  if (tid == 0) s_events = 0ull;

  // ---- spikes, surrogate derivative, ordered compaction of the spike list
  double vr[FWD_MAX_ITEMS], ar[FWD_MAX_ITEMS];
  bool zr[FWD_MAX_ITEMS];
  int nz = 0;
#pragma unroll
  for (int it = 0; it < FWD_MAX_ITEMS; ++it) {
    if (it >= items) break;
    const int j = it * FWD_NT + tid;
    bool z = false;
    vr[it] = 0.0;
    ar[it] = 0.0;
    if (j < a.n_rec) {
      const double v = a.V[(int64_t)b * a.n_rec + j], ad = a.A[(int64_t)b * a.n_rec + j];
      const double thr = a.v_thr + a.beta * ad;
      z = v >= thr;
      const double h = 1.0 - fabs(v - thr) / a.v_thr;
      a.psiT[(int64_t)j * B + b] = (float)(a.psi_scale * fmax(h, 0.0));
      a.z[(int64_t)b * a.n_rec + j] = (uint8_t)z;
      acc[j] = 0ll;
      vr[it] = v;
      ar[it] = ad;
    }
    zr[it] = z;
    int tot;
    int off = block_scan_flag_fwd(z, s_wave, &tot);
    if (z) zlist[nz + off] = j;
    nz += tot;
  }

  // ---- input spikes of (t, b)
  const int xq = a.t_local * B + b;
  const int xbeg = a.x_off[xq], nx = a.x_off[xq + 1] - xbeg;
  for (int q = tid; q < nx; q += FWD_NT) {
    const int i = a.x_idx[xbeg + q];
    if ((unsigned)i < (unsigned)a.n_in) atomicOr(&xflags[i >> 5], 1u << (i & 31));
  }
  __syncthreads();

  // ---- propagation: one wave per spiking row, lanes over the row's slots
  unsigned long long ev = 0ull;
  for (int r = wv; r < nx + nz; r += FWD_NT / WAVE) {
    const bool from_in = r < nx;
    const int i = from_in ? a.x_idx[xbeg + r] : zlist[r - nx];
    if (from_in && (unsigned)i >= (unsigned)a.n_in) continue;  // rejected at set_input; never read
    const int* lenp = from_in ? a.len_in : a.len_rec;
    const int* ind = from_in ? a.ind_in : a.ind_rec;
    const float* w = from_in ? a.w_in : a.w_rec;
    const int cap = from_in ? a.cap_in : a.cap_rec;
    const int n = lenp[i];
    const int64_t base = (int64_t)i * cap;
    ev += (unsigned long long)n;
    for (int k = lane; k < n; k += WAVE) {
      const int j = ind[base + k];
      const long long q = __double2ll_rn((double)w[base + k] * FIX_SCALE);
      atomicAdd((unsigned long long*)&acc[j], (unsigned long long)q);
    }
  }
  if (lane == 0 && ev) atomicAdd(&s_events, ev);
  __syncthreads();

  // ---- neuron update, recurrent trace
#pragma unroll
  for (int it = 0; it < FWD_MAX_ITEMS; ++it) {
    if (it >= items) break;
    const int j = it * FWD_NT + tid;
    if (j < a.n_rec) {
      const double I = (double)acc[j] * FIX_INV;
      const double zf = zr[it] ? 1.0 : 0.0;
      a.V[(int64_t)b * a.n_rec + j] = a.alpha * (vr[it] - zf * a.v_thr) + I;
      a.A[(int64_t)b * a.n_rec + j] = a.rho * ar[it] + zf;
      const int64_t m = (int64_t)b * a.n_rec + j, q = (int64_t)j * B + b;
      const double zb = a.zbar[m];
      const double zb1 = a.alpha * zb + zf;
      a.zbar[m] = zb1;
      a.zbar_prevT[q] = (float)zb;
      a.zbar_newT[q] = (float)zb1;
    }
  }
  // ---- input trace
  for (int i = tid; i < a.n_in; i += FWD_NT) {
    const double x = ((xflags[i >> 5] >> (i & 31)) & 1u) ? 1.0 : 0.0;
    const int64_t m = (int64_t)b * a.n_in + i;
    const double xb = a.xbar[m];
    a.xbar[m] = a.alpha * xb + x;
    a.xbar_prevT[(int64_t)i * B + b] = (float)xb;
  }

  // ---- leaky readout: one wave per output unit over the spike list
  for (int k = wv; k < a.n_out; k += FWD_NT / WAVE) {
    float s = 0.0f;
    const float* wk = a.Wout + (int64_t)k * a.n_rec;
    for (int l = lane; l < nz; l += WAVE) s += wk[zlist[l]];
    s = wave_sum(s);
    if (lane == 0) {
      const double y = a.alpha * a.Y[(int64_t)b * a.n_out + k] + (double)s + (double)a.bout[k];
      a.Y[(int64_t)b * a.n_out + k] = y;
      ylds[k] = (float)y;
    }
  }
  __syncthreads();

  // ---- softmax and output error (wave 0)
  if (wv == 0) {
    float m = -INFINITY;
    for (int k = lane; k < a.n_out; k += WAVE) m = fmaxf(m, ylds[k]);
    m = wave_max(m);
    float den = 0.0f;
    for (int k = lane; k < a.n_out; k += WAVE) den += expf(ylds[k] - m);
    den = wave_sum(den);
    const int label = a.labels[b];
    for (int k = lane; k < a.n_out; k += WAVE) {
      const float d = expf(ylds[k] - m) / den - (k == label ? 1.0f : 0.0f);
      dlds[k] = d;
      a.deltaT[(int64_t)k * B + b] = d;
    }
  }
  if (tid == 0) {
    atomicAdd(&a.counters[0], s_events);
    atomicAdd(&a.counters[1], (unsigned long long)nz);
  }
  __syncthreads();

  // ---- learning signal through B = W_out^T
#pragma unroll
  for (int it = 0; it < FWD_MAX_ITEMS; ++it) {
    if (it >= items) break;
    const int j = it * FWD_NT + tid;
    if (j < a.n_rec) {
      float l = 0.0f;
      for (int k = 0; k < a.n_out; ++k) l += a.Wout[(int64_t)k * a.n_rec + j] * dlds[k];
      a.LT[(int64_t)j * B + b] = l;
    }
  }
}

size_t fwd_smem_bytes(const FwdArgs& a) {
  return (size_t)a.n_rec * (8 + 4) + (size_t)((a.n_in + 31) / 32) * 4 + (size_t)a.n_out * 8;
}

void launch_fwd(hipStream_t s, const FwdArgs& a) {
  size_t sm = fwd_smem_bytes(a);
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)k_fwd, 150 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_fwd, dim3(a.B), dim3(FWD_NT), sm, s, a);
}

// ---------------------------------------------------------------------------
// Eligibility traces and gradients.
// Wide form (B % 4 == 0, B >= 64): a 256-thread workgroup owns one presynaptic
// row; each wave walks every 4th synapse of the row and each lane carries four
// consecutive batch instances, so every load/store of eps, ebar, psi, L and the
// presynaptic trace is a contiguous 1 KB wave access.
constexpr int EP_NT = 256;
constexpr int EP_WAVES = EP_NT / WAVE;

template <bool ALIF>
__device__ __forceinline__ float synapse_update(const EpropArgs& a, const float* __restrict__ psiT,
                                                const float* __restrict__ LT, float* __restrict__ eps,
                                                float* __restrict__ ebar, int64_t s, int j, int c, f4 p) {
  const int B = a.B;
  const f4 psi = *(const f4*)&psiT[(int64_t)j * B + 4 * c];
  const f4 L = *(const f4*)&LT[(int64_t)j * B + 4 * c];
  const d4 dpsi = __builtin_convertvector(psi, d4), dp = __builtin_convertvector(p, d4);
  const f4 eb0 = __builtin_nontemporal_load((const f4*)&ebar[s * B + 4 * c]);
  d4 e;
  if (ALIF) {
    const d4 ep = __builtin_convertvector(__builtin_nontemporal_load((const f4*)&eps[s * B + 4 * c]), d4);
    e = dpsi * (dp - a.beta * ep);
    const d4 ep1 = dpsi * dp + (a.rho - dpsi * a.beta) * ep;
    __builtin_nontemporal_store(__builtin_convertvector(ep1, f4), (f4*)&eps[s * B + 4 * c]);
  } else {
    e = dpsi * dp;
  }
  const f4 eb = __builtin_convertvector(a.alpha * __builtin_convertvector(eb0, d4) + e, f4);
  __builtin_nontemporal_store(eb, (f4*)&ebar[s * B + 4 * c]);
  return (L.x * eb.x + L.y * eb.y) + (L.z * eb.z + L.w * eb.w);
}

// One eligibility step for four batch instances held by a lane; returns the
// lane's part of sum_b L ebar.
template <bool ALIF>
__device__ __forceinline__ float trace_step(const EpropArgs& a, f4 psi, f4 L, f4 p, f4 eb0, f4 ep0,
                                            float* __restrict__ ebar_out, float* __restrict__ eps_out) {
  const d4 dpsi = __builtin_convertvector(psi, d4), dp = __builtin_convertvector(p, d4);
  d4 e;
  if (ALIF) {
    const d4 ep = __builtin_convertvector(ep0, d4);
    e = dpsi * (dp - a.beta * ep);
    const d4 ep1 = dpsi * dp + (a.rho - dpsi * a.beta) * ep;
    __builtin_nontemporal_store(__builtin_convertvector(ep1, f4), (f4*)eps_out);
  } else {
    e = dpsi * dp;
  }
  const f4 eb = __builtin_convertvector(a.alpha * __builtin_convertvector(eb0, d4) + e, f4);
  __builtin_nontemporal_store(eb, (f4*)ebar_out);
  return (L.x * eb.x + L.y * eb.y) + (L.z * eb.z + L.w * eb.w);
}

__device__ __forceinline__ void readout_grad_wave(const EpropArgs& a, int j, int lane) {
  const int B = a.B, nb4 = B / 4;
  if (j < a.n_rec) {
    for (int k = 0; k < a.n_out; ++k) {
      float g = 0.0f;
      for (int c = lane; c < nb4; c += WAVE) {
        const f4 z = *(const f4*)&a.zbar_new[(int64_t)j * B + 4 * c];
        const f4 d = *(const f4*)&a.deltaT[(int64_t)k * B + 4 * c];
        g += (d.x * z.x + d.y * z.y) + (d.z * z.z + d.w * z.w);
      }
      g = wave_sum(g);
      if (lane == 0) a.Gout[(int64_t)k * a.n_rec + j] += g;
    }
  } else if (j == a.n_rec) {
    for (int k = 0; k < a.n_out; ++k) {
      float g = 0.0f;
      for (int c = lane; c < nb4; c += WAVE) {
        const f4 d = *(const f4*)&a.deltaT[(int64_t)k * B + 4 * c];
        g += (d.x + d.y) + (d.z + d.w);
      }
      g = wave_sum(g);
      if (lane == 0) a.Gb[k] += g;
    }
  }
}

template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_wide(EpropArgs a) {
  const int row = blockIdx.x, wv = threadIdx.x / WAVE, lane = lane_id();
  const int n_rows = a.n_in + a.n_rec;
  if (row >= n_rows) {
    readout_grad_wave(a, (row - n_rows) * EP_WAVES + wv, lane);
    return;
  }
  const bool from_in = row < a.n_in;
  const int i = from_in ? row : row - a.n_in;
  const int cap = from_in ? a.in.cap : a.rec.cap;
  const int n = from_in ? a.in.len[i] : a.rec.len[i];
  const int* __restrict__ ind = from_in ? a.in.ind : a.rec.ind;
  float* __restrict__ G = from_in ? a.in.G : a.rec.G;
  float* __restrict__ eps = from_in ? a.in.eps : a.rec.eps;
  float* __restrict__ ebar = from_in ? a.in.ebar : a.rec.ebar;
  const float* __restrict__ pre = from_in ? a.xbar_prev : a.zbar_prev;
  const int B = a.B, nb4 = B / 4;
  const int64_t base = (int64_t)i * cap;
  if (nb4 <= WAVE) {
    // Wave wv owns slots k = wv + 4q.  Per chunk of 64 such slots, lane q holds
    // the target index and gradient of slot wv + 4(64c + q); synapses are then
    // processed two at a time with every load issued before any arithmetic.
    const bool act = lane < nb4;
    const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
    const f4 p = act ? *(const f4*)&pre[(int64_t)i * B + 4 * lane] : zero4;
    for (int c0 = 0; wv + 4 * c0 < n; c0 += WAVE) {
      const int kl = wv + 4 * (c0 + lane);
      const bool own = kl < n;
      const int my_j = own ? ind[base + kl] : 0;
      float my_g = own ? G[base + kl] : 0.0f;
      const int cnt = min(WAVE, (n - wv - 4 * c0 + 3) / 4);
      int q = 0;
      for (; q + 1 < cnt; q += 2) {
        const int j0 = __builtin_amdgcn_readlane(my_j, q), j1 = __builtin_amdgcn_readlane(my_j, q + 1);
        const int64_t s0 = base + wv + 4 * (c0 + q), s1 = s0 + 4;
        float g0 = 0.f, g1 = 0.f;
        if (act) {
          const f4 psi0 = *(const f4*)&a.psiT[(int64_t)j0 * B + 4 * lane];
          const f4 L0 = *(const f4*)&a.LT[(int64_t)j0 * B + 4 * lane];
          const f4 psi1 = *(const f4*)&a.psiT[(int64_t)j1 * B + 4 * lane];
          const f4 L1 = *(const f4*)&a.LT[(int64_t)j1 * B + 4 * lane];
          const f4 eb0 = __builtin_nontemporal_load((const f4*)&ebar[s0 * B + 4 * lane]);
          const f4 eb1 = __builtin_nontemporal_load((const f4*)&ebar[s1 * B + 4 * lane]);
          f4 ep0 = zero4, ep1 = zero4;
          if (ALIF) {
            ep0 = __builtin_nontemporal_load((const f4*)&eps[s0 * B + 4 * lane]);
            ep1 = __builtin_nontemporal_load((const f4*)&eps[s1 * B + 4 * lane]);
          }
          g0 = trace_step<ALIF>(a, psi0, L0, p, eb0, ep0, &ebar[s0 * B + 4 * lane], &eps[s0 * B + 4 * lane]);
          g1 = trace_step<ALIF>(a, psi1, L1, p, eb1, ep1, &ebar[s1 * B + 4 * lane], &eps[s1 * B + 4 * lane]);
        }
        g0 = wave_sum(g0);
        g1 = wave_sum(g1);
        my_g += (lane == q) ? g0 : ((lane == q + 1) ? g1 : 0.0f);
      }
      if (q < cnt) {
        const int j0 = __builtin_amdgcn_readlane(my_j, q);
        const int64_t s0 = base + wv + 4 * (c0 + q);
        float g0 = 0.f;
        if (act) {
          const f4 psi0 = *(const f4*)&a.psiT[(int64_t)j0 * B + 4 * lane];
          const f4 L0 = *(const f4*)&a.LT[(int64_t)j0 * B + 4 * lane];
          const f4 eb0 = __builtin_nontemporal_load((const f4*)&ebar[s0 * B + 4 * lane]);
          f4 ep0 = zero4;
          if (ALIF) ep0 = __builtin_nontemporal_load((const f4*)&eps[s0 * B + 4 * lane]);
          g0 = trace_step<ALIF>(a, psi0, L0, p, eb0, ep0, &ebar[s0 * B + 4 * lane], &eps[s0 * B + 4 * lane]);
        }
        g0 = wave_sum(g0);
        my_g += (lane == q) ? g0 : 0.0f;
      }
      if (own) G[base + kl] = my_g;
    }
  } else {
    for (int k = wv; k < n; k += EP_WAVES) {
      const int64_t s = base + k;
      const int j = ind[s];
      float g = 0.0f;
      for (int c = lane; c < nb4; c += WAVE) {
        const f4 p = *(const f4*)&pre[(int64_t)i * B + 4 * c];
        g += synapse_update<ALIF>(a, a.psiT, a.LT, eps, ebar, s, j, c, p);
      }
      g = wave_sum(g);
      if (lane == 0) G[s] += g;
    }
  }
}

// Narrow form (any B): threads over a row's synapses, each looping over the
// batch; used for small batches such as single-instance online learning.
template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_narrow(EpropArgs a) {
  const int row = blockIdx.x, tid = threadIdx.x;
  const int n_rows = a.n_in + a.n_rec;
  const int B = a.B;
  if (row >= n_rows) {
    const int j = (row - n_rows) * EP_NT + tid;
    if (j < a.n_rec) {
      for (int k = 0; k < a.n_out; ++k) {
        float g = 0.0f;
        for (int b = 0; b < B; ++b) g += a.deltaT[(int64_t)k * B + b] * a.zbar_new[(int64_t)j * B + b];
        a.Gout[(int64_t)k * a.n_rec + j] += g;
      }
    } else if (j == a.n_rec) {
      for (int k = 0; k < a.n_out; ++k) {
        float g = 0.0f;
        for (int b = 0; b < B; ++b) g += a.deltaT[(int64_t)k * B + b];
        a.Gb[k] += g;
      }
    }
    return;
  }
  const bool from_in = row < a.n_in;
  const int i = from_in ? row : row - a.n_in;
  const int cap = from_in ? a.in.cap : a.rec.cap;
  const int n = from_in ? a.in.len[i] : a.rec.len[i];
  const int* ind = from_in ? a.in.ind : a.rec.ind;
  float* G = from_in ? a.in.G : a.rec.G;
  float* eps = from_in ? a.in.eps : a.rec.eps;
  float* ebar = from_in ? a.in.ebar : a.rec.ebar;
  const float* pre = from_in ? a.xbar_prev : a.zbar_prev;
  for (int k = tid; k < n; k += EP_NT) {
    const int64_t s = (int64_t)i * cap + k;
    const int j = ind[s];
    float g = 0.0f;
    for (int b = 0; b < B; ++b) {
      const double p = pre[(int64_t)i * B + b];
      const double psi = a.psiT[(int64_t)j * B + b];
      double e;
      if (ALIF) {
        const double ep = eps[s * B + b];
        e = psi * (p - a.beta * ep);
        eps[s * B + b] = (float)(psi * p + (a.rho - psi * a.beta) * ep);
      } else {
        e = psi * p;
      }
      const float eb = (float)(a.alpha * (double)ebar[s * B + b] + e);
      ebar[s * B + b] = eb;
      g += a.LT[(int64_t)j * B + b] * eb;
    }
    G[s] += g;
  }
}

void launch_eprop(hipStream_t s, const EpropArgs& a) {
  const int n_rows = a.n_in + a.n_rec;
  if (a.B % 4 == 0 && a.B >= 64) {
    const int extra = (a.n_rec + 1 + EP_WAVES - 1) / EP_WAVES;
    if (a.alif) hipLaunchKernelGGL(k_eprop_wide<true>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_wide<false>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
  } else {
    const int extra = (a.n_rec + 1 + EP_NT - 1) / EP_NT;
    if (a.alif) hipLaunchKernelGGL(k_eprop_narrow<true>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_narrow<false>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
  }
}

}  // namespace rs
