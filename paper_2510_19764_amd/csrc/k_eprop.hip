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

// LDS layout of k_fwd (offsets 16-byte aligned):
//   acc      int64[n_rec]        fixed-point input current of the step
//   zlist    int[n_rec]          ordered spike list of the step
//   len_in   int[n_in], len_rec int[n_rec]   row lengths, staged per launch
//   xflags   u32[ceil(n_in/32)]  input spikes of the step as bits
//   xpos     int[33]             start of each step's input list in xbuf
//   xbuf     int[xcap]           the launch's input spike lists
//   yst      double[n_out], ylds/dlds float[n_out]
//   wout     float[n_out*n_rec]  readout weights (when wout_lds)
struct FwdLds {
  size_t acc, zlist, len_in, len_rec, xflags, xpos, xbuf, yst, ylds, dlds, wout, total;
};
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline FwdLds fwd_lds_layout(int n_in, int n_rec, int n_out, int xcap, int wout_lds) {
  FwdLds L;
  size_t o = 0;
  L.acc = o; o = align16(o + (size_t)n_rec * 8);
  L.zlist = o; o = align16(o + (size_t)n_rec * 4);
  L.len_in = o; o = align16(o + (size_t)n_in * 4);
  L.len_rec = o; o = align16(o + (size_t)n_rec * 4);
  L.xflags = o; o = align16(o + (size_t)((n_in + 31) / 32) * 4);
  L.xpos = o; o = align16(o + 33 * 4);
  L.xbuf = o; o = align16(o + (size_t)xcap * 4);
  L.yst = o; o = align16(o + (size_t)n_out * 8);
  L.ylds = o; o = align16(o + (size_t)n_out * 4);
  L.dlds = o; o = align16(o + (size_t)n_out * 4);
  L.wout = o; o = align16(o + (wout_lds ? (size_t)n_out * n_rec * 4 : 0));
  L.total = o;
  return L;
}

template <int ITEMS>
__global__ void __launch_bounds__(FWD_NT) k_fwd(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const FwdLds lay = fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds);
  long long* acc = (long long*)(smem + lay.acc);
  int* zlist = (int*)(smem + lay.zlist);
  int* len_in = (int*)(smem + lay.len_in);
  int* len_rec = (int*)(smem + lay.len_rec);
  uint32_t* xflags = (uint32_t*)(smem + lay.xflags);
  int* xpos = (int*)(smem + lay.xpos);
  int* xbuf = (int*)(smem + lay.xbuf);
  double* yst = (double*)(smem + lay.yst);
  float* ylds = (float*)(smem + lay.ylds);
  float* dlds = (float*)(smem + lay.dlds);
  const float* wout = a.wout_lds ? (const float*)(smem + lay.wout) : a.Wout;
  const int xwords = (a.n_in + 31) >> 5;
  __shared__ int s_wave[FWD_NT / WAVE];
  __shared__ unsigned long long s_events;
  __shared__ int s_xsrc[33], s_xcnt[33];
  __shared__ int s_xstaged;

  const int b = blockIdx.x, tid = threadIdx.x, B = a.B;
  const int lane = lane_id(), wv = tid / WAVE;
  const int items = (a.n_rec + FWD_NT - 1) / FWD_NT;
  const int xitems = (a.n_in + FWD_NT - 1) / FWD_NT;

  // ---- stage the launch's constants: row lengths, readout weights, input lists
  for (int i = tid; i < a.n_in; i += FWD_NT) len_in[i] = a.len_in[i];
  for (int i = tid; i < a.n_rec; i += FWD_NT) len_rec[i] = a.len_rec[i];
  if (a.wout_lds) {
    float* w = (float*)(smem + lay.wout);
    const int nw = a.n_out * a.n_rec;
    for (int q = tid; q < nw; q += FWD_NT) w[q] = a.Wout[q];
  }
  if (tid <= a.nsteps) {
    const int tau = tid < a.nsteps ? tid : a.nsteps - 1;
    const int xq = ((a.t0 + tau) % a.sample_steps) * B + b;
    // clamp the caller's offsets into the index array
    const long long lo = min(max((long long)a.x_off[xq], 0ll), a.n_idx);
    const long long hi = min(max((long long)a.x_off[xq + 1], lo), a.n_idx);
    s_xsrc[tid] = tid < a.nsteps ? (int)lo : 0;
    s_xcnt[tid] = tid < a.nsteps ? (int)(hi - lo) : 0;
  }
  __syncthreads();
  if (tid == 0) {  // starts of each step's list in xbuf, staged only if all fit
    long long run = 0;
    for (int t = 0; t < a.nsteps; ++t) {
      xpos[t] = (int)min(run, (long long)a.xcap);
      run += s_xcnt[t];
    }
    xpos[a.nsteps] = (int)min(run, (long long)a.xcap);
    s_xstaged = run <= (long long)a.xcap;
  }
  __syncthreads();
  const bool xstaged = s_xstaged != 0;
  if (xstaged) {
    for (int t = wv; t < a.nsteps; t += FWD_NT / WAVE) {
      const int n = s_xcnt[t];
      for (int l = lane; l < n; l += WAVE) xbuf[xpos[t] + l] = a.x_idx[s_xsrc[t] + l];
    }
  }

  // neuron, trace and readout state of this instance stays on chip for the block
  double vr[ITEMS], ar[ITEMS], zbr[ITEMS], xbr[ITEMS];
  bool zr[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int j = it * FWD_NT + tid;
    const bool ok = it < items && j < a.n_rec;
    vr[it] = ok ? a.V[(int64_t)b * a.n_rec + j] : 0.0;
    ar[it] = ok ? a.A[(int64_t)b * a.n_rec + j] : 0.0;
    zbr[it] = ok ? a.zbar[(int64_t)b * a.n_rec + j] : 0.0;
    const int i = it * FWD_NT + tid;
    xbr[it] = (it < xitems && i < a.n_in) ? a.xbar[(int64_t)b * a.n_in + i] : 0.0;
    zr[it] = false;
  }
  for (int k = tid; k < a.n_out; k += FWD_NT) yst[k] = a.Y[(int64_t)b * a.n_out + k];
  if (tid == 0) s_events = 0ull;
  unsigned long long spikes = 0ull;
  const int label = a.labels[b];
  __syncthreads();

  for (int tau = 0; tau < a.nsteps; ++tau) {
    for (int q = tid; q < xwords; q += FWD_NT) xflags[q] = 0u;
    // ---- spikes, surrogate derivative, ordered compaction of the spike list
    int nz = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (it >= items) break;
      const int j = it * FWD_NT + tid;
      bool z = false;
      if (j < a.n_rec) {
        const double thr = a.v_thr + a.beta * ar[it];
        z = vr[it] >= thr;
        const double h = 1.0 - fabs(vr[it] - thr) / a.v_thr;
        a.psi[((int64_t)tau * B + b) * a.n_rec + j] = (float)(a.psi_scale * fmax(h, 0.0));
        acc[j] = 0ll;
      }
      zr[it] = z;
      int tot;
      const int off = block_scan_flag_fwd(z, s_wave, &tot);
      if (z) zlist[nz + off] = j;
      nz += tot;
    }
    spikes += (unsigned long long)nz;

    // ---- input spikes of (t, b)
    const int nx = s_xcnt[tau];
    const int* xs = xstaged ? xbuf + xpos[tau] : a.x_idx + s_xsrc[tau];
    for (int q = tid; q < nx; q += FWD_NT) {
      const int i = xs[q];
      if ((unsigned)i < (unsigned)a.n_in) atomicOr(&xflags[i >> 5], 1u << (i & 31));
    }
    __syncthreads();

    // ---- propagation: one wave per spiking row, lanes over the row's slots
    unsigned long long ev = 0ull;
    for (int r = wv; r < nx + nz; r += FWD_NT / WAVE) {
      const bool from_in = r < nx;
      const int i = from_in ? xs[r] : zlist[r - nx];
      if (from_in && (unsigned)i >= (unsigned)a.n_in) continue;  // rejected at set_input; never read
      const int* ind = from_in ? a.ind_in : a.ind_rec;
      const float* w = from_in ? a.w_in : a.w_rec;
      const int cap = from_in ? a.cap_in : a.cap_rec;
      const int n = from_in ? len_in[i] : len_rec[i];
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

    // ---- neuron update, traces
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (it >= items) break;
      const int j = it * FWD_NT + tid;
      if (j < a.n_rec) {
        const double I = (double)acc[j] * FIX_INV;
        const double zf = zr[it] ? 1.0 : 0.0;
        vr[it] = a.alpha * (vr[it] - zf * a.v_thr) + I;
        ar[it] = a.rho * ar[it] + zf;
        const int64_t q = ((int64_t)tau * B + b) * a.n_rec + j;
        a.zbar_prev[q] = (float)zbr[it];
        zbr[it] = a.alpha * zbr[it] + zf;
        a.zbar_new[q] = (float)zbr[it];
      }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (it >= xitems) break;
      const int i = it * FWD_NT + tid;
      if (i < a.n_in) {
        const double x = ((xflags[i >> 5] >> (i & 31)) & 1u) ? 1.0 : 0.0;
        a.xbar_prev[((int64_t)tau * B + b) * a.n_in + i] = (float)xbr[it];
        xbr[it] = a.alpha * xbr[it] + x;
      }
    }

    // ---- leaky readout: one wave per output unit over the spike list
    for (int k = wv; k < a.n_out; k += FWD_NT / WAVE) {
      float s = 0.0f;
      const float* wk = wout + (int64_t)k * a.n_rec;
      for (int l = lane; l < nz; l += WAVE) s += wk[zlist[l]];
      s = wave_sum(s);
      if (lane == 0) {
        const double y = a.alpha * yst[k] + (double)s + (double)a.bout[k];
        yst[k] = y;
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
      for (int k = lane; k < a.n_out; k += WAVE) {
        const float d = expf(ylds[k] - m) / den - (k == label ? 1.0f : 0.0f);
        dlds[k] = d;
        a.delta[((int64_t)tau * B + b) * a.n_out + k] = d;
      }
    }
    __syncthreads();

    // ---- learning signal through B = W_out^T
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (it >= items) break;
      const int j = it * FWD_NT + tid;
      if (j < a.n_rec) {
        float l = 0.0f;
        for (int k = 0; k < a.n_out; ++k) l += wout[(int64_t)k * a.n_rec + j] * dlds[k];
        a.L[((int64_t)tau * B + b) * a.n_rec + j] = l;
      }
    }
    __syncthreads();  // LDS (acc, zlist, xflags, dlds) is reused by the next step
  }

  // ---- write back the state and the last step's spikes
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (it >= items) break;
    const int j = it * FWD_NT + tid;
    if (j < a.n_rec) {
      const int64_t m = (int64_t)b * a.n_rec + j;
      a.V[m] = vr[it];
      a.A[m] = ar[it];
      a.zbar[m] = zbr[it];
      a.z[m] = (uint8_t)zr[it];
    }
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (it >= xitems) break;
    const int i = it * FWD_NT + tid;
    if (i < a.n_in) a.xbar[(int64_t)b * a.n_in + i] = xbr[it];
  }
  for (int k = tid; k < a.n_out; k += FWD_NT) a.Y[(int64_t)b * a.n_out + k] = yst[k];
  if (tid == 0) {
    atomicAdd(&a.counters[0], s_events);
    atomicAdd(&a.counters[1], spikes);
  }
}

// Items per thread: neurons (and input channels) handled by each of the
// workgroup's threads, kept in registers across the block of steps.
void launch_fwd(hipStream_t s, const FwdArgs& a_in) {
  // LDS budget: stage W_out and up to 2048 input spikes when they fit
  static int lds_cap = 0;
  if (!lds_cap) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds_cap = 64 * 1024;
    (void)hipGetLastError();
    lds_cap = (lds_cap < 150 * 1024 ? lds_cap : 150 * 1024) - 1024;
  }
  FwdArgs a = a_in;
  a.xcap = 2048;
  a.wout_lds = 1;
  if (fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, 1).total > (size_t)lds_cap) a.wout_lds = 0;
  while (fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds).total > (size_t)lds_cap && a.xcap > 0)
    a.xcap /= 2;
  const size_t sm = fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds).total;
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)k_fwd<1>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<2>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<4>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<8>, 150 * 1024);
    attr_set = true;
  }
  const int need = (max(a.n_rec, a.n_in) + FWD_NT - 1) / FWD_NT;
  if (need <= 1) hipLaunchKernelGGL(k_fwd<1>, dim3(a.B), dim3(FWD_NT), sm, s, a);
  else if (need <= 2) hipLaunchKernelGGL(k_fwd<2>, dim3(a.B), dim3(FWD_NT), sm, s, a);
  else if (need <= 4) hipLaunchKernelGGL(k_fwd<4>, dim3(a.B), dim3(FWD_NT), sm, s, a);
  else hipLaunchKernelGGL(k_fwd<8>, dim3(a.B), dim3(FWD_NT), sm, s, a);
}

// ---------------------------------------------------------------------------
// Eligibility traces and gradients over a block of steps.
// The forward pass does not depend on the traces, so it runs ahead and leaves
// psi, L and the presynaptic traces of every step in a ring of slots; one
// launch then applies `nsteps` steps per synapse while its eps/ebar stay in
// registers: the trace stream crosses HBM once per block instead of once per
// step.  Each step rounds eps/ebar to float and adds its batch sum to G in
// step order, so the result is bit-identical for every block length.
// Wide form (B % 4 == 0, B >= 64): a 256-thread workgroup owns one presynaptic
// row, wave w the slots w, w+4, ...; each lane carries four consecutive batch
// instances, so every access of eps, ebar, psi, L and the presynaptic trace is
// a contiguous 1 KB wave access.
constexpr int EP_NT = 256;
constexpr int EP_WAVES = EP_NT / WAVE;

// One eligibility step for the four instances a lane holds (eq. eprop_elig_1/2,
// eprop_elig_lif); returns the lane's part of sum_b L ebar.  The eps update
// eps' = psi p + (rho - psi beta) eps is evaluated as
// eps + (psi p - ((1 - rho) + psi beta) eps): rho is within 5e-4 of one, and a
// float rho would shift its 2000-step decay by a systematic 3e-8 per step,
// whereas 1 - rho in float is accurate to 3e-8 of itself.
template <bool ALIF>
__device__ __forceinline__ float trace_step(const EpropArgs& a, f4 psi, f4 L, f4 p, f4& eb, f4& ep) {
  f4 e;
  if (ALIF) {
    e = psi * (p - a.beta * ep);
    const f4 k = psi * a.beta + a.one_m_rho;
    ep = ep + (psi * p - k * ep);
  } else {
    e = psi * p;
  }
  eb = a.alpha * eb + e;
  return (L.x * eb.x + L.y * eb.y) + (L.z * eb.z + L.w * eb.w);
}

__device__ __forceinline__ int64_t ring(const EpropArgs& a, int n, int tau) {
  return ((int64_t)n * a.nslot + a.slot0 + tau) * a.B;
}

__device__ __forceinline__ void readout_grad_wave(const EpropArgs& a, int j, int lane) {
  const int nb4 = a.B / 4;
  for (int tau = 0; tau < a.nsteps; ++tau) {
    if (j < a.n_rec) {
      for (int k = 0; k < a.n_out; ++k) {
        float g = 0.0f;
        for (int c = lane; c < nb4; c += WAVE) {
          const f4 z = *(const f4*)&a.zbar_new[ring(a, j, tau) + 4 * c];
          const f4 d = *(const f4*)&a.deltaT[ring(a, k, tau) + 4 * c];
          g += (d.x * z.x + d.y * z.y) + (d.z * z.z + d.w * z.w);
        }
        g = wave_sum(g);
        if (lane == 0) a.Gout[(int64_t)k * a.n_rec + j] += g;
      }
    } else if (j == a.n_rec) {
      for (int k = 0; k < a.n_out; ++k) {
        float g = 0.0f;
        for (int c = lane; c < nb4; c += WAVE) {
          const f4 d = *(const f4*)&a.deltaT[ring(a, k, tau) + 4 * c];
          g += (d.x + d.y) + (d.z + d.w);
        }
        g = wave_sum(g);
        if (lane == 0) a.Gb[k] += g;
      }
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
  const int B = a.B, nb4 = B / 4, T = a.nsteps;
  const int64_t base = (int64_t)i * cap;
  const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
  if (nb4 <= WAVE) {
    // lane q of wave wv holds the target index and gradient of slot
    // wv + 4(c0 + q); synapses go two at a time, every load issued up front
    const bool act = lane < nb4;
    const int lo = 4 * lane;
    for (int c0 = 0; wv + 4 * c0 < n; c0 += WAVE) {
      const int kl = wv + 4 * (c0 + lane);
      const bool own = kl < n;
      const int my_j = own ? ind[base + kl] : 0;
      float my_g = own ? G[base + kl] : 0.0f;
      const int cnt = min(WAVE, (n - wv - 4 * c0 + 3) / 4);
      for (int q = 0; q < cnt; q += 2) {
        const bool two = q + 1 < cnt;
        const int j0 = __builtin_amdgcn_readlane(my_j, q);
        const int j1 = two ? __builtin_amdgcn_readlane(my_j, q + 1) : j0;
        const int64_t s0 = base + wv + 4 * (c0 + q), s1 = two ? s0 + 4 : s0;
        f4 eb0 = zero4, eb1 = zero4, ep0 = zero4, ep1 = zero4;
        if (act) {
          eb0 = __builtin_nontemporal_load((const f4*)&ebar[s0 * B + lo]);
          if (two) eb1 = __builtin_nontemporal_load((const f4*)&ebar[s1 * B + lo]);
          if (ALIF) {
            ep0 = __builtin_nontemporal_load((const f4*)&eps[s0 * B + lo]);
            if (two) ep1 = __builtin_nontemporal_load((const f4*)&eps[s1 * B + lo]);
          }
        }
        for (int tau = 0; tau < T; ++tau) {
          float g0 = 0.f, g1 = 0.f;
          if (act) {
            const f4 p = *(const f4*)&pre[ring(a, i, tau) + lo];
            const f4 psi0 = *(const f4*)&a.psiT[ring(a, j0, tau) + lo];
            const f4 L0 = *(const f4*)&a.LT[ring(a, j0, tau) + lo];
            const f4 psi1 = *(const f4*)&a.psiT[ring(a, j1, tau) + lo];
            const f4 L1 = *(const f4*)&a.LT[ring(a, j1, tau) + lo];
            g0 = trace_step<ALIF>(a, psi0, L0, p, eb0, ep0);
            g1 = trace_step<ALIF>(a, psi1, L1, p, eb1, ep1);
          }
          g0 = wave_sum(g0);
          g1 = wave_sum(g1);
          if (lane == q) my_g += g0;
          if (two && lane == q + 1) my_g += g1;
        }
        if (act) {
          __builtin_nontemporal_store(eb0, (f4*)&ebar[s0 * B + lo]);
          if (ALIF) __builtin_nontemporal_store(ep0, (f4*)&eps[s0 * B + lo]);
          if (two) {
            __builtin_nontemporal_store(eb1, (f4*)&ebar[s1 * B + lo]);
            if (ALIF) __builtin_nontemporal_store(ep1, (f4*)&eps[s1 * B + lo]);
          }
        }
      }
      if (own) G[base + kl] = my_g;
    }
  } else {
    // more than 256 instances: lanes loop over 256-instance chunks
    for (int k = wv; k < n; k += EP_WAVES) {
      const int64_t s = base + k;
      const int j = ind[s];
      float gsum = G[s];
      float gstep[32];
      for (int tau = 0; tau < T; ++tau) gstep[tau] = 0.0f;
      for (int c = lane; c < nb4; c += WAVE) {
        f4 eb = __builtin_nontemporal_load((const f4*)&ebar[s * B + 4 * c]);
        f4 ep = ALIF ? __builtin_nontemporal_load((const f4*)&eps[s * B + 4 * c]) : zero4;
        for (int tau = 0; tau < T; ++tau) {
          const f4 p = *(const f4*)&pre[ring(a, i, tau) + 4 * c];
          const f4 psi = *(const f4*)&a.psiT[ring(a, j, tau) + 4 * c];
          const f4 L = *(const f4*)&a.LT[ring(a, j, tau) + 4 * c];
          gstep[tau] += trace_step<ALIF>(a, psi, L, p, eb, ep);
        }
        __builtin_nontemporal_store(eb, (f4*)&ebar[s * B + 4 * c]);
        if (ALIF) __builtin_nontemporal_store(ep, (f4*)&eps[s * B + 4 * c]);
      }
      for (int tau = 0; tau < T; ++tau) gsum += wave_sum(gstep[tau]);
      if (lane == 0) G[s] = gsum;
    }
  }
}

// Hand-off transpose: [tau][B][n] -> [n][nslot][B] through a 64 x 64 LDS tile
// (both sides coalesced).  blockIdx.z = array * nsteps + tau.
__global__ void __launch_bounds__(256) k_handoff_transpose(HandoffArrays h, int B, int nsteps, int slot0,
                                                           int nslot) {
  __shared__ float tile[64][65];
  const int arr = blockIdx.z / nsteps, tau = blockIdx.z % nsteps;
  const int n = h.n[arr];
  const int n0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
  if (n0 >= n || b0 >= B) return;
  const float* src = h.src[arr] + (int64_t)tau * B * n;
  float* dst = h.dst[arr];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const int b = b0 + r, j = n0 + tx;
    tile[r][tx] = (b < B && j < n) ? src[(int64_t)b * n + j] : 0.0f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = n0 + r, b = b0 + tx;
    if (j < n && b < B) dst[((int64_t)j * nslot + slot0 + tau) * B + b] = tile[tx][r];
  }
}

void launch_handoff_transpose(hipStream_t s, const HandoffArrays& h, int B, int nsteps, int slot0, int nslot) {
  int nmax = 0;
  for (int q = 0; q < 6; ++q) nmax = max(nmax, h.n[q]);
  dim3 grid((nmax + 63) / 64, (B + 63) / 64, 6 * nsteps);
  hipLaunchKernelGGL(k_handoff_transpose, grid, dim3(256), 0, s, h, B, nsteps, slot0, nslot);
}

// XCD-aware form (B % 4 == 0, 64 <= B <= 256): workgroup w = row*8 + o takes
// the row's synapses whose target lies in octant o.  Workgroups are handed to
// the 8 XCDs round-robin, so each XCD's L2 only ever holds psi and L of its own
// eighth of the targets.  One wave per workgroup; same arithmetic and order as
// the row form.
template <bool ALIF>
__global__ void __launch_bounds__(WAVE) k_eprop_oct(EpropArgs a) {
  const int lane = lane_id();
  const int n_rows = a.n_in + a.n_rec;
  const int wg = blockIdx.x;
  if (wg >= n_rows * 8) {
    readout_grad_wave(a, wg - n_rows * 8, lane);
    return;
  }
  const int row = wg >> 3, oct = wg & 7;
  const bool from_in = row < a.n_in;
  const ProjDev& P = from_in ? a.in : a.rec;
  const int i = from_in ? row : row - a.n_in;
  const int cap = P.cap;
  const int q0 = P.oct_off[i * 9 + oct], q1 = P.oct_off[i * 9 + oct + 1];
  if (q1 <= q0) return;
  const int* __restrict__ ind = P.ind;
  const int* __restrict__ perm = P.perm;
  float* __restrict__ G = P.G;
  float* __restrict__ eps = P.eps;
  float* __restrict__ ebar = P.ebar;
  const int B = a.B, nb4 = B / 4, T = a.nsteps;
  const int64_t base = (int64_t)i * cap;
  const bool act = lane < nb4;
  const int lo = act ? 4 * lane : 0;  // inactive lanes read instance 0, never store
  const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
  const float* __restrict__ pre = (from_in ? a.xbar_prev : a.zbar_prev) + ring(a, i, 0) + lo;
  for (int c0 = q0; c0 < q1; c0 += WAVE) {
    const bool own = c0 + lane < q1;
    const int my_s = own ? perm[base + c0 + lane] : 0;
    const int my_j = own ? ind[base + my_s] : 0;
    float my_g = own ? G[base + my_s] : 0.0f;
    const int cnt = min(WAVE, q1 - c0);
    for (int q = 0; q < cnt; q += 2) {
      const bool two = q + 1 < cnt;
      const int j0 = __builtin_amdgcn_readlane(my_j, q);
      const int j1 = two ? __builtin_amdgcn_readlane(my_j, q + 1) : j0;
      const int64_t s0 = base + __builtin_amdgcn_readlane(my_s, q);
      const int64_t s1 = two ? base + __builtin_amdgcn_readlane(my_s, q + 1) : s0;
      const float* __restrict__ psi0p = a.psiT + ring(a, j0, 0) + lo;
      const float* __restrict__ L0p = a.LT + ring(a, j0, 0) + lo;
      const float* __restrict__ psi1p = a.psiT + ring(a, j1, 0) + lo;
      const float* __restrict__ L1p = a.LT + ring(a, j1, 0) + lo;
      f4 eb0 = __builtin_nontemporal_load((const f4*)&ebar[s0 * B + lo]);
      f4 eb1 = __builtin_nontemporal_load((const f4*)&ebar[s1 * B + lo]);
      f4 ep0 = zero4, ep1 = zero4;
      if (ALIF) {
        ep0 = __builtin_nontemporal_load((const f4*)&eps[s0 * B + lo]);
        ep1 = __builtin_nontemporal_load((const f4*)&eps[s1 * B + lo]);
      }
      // software pipeline over the block's steps: step tau+1's inputs are in
      // flight while step tau is computed
      f4 p = *(const f4*)pre, psi0 = *(const f4*)psi0p, L0 = *(const f4*)L0p;
      f4 psi1 = *(const f4*)psi1p, L1 = *(const f4*)L1p;
      for (int tau = 0; tau < T; ++tau) {
        const int nx = (tau + 1 < T ? tau + 1 : tau) * B;
        const f4 pn = *(const f4*)(pre + nx), psi0n = *(const f4*)(psi0p + nx), L0n = *(const f4*)(L0p + nx);
        const f4 psi1n = *(const f4*)(psi1p + nx), L1n = *(const f4*)(L1p + nx);
        float g0 = trace_step<ALIF>(a, psi0, L0, p, eb0, ep0);
        float g1 = trace_step<ALIF>(a, psi1, L1, p, eb1, ep1);
        if (!act) { g0 = 0.f; g1 = 0.f; }
        g0 = wave_sum(g0);
        g1 = wave_sum(g1);
        if (lane == q) my_g += g0;
        if (two && lane == q + 1) my_g += g1;
        p = pn; psi0 = psi0n; L0 = L0n; psi1 = psi1n; L1 = L1n;
      }
      if (act) {
        __builtin_nontemporal_store(eb0, (f4*)&ebar[s0 * B + lo]);
        if (ALIF) __builtin_nontemporal_store(ep0, (f4*)&eps[s0 * B + lo]);
        if (two) {
          __builtin_nontemporal_store(eb1, (f4*)&ebar[s1 * B + lo]);
          if (ALIF) __builtin_nontemporal_store(ep1, (f4*)&eps[s1 * B + lo]);
        }
      }
    }
    if (own) G[base + my_s] = my_g;
  }
}

// Octant permutation of every row: one wave per row, stable counting sort of
// the row's slots by target octant.
__global__ void __launch_bounds__(WAVE) k_octant_perm(ProjDev P) {
  __shared__ int cnt[9];
  const int i = blockIdx.x, lane = lane_id();
  const int n = P.len[i];
  const int64_t base = (int64_t)i * P.cap;
  if (lane < 9) cnt[lane] = 0;
  __syncthreads();
  int run[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // per-octant running offset (uniform)
  // first pass: octant sizes
  for (int c = 0; c < n; c += WAVE) {
    const int k = c + lane;
    const int o = k < n ? min(P.ind[base + k] / P.oct_size, 7) : 8;
#pragma unroll
    for (int b = 0; b < 8; ++b) run[b] += __popcll(ballot(o == b));
  }
  int off[9];
  off[0] = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) off[b + 1] = off[b] + run[b];
  if (lane < 9) P.oct_off[i * 9 + lane] = off[lane];
  // second pass: stable placement
#pragma unroll
  for (int b = 0; b < 8; ++b) run[b] = off[b];
  for (int c = 0; c < n; c += WAVE) {
    const int k = c + lane;
    const int o = k < n ? min(P.ind[base + k] / P.oct_size, 7) : 8;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = ballot(o == b);
      if (o == b) P.perm[base + run[b] + __popcll(m & lanemask_lt())] = k;
      run[b] += __popcll(m);
    }
  }
}

void launch_octant_perm(hipStream_t s, const ProjDev& P) {
  if (!P.perm) return;
  hipLaunchKernelGGL(k_octant_perm, dim3(P.n_pre), dim3(WAVE), 0, s, P);
}

// Narrow form (any B): threads over a row's synapses, each looping over steps
// and instances; used for small batches such as single-instance learning.
template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_narrow(EpropArgs a) {
  const int row = blockIdx.x, tid = threadIdx.x;
  const int n_rows = a.n_in + a.n_rec;
  const int B = a.B;
  if (row >= n_rows) {
    const int j = (row - n_rows) * EP_NT + tid;
    for (int tau = 0; tau < a.nsteps; ++tau) {
      if (j < a.n_rec) {
        for (int k = 0; k < a.n_out; ++k) {
          float g = 0.0f;
          for (int b = 0; b < B; ++b) g += a.deltaT[ring(a, k, tau) + b] * a.zbar_new[ring(a, j, tau) + b];
          a.Gout[(int64_t)k * a.n_rec + j] += g;
        }
      } else if (j == a.n_rec) {
        for (int k = 0; k < a.n_out; ++k) {
          float g = 0.0f;
          for (int b = 0; b < B; ++b) g += a.deltaT[ring(a, k, tau) + b];
          a.Gb[k] += g;
        }
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
    float gsum = G[s];
    for (int tau = 0; tau < a.nsteps; ++tau) {
      float g = 0.0f;
      for (int b = 0; b < B; ++b) {
        const float p = pre[ring(a, i, tau) + b];
        const float psi = a.psiT[ring(a, j, tau) + b];
        float e;
        if (ALIF) {
          const float ep = eps[s * B + b];
          e = psi * (p - a.beta * ep);
          const float k = psi * a.beta + a.one_m_rho;
          eps[s * B + b] = ep + (psi * p - k * ep);
        } else {
          e = psi * p;
        }
        const float eb = a.alpha * ebar[s * B + b] + e;
        ebar[s * B + b] = eb;
        g += a.LT[ring(a, j, tau) + b] * eb;
      }
      gsum += g;
    }
    G[s] = gsum;
  }
}

void launch_eprop(hipStream_t s, const EpropArgs& a) {
  const int n_rows = a.n_in + a.n_rec;
  if (a.nsteps <= 0) return;
  if (a.B % 4 == 0 && a.B >= 64 && a.B <= 256 && a.in.perm && a.rec.perm) {
    const int blocks = n_rows * 8 + a.n_rec + 1;
    if (a.alif) hipLaunchKernelGGL(k_eprop_oct<true>, dim3(blocks), dim3(WAVE), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_oct<false>, dim3(blocks), dim3(WAVE), 0, s, a);
  } else if (a.B % 4 == 0 && a.B >= 64) {
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
