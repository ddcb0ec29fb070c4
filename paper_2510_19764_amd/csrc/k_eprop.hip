// Per-timestep kernels of the e-prop classifier (paper, recurrent classifier
// section; eligibility traces eq. eprop_elig_1/2 and eprop_elig_lif).
//
// k_fwd: one workgroup per batch instance b runs a block of steps.  Spikes and
//   surrogate derivatives from the state at the start of the step, ordered
//   spike compaction with ballots, propagation of input and recurrent spikes
//   through the ragged rows (one wave per spiking row, lanes over its slots,
//   accumulation into LDS), neuron update with subtractive reset, presynaptic
//   traces F <- fma(alpha, F, spike) in float, and the readout drive
//   u_k = sum_j W_out[k][j] z_j of the step.  Per block it hands over psi of
//   every step, the traces at the block start and the block's spike bits.
//   Input currents are accumulated as 64-bit fixed point (2^-36 resolution) so
//   the sum does not depend on the order of the LDS atomics.
// k_readout / k_learning_signal: leaky readout, softmax error and learning
//   signal L_j = sum_k W_out[k][j] delta_k for the whole block, off the
//   forward kernel's sequential path.
// k_eprop_*: per-synapse eligibility traces over every batch instance and the
//   batch-summed gradient G_ji += sum_b L_j ebar_ji; further workgroups
//   accumulate the readout delta rule.  State is laid out batch-innermost
//   ([slot][B], [neuron][B]) so a wave reads consecutive instances.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int FWD_NT = 1024;
constexpr int FWD_MAX_ITEMS = 8;  // n_rec <= FWD_NT * FWD_MAX_ITEMS

// Ordered position of a flagged thread among the workgroup's flagged threads,
// and their total.  s_wave alternates between two buffers on consecutive calls
// so that no trailing barrier is needed: a buffer is written again only after
// the intervening call's barrier.
__device__ __forceinline__ int block_scan_flag_fwd(bool f, int* s_wave, int* total) {
  uint64_t m = ballot(f);
  int lane = lane_id(), w = wave_id();
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
  *total = tot;
  return base + pre;
}

// LDS layout of k_fwd (offsets 16-byte aligned):
//   acc      int64[n_rec]        fixed-point input current of the step
//   zlist    int[n_rec]          ordered spike list of the step
//   len_in   int[n_in], len_rec int[n_rec]   row lengths, staged per launch
//   xflags   u32[2][ceil(n_in/32)] input spikes of the step as bits, by step parity
//   xpos     int[33]             start of each step's input list in xbuf
//   xbuf     int[xcap]           the launch's input spike lists
//   wout     float[n_out*n_rec]  readout weights (when wout_lds)
struct FwdLds {
  size_t acc, zlist, len_in, len_rec, xflags, xpos, xbuf, wout, total;
};
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline FwdLds fwd_lds_layout(int n_in, int n_rec, int n_out, int xcap, int wout_lds) {
  FwdLds L;
  size_t o = 0;
  L.acc = o; o = align16(o + (size_t)n_rec * 8);
  L.zlist = o; o = align16(o + (size_t)n_rec * 4);
  L.len_in = o; o = align16(o + (size_t)n_in * 4);
  L.len_rec = o; o = align16(o + (size_t)n_rec * 4);
  L.xflags = o; o = align16(o + (size_t)((n_in + 31) / 32) * 8);
  L.xpos = o; o = align16(o + 33 * 4);
  L.xbuf = o; o = align16(o + (size_t)xcap * 4);
  L.wout = o; o = align16(o + (wout_lds ? (size_t)n_out * n_rec * 4 : 0));
  L.total = o;
  return L;
}

constexpr int PROP_U = 4;  // slots per lane loaded ahead of the LDS atomics

template <int ITEMS>
__global__ void __launch_bounds__(FWD_NT) k_fwd(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const FwdLds lay = fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds);
  long long* acc = (long long*)(smem + lay.acc);
  int* zlist = (int*)(smem + lay.zlist);
  int* len_in = (int*)(smem + lay.len_in);
  int* len_rec = (int*)(smem + lay.len_rec);
  uint32_t* xflags2 = (uint32_t*)(smem + lay.xflags);
  int* xpos = (int*)(smem + lay.xpos);
  int* xbuf = (int*)(smem + lay.xbuf);
  const float* wout = a.wout_lds ? (const float*)(smem + lay.wout) : a.Wout;
  const int xwords = (a.n_in + 31) >> 5;
  __shared__ int s_wave[2][FWD_NT / WAVE];
  __shared__ unsigned long long s_events;
  __shared__ int s_xsrc[33], s_xcnt[33];
  __shared__ int s_xstaged;

  const int b = blockIdx.x, tid = threadIdx.x, B = a.B;
  const int lane = lane_id(), wv = wave_id();
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
  const int* xsrc_base;  // the step lists: the caller's raster, or drawn below
  if (a.x_thr) {
    // Poisson source: one Bernoulli draw per (step, channel) of the block,
    // spread over the workgroup; spikes are appended to each step's list in
    // arrival order (the propagation sums are order-independent)
    xsrc_base = a.x_list;
    if (tid < 33) s_xcnt[tid] = 0;
    __syncthreads();
    const uint64_t* thr = a.x_thr + (int64_t)b * a.x_thr_stride;
    const int total = a.nsteps * a.n_in;
    for (int q = tid; q < total; q += FWD_NT) {
      const int tau = q / a.n_in, i = q - tau * a.n_in;
      const uint32_t u = draw_u32(a.seed, TAG_INPUT, 0, a.step0 + (uint64_t)tau, (uint64_t)b, (uint64_t)i, 0);
      if ((uint64_t)u < thr[i]) {
        const int pos = atomicAdd(&s_xcnt[tau], 1);
        a.x_list[((int64_t)tau * B + b) * a.n_in + pos] = i;
      }
    }
    if (tid < a.nsteps) s_xsrc[tid] = (tid * B + b) * a.n_in;
  } else {
    xsrc_base = a.x_idx;
    if (tid <= a.nsteps) {
      const int tau = tid < a.nsteps ? tid : a.nsteps - 1;
      const int xq = ((a.t0 + tau) % a.sample_steps) * B + b;
      // clamp the caller's offsets into the index array
      const long long lo = min(max((long long)a.x_off[xq], 0ll), a.n_idx);
      const long long hi = min(max((long long)a.x_off[xq + 1], lo), a.n_idx);
      s_xsrc[tid] = tid < a.nsteps ? (int)lo : 0;
      s_xcnt[tid] = tid < a.nsteps ? (int)(hi - lo) : 0;
    }
  }
  for (int q = tid; q < 2 * xwords; q += FWD_NT) xflags2[q] = 0u;
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
      for (int l = lane; l < n; l += WAVE) xbuf[xpos[t] + l] = xsrc_base[s_xsrc[t] + l];
    }
  }

  // neuron and trace state of this instance stays on chip for the block; the
  // traces at the block start and the block's spike bits go to the e-prop
  // hand-off, which rebuilds every step's traces from them
  double vr[ITEMS], ar[ITEMS];
  float zbr[ITEMS], xbr[ITEMS];
  uint32_t zbits[ITEMS], xbits[ITEMS];
  bool zr[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int j = it * FWD_NT + tid;
    const bool ok = it < items && j < a.n_rec;
    vr[it] = ok ? a.V[(int64_t)b * a.n_rec + j] : 0.0;
    ar[it] = ok ? a.A[(int64_t)b * a.n_rec + j] : 0.0;
    zbr[it] = ok ? a.zbar[(int64_t)b * a.n_rec + j] : 0.0f;
    if (ok) a.z0[(int64_t)b * a.n_rec + j] = zbr[it];
    const int i = it * FWD_NT + tid;
    const bool oki = it < xitems && i < a.n_in;
    xbr[it] = oki ? a.xbar[(int64_t)b * a.n_in + i] : 0.0f;
    if (oki) a.x0[(int64_t)b * a.n_in + i] = xbr[it];
    zr[it] = false;
    zbits[it] = 0u;
    xbits[it] = 0u;
  }
  if (tid == 0) s_events = 0ull;
  unsigned long long spikes = 0ull;
  int scan_buf = 0;
  __syncthreads();

  // Barriers per step: the scan's, one before propagation and one before the
  // neuron update.  Nothing needs one at the end of a step: each thread
  // clears only the acc entries it read itself, the input bits alternate
  // between two buffers (a buffer is cleared after the next scan's barrier),
  // and zlist is rewritten only after the next scan's barrier.
  for (int tau = 0; tau < a.nsteps; ++tau) {
    uint32_t* xflags = xflags2 + (tau & 1) * xwords;
    // ---- spikes, surrogate derivative, ordered compaction of the spike list
    int nz = 0;
    const int nx = s_xcnt[tau];
    const int* xs = xstaged ? xbuf + xpos[tau] : xsrc_base + s_xsrc[tau];
    // input spikes of (t, b) as bits, published by the scan's barrier
    for (int q = tid; q < nx; q += FWD_NT) {
      const int i = xs[q];
      if ((unsigned)i < (unsigned)a.n_in) atomicOr(&xflags[i >> 5], 1u << (i & 31));
    }
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
      const int off = block_scan_flag_fwd(z, s_wave[scan_buf], &tot);
      scan_buf ^= 1;
      if (z) zlist[nz + off] = j;
      nz += tot;
    }
    spikes += (unsigned long long)nz;
    __syncthreads();  // zlist, acc and xflags complete
    // the other parity's bits were last read in the previous step's update,
    // before this step's scan barrier, and are next set after this step's
    // update barrier
    for (int q = tid; q < xwords; q += FWD_NT) xflags2[((tau + 1) & 1) * xwords + q] = 0u;

    // ---- propagation: one wave per spiking row, lanes over the row's slots;
    // up to PROP_U slots per lane are loaded before any LDS atomic, so a row
    // of up to 256 slots costs one memory latency
    unsigned long long ev = 0ull;
    for (int r = wv; r < nx + nz; r += FWD_NT / WAVE) {
      const bool from_in = r < nx;
      const int i = from_in ? xs[r] : zlist[r - nx];
      if (from_in && (unsigned)i >= (unsigned)a.n_in) continue;  // out-of-range channel: ignored
      const int* ind = from_in ? a.ind_in : a.ind_rec;
      const float* w = from_in ? a.w_in : a.w_rec;
      const int cap = from_in ? a.cap_in : a.cap_rec;
      const int n = from_in ? len_in[i] : len_rec[i];
      const int64_t base = (int64_t)i * cap;
      ev += (unsigned long long)n;
      for (int c0 = 0; c0 < n; c0 += PROP_U * WAVE) {
        int jj[PROP_U];
        float ww[PROP_U];
#pragma unroll
        for (int u = 0; u < PROP_U; ++u) {
          const int k = c0 + u * WAVE + lane;
          jj[u] = k < n ? ind[base + k] : -1;
          ww[u] = k < n ? w[base + k] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < PROP_U; ++u)
          if (jj[u] >= 0)
            atomicAdd((unsigned long long*)&acc[jj[u]], (unsigned long long)__double2ll_rn((double)ww[u] * FIX_SCALE));
      }
    }
    if (lane == 0 && ev) atomicAdd(&s_events, ev);

    // ---- readout drive u_k = sum_j W_out[k][j] z_j: one wave per output unit
    for (int k = wv; k < a.n_out; k += FWD_NT / WAVE) {
      float s = 0.0f;
      const float* wk = wout + (int64_t)k * a.n_rec;
      for (int l = lane; l < nz; l += WAVE) s += wk[zlist[l]];
      s = wave_sum(s);
      if (lane == 0) a.u[((int64_t)tau * B + b) * a.n_out + k] = s;
    }
    __syncthreads();  // acc complete

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
        zbr[it] = fmaf(a.alpha_f, zbr[it], zr[it] ? 1.0f : 0.0f);
        zbits[it] |= (zr[it] ? 1u : 0u) << tau;
      }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (it >= xitems) break;
      const int i = it * FWD_NT + tid;
      if (i < a.n_in) {
        const uint32_t x = (xflags[i >> 5] >> (i & 31)) & 1u;
        xbr[it] = fmaf(a.alpha_f, xbr[it], (float)x);
        xbits[it] |= x << tau;
      }
    }
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
      a.zbits[m] = zbits[it];
      a.zcount[m] += (uint32_t)__popc(zbits[it]);
    }
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (it >= xitems) break;
    const int i = it * FWD_NT + tid;
    if (i < a.n_in) {
      a.xbar[(int64_t)b * a.n_in + i] = xbr[it];
      a.xbits[(int64_t)b * a.n_in + i] = xbits[it];
    }
  }
  __syncthreads();
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

// Leaky readout and softmax error over a block (recurrent classifier
// section): one wave per instance b, lane k (and k + 64, ...) carrying output
// k through the block's steps,
//   y_k <- alpha y_k + u_k + b_k   (double),   delta_k = softmax(y)_k - [k == label_b],
// with the softmax maximum and denominator reduced across the wave.  delta
// goes into the ring [k][slot][b].  Labels outside 0..n_out-1 contribute no
// target term.
constexpr int RO_KMAX = 4;  // n_out <= 4 * WAVE
__global__ void __launch_bounds__(256) k_readout(ReadoutArgs a) {
  const int b = blockIdx.x * 4 + wave_id(), lane = lane_id();
  if (b >= a.B) return;
  const int label = a.labels[b];
  double y[RO_KMAX];
  float bias[RO_KMAX];
#pragma unroll
  for (int q = 0; q < RO_KMAX; ++q) {
    const int k = q * WAVE + lane;
    y[q] = k < a.n_out ? a.Y[(int64_t)b * a.n_out + k] : 0.0;
    bias[q] = k < a.n_out ? a.bout[k] : 0.0f;
  }
  for (int tau = 0; tau < a.nsteps; ++tau) {
    const float* u = a.u + ((int64_t)tau * a.B + b) * a.n_out;
    float m = -INFINITY;
#pragma unroll
    for (int q = 0; q < RO_KMAX; ++q) {
      const int k = q * WAVE + lane;
      if (k < a.n_out) {
        y[q] = a.alpha * y[q] + (double)u[k] + (double)bias[q];
        m = fmaxf(m, (float)y[q]);
      }
    }
    m = wave_max(m);
    float den = 0.0f;
#pragma unroll
    for (int q = 0; q < RO_KMAX; ++q)
      if (q * WAVE + lane < a.n_out) den += expf((float)y[q] - m);
    den = wave_sum(den);
#pragma unroll
    for (int q = 0; q < RO_KMAX; ++q) {
      const int k = q * WAVE + lane;
      if (k < a.n_out) {
        const float d = expf((float)y[q] - m) / den - (k == label ? 1.0f : 0.0f);
        a.deltaT[((int64_t)k * a.nslot + a.slot0 + tau) * a.B + b] = d;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RO_KMAX; ++q) {
    const int k = q * WAVE + lane;
    if (k < a.n_out) a.Y[(int64_t)b * a.n_out + k] = y[q];
  }
}

// Learning signal L_j = sum_k W_out[k][j] delta_k (recurrent classifier
// section), written straight into the ring [j][slot][b]: lanes over
// instances, each thread 16 consecutive neurons of a 64-neuron tile whose
// readout weights are staged in LDS.  blockIdx = (neuron tile, instance tile,
// step).
__global__ void __launch_bounds__(256) k_learning_signal(ReadoutArgs a) {
  __shared__ float w[64][65];  // [k in chunk][j in tile]
  const int j0 = blockIdx.x * 64, b = blockIdx.y * 64 + lane_id(), tau = blockIdx.z;
  const int jq = wave_id() * 16;  // this wave's 16 neurons of the tile
  const bool act = b < a.B;
  float acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
  for (int k0 = 0; k0 < a.n_out; k0 += 64) {
    const int kn = min(64, a.n_out - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int kk = e / 64, jj = e % 64;
      w[kk][jj] = (kk < kn && j0 + jj < a.n_rec) ? a.Wout[(int64_t)(k0 + kk) * a.n_rec + j0 + jj] : 0.0f;
    }
    __syncthreads();
    for (int kk = 0; kk < kn; ++kk) {
      const float d = act ? a.deltaT[((int64_t)(k0 + kk) * a.nslot + a.slot0 + tau) * a.B + b] : 0.0f;
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = fmaf(w[kk][jq + q], d, acc[q]);
    }
  }
  if (!act) return;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = j0 + jq + q;
    if (j < a.n_rec) a.LT[((int64_t)j * a.nslot + a.slot0 + tau) * a.B + b] = acc[q];
  }
}

void launch_readout(hipStream_t s, const ReadoutArgs& a, bool learning_signal) {
  if (a.nsteps <= 0) return;
  hipLaunchKernelGGL(k_readout, dim3((a.B + 3) / 4), dim3(256), 0, s, a);
  if (learning_signal)
    hipLaunchKernelGGL(k_learning_signal, dim3((a.n_rec + 63) / 64, (a.B + 63) / 64, a.nsteps), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// Eligibility traces and gradients over a block of steps.
// The forward pass does not depend on the traces, so it runs ahead and leaves
// psi, L and the presynaptic traces of every step in a ring of slots; one
// launch then applies up to COL_TB steps per synapse while its eps/ebar stay in
// registers: the trace stream crosses HBM once per block instead of once per
// step.  Each step rounds eps/ebar to float, so they are bit-identical for
// every block length; the gradient is summed over the block's steps per lane
// before the batch reduction, so G depends on the block length only through
// float rounding.
constexpr int EP_NT = 256;
// Steps per launch of the target-major kernel.  20 divides the usual update
// intervals (100 steps), so no block ends in a short tail launch; psi and L of
// 20 steps take 40 KB of LDS, four workgroups per CU.
constexpr int COL_TB = 20;
constexpr int COL_OCT = 8;  // source octants, one per XCD

__device__ __forceinline__ int64_t ring(const EpropArgs& a, int n, int tau) {
  return ((int64_t)n * a.nslot + a.slot0 + tau) * a.B;
}

// Raw buffer access: a 128-bit resource (base, byte size) in scalar registers
// plus a 32-bit per-lane byte offset and a uniform byte offset, so a load
// costs no vector address arithmetic.  Offsets at or past the size read zero
// and drop stores; every offset used here is in range by construction.
constexpr int BUF_FLAGS = 0x00020000;  // 32-bit data format (gfx9 family)
constexpr int BUF_NT = 2;              // non-temporal
// The base and size are wave-uniform; readfirstlane states it to the compiler.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  const uint64_t v = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  void* u = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, 0, (int)__builtin_amdgcn_readfirstlane(bytes), BUF_FLAGS);
}
template <int AUX = 0>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, 0, AUX);
}
typedef unsigned v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 buf_ld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
template <int AUX>
__device__ __forceinline__ f4 buf_ld4x(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ void buf_st4(f4 v, __amdgpu_buffer_rsrc_t r, uint32_t voff) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, v), r, (int)voff, 0, AUX);
}


// Vectors of IPL consecutive instances (2 or 4) held by one lane.
template <int IPL> struct VecT;
template <> struct VecT<2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecT<4> { typedef float type __attribute__((ext_vector_type(4))); };

template <int IPL>
__device__ __forceinline__ typename VecT<IPL>::type buf_ldv(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  typedef typename VecT<IPL>::type V;
  if constexpr (IPL == 4)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <int IPL>
__device__ __forceinline__ typename VecT<IPL>::type buf_ldv_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  typedef typename VecT<IPL>::type V;
  if constexpr (IPL == 4)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, BUF_NT));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, BUF_NT));
}
template <int IPL>
__device__ __forceinline__ void buf_stv_nt(typename VecT<IPL>::type v, __amdgpu_buffer_rsrc_t r, uint32_t voff) {
  typedef unsigned U __attribute__((ext_vector_type(IPL)));
  if constexpr (IPL == 4)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, (int)voff, 0, BUF_NT);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, (int)voff, 0, BUF_NT);
}
// One step of a presynaptic trace for each of a lane's instances:
// F <- fma(alpha, F, spike t), the forward pass's own float recursion.
template <int IPL>
__device__ __forceinline__ typename VecT<IPL>::type trace_next(
    typename VecT<IPL>::type f, float alpha, unsigned __attribute__((ext_vector_type(IPL))) w, int t) {
#pragma unroll
  for (int e = 0; e < IPL; ++e) f[e] = fmaf(alpha, f[e], (float)((w[e] >> t) & 1u));
  return f;
}

template <int IPL>
__device__ __forceinline__ float hsum(typename VecT<IPL>::type v) {
  if constexpr (IPL == 4) return (v.x + v.y) + (v.z + v.w);
  else return v.x + v.y;
}

// Readout delta rule over the launch's steps (recurrent classifier section):
// wave j < n_rec adds sum_t sum_b delta_k z_j to Gout[k][j] for every output
// k, where z_j after step t is rebuilt from the block's start trace and spike
// bits; wave n_rec adds the bias gradient sum_t sum_b delta_k.  Steps are read
// four at a time with independent loads.
__device__ __forceinline__ void readout_grad(const EpropArgs& a, int j, int lane) {
  if (j > a.n_rec) return;
  const int B = a.B, T = a.nsteps;
  const bool wt = j < a.n_rec;
  const uint32_t step_bytes = (uint32_t)B * 4u, blk = (uint32_t)T * step_bytes;
  const auto rz = buf_rsrc(a.z0 + (int64_t)(wt ? j : 0) * B, step_bytes);
  const auto rb = buf_rsrc(a.zbits + (int64_t)(wt ? j : 0) * B, step_bytes);
  const int ipl = B % 4 == 0 ? 4 : 1;  // instances per lane
  for (int k = 0; k < a.n_out; ++k) {
    const auto rd = buf_rsrc(a.deltaT + ring(a, k, 0), blk);
    float g = 0.0f;
    for (int c = ipl * lane; c < B; c += ipl * WAVE) {
      const uint32_t off = (uint32_t)c * 4u;
      f4 z = {1.f, 1.f, 1.f, 1.f};
      v4u w = {0u, 0u, 0u, 0u};
      if (wt) {
        if (ipl == 4) {
          z = buf_ldv<4>(rz, off, 0);
          w = __builtin_bit_cast(v4u, buf_ldv<4>(rb, off, 0));
        } else {
          z.x = buf_ld(rz, off, 0);
          w.x = __builtin_bit_cast(uint32_t, buf_ld(rb, off, 0));
        }
        for (int t = 0; t < a.tofs; ++t) z = trace_next<4>(z, a.alpha, w, t);
      }
      for (int t0 = 0; t0 < T; t0 += 4) {
        f4 d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t so = (uint32_t)min(t0 + u, T - 1) * step_bytes;
          if (ipl == 4) d[u] = buf_ldv<4>(rd, off, so);
          else d[u].x = buf_ld(rd, off, so);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (t0 + u < T) {
            if (wt) z = trace_next<4>(z, a.alpha, w, a.tofs + t0 + u);  // the trace after the step
            if (ipl == 4) g += (d[u].x * z.x + d[u].y * z.y) + (d[u].z * z.z + d[u].w * z.w);
            else g = fmaf(d[u].x, z.x, g);
          }
        }
      }
    }
    g = wave_sum(g);
    if (lane == 0) {
      if (wt) a.Gout[(int64_t)k * a.n_rec + j] += g;
      else a.Gb[k] += g;
    }
  }
}

// Workgroups of an e-prop launch: the readout waves come first (they form a
// long dependent chain per wave and would otherwise trail the launch), padded
// to a multiple of 8 so that workgroup n_ro + 8j + o still lands on XCD o.
__host__ __device__ inline int readout_groups(int n_rec, int nw) {
  return ((n_rec + 1 + nw - 1) / nw + 7) & ~7;
}

// Target-major form (B % 4 == 0).  Workgroup n_ro + 8j + o owns target
// neuron j and the synapses onto it from rows r with r % 8 == o (r = i for
// input rows, n_in + i for recurrent rows).  Workgroups are dealt to the 8 XCDs
// in turn, so XCD o only gathers the presynaptic traces of its own eighth of
// the rows, which fits its L2.  Every lane holds four consecutive instances,
// so one wave covers 256 instances of a synapse with 16-byte accesses; wave w
// takes synapses w, w + 4, ... of the list.  psi_j and L_j of the block's
// steps for the current 256-instance chunk are staged once in LDS (32 KB) and
// shared by the workgroup's waves, so a synapse step costs one gathered
// presynaptic trace and six float operations per instance (ALIF):
//   e = psi (p - beta eps),  d = e - (1 - rho) eps,  eps' = eps + d,
//   ebar' = alpha ebar + e,  g += L ebar'
// which is eq. eprop_elig_1/2 (eprop_elig_lif without eps), with
// eps' = psi p + (rho - psi beta) eps.  rho is within 5e-4 of one: carrying
// 1 - rho instead of a float rho keeps the slow eps decay free of a
// systematic 3e-8 per step.  The gradient is summed per lane over the steps
// and its four instances, reduced once per synapse and chunk, and added to G
// in chunk order by the one wave that owns the synapse, so the result does
// not depend on scheduling or on the order of the column list.
constexpr int WL_CH = 4 * WAVE;  // instances per LDS chunk
constexpr int WL_IPL = 4;  // instances per lane

// IPL = 4 instances per lane: a workgroup's 4 waves share a chunk of 256
// instances and wave w works on synapses w, w + 4, ...
template <bool ALIF, int IPL>
__global__ void __launch_bounds__(256 * (4 / IPL)) k_eprop_wl(EpropArgs a) {
  typedef typename VecT<IPL>::type V;
  typedef unsigned U __attribute__((ext_vector_type(IPL)));
  static_assert(IPL == 4, "one wave covers a 256-instance chunk");
  constexpr int LPC = WL_CH / IPL;  // vectors across a chunk
  // 32 KB: with more, the compiler budgets registers for fewer waves
  __shared__ V s_psi[COL_TB][LPC], s_L[COL_TB][LPC];
  const int wv = wave_id(), lane = lane_id();
  const int nw = blockDim.x / WAVE;
  const int n_ro = readout_groups(a.n_rec, nw);
  if ((int)blockIdx.x < n_ro) {
    readout_grad(a, blockIdx.x * nw + wv, lane);
    return;
  }
  const int wg = blockIdx.x - n_ro;
  const int j = wg / COL_OCT;
  const int q0 = a.col_off[wg], q1 = a.col_off[wg + 1];
  if (q1 <= q0) return;
  const int sub = wv;
  const int B = a.B, T = a.nsteps;
  const int n_ch = (B + WL_CH - 1) / WL_CH;
  const uint32_t step_bytes = (uint32_t)B * 4u, blk_bytes = (uint32_t)T * step_bytes;
  const float alpha = a.alpha, omr = a.one_m_rho, beta = a.beta;
  V zero;
#pragma unroll
  for (int e = 0; e < IPL; ++e) zero[e] = 0.0f;
  auto st_off = [&](int t) { return (uint32_t)(t < T ? t : T - 1) * step_bytes; };
  for (int m = 0; m < n_ch; ++m) {
    const int lv = lane;  // this lane's vector within the chunk
    const int b0 = m * WL_CH + IPL * lv;
    const bool act = b0 < B;
    const uint32_t off = (uint32_t)(act ? b0 : 0) * 4u;  // idle lanes read instance 0, never store
    __syncthreads();  // the previous chunk's psi/L are no longer read
    {
      const auto rp = buf_rsrc(a.psiT + ring(a, j, 0), blk_bytes);
      const auto rl = buf_rsrc(a.LT + ring(a, j, 0), blk_bytes);
      for (int t = sub; t < COL_TB; t += 4) {
        s_psi[t][lv] = t < T ? buf_ldv<IPL>(rp, off, st_off(t)) : zero;
        s_L[t][lv] = act && t < T ? buf_ldv<IPL>(rl, off, st_off(t)) : zero;
      }
    }
    __syncthreads();
    for (int sc = q0; sc < q1; sc += WAVE) {  // chunks of 64 list entries
      const int ns = min(WAVE, q1 - sc);
#pragma unroll 1
      for (int k = sub; k < ns; k += 4) {
        // keeps the per-step LDS reads and the trace loads inside their
        // groups (hoisted, they would cost registers, hence occupancy)
        __asm__ volatile("" ::: "memory");
        const int2 ent = a.col[sc + k];
        const bool fin = ent.x < a.n_in;
        const int i = fin ? ent.x : ent.x - a.n_in;
        const int64_t rec = (int64_t)ent.y * B;
        const auto reb = buf_rsrc((fin ? a.in.ebar : a.rec.ebar) + rec, step_bytes);
        const auto rep = buf_rsrc(ALIF ? (fin ? a.in.eps : a.rec.eps) + rec : a.in.ebar, step_bytes);
        // presynaptic trace of the block start and the block's spike bits;
        // the trace of each step is rebuilt with the forward pass's float
        // recursion F <- fma(alpha, F, spike), so it equals the forward's value
        const auto rx0 = buf_rsrc((fin ? a.x0 : a.z0) + (int64_t)i * B, step_bytes);
        const auto rbt = buf_rsrc((fin ? a.xbits : a.zbits) + (int64_t)i * B, step_bytes);
        V eb = buf_ldv_nt<IPL>(reb, off);
        V ep = ALIF ? buf_ldv_nt<IPL>(rep, off) : zero;
        V pr = buf_ldv<IPL>(rx0, off, 0);
        const U bits = __builtin_bit_cast(U, buf_ldv<IPL>(rbt, off, 0));
        for (int t = 0; t < a.tofs; ++t) pr = trace_next<IPL>(pr, alpha, bits, t);
        V g = zero;
#pragma unroll
        for (int t = 0; t < COL_TB; ++t) {
          // step groups of four: the launch's steps end at a group boundary
          // or inside the last group; LDS reads stay inside their group
          if (t % 4 == 0) {
            if (t >= T) break;
            __asm__ volatile("" ::: "memory");
          }
          const V psi = s_psi[t][lv], L = s_L[t][lv];
          // decay factors (alpha, 1 - rho) for the launch's steps and (1, 0)
          // past them, where psi = L = 0 as well: padded steps change nothing
          const float da = t < T ? alpha : 1.0f, dr = t < T ? omr : 0.0f;
          if (ALIF) {
            const V e = psi * (pr - beta * ep);
            const V d = e - dr * ep;
            ep = ep + d;
            eb = da * eb + e;
          } else {
            eb = da * eb + psi * pr;
          }
          g = g + L * eb;
          pr = trace_next<IPL>(pr, alpha, bits, a.tofs + t);
        }
        if (act) {
          buf_stv_nt<IPL>(eb, reb, off);
          if (ALIF) buf_stv_nt<IPL>(ep, rep, off);
        }
        const float gs = wave_sum(hsum<IPL>(g));
        if (lane == 0) (fin ? a.in.G : a.rec.G)[ent.y] += gs;
      }
    }
  }
}

// Column view of both projections for k_eprop_wl: entries
// col[col_off[j*8+o] .. col_off[j*8+o+1]) are (r, slot) of every synapse of a
// row r with r % 8 == o onto target j.  Rebuilt whenever rows change; the
// order inside a list is arbitrary.
__global__ void __launch_bounds__(WAVE) k_col_count(ProjDev in, ProjDev rec, int* cnt) {
  const int r = blockIdx.x;
  const bool fin = r < in.n_pre;
  const ProjDev& P = fin ? in : rec;
  const int i = fin ? r : r - in.n_pre;
  const int n = P.len[i];
  const int64_t base = (int64_t)i * P.cap;
  for (int k = lane_id(); k < n; k += WAVE) atomicAdd(&cnt[P.ind[base + k] * COL_OCT + (r & 7)], 1);
}

// Exclusive scan of n counts (one workgroup): off[0..n]; cnt becomes the fill
// cursor (= off).
__global__ void __launch_bounds__(1024) k_col_scan(int* cnt, int* off, int n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(t * per, n), hi = min(lo + per, n);
  int s = 0;
  for (int q = lo; q < hi; ++q) s += cnt[q];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
    const int v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t ? part[t - 1] : 0;
  for (int q = lo; q < hi; ++q) {
    const int c = cnt[q];
    off[q] = run;
    cnt[q] = run;
    run += c;
  }
  if (t == 1023) off[n] = part[1023];
}

__global__ void __launch_bounds__(WAVE) k_col_fill(ProjDev in, ProjDev rec, int* cur, int2* col) {
  const int r = blockIdx.x;
  const bool fin = r < in.n_pre;
  const ProjDev& P = fin ? in : rec;
  const int i = fin ? r : r - in.n_pre;
  const int n = P.len[i];
  const int64_t base = (int64_t)i * P.cap;
  for (int k = lane_id(); k < n; k += WAVE) {
    const int pos = atomicAdd(&cur[P.ind[base + k] * COL_OCT + (r & 7)], 1);
    col[pos] = make_int2(r, (int)(base + k));
  }
}

void launch_columns(hipStream_t s, const ProjDev& in, const ProjDev& rec, const ColumnView& cv) {
  const int n = rec.n_post * COL_OCT;
  launch_fill_zero(s, cv.cnt, (size_t)n * 4);
  hipLaunchKernelGGL(k_col_count, dim3(in.n_pre + rec.n_pre), dim3(WAVE), 0, s, in, rec, cv.cnt);
  hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(1024), 0, s, cv.cnt, cv.off, n);
  hipLaunchKernelGGL(k_col_fill, dim3(in.n_pre + rec.n_pre), dim3(WAVE), 0, s, in, rec, cv.cnt, cv.col);
}

// Hand-off transpose: [step][B][n] -> [n][nslot][B] (slot slot0 + step) through
// a 64 x 64 LDS tile, both sides coalesced; 32-bit words are moved unchanged.
// blockIdx.z enumerates (array, step) pairs.
__global__ void __launch_bounds__(256) k_handoff_transpose(HandoffArrays h, int B) {
  __shared__ uint32_t tile[64][65];
  int z = blockIdx.z, arr = 0;
  while (arr + 1 < HANDOFF_ARRAYS && z >= h.steps[arr]) z -= h.steps[arr++];
  const int tau = z, n = h.n[arr];
  const int n0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
  if (n0 >= n || b0 >= B || tau >= h.steps[arr]) return;
  const uint32_t* src = h.src[arr] + (int64_t)tau * B * n;
  uint32_t* dst = h.dst[arr];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const int b = b0 + r, j = n0 + tx;
    tile[r][tx] = (b < B && j < n) ? src[(int64_t)b * n + j] : 0u;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = n0 + r, b = b0 + tx;
    if (j < n && b < B) dst[((int64_t)j * h.nslot[arr] + h.slot0[arr] + tau) * B + b] = tile[tx][r];
  }
}

void launch_handoff_transpose(hipStream_t s, const HandoffArrays& h, int B) {
  int nmax = 0, zs = 0;
  for (int q = 0; q < HANDOFF_ARRAYS; ++q) {
    nmax = max(nmax, h.n[q]);
    zs += h.steps[q];
  }
  if (zs <= 0) return;
  dim3 grid((nmax + 63) / 64, (B + 63) / 64, zs);
  hipLaunchKernelGGL(k_handoff_transpose, grid, dim3(256), 0, s, h, B);
}

// Narrow form (B % 4 != 0): threads over a row's synapses, each looping over
// instances and steps; used for small or odd batches such as single-instance
// learning.  Same trace recursion and arithmetic as the target-major form.
template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_narrow(EpropArgs a) {
  const int row = blockIdx.x, tid = threadIdx.x;
  const int n_rows = a.n_in + a.n_rec;
  const int B = a.B;
  if (row >= n_rows) {
    const int j = (row - n_rows) * EP_NT + tid;
    if (j > a.n_rec) return;
    const bool wt = j < a.n_rec;
    for (int k = 0; k < a.n_out; ++k) {
      float g = 0.0f;
      for (int b = 0; b < B; ++b) {
        float z = wt ? a.z0[(int64_t)j * B + b] : 1.0f;
        const uint32_t w = wt ? a.zbits[(int64_t)j * B + b] : 0u;
        if (wt)
          for (int t = 0; t < a.tofs; ++t) z = fmaf(a.alpha, z, (float)((w >> t) & 1u));
        for (int tau = 0; tau < a.nsteps; ++tau) {
          if (wt) z = fmaf(a.alpha, z, (float)((w >> (a.tofs + tau)) & 1u));
          g = fmaf(a.deltaT[ring(a, k, tau) + b], z, g);
        }
      }
      if (wt) a.Gout[(int64_t)k * a.n_rec + j] += g;
      else a.Gb[k] += g;
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
  const float* x0 = (from_in ? a.x0 : a.z0) + (int64_t)i * B;
  const uint32_t* bits = (from_in ? a.xbits : a.zbits) + (int64_t)i * B;
  for (int k = tid; k < n; k += EP_NT) {
    const int64_t s = (int64_t)i * cap + k;
    const int j = ind[s];
    float gsum = 0.0f;
    for (int b = 0; b < B; ++b) {
      float p = x0[b];
      const uint32_t w = bits[b];
      for (int t = 0; t < a.tofs; ++t) p = fmaf(a.alpha, p, (float)((w >> t) & 1u));
      float ep = ALIF ? eps[s * B + b] : 0.0f, eb = ebar[s * B + b];
      for (int tau = 0; tau < a.nsteps; ++tau) {
        const float psi = a.psiT[ring(a, j, tau) + b];
        if (ALIF) {
          const float e = psi * (p - a.beta * ep);
          const float d = e - a.one_m_rho * ep;
          ep = ep + d;
          eb = a.alpha * eb + e;
        } else {
          eb = a.alpha * eb + psi * p;
        }
        gsum = fmaf(a.LT[ring(a, j, tau) + b], eb, gsum);
        p = fmaf(a.alpha, p, (float)((w >> (a.tofs + tau)) & 1u));
      }
      if (ALIF) eps[s * B + b] = ep;
      ebar[s * B + b] = eb;
    }
    G[s] += gsum;
  }
}

void launch_eprop(hipStream_t s, const EpropArgs& a) {
  if (a.nsteps <= 0) return;
  if (a.B % 4 == 0 && a.col && a.col_off) {
    const int nw = 4;
    const int blocks = readout_groups(a.n_rec, nw) + a.n_rec * COL_OCT;
    for (int t0 = 0; t0 < a.nsteps; t0 += COL_TB) {  // blocks longer than COL_TB in parts
      EpropArgs p = a;
      p.slot0 = a.slot0 + t0;
      p.tofs = a.tofs + t0;
      p.nsteps = min(COL_TB, a.nsteps - t0);
      // the step count stays a runtime value: fixed at 16, the compiler
      // schedules for registers beyond the occupancy the LDS allows
      if (a.alif) hipLaunchKernelGGL((k_eprop_wl<true, WL_IPL>), dim3(blocks), dim3(nw * WAVE), 0, s, p);
      else hipLaunchKernelGGL((k_eprop_wl<false, WL_IPL>), dim3(blocks), dim3(nw * WAVE), 0, s, p);
    }
  } else {
    const int n_rows = a.n_in + a.n_rec;
    const int extra = (a.n_rec + 1 + EP_NT - 1) / EP_NT;
    if (a.alif) hipLaunchKernelGGL(k_eprop_narrow<true>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_narrow<false>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
  }
}

}  // namespace rs
