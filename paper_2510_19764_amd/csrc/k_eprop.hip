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
//   batch-summed gradient G_ji += sum_b L_j ebar_ji; the last workgroups
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
// launch then applies up to COL_TB steps per synapse while its eps/ebar stay in
// registers: the trace stream crosses HBM once per block instead of once per
// step.  Each step rounds eps/ebar to float, so they are bit-identical for
// every block length; the gradient is summed over the block's steps per lane
// before the batch reduction, so G depends on the block length only through
// float rounding.
constexpr int EP_NT = 256;
constexpr int COL_TB = 16;  // steps per launch of the column kernel
constexpr int COL_OCT = 8;  // source octants, one per XCD

__device__ __forceinline__ int64_t ring(const EpropArgs& a, int n, int tau) {
  return ((int64_t)n * a.nslot + a.slot0 + tau) * a.B;
}

// Readout delta rule over the launch's steps (recurrent classifier section):
// wave j < n_rec adds sum_t sum_b delta_k z_j to Gout[k][j] for every output
// k, wave n_rec the bias gradient sum_t sum_b delta_k.
__device__ __forceinline__ void readout_grad(const EpropArgs& a, int j, int lane) {
  if (j > a.n_rec) return;
  const int B = a.B, T = a.nsteps;
  const bool wt = j < a.n_rec;
  for (int k = 0; k < a.n_out; ++k) {
    float g = 0.0f;
    for (int t = 0; t < T; ++t) {
      const float* __restrict__ d = a.deltaT + ring(a, k, t);
      const float* __restrict__ z = a.zbar_new + ring(a, wt ? j : 0, t);
      if (B % 4 == 0) {
        for (int c = lane; c < B / 4; c += WAVE) {
          const f4 d4 = *(const f4*)&d[4 * c];
          if (wt) {
            const f4 z4 = *(const f4*)&z[4 * c];
            g += (d4.x * z4.x + d4.y * z4.y) + (d4.z * z4.z + d4.w * z4.w);
          } else {
            g += (d4.x + d4.y) + (d4.z + d4.w);
          }
        }
      } else {
        for (int b = lane; b < B; b += WAVE) g += wt ? d[b] * z[b] : d[b];
      }
    }
    g = wave_sum(g);
    if (lane == 0) {
      if (wt) a.Gout[(int64_t)k * a.n_rec + j] += g;
      else a.Gb[k] += g;
    }
  }
}

// Target-major form (B >= 32).  Workgroup g = j*8 + o owns target neuron j
// and the synapses onto it from rows r with r % 8 == o (r = i for input rows,
// n_in + i for recurrent rows).  Workgroups are handed to the 8 XCDs
// round-robin, so XCD o only gathers the presynaptic traces of its own eighth
// of the rows.  Wave w takes 64-instance chunks w, w + nw, ... with one
// instance per lane; psi_j, L_j and the eps decay factor of the block's steps
// sit in registers, so each synapse step costs one gathered float (the
// presynaptic trace) and six float operations (ALIF):
//   u = psi p,  d = u - ((1 - rho) + psi beta) eps,  e = d + (1 - rho) eps,
//   eps' = eps + d,  ebar' = alpha ebar + e,  g += L ebar'
// which is e = psi (p - beta eps) and eps' = psi p + (rho - psi beta) eps of
// eq. eprop_elig_1/2 (eprop_elig_lif without eps).  rho is within 5e-4 of one:
// carrying 1 - rho instead of a float rho keeps the slow eps decay free of a
// systematic 3e-8 per step.  Lane sums over the steps are reduced per synapse
// with DPP, per wave in chunk order and across waves in wave order, so the
// result does not depend on scheduling or on the order of the column list.
template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_col(EpropArgs a) {
  __shared__ float gpart[EP_NT / WAVE][WAVE];
  const int wv = threadIdx.x / WAVE, lane = lane_id();
  const int nw = blockDim.x / WAVE;
  const int ncol = a.n_rec * COL_OCT;
  const int wg = blockIdx.x;
  if (wg >= ncol) {
    readout_grad(a, (wg - ncol) * nw + wv, lane);
    return;
  }
  const int j = wg / COL_OCT;
  const int q0 = a.col_off[wg], q1 = a.col_off[wg + 1];
  const int B = a.B, T = a.nsteps, n_ic = (B + WAVE - 1) / WAVE;
  const float alpha = a.alpha, omr = a.one_m_rho, beta = a.beta;
  for (int sc = q0; sc < q1; sc += WAVE) {  // uniform over the workgroup
    const int ns = min(WAVE, q1 - sc);
    float my_g = 0.0f;  // lane k: this wave's part of the gradient of entry sc + k
    for (int ic = wv; ic < n_ic; ic += nw) {
      const int b = ic * WAVE + lane;
      const bool act = b < B;
      const int bb = act ? b : 0;  // idle lanes read instance 0 and never store
      float psi[COL_TB], L[COL_TB], c[COL_TB];
      const float* __restrict__ pj = a.psiT + ring(a, j, 0) + bb;
      const float* __restrict__ lj = a.LT + ring(a, j, 0) + bb;
#pragma unroll
      for (int t = 0; t < COL_TB; ++t) {
        const int tt = t < T ? t : T - 1;  // loads stay inside the block
        psi[t] = pj[(int64_t)tt * B];
        L[t] = act ? lj[(int64_t)tt * B] : 0.0f;
        c[t] = ALIF ? fmaf(psi[t], beta, omr) : 0.0f;
      }
      for (int k = 0; k < ns; ++k) {
        const int2 ent = a.col[sc + k];
        const bool fin = ent.x < a.n_in;
        const int i = fin ? ent.x : ent.x - a.n_in;
        const float* __restrict__ pre = (fin ? a.xbar_prev : a.zbar_prev) + ring(a, i, 0) + bb;
        const int64_t rec = (int64_t)ent.y * B + bb;
        float* __restrict__ ebp = (fin ? a.in.ebar : a.rec.ebar) + rec;
        float* __restrict__ epp = ALIF ? (fin ? a.in.eps : a.rec.eps) + rec : nullptr;
        float p[COL_TB];
#pragma unroll
        for (int t = 0; t < COL_TB; ++t) p[t] = pre[(int64_t)(t < T ? t : T - 1) * B];
        float eb = __builtin_nontemporal_load(ebp);
        float ep = ALIF ? __builtin_nontemporal_load(epp) : 0.0f;
        float g = 0.0f;
#pragma unroll
        for (int t = 0; t < COL_TB; ++t) {
          if (t < T) {
            const float u = psi[t] * p[t];
            if (ALIF) {
              const float d = fmaf(-c[t], ep, u);
              const float e = fmaf(omr, ep, d);
              ep = ep + d;
              eb = fmaf(alpha, eb, e);
            } else {
              eb = fmaf(alpha, eb, u);
            }
            g = fmaf(L[t], eb, g);
          }
        }
        if (act) {
          __builtin_nontemporal_store(eb, ebp);
          if (ALIF) __builtin_nontemporal_store(ep, epp);
        }
        const float gs = wave_sum(g);
        if (lane == k) my_g += gs;
      }
    }
    gpart[wv][lane] = my_g;
    __syncthreads();
    if ((int)threadIdx.x < ns) {
      const int2 ent = a.col[sc + threadIdx.x];
      float gsum = 0.0f;
      for (int w = 0; w < nw; ++w) gsum += gpart[w][threadIdx.x];
      float* G = ent.x < a.n_in ? a.in.G : a.rec.G;
      G[ent.y] += gsum;
    }
    __syncthreads();
  }
}

// Column view of both projections for k_eprop_col: entries
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

// Narrow form (B < 32): threads over a row's synapses, each looping over steps
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
  if (a.nsteps <= 0) return;
  if (a.B >= 32 && a.col && a.col_off) {
    const int nw = min(EP_NT / WAVE, (a.B + WAVE - 1) / WAVE);
    const int blocks = a.n_rec * COL_OCT + (a.n_rec + 1 + nw - 1) / nw;
    for (int t0 = 0; t0 < a.nsteps; t0 += COL_TB) {  // blocks longer than COL_TB in parts
      EpropArgs p = a;
      p.slot0 = a.slot0 + t0;
      p.nsteps = min(COL_TB, a.nsteps - t0);
      if (a.alif) hipLaunchKernelGGL(k_eprop_col<true>, dim3(blocks), dim3(nw * WAVE), 0, s, p);
      else hipLaunchKernelGGL(k_eprop_col<false>, dim3(blocks), dim3(nw * WAVE), 0, s, p);
    }
  } else {
    const int n_rows = a.n_in + a.n_rec;
    const int extra = (a.n_rec + 1 + EP_NT - 1) / EP_NT;
    if (a.alif) hipLaunchKernelGGL(k_eprop_narrow<true>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_narrow<false>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
  }
}

}  // namespace rs
