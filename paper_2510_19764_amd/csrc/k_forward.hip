// Forward-pass kernels of the e-prop classifier (paper, recurrent classifier
// section).
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
//   the sum does not depend on the order of the LDS atomics.  Input spikes come
//   from the caller's raster or are drawn by the kernel (Poisson source).
// k_readout / k_learning_signal: leaky readout, softmax error and learning
//   signal L_j = sum_k W_out[k][j] delta_k for the whole block, off the
//   forward kernel's sequential path.
// k_handoff_transpose: the forward kernel's instance-major staging into the
//   neuron-major rings the eligibility kernels read.
#include <mutex>

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
//   rows     int[n_in*cap_in], float[n_in*cap_in], int[n_rec*cap_rec],
//            float[n_rec*cap_rec]  both projections' rows (when rows_lds)
struct FwdLds {
  size_t acc, zlist, len_in, len_rec, xflags, xpos, xbuf, wout, ind_in, w_in, ind_rec, w_rec, total;
};
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline FwdLds fwd_lds_layout(int n_in, int n_rec, int n_out, int xcap, int wout_lds,
                                                 int rows_lds = 0, int cap_in = 0, int cap_rec = 0) {
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
  const size_t si = rows_lds ? (size_t)n_in * cap_in * 4 : 0, sr = rows_lds ? (size_t)n_rec * cap_rec * 4 : 0;
  L.ind_in = o; o = align16(o + si);
  L.w_in = o; o = align16(o + si);
  L.ind_rec = o; o = align16(o + sr);
  L.w_rec = o; o = align16(o + sr);
  L.total = o;
  return L;
}

constexpr int PROP_U = 4;  // slots per lane loaded ahead of the LDS atomics
constexpr size_t WOUT_LDS_MAX = 16 * 1024;  // largest readout matrix staged in LDS

// ROWS: both projections' rows are staged in LDS for the launch (small
// networks), so propagation reads no global memory.
template <int ITEMS, bool ROWS>
__device__ __forceinline__ void fwd_body(const FwdArgs& a, const int b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const FwdLds lay = fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds, ROWS, a.cap_in, a.cap_rec);
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

  const int tid = threadIdx.x, B = a.B;
  // Poisson draws are keyed by the absolute step: the block's first step,
  // plus the device step count where a recorded launch replays
  const uint64_t step0 = a.step0 + (a.step_base ? *a.step_base : 0ull);
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
  const int cap_in = a.cap_in, cap_rec = a.cap_rec;
  const int* ind_in = a.ind_in;
  const float* w_in = a.w_in;
  const int* ind_rec = a.ind_rec;
  const float* w_rec = a.w_rec;
  if constexpr (ROWS) {
    int* si = (int*)(smem + lay.ind_in);
    float* sw = (float*)(smem + lay.w_in);
    int* sir = (int*)(smem + lay.ind_rec);
    float* swr = (float*)(smem + lay.w_rec);
    const int ni = a.n_in * a.cap_in, nr = a.n_rec * a.cap_rec;
    for (int q = tid; q < ni; q += FWD_NT) {
      si[q] = a.ind_in[q];
      sw[q] = a.w_in[q];
    }
    for (int q = tid; q < nr; q += FWD_NT) {
      sir[q] = a.ind_rec[q];
      swr[q] = a.w_rec[q];
    }
    ind_in = si;
    w_in = sw;
    ind_rec = sir;
    w_rec = swr;
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
      const uint32_t u = draw_u32(a.seed, TAG_INPUT, 0, step0 + (uint64_t)tau, (uint64_t)b, (uint64_t)i, 0);
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
    if (ok && a.z0) a.z0[(int64_t)b * a.n_rec + j] = zbr[it];
    const int i = it * FWD_NT + tid;
    const bool oki = it < xitems && i < a.n_in;
    xbr[it] = oki ? a.xbar[(int64_t)b * a.n_in + i] : 0.0f;
    if (oki && a.x0) a.x0[(int64_t)b * a.n_in + i] = xbr[it];
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
        if (a.psi) a.psi[((int64_t)tau * B + b) * a.n_rec + j] = (float)(a.psi_scale * fmax(h, 0.0));
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

    // ---- propagation: one wave per spiking row, lanes over the row's slots.
    // All PROP_U slots per lane are loaded, unconditionally (lanes past the
    // row's end read its last slot again), before any is used, so a row of up
    // to 256 slots costs one memory latency: loads under a lane condition
    // would each be waited for before the next is issued.
    unsigned long long ev = 0ull;
    // the readout drive's weights are loaded first, beside the rows: with at
    // most 64 spikes and 32 outputs, wave wv's outputs wv and wv + 16 need one
    // weight per lane each (lanes past the spike list read a valid weight and
    // drop it)
    constexpr int NWV = FWD_NT / WAVE;
    const bool ro_fast = nz <= WAVE && a.n_out <= 2 * NWV;
    float ro_w0 = 0.0f, ro_w1 = 0.0f;
    bool ro_issued = !ro_fast || wv >= a.n_out;
    // the readout drive's weights: with at most 64 spikes and 32 outputs, wave
    // wv's outputs wv and wv + 16 need one weight per lane each (lanes past
    // the spike list read a valid weight and drop it).  They are requested
    // right after the wave's first row, so that the row's wait leaves them in
    // flight.
    auto issue_readout = [&]() {
      const int jz = nz > 0 ? zlist[min(lane, nz - 1)] : 0;
      const int64_t o0 = (int64_t)wv * a.n_rec + jz, o1 = (int64_t)min(wv + NWV, a.n_out - 1) * a.n_rec + jz;
      if (a.wout_lds) {
        const float* wl = (const float*)(smem + lay.wout);
        ro_w0 = wl[o0];
        ro_w1 = wl[o1];
      } else {
        ro_w0 = ld_global(a.Wout + o0);
        ro_w1 = ld_global(a.Wout + o1);
      }
      ro_issued = true;
    };
    // The wave's rows r = wv, wv + 16, ... in groups of 64: lane k reads row
    // wv + 16 (g + k)'s index and length, and the loop reads them by readlane.
    const int nr_w = nx + nz > wv ? (nx + nz - wv + NWV - 1) / NWV : 0;
    for (int g = 0; g < nr_w; g += WAVE) {
      int my_i = -1, my_n = 0;
      if (g + lane < nr_w) {
        const int r = wv + (g + lane) * NWV;
        if (r >= nx) {
          my_i = zlist[r - nx];
          my_n = len_rec[my_i];
        } else {
          const int i = xstaged ? xbuf[xpos[tau] + r] : ld_global(xsrc_base + s_xsrc[tau] + r);
          if ((unsigned)i < (unsigned)a.n_in) {  // out-of-range channel: ignored
            my_i = i;
            my_n = len_in[i];
          }
        }
      }
      const int kn = min(WAVE, nr_w - g);
      for (int k = 0; k < kn; ++k) {
        const int i = __builtin_amdgcn_readlane(my_i, k), n = __builtin_amdgcn_readlane(my_n, k);
        if (i < 0 || n <= 0) continue;
        const bool from_in = wv + (g + k) * NWV < nx;
        const int* ind = from_in ? ind_in : ind_rec;
        const float* w = from_in ? w_in : w_rec;
        const int64_t base = (int64_t)i * (from_in ? cap_in : cap_rec);
        ev += (unsigned long long)n;
        for (int c0 = 0; c0 < n; c0 += PROP_U * WAVE) {
          int jj[PROP_U];
          float ww[PROP_U];
#pragma unroll
          for (int u = 0; u < PROP_U; ++u) {
            const int64_t q = base + min(c0 + u * WAVE + lane, n - 1);
            jj[u] = ind[q];
            ww[u] = w[q];
          }
          if (!ro_issued) issue_readout();
#pragma unroll
          for (int u = 0; u < PROP_U; ++u)
            if (c0 + u * WAVE + lane < n)
              atomicAdd((unsigned long long*)&acc[jj[u]],
                        (unsigned long long)__double2ll_rn((double)ww[u] * FIX_SCALE));
        }
      }
    }
    if (!ro_issued) issue_readout();  // a wave without rows
    if (lane == 0 && ev) atomicAdd(&s_events, ev);

    // ---- readout drive u_k = sum_j W_out[k][j] z_j: one wave per output unit
    if (ro_fast) {
      if (wv < a.n_out) {
        const float s0 = wave_sum(lane < nz ? ro_w0 : 0.0f);
        const float s1 = wave_sum(lane < nz ? ro_w1 : 0.0f);
        if (lane == 0) {
          a.u[((int64_t)tau * B + b) * a.n_out + wv] = s0;
          if (wv + NWV < a.n_out) a.u[((int64_t)tau * B + b) * a.n_out + wv + NWV] = s1;
        }
      }
    } else {
      for (int k = wv; k < a.n_out; k += FWD_NT / WAVE) {
        float s = 0.0f;
        const float* wk = wout + (int64_t)k * a.n_rec;
        for (int l = lane; l < nz; l += WAVE) s += wk[zlist[l]];
        s = wave_sum(s);
        if (lane == 0) a.u[((int64_t)tau * B + b) * a.n_out + k] = s;
      }
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
      if (a.zbits) a.zbits[m] = zbits[it];
      a.zcount[m] += (uint32_t)__popc(zbits[it]);
    }
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (it >= xitems) break;
    const int i = it * FWD_NT + tid;
    if (i < a.n_in) {
      a.xbar[(int64_t)b * a.n_in + i] = xbr[it];
      if (a.xbits) a.xbits[(int64_t)b * a.n_in + i] = xbits[it];
    }
  }
  __syncthreads();
  if (tid == 0) {
    atomicAdd(&a.counters[0], s_events);
    atomicAdd(&a.counters[1], spikes);
  }
}

template <int ITEMS, bool ROWS>
__global__ void __launch_bounds__(FWD_NT) k_fwd(FwdArgs a) {
  fwd_body<ITEMS, ROWS>(a, blockIdx.x);
}

// Several networks in one launch: workgroup g runs batch instance work[g].y of
// network work[g].x, whose arguments are A[work[g].x].
// The arguments are copied out of the table first: read through the table,
// every field would be read again after each store the kernel makes.
template <int ITEMS>
__global__ void __launch_bounds__(FWD_NT) k_fwd_multi(const FwdArgs* __restrict__ A,
                                                      const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const FwdArgs a = A[w.x];
  fwd_body<ITEMS, false>(a, w.y);
}

// Items per thread: neurons (and input channels) handled by each of the
// workgroup's threads, kept in registers across the block of steps.
// LDS a forward workgroup may take: the device's limit, at most 150 KB, less
// 1 KB for the kernel's static arrays.
static int fwd_lds_cap() {
  static const int lds_cap = [] {
    int dev = 0, cap = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      cap = 64 * 1024;
    (void)hipGetLastError();
    return (cap < 150 * 1024 ? cap : 150 * 1024) - 1024;
  }();
  return lds_cap;
}

bool fwd_fits(int n_in, int n_rec, int n_out) {
  return fwd_lds_layout(n_in, n_rec, n_out, 0, 0).total <= (size_t)fwd_lds_cap();
}

size_t fwd_plan(FwdArgs& a) {
  // LDS budget: stage W_out and up to 2048 input spikes when they fit
  const int lds_cap = fwd_lds_cap();
  a.xcap = 2048;
  // W_out is staged only while small: the forward workgroups stay resident on
  // their CUs beside the e-prop launch of the previous block, and every
  // kilobyte of LDS they hold is taken from the e-prop workgroups' share
  a.wout_lds = (size_t)a.n_out * a.n_rec * 4 <= WOUT_LDS_MAX ? 1 : 0;
  if (fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds).total > (size_t)lds_cap) a.wout_lds = 0;
  while (fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds).total > (size_t)lds_cap && a.xcap > 0)
    a.xcap /= 2;
  return fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds).total;
}

int fwd_items(int n_in, int n_rec) {
  const int need = (max(n_rec, n_in) + FWD_NT - 1) / FWD_NT;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

void fwd_attrs() {
  static std::once_flag once;
  std::call_once(once, [] {
    allow_dynamic_lds((const void*)k_fwd<1, true>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<1, false>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<2, false>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<4, false>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd<8, false>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd_multi<1>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd_multi<2>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd_multi<4>, 150 * 1024);
    allow_dynamic_lds((const void*)k_fwd_multi<8>, 150 * 1024);
  });
}

void launch_fwd_multi(hipStream_t s, const FwdArgs* A, const int2* work, int n_work, int items, size_t lds) {
  if (n_work <= 0) return;
  fwd_attrs();
  if (items <= 1) hipLaunchKernelGGL(k_fwd_multi<1>, dim3(n_work), dim3(FWD_NT), lds, s, A, work);
  else if (items <= 2) hipLaunchKernelGGL(k_fwd_multi<2>, dim3(n_work), dim3(FWD_NT), lds, s, A, work);
  else if (items <= 4) hipLaunchKernelGGL(k_fwd_multi<4>, dim3(n_work), dim3(FWD_NT), lds, s, A, work);
  else hipLaunchKernelGGL(k_fwd_multi<8>, dim3(n_work), dim3(FWD_NT), lds, s, A, work);
}

void launch_fwd(hipStream_t s, const FwdArgs& a_in) {
  const int lds_cap = fwd_lds_cap();
  FwdArgs a = a_in;
  fwd_plan(a);
  const int need = (max(a.n_rec, a.n_in) + FWD_NT - 1) / FWD_NT;
  // rows in LDS when asked for, one neuron per thread and everything fits
  const bool rows = a.rows_lds && need <= 1 &&
                    fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds, 1, a.cap_in, a.cap_rec).total <=
                        (size_t)lds_cap;
  const size_t sm = fwd_lds_layout(a.n_in, a.n_rec, a.n_out, a.xcap, a.wout_lds, rows, a.cap_in, a.cap_rec).total;
  fwd_attrs();
  if (rows) hipLaunchKernelGGL((k_fwd<1, true>), dim3(a.B), dim3(FWD_NT), sm, s, a);
  else if (need <= 1) hipLaunchKernelGGL((k_fwd<1, false>), dim3(a.B), dim3(FWD_NT), sm, s, a);
  else if (need <= 2) hipLaunchKernelGGL((k_fwd<2, false>), dim3(a.B), dim3(FWD_NT), sm, s, a);
  else if (need <= 4) hipLaunchKernelGGL((k_fwd<4, false>), dim3(a.B), dim3(FWD_NT), sm, s, a);
  else hipLaunchKernelGGL((k_fwd<8, false>), dim3(a.B), dim3(FWD_NT), sm, s, a);
}

// Leaky readout and softmax error over a block (recurrent classifier
// section): one wave per instance b, lane k (and k + 64, ...) carrying output
// k through the block's steps,
//   y_k <- alpha y_k + u_k + b_k   (double),   delta_k = softmax(y)_k - [k == label_b],
// with the softmax maximum and denominator reduced across the wave.  delta
// goes into the ring [k][slot][b].  Labels outside 0..n_out-1 contribute no
// target term.
constexpr int RO_KMAX = 4;  // n_out <= 4 * WAVE
// KMAX output chunks of 64 per lane (KMAX = 1 for n_out <= 64: fewer registers,
// so a workgroup fits beside the e-prop launch's)
template <int KMAX>
__device__ __forceinline__ void readout_body(const ReadoutArgs& a, const int bx) {
  const int b = bx * 4 + wave_id(), lane = lane_id();
  if (b >= a.B) return;
  const int label = a.labels[b];
  double y[KMAX];
  float bias[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int k = q * WAVE + lane;
    y[q] = k < a.n_out ? a.Y[(int64_t)b * a.n_out + k] : 0.0;
    bias[q] = k < a.n_out ? a.bout[k] : 0.0f;
  }
  // Steps go in groups of RO_TC: the group's drive is loaded before any of it
  // is used (one memory latency per group), the leaky outputs of its steps
  // are advanced in order, and then the group's softmaxes, which depend only
  // on their own step's outputs, are reduced side by side.
  constexpr int RO_TC = 8;
  for (int t0 = 0; t0 < a.nsteps; t0 += RO_TC) {
    const int nt = min(RO_TC, a.nsteps - t0);
    float uc[RO_TC][KMAX];
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) {
      const int64_t row = ((int64_t)min(t0 + t, a.nsteps - 1) * a.B + b) * a.n_out;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) uc[t][q] = ld_global(a.u + row + min(q * WAVE + lane, a.n_out - 1));
    }
    // outputs after each step of the group (steps past the block leave y as it is)
    float yf[RO_TC][KMAX], m[RO_TC];
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) {
      m[t] = -INFINITY;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        if (t < nt && q * WAVE + lane < a.n_out) y[q] = a.alpha * y[q] + (double)uc[t][q] + (double)bias[q];
        yf[t][q] = (float)y[q];
        if (q * WAVE + lane < a.n_out) m[t] = fmaxf(m[t], yf[t][q]);
      }
    }
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) m[t] = wave_max(m[t]);
    float ex[RO_TC][KMAX], den[RO_TC];
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) {
      den[t] = 0.0f;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        ex[t][q] = expf(yf[t][q] - m[t]);
        if (q * WAVE + lane < a.n_out) den[t] += ex[t][q];
      }
    }
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) den[t] = wave_sum(den[t]);
#pragma unroll
    for (int t = 0; t < RO_TC; ++t) {
      if (t >= nt) break;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        const int k = q * WAVE + lane;
        if (k < a.n_out) {
          const float d = ex[t][q] / den[t] - (k == label ? 1.0f : 0.0f);
          a.deltaT[((int64_t)k * a.nslot + a.slot0 + t0 + t) * a.B + b] = d;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int k = q * WAVE + lane;
    if (k < a.n_out) a.Y[(int64_t)b * a.n_out + k] = y[q];
  }
}
template <int KMAX>
__global__ void __launch_bounds__(256) k_readout(ReadoutArgs a) { readout_body<KMAX>(a, blockIdx.x); }

// Learning signal L_j = sum_k W_out[k][j] delta_k (recurrent classifier
// section), written straight into the ring [j][slot][b]: lanes over
// instances, each thread 16 consecutive neurons of a 64-neuron tile whose
// readout weights are staged in LDS.  blockIdx = (neuron tile, instance tile,
// step).  A thread requests its weights and up to LS_KC deltas before using
// any (rows and outputs past the ends are read again, clamped, and not used),
// and the products are added in output order.  The staged weights take
// min(n_out, 64) rows of LDS (5.2 KB for 20 outputs), so a workgroup fits on
// a CU beside three e-prop workgroups.
constexpr int LS_KC = 16;
constexpr int LS_LD = 65;  // LDS row pitch in floats
inline size_t ls_lds_bytes(int n_out) { return (size_t)(n_out < 64 ? n_out : 64) * LS_LD * sizeof(float); }
__device__ __forceinline__ void learning_signal_body(const ReadoutArgs& a, const int bx, const int by, const int bz,
                                                     float* w /* [min(n_out, 64)][LS_LD]: [k in chunk][j in tile] */) {
  const int lane = lane_id(), wv = wave_id();
  const int j0 = bx * 64, b = by * 64 + lane, tau = bz;
  const int jq = wv * 16;  // this wave's 16 neurons of the tile
  const int bl = min(b, a.B - 1), jl = min(j0 + lane, a.n_rec - 1);
  const int64_t dcol = (int64_t)a.slot0 + tau;
  float acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
  for (int k0 = 0; k0 < a.n_out; k0 += 64) {
    const int kn = min(64, a.n_out - k0);
    float wl[16], d[LS_KC];
#pragma unroll
    for (int i = 0; i < 16; ++i) wl[i] = ld_global(a.Wout + (int64_t)(k0 + min(wv + 4 * i, kn - 1)) * a.n_rec + jl);
    auto load_d = [&](int kc) {
#pragma unroll
      for (int i = 0; i < LS_KC; ++i)
        d[i] = ld_global(a.deltaT + ((int64_t)(k0 + min(kc + i, kn - 1)) * a.nslot + dcol) * a.B + bl);
    };
    load_d(0);
    __syncthreads();  // the previous chunk's reads of w are done
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int kk = wv + 4 * i;
      if (kk < kn) w[kk * LS_LD + lane] = j0 + lane < a.n_rec ? wl[i] : 0.0f;
    }
    __syncthreads();
    for (int kc = 0; kc < kn; kc += LS_KC) {
      if (kc > 0) load_d(kc);
#pragma unroll
      for (int i = 0; i < LS_KC; ++i) {
        if (kc + i >= kn) break;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = fmaf(w[(kc + i) * LS_LD + jq + q], d[i], acc[q]);
      }
    }
  }
  if (b >= a.B) return;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = j0 + jq + q;
    if (j < a.n_rec) a.LT[((int64_t)j * a.nslot + dcol) * a.B + b] = acc[q];
  }
}
__global__ void __launch_bounds__(256) k_learning_signal(ReadoutArgs a) {
  extern __shared__ float ls_w[];
  learning_signal_body(a, blockIdx.x, blockIdx.y, blockIdx.z, ls_w);
}

int readout_grid(const ReadoutArgs& a) { return (a.B + 3) / 4; }
void learning_signal_grid(const ReadoutArgs& a, int g[3]) {
  g[0] = (a.n_rec + 63) / 64;
  g[1] = (a.B + 63) / 64;
  g[2] = a.nsteps;
}

void launch_readout(hipStream_t s, const ReadoutArgs& a, bool learning_signal) {
  if (a.nsteps <= 0) return;
  if (a.n_out <= WAVE) hipLaunchKernelGGL(k_readout<1>, dim3(readout_grid(a)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_readout<RO_KMAX>, dim3(readout_grid(a)), dim3(256), 0, s, a);
  if (learning_signal) {
    int g[3];
    learning_signal_grid(a, g);
    hipLaunchKernelGGL(k_learning_signal, dim3(g[0], g[1], g[2]), dim3(256), ls_lds_bytes(a.n_out), s, a);
  }
}

// Hand-off transpose: [step][B][n] -> [n][nslot][B] (slot slot0 + step) through
// a 32 (instances) x 64 (neurons) LDS tile, both sides coalesced; 32-bit words
// are moved unchanged.  blockIdx.z enumerates (array, step) pairs.  A thread's
// eight loads are all issued before the first is used (past the array's edges
// the last row or column is read again and not stored), so a workgroup waits
// for memory once.  The tile's 8.3 KB fit on a CU beside three e-prop
// workgroups.
constexpr int HO_TB = 32;  // instances per transpose tile
__device__ __forceinline__ void handoff_body(const HandoffArrays& h, const int B, const int bx, const int by,
                                             const int bz) {
  __shared__ uint32_t tile[HO_TB][65];
  int z = bz, arr = 0;
  while (arr + 1 < HANDOFF_ARRAYS && z >= h.steps[arr]) z -= h.steps[arr++];
  const int tau = z, n = h.n[arr];
  const int n0 = bx * 64, b0 = by * HO_TB;
  if (n0 >= n || b0 >= B || tau >= h.steps[arr]) return;
  const uint32_t* src = h.src[arr] + (int64_t)tau * B * n;
  uint32_t* dst = h.dst[arr];
  // loads: 64 neurons (lanes) x 4 rows of instances per pass
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int jl = min(n0 + tx, n - 1);
  uint32_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = ld_global(src + (int64_t)min(b0 + ty + 4 * i, B - 1) * n + jl);
#pragma unroll
  for (int i = 0; i < 8; ++i) tile[ty + 4 * i][tx] = v[i];
  __syncthreads();
  // stores: 32 instances (lanes) x 8 neurons per pass
  const int sx = threadIdx.x & 31, sy = threadIdx.x >> 5;
  const int b = b0 + sx;
  if (b >= B) return;
  const int64_t col = (int64_t)h.slot0[arr] + tau, nslot = h.nslot[arr], es = h.es[arr];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = tile[sx][sy + 8 * i];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int j = n0 + sy + 8 * i;
    if (j < n) dst[(((int64_t)j * nslot + col) * B + b) * es] = v[i];
  }
}
__global__ void __launch_bounds__(256) k_handoff_transpose(HandoffArrays h, int B) {
  handoff_body(h, B, blockIdx.x, blockIdx.y, blockIdx.z);
}

// The three block kernels above for several networks in one launch: workgroup
// g runs tile (work[g].y, work[g].z, work[g].w) of network work[g].x.
__global__ void __launch_bounds__(256) k_handoff_multi(const HandoffArrays* __restrict__ H,
                                                       const int* __restrict__ Bs, const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  const HandoffArrays h = H[w.x];
  handoff_body(h, Bs[w.x], w.y, w.z, w.w);
}
__global__ void __launch_bounds__(256) k_readout_multi(const ReadoutArgs* __restrict__ A,
                                                       const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  const ReadoutArgs a = A[w.x];
  readout_body<RO_KMAX>(a, w.y);
}
__global__ void __launch_bounds__(256) k_learning_signal_multi(const ReadoutArgs* __restrict__ A,
                                                               const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  const ReadoutArgs a = A[w.x];
  __shared__ float w_tile[64 * LS_LD];  // networks of any output count
  learning_signal_body(a, w.y, w.z, w.w, w_tile);
}

void handoff_grid(const HandoffArrays& h, int B, int g[3]) {
  int nmax = 0, zs = 0;
  for (int q = 0; q < HANDOFF_ARRAYS; ++q) {
    nmax = max(nmax, h.n[q]);
    zs += h.steps[q];
  }
  g[0] = (nmax + 63) / 64;
  g[1] = (B + HO_TB - 1) / HO_TB;
  g[2] = zs;
}

void launch_handoff_transpose(hipStream_t s, const HandoffArrays& h, int B) {
  int g[3];
  handoff_grid(h, B, g);
  if (g[2] <= 0) return;
  hipLaunchKernelGGL(k_handoff_transpose, dim3(g[0], g[1], g[2]), dim3(256), 0, s, h, B);
}

void launch_handoff_multi(hipStream_t s, const HandoffArrays* H, const int* Bs, const int4* work, int n_work) {
  if (n_work > 0) hipLaunchKernelGGL(k_handoff_multi, dim3(n_work), dim3(256), 0, s, H, Bs, work);
}

void launch_readout_multi(hipStream_t s, const ReadoutArgs* A, const int4* ro_work, int n_ro, const int4* ls_work,
                          int n_ls) {
  if (n_ro > 0) hipLaunchKernelGGL(k_readout_multi, dim3(n_ro), dim3(256), 0, s, A, ro_work);
  if (n_ls > 0) hipLaunchKernelGGL(k_learning_signal_multi, dim3(n_ls), dim3(256), 0, s, A, ls_work);
}

}  // namespace rs
