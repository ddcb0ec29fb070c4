// Topographic-map simulation over several workgroups (topographic-map model,
// Tab. A-H; scaled maps L = 16 s of the scaling paragraph), with the optional
// lateral projection (target -> target rows, Tab. A "feed-forward and lateral
// connections", Tab. G lateral formation parameters).
//
// The target sheet is cut into tiles of TOPO_TILE neurons; workgroup g owns
// targets [256 g, 256 g + 256), one per thread, and the source channels with
// the same indices.  Every synapse's weight is read and written only by the
// workgroup owning its target (delivery filters each spiking row to the tile;
// potentiation walks the tile's columns), so the tiles never write the same
// word.  What a tile needs from the others is, per step: which sources and
// which targets spiked (bitmasks) and the presynaptic traces x, xl of any
// source or target whose synapse onto the tile is potentiated.  Each tile
// publishes its share of these at the end of its step into a double-buffered
// exchange (buffer 0 is the state arrays zin, zout, x, xl; buffer 1 the copies
// zin_b, ...), then counts itself in at a device-wide barrier; the next step
// waits for every tile's arrival before reading.  One barrier per step:
//   - the spikes of step t are delivered at t+1 (delay h), so the bitmasks of
//     step t are exactly what step t+1 delivers;
//   - x_i(t+1) = x_i(t) exp(-h/tau_+) + [i spiked at t]: a reader computes it
//     from the published x_i(t) and the bitmask with the same float
//     operations as the owner, so every tile sees the same value.
// The barrier is one flag per tile holding the count of barriers the tile has
// passed, which only grows: a launch starts from the count the last one ended
// at, so nothing is reset between launches.  A workgroup's wait is bounded: past the spin limit it
// raises the error flag and the launch ends early on every workgroup (the host
// reports the flag); the host launches no more tiles than the device keeps
// resident at once.
//
// Step t on tile g (the order of the model readings, as in the one-workgroup
// kernel):
//   A  draw the tile's source spikes of step t (waves 1.., eight channels per
//      generator call), while wave 0 waits for the step barrier
//   B  decay the traces, list the spiking sources (and targets) of step t-1
//      from the exchange with their row lengths, and deliver their rows to
//      the tile's targets with depression: every (spike, slot) pair up to the
//      longest listed row is one work item, so all row loads of the step are
//      in flight together
//   C  neuron update (registers), publish the tile's spike words and traces
//   D  potentiation along the columns of the tile's spiking targets
#include <mutex>

#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int TT_NT = TOPO_TILE;  // threads per workgroup = targets per tile
constexpr int TT_WORDS = TT_NT / 32;  // spike words per tile
constexpr unsigned TT_SPIN_LIMIT = 1u << 22;  // polls of the barrier count before giving up
constexpr int TT_DRAW_WAVES = (TT_NT / 8 + WAVE - 1) / WAVE;  // waves drawing the tile's source channels
static_assert(TT_NT % WAVE == 0 && TT_NT / WAVE > TT_DRAW_WAVES, "drawing waves beside the waiting one");
static_assert((TT_NT / 8) % 4 == 0, "four drawing lanes make one spike word");

size_t topo_tiles_lds_bytes(int N, bool lateral) {
  return (size_t)TT_NT * (8 + 4 + 4 + 4 + 4) + (size_t)N * 4 * (lateral ? 2 : 1);
}

int topo_tiles_grid(int N) { return (N + TT_NT - 1) / TT_NT; }

__device__ __forceinline__ int axis_dist_t(int L, int a, int b) {
  const int d = abs(a - b);
  return min(d, L - d);
}

__device__ __forceinline__ uint32_t bit_of(const uint32_t* bits, int i) { return (bits[i >> 5] >> (i & 31)) & 1u; }

// The step barrier: tile g's flag (one per 128 bytes) holds the number of
// barriers it has passed since the simulation was attached, a count that
// only grows.  Arrival: every thread's stores are made visible device-wide,
// then one thread stores the new count with release order.  No two tiles
// write one line, and no read-modify-write is serialised on one address.
constexpr int TT_FLAG_STRIDE = 16;  // 64-bit words between two tiles' flags
__device__ __forceinline__ void tiles_arrive(unsigned long long* flags, unsigned long long count) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&flags[(size_t)blockIdx.x * TT_FLAG_STRIDE], count, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every tile's flag reaches `count`: wave 0 polls one flag per
// lane (at most 64 tiles); false (on every thread) if the wait gave up or
// another workgroup raised the error flag.
__device__ __forceinline__ bool tiles_wait(unsigned long long* flags, unsigned long long count, int* err,
                                           int* s_ok) {
  if (threadIdx.x < WAVE) {
    const int l = threadIdx.x;
    const bool mine = l < (int)gridDim.x;
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      // relaxed polls (an acquire per poll would invalidate the caches each
      // time); the acquire fences below order what follows after the last one
      const unsigned long long v =
          mine ? __hip_atomic_load(&flags[(size_t)l * TT_FLAG_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : count;
      if (ballot(v < count) == 0ull) break;
      if (++spins > TT_SPIN_LIMIT || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok && l == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (l == 0) *s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *s_ok != 0;
}

// List the set bits of bits[0 .. words) with their rows' lengths, packed as
// i << 11 | len (i < 2^14, len <= 1024), and the longest such row.
constexpr int TT_LEN_BITS = 11;
__device__ __forceinline__ void list_rows(const uint32_t* bits, int words, const int* len, int* list, int* s_n,
                                          int* s_max) {
  int mx = 0;
  for (int q = threadIdx.x; q < words; q += TT_NT) {
    uint32_t w = bits[q];
    if (!w) continue;
    int pos = atomicAdd(s_n, __popc(w));
    while (w) {
      const int i = q * 32 + __builtin_ctz(w);
      w &= w - 1;
      const int n = len[i];
      mx = max(mx, n);
      list[pos++] = (i << TT_LEN_BITS) | n;
    }
  }
  if (mx) atomicMax(s_max, mx);
}

// Deliver the listed rows to this tile's targets: conductance in fixed point,
// depression by A_- y_target.  Work item e is slot e % mx of row e / mx, mx
// the longest listed row, so every load of the step is issued together.
__device__ __forceinline__ void deliver_rows(const ProjDev& Q, const int* list, int n, int mx, int j0,
                                             long long* acc, const float* y, const TopoSimDev& sd) {
  const int total = n * mx;
  for (int e = threadIdx.x; e < total; e += TT_NT) {
    const int q = e / mx, s = e - q * mx;
    const int v = list[q];
    if (s >= (v & ((1 << TT_LEN_BITS) - 1))) continue;
    const int64_t k = (int64_t)(v >> TT_LEN_BITS) * Q.cap + s;
    const int jj = Q.ind[k] - j0;
    const float w = Q.w[k];
    if ((unsigned)jj < (unsigned)TT_NT) {
      atomicAdd((unsigned long long*)&acc[jj], (unsigned long long)__double2ll_rn((double)w * FIX_SCALE));
      if (sd.stdp) Q.w[k] = fmaxf(0.f, w - sd.A_minus * y[jj]);
    }
  }
}

// Potentiate the synapses of column j (slots into Q's rows) by A_+ times the
// presynaptic trace of this step, computed from the exchange.
__device__ __forceinline__ void potentiate_col(const ProjDev& Q, const int* col, int n, const float* Xcur,
                                               const uint32_t* Zcur, const TopoSimDev& sd) {
  for (int e = lane_id(); e < n; e += WAVE) {
    const int slot = col[e];
    if (slot < 0) continue;  // removed by a rewire
    const int i = slot / Q.cap;
    const float xi = Xcur[i] * sd.dx + (float)bit_of(Zcur, i);
    Q.w[slot] = fminf(Q.w[slot] + sd.A_plus * xi, sd.g_max);
  }
}

__device__ __forceinline__ void tiles_mark(long long& acc, long long& prev) {
  const long long now = (long long)wall_clock64();
  acc += now - prev;
  prev = now;
}

template <bool TIMED, bool LAT>
__global__ void __launch_bounds__(TT_NT) k_topo_tiles(uint64_t seed, ProjDev P, ProjDev PL, TopoSimDev sd,
                                                      uint64_t t0, int n_steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_nS, s_nZ, s_mS, s_mZ, s_npost, s_ok;
  __shared__ int s_stim[3];
  __shared__ uint32_t s_sbits[TT_WORDS];
  if (*sd.err) return;  // an earlier launch gave up: leave the state alone
  const int N = sd.N, tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int j0 = blockIdx.x * TT_NT, j = j0 + tid;
  const bool own = j < N;
  const int words = (N + 31) / 32, wb = j0 >> 5;
  long long* acc = (long long*)smem;  // [T] delivered conductance, fixed point
  float* y = (float*)(acc + TT_NT);   // [T] post trace
  int* post = (int*)(y + TT_NT);      // [T] tile's targets that spiked this step
  int* clf = post + TT_NT;            // [T] feed-forward column lengths
  int* cll = clf + TT_NT;             // [T] lateral column lengths
  int* listS = cll + TT_NT;           // [N] spiking sources of the step before
  int* listZ = listS + N;             // [N] spiking targets of the step before (lateral)
  const bool tm = TIMED && blockIdx.x == 0 && tid == 0;
  long long tprev = tm ? (long long)wall_clock64() : 0, tk[TOPO_PHASES] = {0, 0, 0, 0};

  if (t0 == STEP_FROM_DEVICE) t0 = *sd.step_dev;  // read before the first arrival; written after the last
  // every tile's flag equals the count the last launch ended at
  unsigned long long target = sd.bar[(size_t)blockIdx.x * TT_FLAG_STRIDE];
  const int dirty = *sd.col_dirty || (LAT && *sd.col_dirty_l);
  // this tile's state: neurons and both presynaptic traces in registers
  float V = 0.f, gr = 0.f, xr = 0.f, xlr = 0.f;
  int ref = 0;
  uint32_t cnt = 0;
  if (own) {
    V = sd.V[j];
    gr = sd.g[j];
    ref = sd.ref[j];
    cnt = sd.count[j];
    xr = sd.x[j];
    if (LAT) xlr = sd.xl[j];
    y[tid] = sd.y[j];
  } else {
    y[tid] = 0.f;
  }
  acc[tid] = 0;
  const int L = sd.L, Ls = sd.stim_L;
  if (tid < 3) {  // stimulus position of t0's epoch
    const uint32_t u = draw_u32(seed, TAG_STIM, 0, t0 / (uint64_t)sd.stim_steps, (uint64_t)tid, 0, 0);
    s_stim[tid] = tid < 2 ? (int)below(u, (uint32_t)Ls) : (int)(u & 1u);
  }
  if (tid == 0) {
    s_nS = 0;
    s_nZ = 0;
    s_mS = 0;
    s_mZ = 0;
  }
  if (dirty) {
    // rebuild both column views: clear the tile's columns, then let every
    // tile append its own rows' slots (any order: potentiation is per slot)
    if (own) {
      sd.col_len[j] = 0;
      if (LAT) sd.col_len_l[j] = 0;
    }
    tiles_arrive(sd.bar, ++target);
    if (!tiles_wait(sd.bar, target, sd.err, &s_ok)) return;
    if (own) {
      const int n = P.len[j];
      for (int s = 0; s < n; ++s) {
        const int jj = P.ind[(int64_t)j * P.cap + s];
        const int pos = atomicAdd(&sd.col_len[jj], 1);
        if (pos < sd.col_cap) sd.col_ent[(int64_t)jj * sd.col_cap + pos] = j * P.cap + s;
      }
      if (LAT) {
        const int nl = PL.len[j];
        for (int s = 0; s < nl; ++s) {
          const int jj = PL.ind[(int64_t)j * PL.cap + s];
          const int pos = atomicAdd(&sd.col_len_l[jj], 1);
          if (pos < sd.col_cap) sd.col_ent_l[(int64_t)jj * sd.col_cap + pos] = j * PL.cap + s;
        }
      }
    }
    tiles_arrive(sd.bar, ++target);
    if (!tiles_wait(sd.bar, target, sd.err, &s_ok)) return;
  }
  clf[tid] = own ? min(sd.col_len[j], sd.col_cap) : 0;
  cll[tid] = (LAT && own) ? min(sd.col_len_l[j], sd.col_cap) : 0;
  uint64_t thr[8];  // the drawing lanes' source thresholds for the current stimulus epoch
  __syncthreads();
  if (tm) tiles_mark(tk[3], tprev);

  for (int k = 0; k < n_steps; ++k) {
    const uint64_t t = t0 + (uint64_t)k;
    const int cb = k & 1;
    const uint32_t* Scur = cb ? sd.zin_b : sd.zin;
    const uint32_t* Zcur = cb ? sd.zout_b : sd.zout;
    const float* Xcur = cb ? sd.x_b : sd.x;
    const float* XLcur = cb ? sd.xl_b : sd.xl;
    uint32_t* Snxt = cb ? sd.zin : sd.zin_b;
    uint32_t* Znxt = cb ? sd.zout : sd.zout_b;
    float* Xnxt = cb ? sd.x : sd.x_b;
    float* XLnxt = cb ? sd.xl : sd.xl_b;
    // ---- A: this tile's source spikes of step t (published at C), drawn by
    // wave 1 while wave 0 waits for the step before
    const int c = (wv - 1) * WAVE + lane;  // generator call of this lane: channels j0 + 8c .. j0 + 8c + 7
    if (wv >= 1 && wv <= TT_DRAW_WAVES && c < TT_NT / 8) {
      if (k == 0 || t % (uint64_t)sd.stim_steps == 0) {
        const int cx = s_stim[0], cy = s_stim[1], orient = s_stim[2];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int i = j0 + 8 * c + b;
          thr[b] = 0;  // channels beyond the sheet never fire
          if (i < N) {
            const int dxs = axis_dist_t(Ls, (i % L) % Ls, cx), dys = axis_dist_t(Ls, (i / L) % Ls, cy);
            const int d2 = sd.stim_kind ? (orient ? dys * dys : dxs * dxs) : dxs * dxs + dys * dys;
            thr[b] = sd.T_in[d2];
          }
        }
      }
      const U64x4 o = philox(seed, (uint64_t)TAG_TP_INPUT, t, (uint64_t)((j0 >> 3) + c), 0, 0);
      const uint64_t wd[4] = {o.x0, o.x1, o.x2, o.x3};
      uint32_t byte = 0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint32_t u = (b & 1) ? (uint32_t)wd[b >> 1] : (uint32_t)(wd[b >> 1] >> 32);
        if ((uint64_t)u < thr[b]) byte |= 1u << b;
      }
      uint32_t wbits = byte << (8 * (lane & 3));  // four lanes make one word
      wbits |= __shfl_xor(wbits, 1, WAVE);
      wbits |= __shfl_xor(wbits, 2, WAVE);
      if ((lane & 3) == 0) s_sbits[c >> 2] = wbits;
    }
    if (k > 0 && !tiles_wait(sd.bar, target, sd.err, &s_ok)) return;
    if (tm) tiles_mark(tk[3], tprev);
    // ---- B: traces, lists, delivery
    if (tid == 0) s_npost = 0;
    if (own) {
      xr = xr * sd.dx + (float)bit_of(Scur, j);
      if (LAT) xlr = xlr * sd.dx + (float)bit_of(Zcur, j);
      y[tid] *= sd.dy;
    }
    list_rows(Scur, words, P.len, listS, &s_nS, &s_mS);
    if (LAT) list_rows(Zcur, words, PL.len, listZ, &s_nZ, &s_mZ);
    __syncthreads();
    deliver_rows(P, listS, s_nS, s_mS, j0, acc, y, sd);
    if (LAT) deliver_rows(PL, listZ, s_nZ, s_mZ, j0, acc, y, sd);
    __syncthreads();
    if (tm) tiles_mark(tk[0], tprev);
    // ---- C: neurons, then publish the tile's spikes and traces
    bool z = false;
    if (own) {
      const float gj = gr + (float)((double)acc[tid] * FIX_INV);
      acc[tid] = 0;
      float v = V;
      if (ref > 0) {
        ref -= 1;
        v = sd.V_reset;
      } else {
        const float I = gj * (sd.E_exc - v);
        const float RI = sd.R * I;
        v = sd.V_rest + RI + (v - sd.V_rest - RI) * sd.em;
        if (v >= sd.V_th) {
          z = true;
          v = sd.V_reset;
          ref = sd.ref_steps;
          cnt += 1u;
          post[atomicAdd(&s_npost, 1)] = tid;
        }
      }
      V = v;
      gr = gj * sd.es;
      y[tid] += z ? 1.f : 0.f;
      Xnxt[j] = xr;
      if (LAT) XLnxt[j] = xlr;
    }
    const uint64_t mz = ballot(z);
    if (lane == 0) {
      const int w0 = wb + wv * (WAVE / 32);
      if (w0 < words) Znxt[w0] = (uint32_t)mz;
      if (w0 + 1 < words) Znxt[w0 + 1] = (uint32_t)(mz >> 32);
    }
    if (tid < TT_WORDS && wb + tid < words) Snxt[wb + tid] = s_sbits[tid];
    if (tid == 0) {
      s_nS = 0;  // read in B before the barrier above
      s_nZ = 0;
      s_mS = 0;
      s_mZ = 0;
    }
    __syncthreads();
    if (tm) tiles_mark(tk[1], tprev);
    // ---- D: potentiation along the columns of the tile's spiking targets
    const int npost = s_npost;
    if (sd.stdp) {
      for (int q = wv; q < npost; q += TT_NT / WAVE) {
        const int tj = post[q];
        const int64_t jg = j0 + tj;
        potentiate_col(P, sd.col_ent + jg * sd.col_cap, clf[tj], Xcur, Scur, sd);
        if (LAT) potentiate_col(PL, sd.col_ent_l + jg * sd.col_cap, cll[tj], XLcur, Zcur, sd);
      }
    }
    // stimulus position of the next step's epoch
    if (tid < 3 && (t + 1) % (uint64_t)sd.stim_steps == 0) {
      const uint32_t u = draw_u32(seed, TAG_STIM, 0, (t + 1) / (uint64_t)sd.stim_steps, (uint64_t)tid, 0, 0);
      s_stim[tid] = tid < 2 ? (int)below(u, (uint32_t)Ls) : (int)(u & 1u);
    }
    if (tm) tiles_mark(tk[2], tprev);
    tiles_arrive(sd.bar, ++target);
  }
  // every tile has finished reading the exchange once the last step's
  // arrivals are all in; then the state goes back, the last step's exchange
  // buffer into the state arrays
  if (!tiles_wait(sd.bar, target, sd.err, &s_ok)) return;
  if (own) {
    sd.V[j] = V;
    sd.g[j] = gr;
    sd.ref[j] = ref;
    sd.count[j] = cnt;
    sd.y[j] = y[tid];
    if (n_steps & 1) {
      sd.x[j] = xr;
      if (LAT) sd.xl[j] = xlr;
    }
  }
  if ((n_steps & 1) && tid < TT_WORDS && wb + tid < words) {
    sd.zin[wb + tid] = sd.zin_b[wb + tid];
    sd.zout[wb + tid] = sd.zout_b[wb + tid];
  }
  if (blockIdx.x == 0 && tid == 0) {
    *sd.step_dev = t0 + (uint64_t)n_steps;
    if (dirty) {
      *sd.col_dirty = 0;
      if (LAT) *sd.col_dirty_l = 0;
    }
  }
  if (tm) {
    tiles_mark(tk[3], tprev);
    for (int q = 0; q < TOPO_PHASES; ++q) atomicAdd(&sd.ticks[q], (unsigned long long)tk[q]);
  }
}

static void topo_tiles_attrs() {
  static std::once_flag once;
  std::call_once(once, [] {
    allow_dynamic_lds((const void*)k_topo_tiles<false, false>, 160 * 1024);
    allow_dynamic_lds((const void*)k_topo_tiles<false, true>, 160 * 1024);
    allow_dynamic_lds((const void*)k_topo_tiles<true, false>, 160 * 1024);
    allow_dynamic_lds((const void*)k_topo_tiles<true, true>, 160 * 1024);
  });
}

int topo_tiles_resident(int N, bool lateral) {
  topo_tiles_attrs();
  int dev = 0, cus = 0, per = 0;
  const void* k = lateral ? (const void*)k_topo_tiles<true, true> : (const void*)k_topo_tiles<true, false>;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, TT_NT, topo_tiles_lds_bytes(N, lateral)) !=
          hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cus * per;
}

void launch_topo_tiles(hipStream_t s, uint64_t seed, const ProjDev& P, const ProjDev& PL, const TopoSimDev& sd,
                       uint64_t t0, int n_steps) {
  topo_tiles_attrs();
  const bool lat = PL.n_pre > 0;
  const dim3 grid(topo_tiles_grid(sd.N)), block(TT_NT);
  const size_t lds = topo_tiles_lds_bytes(sd.N, lat);
  if (sd.ticks) {
    if (lat) hipLaunchKernelGGL((k_topo_tiles<true, true>), grid, block, lds, s, seed, P, PL, sd, t0, n_steps);
    else hipLaunchKernelGGL((k_topo_tiles<true, false>), grid, block, lds, s, seed, P, PL, sd, t0, n_steps);
  } else {
    if (lat) hipLaunchKernelGGL((k_topo_tiles<false, true>), grid, block, lds, s, seed, P, PL, sd, t0, n_steps);
    else hipLaunchKernelGGL((k_topo_tiles<false, false>), grid, block, lds, s, seed, P, PL, sd, t0, n_steps);
  }
}

}  // namespace rs
