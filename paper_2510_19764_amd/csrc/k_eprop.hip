// Eligibility-trace kernels of the e-prop classifier (paper, recurrent
// classifier section; eligibility traces eq. eprop_elig_1/2 and
// eprop_elig_lif).
//
// k_eprop_*: per-synapse eligibility traces over every batch instance and the
//   batch-summed gradient G_ji += sum_b L_j ebar_ji; further workgroups
//   accumulate the readout delta rule.  State is laid out batch-innermost
//   ([slot][B], [neuron][B]) so a wave reads consecutive instances.
// k_col_*: the column view (synapses grouped by target) the target-major
//   kernel walks, rebuilt by a counting sort whenever rows change.
#include <algorithm>
#include <mutex>

#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

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
static_assert(COL_TB % 4 == 0, "the step loop runs in groups of four");
// Source groups per target: the synapses onto target j are split by row
// r % COL_GRP.  Group g's workgroups land on XCDs g and g + 4, so each XCD
// gathers presynaptic traces from a quarter of the rows; psi_j and L_j are
// fetched once per group.  Eight groups (one per XCD) fetched psi/L eight
// times; one or two groups gathered from too many rows per XCD.
constexpr int COL_GRP = 4;
static_assert(COL_GRP <= COL_GROUPS_MAX && 8 % COL_GRP == 0, "groups must divide the 8 XCDs");

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
// The spike bits of steps t .. t+3 moved to bit 0 of bytes 0 .. 3: with
// x = b0 + 2 b1 + 4 b2 + 8 b3, x * (1 + 2^7 + 2^14 + 2^21) puts b_k at bit
// k + 7m for the m-th term, sixteen distinct positions (no carries), of which
// the mask keeps 0, 8, 16 and 24.  A step's spike is then one byte conversion
// (v_cvt_f32_ubyteN).  The mask is applied in asm: seen by the compiler, the
// known-zero bits would turn those conversions back into bit extracts.
__device__ __forceinline__ uint32_t spikes4(uint32_t w, int t) {
  const uint32_t m = __umul24((w >> t) & 15u, 0x204081u);
  uint32_t r;
  __asm__("v_and_b32 %0, 0x1010101, %1" : "=v"(r) : "v"(m));
  return r;
}
template <int IPL>
__device__ __forceinline__ typename VecT<IPL>::type trace_next_byte(
    typename VecT<IPL>::type f, float alpha, unsigned __attribute__((ext_vector_type(IPL))) sp, int byte) {
#pragma unroll
  for (int e = 0; e < IPL; ++e) f[e] = fmaf(alpha, f[e], (float)((sp[e] >> (8 * byte)) & 0xFFu));
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
  // (trace, word) pairs: B % 4 == 0 there, four instances are two 16-byte loads
  const bool pairs = a.tr_es == 2;
  const auto rz = buf_rsrc(a.z0 + (int64_t)(wt ? j : 0) * B * (pairs ? 2 : 1), pairs ? 2 * step_bytes : step_bytes);
  const auto rb = buf_rsrc(a.zbits + (int64_t)(wt ? j : 0) * B * (pairs ? 2 : 1), pairs ? 2 * step_bytes : step_bytes);
  const int ipl = B % 4 == 0 ? 4 : 1;  // instances per lane
  for (int k = 0; k < a.n_out; ++k) {
    const auto rd = buf_rsrc(a.deltaT + ring(a, k, 0), blk);
    float g = 0.0f;
    for (int c = ipl * lane; c < B; c += ipl * WAVE) {
      const uint32_t off = (uint32_t)c * 4u;
      f4 z = {1.f, 1.f, 1.f, 1.f};
      v4u w = {0u, 0u, 0u, 0u};
      if (wt) {
        if (pairs) {
          const f4 p0 = buf_ldv<4>(rz, 2 * off, 0), p1 = buf_ldv<4>(rz, 2 * off + 16u, 0);
          z = (f4){p0.x, p0.z, p1.x, p1.z};
          w = (v4u){__float_as_uint(p0.y), __float_as_uint(p0.w), __float_as_uint(p1.y), __float_as_uint(p1.w)};
        } else if (ipl == 4) {
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
// to a multiple of 8 so that workgroup n_ro + COL_GRP*j + g lands on XCD
// (COL_GRP*j + g) % 8.
__host__ __device__ inline int readout_groups(int n_rec, int nw) {
  return ((n_rec + 1 + nw - 1) / nw + 7) & ~7;
}

// Target-major form (B % 4 == 0).  Workgroup n_ro + COL_GRP*j + g owns target
// neuron j and the synapses onto it from rows r with r % COL_GRP == g (r = i
// for input rows, n_in + i for recurrent rows).  Workgroups are dealt to the 8
// XCDs in turn, so an XCD only gathers the presynaptic traces of one group of
// rows, which fits its L2.  Every lane holds four consecutive instances,
// so one wave covers 256 instances of a synapse with 16-byte accesses; wave w
// takes synapses w, w + WL_NW, ... of the list.  psi_j and L_j of the block's
// steps for the current 256-instance chunk are staged once in LDS (40 KB) and
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
// One synapse's inputs to a launch: its eps/ebar records, the presynaptic
// start trace and spike mask of the lane's instances, and its gradient before
// the launch.  r = i (input row) or n_in + i (recurrent row) and
// slot = i * cap + k are wave-uniform.
template <int IPL>
struct SynIn {
  typedef typename VecT<IPL>::type V;
  typedef unsigned U __attribute__((ext_vector_type(IPL)));
  V eb, ep, pr;
  U bits;
  float g0;
  int fin, slot;
};
template <bool ALIF, int IPL>
__device__ __forceinline__ void syn_load(const EpropArgs& a, int r, int slot, uint32_t off,
                                         uint32_t step_bytes, SynIn<IPL>& s) {
  s.fin = r < a.n_in;
  s.slot = slot;
  const int i = s.fin ? r : r - a.n_in;
  const int64_t rec = (int64_t)slot * a.B;
  const auto reb = buf_rsrc((s.fin ? a.in.ebar : a.rec.ebar) + rec, step_bytes);
  s.eb = buf_ldv_nt<IPL>(reb, off);
  if (ALIF) {
    s.ep = buf_ldv_nt<IPL>(buf_rsrc((s.fin ? a.in.eps : a.rec.eps) + rec, step_bytes), off);
  } else {
#pragma unroll
    for (int e = 0; e < IPL; ++e) s.ep[e] = 0.0f;
  }
  // presynaptic trace of the block start and the block's spike bits; the
  // trace of each step is rebuilt with the forward pass's float recursion
  // F <- fma(alpha, F, spike), so it equals the forward's value
  s.pr = buf_ldv<IPL>(buf_rsrc((s.fin ? a.x0 : a.z0) + (int64_t)i * a.B, step_bytes), off, 0);
  s.bits = __builtin_bit_cast(typename SynIn<IPL>::U,
                              buf_ldv<IPL>(buf_rsrc((s.fin ? a.xbits : a.zbits) + (int64_t)i * a.B, step_bytes), off, 0));
  s.g0 = buf_ld(buf_rsrc((s.fin ? a.in.G : a.rec.G) + slot, 4u), 0u, 0u);  // every lane reads the one word
}
// Write back a synapse's traces and gradient.  The stores are unconditional:
// a lane that must not store passes an offset past the buffer's size, which
// the buffer unit drops, so the wave's memory counter stays path-independent.
template <bool ALIF, int IPL>
__device__ __forceinline__ void syn_store(const EpropArgs& a, const SynIn<IPL>& s, uint32_t soff,
                                          uint32_t step_bytes, typename VecT<IPL>::type eb,
                                          typename VecT<IPL>::type ep, float g, uint32_t goff) {
  // uniform values, restated so the address arithmetic stays scalar
  const int fin = __builtin_amdgcn_readfirstlane(s.fin), slot = __builtin_amdgcn_readfirstlane(s.slot);
  const int64_t rec = (int64_t)slot * a.B;
  buf_stv_nt<IPL>(eb, buf_rsrc((fin ? a.in.ebar : a.rec.ebar) + rec, step_bytes), soff);
  if (ALIF) buf_stv_nt<IPL>(ep, buf_rsrc((fin ? a.in.eps : a.rec.eps) + rec, step_bytes), soff);
  buf_st(g, buf_rsrc((fin ? a.in.G : a.rec.G) + slot, 4u), goff);
}

constexpr int WL_CH = 4 * WAVE;  // instances per LDS chunk
constexpr int WL_IPL = 4;  // instances per lane
// Waves per workgroup.  The 40 KB of staged psi/L are shared by the
// workgroup's waves: with 8 waves, three workgroups (24 waves) fit a CU's
// 160 KB of LDS next to a forward workgroup of the next block, where four
// 4-wave workgroups would leave it no room and lose one of the four.
constexpr int WL_NW = 8;

// IPL = 4 instances per lane: a workgroup's WL_NW waves share a chunk of 256
// instances and wave w works on synapses w, w + WL_NW, ...
template <bool ALIF, int IPL>
__global__ void __launch_bounds__(WL_NW * WAVE) k_eprop_wl(EpropArgs a) {
  typedef typename VecT<IPL>::type V;
  typedef unsigned U __attribute__((ext_vector_type(IPL)));
  static_assert(IPL == 4, "one wave covers a 256-instance chunk");
  constexpr int LPC = WL_CH / IPL;  // vectors across a chunk
  // 40 KB at 20 steps: four workgroups per CU
  __shared__ V s_psi[COL_TB][LPC], s_L[COL_TB][LPC];
  const int wv = wave_id(), lane = lane_id();
  const int nw = blockDim.x / WAVE;
  const int n_ro = readout_groups(a.n_rec, nw);
  if ((int)blockIdx.x < n_ro) {
    readout_grad(a, blockIdx.x * nw + wv, lane);
    return;
  }
  const int wg = blockIdx.x - n_ro;
  const int j = wg / COL_GRP;
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
      for (int t = sub; t < COL_TB; t += WL_NW) {
        s_psi[t][lv] = t < T ? buf_ldv<IPL>(rp, off, st_off(t)) : zero;
        s_L[t][lv] = act && t < T ? buf_ldv<IPL>(rl, off, st_off(t)) : zero;
      }
    }
    __syncthreads();
    // stores of idle lanes (instances past B) and gradient stores of all
    // lanes but 0 go past their buffer and are dropped
    const uint32_t soff = act ? off : 0x40000000u, goff = lane == 0 ? 0u : 0x40000000u;
    // one synapse: the block's steps on its loaded inputs, then the write-back
    auto run = [&](const SynIn<IPL>& in) {
      V eb = in.eb, ep = in.ep, pr = in.pr;
      for (int t = 0; t < a.tofs; ++t) pr = trace_next<IPL>(pr, alpha, in.bits, t);
      V g = zero;
      U sp;  // spikes of the current group of four steps, one per byte
#pragma unroll
      for (int t = 0; t < COL_TB; ++t) {
        // step groups of four: the launch's steps end at a group boundary
        // or inside the last group; LDS reads stay inside their group
        // (hoisted, they would cost registers, hence occupancy)
        if (t % 4 == 0) {
          if (t >= T) break;
          __asm__ volatile("" ::: "memory");
#pragma unroll
          for (int e = 0; e < IPL; ++e) sp[e] = spikes4(in.bits[e], a.tofs + t);
        }
        const V psi = s_psi[t][lv], L = s_L[t][lv];
        // decay factors (alpha, 1 - rho) for the launch's steps and (1, 0)
        // past them, where psi = L = 0 as well: padded steps change nothing
        const float da = t < T ? alpha : 1.0f, dr = t < T ? omr : 0.0f;
        // every product-sum is an explicit fma, so each unrolled copy of the
        // step rounds alike and the result does not depend on the block length
        if (ALIF) {
          const V e = psi * __builtin_elementwise_fma((V)(-beta), ep, pr);
          const V d = __builtin_elementwise_fma((V)(-dr), ep, e);
          ep = ep + d;
          eb = __builtin_elementwise_fma((V)da, eb, e);
        } else {
          eb = __builtin_elementwise_fma((V)da, eb, psi * pr);
        }
        g = __builtin_elementwise_fma(L, eb, g);
        pr = trace_next_byte<IPL>(pr, alpha, sp, t % 4);
      }
      syn_store<ALIF, IPL>(a, in, soff, step_bytes, eb, ep, in.g0 + wave_sum(hsum<IPL>(g)), goff);
    };
    for (int sc = q0; sc < q1; sc += WAVE) {  // chunks of 64 list entries
      const int ns = min(WAVE, q1 - sc);
      if (sub >= ns) break;  // only the last chunk is short
      // the chunk's list entries, one per lane; a synapse's entry is read
      // from its lane, so no memory access waits on it
      const int2 ents = a.col[sc + min(lane, ns - 1)];
      auto load = [&](int k, SynIn<IPL>& in) {
        syn_load<ALIF, IPL>(a, __builtin_amdgcn_readlane(ents.x, k), __builtin_amdgcn_readlane(ents.y, k), off,
                            step_bytes, in);
      };
      // Each synapse's inputs are loaded one synapse ahead, alternating
      // between two register sets: while the wave computes synapse k, the
      // loads of k + WL_NW are in flight, and the gradient is written back
      // without being read again.  The loads are unconditional (past the
      // list the last entry is read again and not used), so the number of
      // memory operations in flight is the same on every path and the waits
      // before a synapse's steps cover only its own loads.
      SynIn<IPL> s0, s1;
      load(sub, s0);
#pragma unroll 1
      for (int k = sub; k < ns; k += 2 * WL_NW) {
        load(min(k + WL_NW, ns - 1), s1);
        run(s0);
        if (k + WL_NW >= ns) break;
        load(min(k + 2 * WL_NW, ns - 1), s0);
        run(s1);
      }
    }
  }
}

// Transfer-coefficient form of the same block (eq. eprop_elig_1/2,
// eprop_elig_lif), one lane per instance.  Within a block the recursions
//   e_t = psi_t (p_t - beta eps_{t-1}),  eps_t = e_t + rho eps_{t-1},
//   ebar_t = alpha ebar_{t-1} + e_t,     g += L_t ebar_t,
//   p_{t+1} = alpha p_t + z_t
// are linear in a synapse's start state (p_0, eps_{-1}, ebar_{-1}) and its
// presynaptic spikes z_t, with coefficients that depend only on the target's
// psi_t and L_t.  A workgroup computes them once for its target and 128
// instances by the adjoint recursion backwards over the block (the gradient,
// ebar at the block end and eps at the block end; for eps the decay product
// is carried as 1 - D, so the slow decay keeps full precision) into LDS.  A
// synapse then costs three multiply-adds per instance for its start state and
// three adds per presynaptic spike of the block: the wave walks the spikes of
// its lanes, lowest step first, for as many rounds as its busiest lane has
// spikes, and lanes without a spike left read a row of zeros.  The results
// equal the step-by-step recursion up to float rounding.
//
// Workgroup n_ro + k owns target j = k / n_ch and instances 128 c .. 128 c +
// 127 (two per lane), c = k % n_ch: with two chunks the XCDs of one parity
// serve one chunk, so the presynaptic traces an XCD gathers are half of all of
// them.  Its TC_NW waves take the target's synapses in turn, each with the
// inputs of its next two synapses in flight.  With one chunk the workgroup
// adds a synapse's gradient to G; with more, each chunk adds its part to an
// array of its own by list position (coalesced, where G's slots are
// scattered), and k_gx_fold adds the arrays to G in chunk order before the
// parameter update, so the sums do not depend on scheduling.
constexpr int TC_NW = 8;
constexpr int TC_IPL = 2;                 // instances per lane
constexpr int TC_CH = TC_IPL * WAVE;      // instances per chunk
constexpr int TC_TB = 31;                 // steps per launch: below the top bit of a 32-bit spike mask
constexpr int TC_MIN_B = 32;  // below, most lanes would idle: the 4-instances-per-lane kernel serves
typedef float tcv __attribute__((ext_vector_type(2)));
typedef unsigned tcu __attribute__((ext_vector_type(2)));
// LDS of a launch of T steps: the coefficients of z_t for the three outputs,
// T rows and a row of zeros each (the first two hold L and psi while the
// coefficients are computed), then those of the start state.
__host__ __device__ inline size_t tc_lds_bytes(int T, bool alif) {
  return ((size_t)(alif ? 3 : 2) * (T + 1) + 8) * TC_CH * sizeof(float);
}
template <bool ALIF>
__global__ void __launch_bounds__(TC_NW * WAVE) k_eprop_tc(EpropArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = lane_id(), wv = wave_id();
  const int n_ro = readout_groups(a.n_rec, TC_NW);
  if ((int)blockIdx.x < n_ro) {
    readout_grad(a, blockIdx.x * TC_NW + wv, lane);
    return;
  }
  const int B = a.B, T = a.nsteps;
  // coefficients of z_t: step t's rows for the gradient (L while staging),
  // ebar at the block end (psi while staging) and eps at the block end (ALIF)
  // side by side, so one address serves all three; row T is zeros
  constexpr int NA = ALIF ? 3 : 2;
  float* c_z = (float*)smem;                    // [T + 1][NA][TC_CH]
  float* c_k = c_z + (T + 1) * NA * TC_CH;      // [8][TC_CH] gradient: p0, eps, ebar; ebar: p0, eps, ebar; eps: p0, D
  auto cz = [&](int t, int r, int e) -> float& { return c_z[(t * NA + r) * TC_CH + e]; };
  const int n_ch = (B + TC_CH - 1) / TC_CH;
  const int k = blockIdx.x - n_ro;
  const int j = k / n_ch, c = k - j * n_ch;
  const int q0 = a.col_off[j * COL_GRP], q1 = a.col_off[(j + 1) * COL_GRP];
  if (q1 <= q0) return;
  const int b0 = c * TC_CH + TC_IPL * lane;  // this lane's first instance (B is a multiple of 4)
  const bool act = b0 < B;
  const int bi = act ? b0 : B - TC_IPL;      // idle lanes compute on valid instances and store nothing
  const float alpha = a.alpha, beta = a.beta, omr = a.one_m_rho;

  // ---- L and psi of the block for target j and the chunk's instances
  for (int t = wv; t < T; t += TC_NW)
    for (int e = lane; e < TC_CH; e += WAVE) {
      const int be = min(c * TC_CH + e, B - 1);
      cz(t, 0, e) = a.LT[ring(a, j, t) + be];
      cz(t, 1, e) = a.psiT[ring(a, j, t) + be];
    }
  __syncthreads();
  // ---- coefficients, one instance e per lane of waves 0 and 1: the adjoints
  // after step t, A = d out / d eps_t and Bv = d out / d ebar_t, backwards
  // over the block, and P = sum over t' >= t of alpha^(t'-t) d out / d p_t'.
  // The coefficient of z_t is P_{t+1}; slot t of the arrays is written after
  // its L and psi are read, by the same lane.
  if (wv < TC_IPL) {
    const int e = wv * WAVE + lane;
    for (int r = 0; r < NA; ++r) cz(T, r, e) = 0.f;  // read for lanes without a spike left
    float Ag = 0.f, Bg = 0.f, Pg = 0.f;  // gradient
    float Ab = 0.f, Bb = 0.f, Pb = 0.f;  // ebar at the block end
    float De = 0.f, Pe = 0.f;            // eps at the block end: A = 1 - De
    for (int t = T - 1; t >= 0; --t) {
      const float l = cz(t, 0, e), p = cz(t, 1, e);
      cz(t, 0, e) = Pg;
      cz(t, 1, e) = Pb;
      if (ALIF) cz(t, 2, e) = Pe;
      Bg = fmaf(alpha, Bg, l);
      Bb = t == T - 1 ? 1.f : alpha * Bb;
      if (ALIF) {
        const float del = fmaf(beta, p, omr);  // 1 - (rho - beta psi_t)
        const float pb = p * beta;
        Pg = fmaf(alpha, Pg, p * (Ag + Bg));
        Pb = fmaf(alpha, Pb, p * (Ab + Bb));
        Pe = fmaf(alpha, Pe, p * (1.f - De));
        Ag = fmaf(-pb, Bg, fmaf(-Ag, del, Ag));
        Ab = fmaf(-pb, Bb, fmaf(-Ab, del, Ab));
        De = fmaf(-De, del, De + del);
      } else {
        Pg = fmaf(alpha, Pg, p * Bg);
        Pb = fmaf(alpha, Pb, p * Bb);
      }
    }
    c_k[0 * TC_CH + e] = Pg;
    c_k[1 * TC_CH + e] = Ag;
    c_k[2 * TC_CH + e] = alpha * Bg;
    c_k[3 * TC_CH + e] = Pb;
    c_k[4 * TC_CH + e] = Ab;
    c_k[5 * TC_CH + e] = alpha * Bb;
    c_k[6 * TC_CH + e] = Pe;
    c_k[7 * TC_CH + e] = De;
  }
  __syncthreads();
  auto kv = [&](int r) { return *(const tcv*)(c_k + r * TC_CH + TC_IPL * lane); };
  const tcv kg0 = kv(0), kg1 = kv(1), kg2 = kv(2), kb0 = kv(3), kb1 = kv(4), kb2 = kv(5);
  const tcv ke0 = ALIF ? kv(6) : (tcv)0.f, ke1 = ALIF ? kv(7) : (tcv)0.f;
  const float* czl = c_z + TC_IPL * lane;  // this lane's instances of step t at [t * NA * TC_CH + r * TC_CH] (+1)
  const uint32_t tmask = (1u << T) - 1u, sent = 1u << T;  // the launch's steps in the spike words; past them

  // ---- the target's synapses: wave wv takes list entries q0 + wv, q0 + wv + TC_NW, ...
  // Records are addressed from a wave-uniform base plus this lane's offset.
  struct In {
    tcv eb, ep, pr;
    tcu bits;
    int fin, slot, n;
  };
  // list entries of the wave's next 64 synapses, one per lane, read by
  // readlane so that no load waits on another
  int2 ents;
  int base = 0;
  // the batch's gradients, one synapse per lane: the chunk's sum before this
  // launch and this launch's part, gathered as the synapses run and stored
  // once per batch
  float gbat = 0.f, gacc = 0.f;
  float* const gpos = n_ch > 1 ? a.gx + (int64_t)c * a.n_col : nullptr;
  auto load = [&](int n, In& s) {
    const int r = __builtin_amdgcn_readlane(ents.x, n), slot = __builtin_amdgcn_readlane(ents.y, n);
    s.fin = r < a.n_in;
    s.slot = slot;
    s.n = n;
    const int i = s.fin ? r : r - a.n_in;
    const int64_t rec = (int64_t)slot * B + bi;
    const float* el = s.fin ? a.in.ebar : a.rec.ebar;
    if (ALIF) {  // ebar and eps of the lane's two instances, interleaved: one 16-byte record
      const f4 v = __builtin_nontemporal_load((const f4*)(el + 2 * rec));
      s.eb = (tcv){v.x, v.z};
      s.ep = (tcv){v.y, v.w};
    } else {
      s.eb = __builtin_nontemporal_load((const tcv*)(el + rec));
      s.ep = (tcv)0.f;
    }
    // the lane's two instances' block-start traces and spike words: one 16-byte (trace, word) pair record
    const f4 tb = *(const f4*)((s.fin ? a.x0 : a.z0) + ((int64_t)i * B + bi) * 2);
    s.pr = (tcv){tb.x, tb.z};
    s.bits = (tcu){__float_as_uint(tb.y), __float_as_uint(tb.w)};
  };
  auto run = [&](const In& s) {
    tcv pr = s.pr;
    for (int t = 0; t < a.tofs; ++t) {
      const tcv sp = {(float)((s.bits.x >> t) & 1u), (float)((s.bits.y >> t) & 1u)};
      pr = __builtin_elementwise_fma((tcv)alpha, pr, sp);
    }
    tcv g = __builtin_elementwise_fma(kg0, pr, ALIF ? __builtin_elementwise_fma(kg1, s.ep, kg2 * s.eb) : kg2 * s.eb);
    tcv eb = __builtin_elementwise_fma(kb0, pr, ALIF ? __builtin_elementwise_fma(kb1, s.ep, kb2 * s.eb) : kb2 * s.eb);
    tcv ep = ALIF ? __builtin_elementwise_fma(ke0, pr, __builtin_elementwise_fma(-ke1, s.ep, s.ep)) : (tcv)0.f;
    // the block's spikes, lowest step first; z_t = 1 adds the coefficients of step t
    uint32_t mx = (s.bits.x >> a.tofs) & tmask, my = (s.bits.y >> a.tofs) & tmask;
    if (ballot((mx | my) != 0u)) do {
      const float* zx = czl + __builtin_ctz(mx | sent) * (NA * TC_CH);  // row T (zeros) once mx is empty
      const float* zy = czl + __builtin_ctz(my | sent) * (NA * TC_CH) + 1;
      g.x += zx[0];
      g.y += zy[0];
      eb.x += zx[TC_CH];
      eb.y += zy[TC_CH];
      if (ALIF) {
        ep.x += zx[2 * TC_CH];
        ep.y += zy[2 * TC_CH];
      }
      mx &= mx - 1u;
      my &= my - 1u;
    } while (ballot((mx | my) != 0u));
    const int fin = __builtin_amdgcn_readfirstlane(s.fin), slot = __builtin_amdgcn_readfirstlane(s.slot);
    const int64_t rec = (int64_t)slot * B + bi;
    if (act) {
      float* el = fin ? a.in.ebar : a.rec.ebar;
      if (ALIF) __builtin_nontemporal_store((f4){eb.x, ep.x, eb.y, ep.y}, (f4*)(el + 2 * rec));
      else __builtin_nontemporal_store(eb, (tcv*)(el + rec));
    }
    const float part = wave_sum(act ? g.x + g.y : 0.f);
    gacc = lane == s.n ? part : gacc;
  };
  // three register sets in turn: while a synapse runs, the next two load
  // (past the batch the last entry is loaded again and not used)
  In s0, s1, s2;
  for (base = q0 + wv; base < q1; base += TC_NW * WAVE) {
    const int nb = min(WAVE, (q1 - 1 - base) / TC_NW + 1);  // this wave's synapses in the batch
    ents = a.col[base + TC_NW * min(lane, nb - 1)];
    const bool efin = ents.x < a.n_in;
    float* const gl = gpos ? gpos + base + TC_NW * min(lane, nb - 1) : (efin ? a.in.G : a.rec.G) + ents.y;
    gbat = *gl;
    load(0, s0);
    load(min(1, nb - 1), s1);
#pragma unroll 1
    for (int i = 0;;) {
      load(min(i + 2, nb - 1), s2);
      run(s0);
      if (++i >= nb) break;
      load(min(i + 2, nb - 1), s0);
      run(s1);
      if (++i >= nb) break;
      load(min(i + 2, nb - 1), s1);
      run(s2);
      if (++i >= nb) break;
    }
    if (lane < nb) *gl = gbat + gacc;
  }
}

// The chunks' gradients of every listed synapse added to its G in chunk
// order and cleared (each slot is listed once).
__global__ void __launch_bounds__(256) k_gx_fold(EpropArgs a, int n_ch) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= a.col_off[a.n_rec * COL_GRP]) return;
  const int2 e = a.col[q];
  float* G = (e.x < a.n_in ? a.in.G : a.rec.G) + e.y;
  float g = *G;
  for (int c = 0; c < n_ch; ++c) {
    g += a.gx[(int64_t)c * a.n_col + q];
    a.gx[(int64_t)c * a.n_col + q] = 0.0f;
  }
  *G = g;
}

void launch_gx_fold(hipStream_t s, const EpropArgs& a) {
  if (!a.gx || a.n_col <= 0) return;
  const int n_ch = (a.B + TC_CH - 1) / TC_CH;
  hipLaunchKernelGGL(k_gx_fold, dim3((a.n_col + 255) / 256), dim3(256), 0, s, a, n_ch);
}

// Column view of both projections for k_eprop_wl: entries
// col[col_off[j*G+g] .. col_off[j*G+g+1]) (G = COL_GRP) are (r, slot) of every
// synapse of a row r with r % G == g onto target j.  Rebuilt whenever rows change; the
// order inside a list is arbitrary.
__global__ void __launch_bounds__(WAVE) k_col_count(ProjDev in, ProjDev rec, int* cnt) {
  const int r = blockIdx.x;
  const bool fin = r < in.n_pre;
  const ProjDev& P = fin ? in : rec;
  const int i = fin ? r : r - in.n_pre;
  const int n = P.len[i];
  const int64_t base = (int64_t)i * P.cap;
  for (int k = lane_id(); k < n; k += WAVE) atomicAdd(&cnt[P.ind[base + k] * COL_GRP + r % COL_GRP], 1);
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
    const int pos = atomicAdd(&cur[P.ind[base + k] * COL_GRP + r % COL_GRP], 1);
    col[pos] = make_int2(r, (int)(base + k));
  }
}

void launch_columns(hipStream_t s, const ProjDev& in, const ProjDev& rec, const ColumnView& cv) {
  const int n = rec.n_post * COL_GRP;
  launch_fill_zero(s, cv.cnt, (size_t)n * 4);
  hipLaunchKernelGGL(k_col_count, dim3(in.n_pre + rec.n_pre), dim3(WAVE), 0, s, in, rec, cv.cnt);
  hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(1024), 0, s, cv.cnt, cv.off, n);
  hipLaunchKernelGGL(k_col_fill, dim3(in.n_pre + rec.n_pre), dim3(WAVE), 0, s, in, rec, cv.cnt, cv.col);
}

// Narrow form (B % 4 != 0): threads over a row's synapses, each looping over
// instances and steps; used for small or odd batches such as single-instance
// learning.  Same trace recursion and arithmetic as the target-major form.
// Narrow kernel, for any batch size: a row's synapses are spread over `nsub`
// threads (thread `sub` takes slots sub, sub + nsub, ...), each looping over
// the batch instances and the block's steps; the readout delta rule runs on
// further workgroups, one thread per readout column j (j = n_rec: the bias).
template <bool ALIF>
__device__ __forceinline__ void narrow_row(const EpropArgs& a, const int row, const int sub, const int nsub) {
  const int B = a.B;
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
  if (B == 1 && a.nslot % 4 == 0 && a.slot0 % 4 == 0) {
    // One instance: psi_j and L_j of the block's steps are contiguous in the
    // ring, so they are read four steps at a time, the next four loaded while
    // the current ones are applied; each step's arithmetic is the one below.
    for (int k = sub; k < n; k += nsub) {
      const int64_t s = (int64_t)i * cap + k;
      const int j = ind[s];
      const f4* ps = (const f4*)(a.psiT + (int64_t)j * a.nslot + a.slot0);
      const f4* ls = (const f4*)(a.LT + (int64_t)j * a.nslot + a.slot0);
      float p = x0[0];
      const uint32_t w = bits[0];
      for (int t = 0; t < a.tofs; ++t) p = fmaf(a.alpha, p, (float)((w >> t) & 1u));
      float ep = ALIF ? eps[s] : 0.0f, eb = ebar[s], gsum = 0.0f;
      const int nq = (a.nsteps + 3) / 4;
      f4 pv = ps[0], lv = ls[0];
      for (int q = 0; q < nq; ++q) {
        const f4 pc = pv, lc = lv;
        if (q + 1 < nq) {
          pv = ps[q + 1];
          lv = ls[q + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int tau = 4 * q + u;
          if (tau >= a.nsteps) break;
          const float psi = pc[u];
          if (ALIF) {
            const float e = psi * fmaf(-a.beta, ep, p);
            const float d = fmaf(-a.one_m_rho, ep, e);
            ep = ep + d;
            eb = fmaf(a.alpha, eb, e);
          } else {
            eb = fmaf(a.alpha, eb, psi * p);
          }
          gsum = fmaf(lc[u], eb, gsum);
          p = fmaf(a.alpha, p, (float)((w >> (a.tofs + tau)) & 1u));
        }
      }
      if (ALIF) eps[s] = ep;
      ebar[s] = eb;
      G[s] += gsum;
    }
    return;
  }
  for (int k = sub; k < n; k += nsub) {
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
          const float e = psi * fmaf(-a.beta, ep, p);
          const float d = fmaf(-a.one_m_rho, ep, e);
          ep = ep + d;
          eb = fmaf(a.alpha, eb, e);
        } else {
          eb = fmaf(a.alpha, eb, psi * p);
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

__device__ __forceinline__ void narrow_readout(const EpropArgs& a, const int chunk, const int tid) {
  const int B = a.B;
  const int j = chunk * EP_NT + tid;
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
}

template <bool ALIF>
__global__ void __launch_bounds__(EP_NT) k_eprop_narrow(EpropArgs a) {
  const int row = blockIdx.x, n_rows = a.n_in + a.n_rec;
  if (row >= n_rows) narrow_readout(a, row - n_rows, threadIdx.x);
  else narrow_row<ALIF>(a, row, threadIdx.x, EP_NT);
}

// The narrow kernel for several networks, persistent: workgroups stride over
// a work list of row tiles (network work[g].x, rows work[g].y ..
// work[g].y + work[g].z - 1; rows from n_in + n_rec on are readout chunks).
// TPR threads share a row: 256 gives a row the whole workgroup, 64 a wave
// (four rows of the tile at a time).  Every synapse is computed exactly as in
// the one-network kernel, whatever the schedule.
template <bool ALIF, int TPR>
__global__ void __launch_bounds__(EP_NT) k_eprop_narrow_multi(const EpropArgs* __restrict__ A,
                                                              const int4* __restrict__ work, int n_work) {
  const int tid = threadIdx.x;
  for (int g = blockIdx.x; g < n_work; g += gridDim.x) {
    const int4 w = work[g];
    const EpropArgs a = A[w.x];
    const int n_rows = a.n_in + a.n_rec;
    if (w.y >= n_rows) {
      narrow_readout(a, w.y - n_rows, tid);
      continue;
    }
    const int end = min(w.y + w.z, n_rows);
    for (int r = w.y + tid / TPR; r < end; r += EP_NT / TPR) narrow_row<ALIF>(a, r, tid % TPR, TPR);
  }
}

int narrow_readout_chunks(int n_rec) { return (n_rec + 1 + EP_NT - 1) / EP_NT; }

void launch_eprop_narrow_multi(hipStream_t s, const EpropArgs* A, const int4* work, int n_work, bool alif, int tpr,
                               int grid) {
  if (n_work <= 0) return;
  const int g = grid > 0 && grid < n_work ? grid : n_work;
  if (tpr == 64) {
    if (alif) hipLaunchKernelGGL((k_eprop_narrow_multi<true, 64>), dim3(g), dim3(EP_NT), 0, s, A, work, n_work);
    else hipLaunchKernelGGL((k_eprop_narrow_multi<false, 64>), dim3(g), dim3(EP_NT), 0, s, A, work, n_work);
  } else {
    if (alif) hipLaunchKernelGGL((k_eprop_narrow_multi<true, EP_NT>), dim3(g), dim3(EP_NT), 0, s, A, work, n_work);
    else hipLaunchKernelGGL((k_eprop_narrow_multi<false, EP_NT>), dim3(g), dim3(EP_NT), 0, s, A, work, n_work);
  }
}

static void tc_attrs() {
  static std::once_flag once;
  std::call_once(once, [] {
    allow_dynamic_lds((const void*)k_eprop_tc<true>, (int)tc_lds_bytes(TC_TB, true) + 1024);
    allow_dynamic_lds((const void*)k_eprop_tc<false>, (int)tc_lds_bytes(TC_TB, false) + 1024);
  });
}

void eprop_default_schedule(int B, uint32_t update_interval, int* K, int* K0) {
  *K = *K0 = eprop_default_block(B, update_interval);
  const uint32_t U = update_interval;
  if (B % 4 != 0 || B < TC_MIN_B || U <= (uint32_t)TC_TB) return;
  // The first block of an interval is short (a tenth of it), so the first
  // e-prop launch, which waits for that block's forward pass and readout,
  // starts early; the rest of the interval in equal blocks of at most TC_TB
  // steps.  As many launches as equal blocks would take.
  const uint32_t nb = (U + TC_TB - 1) / TC_TB;
  const uint32_t k0 = std::min<uint32_t>((U + 5) / 10, (uint32_t)*K);  // a block holds at most 31 steps
  const uint32_t k = (U - k0 + nb - 2) / (nb - 1);
  if (k > (uint32_t)TC_TB || k0 < 1) return;
  *K = (int)k;
  *K0 = (int)k0;
}

int eprop_default_block(int B, uint32_t update_interval) {
  if (B % 4 != 0 || B < TC_MIN_B) return COL_TB;
  // the update interval in equal blocks of at most TC_TB steps: each launch
  // streams every synapse's eps/ebar once, so fewer, longer blocks move fewer bytes
  if (update_interval == 0) return TC_TB;
  const uint32_t n = (update_interval + TC_TB - 1) / TC_TB;
  return (int)((update_interval + n - 1) / n);
}

bool eprop_tc_path(int B) { return B % 4 == 0 && B >= TC_MIN_B; }
bool eprop_interleaved(int B, bool alif) { return alif && eprop_tc_path(B); }

void launch_eprop(hipStream_t s, const EpropArgs& a) {
  if (a.nsteps <= 0) return;
  if (a.B % 4 == 0 && a.col && a.col_off && a.B >= TC_MIN_B) {
    tc_attrs();
    const int n_ch = (a.B + TC_CH - 1) / TC_CH;
    const int blocks = readout_groups(a.n_rec, TC_NW) + a.n_rec * n_ch;
    for (int t0 = 0; t0 < a.nsteps; t0 += TC_TB) {  // blocks longer than TC_TB in parts
      EpropArgs p = a;
      p.slot0 = a.slot0 + t0;
      p.tofs = a.tofs + t0;
      p.nsteps = min(TC_TB, a.nsteps - t0);
      const size_t lds = tc_lds_bytes(p.nsteps, a.alif);
      if (a.alif) hipLaunchKernelGGL((k_eprop_tc<true>), dim3(blocks), dim3(TC_NW * WAVE), lds, s, p);
      else hipLaunchKernelGGL((k_eprop_tc<false>), dim3(blocks), dim3(TC_NW * WAVE), lds, s, p);
    }
  } else if (a.B % 4 == 0 && a.col && a.col_off) {
    const int nw = WL_NW;
    const int blocks = readout_groups(a.n_rec, nw) + a.n_rec * COL_GRP;
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
    const int extra = narrow_readout_chunks(a.n_rec);
    if (a.alif) hipLaunchKernelGGL(k_eprop_narrow<true>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
    else hipLaunchKernelGGL(k_eprop_narrow<false>, dim3(n_rows + extra), dim3(EP_NT), 0, s, a);
  }
}

}  // namespace rs
