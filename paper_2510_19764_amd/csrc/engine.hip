// Host engine behind the C-ABI of include/ragsnn.h: argument validation,
// device memory plan, build sequence, timestep loop and snapshot access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ragsnn.h"
#include "rs_device.hpp"
#include "rs_host_rng.hpp"
#include "rs_kernels.hpp"

using namespace rs;

namespace {

thread_local std::string g_err;
// The object of the call in progress on this thread: a device error marks it
// unusable (sticky RS_EDEVICE).
thread_local bool* g_dead = nullptr;

rs_status fail(rs_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  if (code == RS_EDEVICE && g_dead) *g_dead = true;
  return code;
}

// Entry of a call on an object: refuses an object an earlier device error
// left unusable, and lets fail() mark this one for the call's duration.
struct CallScope {
  bool* prev;
  explicit CallScope(bool* dead) : prev(g_dead) { g_dead = dead; }
  ~CallScope() { g_dead = prev; }
};
#define ENTER(obj)                                                                                  \
  if (!(obj)) return fail(RS_EINVAL, "NULL object");                                                \
  if ((obj)->dead) return fail(RS_EDEVICE, "an earlier device error left this object unusable"); \
  CallScope call_scope_(&(obj)->dead)

#define HIP_OK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(RS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

uint64_t threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return 1ull << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

// Device allocation list owned by one object: through the caller's
// allocator when one was given (rs_create), else hipMalloc.
struct Arena {
  std::vector<void*> ptrs;
  uint64_t bytes = 0;
  rs_alloc_fn afn = nullptr;
  rs_free_fn ffn = nullptr;
  void* user = nullptr;
  void* raw(size_t b) {
    void* q = nullptr;
    if (afn) return afn(b, user);
    if (hipMalloc(&q, b) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return q;
  }
  void raw_free(void* q) {
    if (ffn) ffn(q, user);
    else (void)hipFree(q);
  }
  template <class T>
  rs_status alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) return RS_OK;
    size_t b = (n * sizeof(T) + 255) & ~(size_t)255;
    void* q = raw(b);
    if (!q) return fail(RS_ENOMEM, "device allocation of %zu bytes failed", b);
    ptrs.push_back(q);
    bytes += b;
    *p = (T*)q;
    return RS_OK;
  }
  void release() {
    for (void* q : ptrs) raw_free(q);
    ptrs.clear();
    bytes = 0;
  }
};

#define TRY(expr)                 \
  do {                            \
    rs_status st_ = (expr);       \
    if (st_ != RS_OK) return st_; \
  } while (0)

struct PhaseTimer {
  int mask = 0;  // phases being timed
  std::vector<hipEvent_t> pool;
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> open;
  double ms[RS_NUM_PHASES] = {0};
  uint64_t count[RS_NUM_PHASES] = {0};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    // timing only: no system-scope fence at the records
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
  }
  bool armed = false;  // the last begin() recorded an event
  void begin(hipStream_t s, int phase) {
    armed = (mask >> phase) & 1;
    if (!armed) return;
    Rec r{phase, get(), get()};
    (void)hipEventRecord(r.a, s);
    open.push_back(r);
  }
  void end(hipStream_t s) {
    if (!armed) return;
    (void)hipEventRecord(open.back().b, s);
    armed = false;
  }
  void collect() {
    for (auto& r : open) {
      float t = 0.f;
      (void)hipEventSynchronize(r.b);
      (void)hipEventElapsedTime(&t, r.a, r.b);
      ms[r.phase] += t;
      count[r.phase] += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    open.clear();
  }
  void destroy() {
    collect();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

}  // namespace

constexpr int RING_MAX = 8;  // hand-off ring segments at most

struct rs_custom_state;
void delete_custom(rs_custom_state* c);

struct rs_eprop {
  rs_eprop_params p;
  hipStream_t stream = nullptr;
  int B = 0;
  Arena arena;
  ProjDev in{}, rec{};
  ColumnView cv{};                                    // target-major view of both projections
  double *V = nullptr, *A = nullptr, *Y = nullptr;   // fp64 neuron and readout state
  float *xbar = nullptr, *zbar = nullptr;             // presynaptic traces [B][n]
  // Hand-off from the forward kernel to the e-prop kernel: a ring of Q
  // segments of K step slots, laid out [n][Q*K][B].  Steps are grouped in
  // blocks of K; the forward pass fills one segment while e-prop launches read
  // earlier ones.  With a segment per block of an update interval (plus one),
  // the forward stream never waits for an e-prop launch inside an interval:
  // the join at each update covers them all.
  float *psiT = nullptr, *LT = nullptr, *deltaT = nullptr;
  // per segment: traces at the block start and the block's spike bits, [Q][n][B]
  // each, or (tr_es = 2, the transfer-coefficient kernel) [Q][n][B][2] with a
  // trace and its spike word side by side (xbitsT = x0T + 1 word, and so on)
  float *x0T = nullptr, *z0T = nullptr;
  uint32_t *xbitsT = nullptr, *zbitsT = nullptr;
  int tr_es = 1;
  // the forward kernel's coalesced staging of a block, one per ring segment,
  // so that a block's transpose can run beside the next block's forward pass
  uint32_t *stg[HANDOFF_ARRAYS] = {};                 // psi [Q][K][B][NR]; x0, z0, xbits, zbits [Q][B][n]
  float *u_stg = nullptr;                             // readout drive [Q segments][K][B][n_out]
  int K = 8, Q = 2, nslot = 16;
  int K0 = 8;  // the first block of an update interval, under automatic updates
  int blk_seg = 0, blk_n = 0, last_slot = 0;
  int last_seg = 0, last_blk_n = 0;                   // the most recently run block
  uint64_t blk_t0 = 0;
  bool blk_learn = false;
  hipStream_t side = nullptr;                         // e-prop / update / rewire stream
  // each block's hand-off transpose and readout, beside the next forward
  // block; at updates the input-projection rewire, beside the recurrent one
  hipStream_t side2 = nullptr;
  bool single = false;                                // small network: everything on the caller's stream
  bool auto_upd = false;                              // inside a step call with RS_AUTO_UPDATE
  hipEvent_t ev_fwd = nullptr, ev_post = nullptr, ev_ep[RING_MAX] = {}, ev_join = nullptr, ev_back = nullptr;
  hipEvent_t ev_loop = nullptr;  // the update boundary's join back to the forward stream
  hipEvent_t ev_upd = nullptr, ev_rw = nullptr;
  bool ep_pending[RING_MAX] = {};  // an e-prop launch reading the segment may still run
  uint8_t* z = nullptr;
  float *Wout = nullptr, *bout = nullptr, *Gout = nullptr, *Gb = nullptr;
  float *Mout = nullptr, *Vout = nullptr, *Mb = nullptr, *Vb = nullptr;
  unsigned long long* counters = nullptr;  // [0] events, [1] spikes
  long long* rw_stats = nullptr;           // [4] DEEP R eliminated, formed, activations distributed,
                                           // activations without a row, since creation
  uint32_t* zcount = nullptr;              // [B][n_rec] spikes per neuron
  const int32_t *x_off = nullptr, *x_idx = nullptr, *labels = nullptr;
  long long n_idx = 0;
  // Poisson input source (instead of a raster): per-step Bernoulli thresholds
  // and the forward kernel's per-block spike lists [K][B][n_in]
  bool poisson = false;
  uint64_t* x_thr = nullptr;               // [B][n_in] capacity
  int x_thr_stride = 0;                    // 0: one table for every instance, n_in: per instance
  int32_t* x_list = nullptr;
  uint64_t step = 0;
  uint32_t adam_k = 0;
  double alpha = 0.0, rho = 0.0, beta = 0.0;  // decay factors exp(-dt/tau) in double
  PhaseTimer timer;
  struct rs_custom_state* custom = nullptr;  // scratch of custom connectivity updates
  bool dead = false;  // a device error occurred: every later call fails with RS_EDEVICE
};

namespace {

rs_status alloc_proj(Arena& ar, ProjDev& P, int B, bool alif, bool deepr, bool interleave) {
  const size_t n = (size_t)P.n_pre * P.cap;
  TRY(ar.alloc(&P.len, (size_t)P.n_pre));
  TRY(ar.alloc(&P.ind, n));
  TRY(ar.alloc(&P.w, n));
  TRY(ar.alloc(&P.m, n));
  TRY(ar.alloc(&P.v, n));
  TRY(ar.alloc(&P.G, n));
  P.erec = alif && interleave ? 2 * B : B;
  TRY(ar.alloc(&P.ebar, n * P.erec));
  if (alif && !interleave) TRY(ar.alloc(&P.eps, n * B));
  TRY(ar.alloc(&P.dormant, (size_t)P.n_pre));
  TRY(ar.alloc(&P.assigned, (size_t)P.n_pre));
  if (deepr) {
    TRY(ar.alloc(&P.conn, (size_t)P.n_pre * P.words));
    TRY(ar.alloc(&P.sign, (size_t)P.n_pre * P.words));
  }
  return RS_OK;
}

void zero_proj_state(hipStream_t s, const ProjDev& P, int B) {
  const size_t n = (size_t)P.n_pre * P.cap;
  launch_fill_zero(s, P.m, n * 4);
  launch_fill_zero(s, P.v, n * 4);
  launch_fill_zero(s, P.G, n * 4);
  launch_fill_zero(s, P.ebar, n * P.erec * 4);
  if (P.eps) launch_fill_zero(s, P.eps, n * B * 4);
  launch_fill_zero(s, P.dormant, (size_t)P.n_pre * 4);
  launch_fill_zero(s, P.assigned, (size_t)P.n_pre * 4);
}

// Count rows on the device, return the longest.
rs_status count_rows(Arena& ar, hipStream_t s, uint64_t seed, ProjDev& P, uint64_t T, int* max_len) {
  int* d_len = (int*)ar.raw(((size_t)P.n_pre * sizeof(int) + 255) & ~(size_t)255);
  if (!d_len) return fail(RS_ENOMEM, "device allocation for row counts failed");
  ProjDev tmp = P;
  tmp.len = d_len;
  tmp.cap = 0;
  launch_fixed_rows(s, seed, tmp, T, 0.0, false);
  std::vector<int> h(P.n_pre);
  hipError_t e = hipMemcpyAsync(h.data(), d_len, sizeof(int) * P.n_pre, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ar.raw_free(d_len);
  if (e != hipSuccess) return fail(RS_EDEVICE, "row count: %s", hipGetErrorString(e));
  *max_len = P.n_pre ? *std::max_element(h.begin(), h.end()) : 0;
  return RS_OK;
}

rs_status validate(const rs_eprop_params* p) {
  if (!p) return fail(RS_EINVAL, "params is NULL");
  if (p->n_in < 1 || p->n_in > 8192) return fail(RS_EINVAL, "n_in must be in 1..8192");
  if (p->n_rec < 1 || p->n_rec > 8192) return fail(RS_EINVAL, "n_rec must be in 1..8192");
  if (p->n_out < 1 || p->n_out > 256) return fail(RS_EINVAL, "n_out must be in 1..256");
  if (p->batch < 1 || p->batch > 65536) return fail(RS_EINVAL, "batch must be in 1..65536");
  if (!(p->dt_ms > 0) || !(p->tau_mem_ms > 0) || !(p->tau_adapt_ms > 0) || !(p->v_thr > 0))
    return fail(RS_EINVAL, "time constants, dt and v_thr must be positive");
  if (!(p->p_in >= 0 && p->p_in <= 1) || !(p->p_rec >= 0 && p->p_rec <= 1))
    return fail(RS_EINVAL, "connection probabilities must be in [0, 1]");
  if (p->deepr_mask > 3) return fail(RS_EINVAL, "deepr_mask must be within bits 0..1");
  if ((p->deepr_mask & 1) && p->n_in > 8192) return fail(RS_EINVAL, "DEEP R input projection: n_in <= 8192");
  if (p->cap_in > p->n_rec || p->cap_rec > p->n_rec)
    return fail(RS_EINVAL, "row capacity cannot exceed the number of targets");
  if (p->sample_steps < 1) return fail(RS_EINVAL, "sample_steps must be >= 1");
  if (p->trace_block > 32) return fail(RS_EINVAL, "trace_block must be in 0..32");
  if (p->reserved != 0) return fail(RS_EINVAL, "reserved must be 0");
  if (!(p->lr >= 0) || !(p->adam_b1 >= 0 && p->adam_b1 < 1) || !(p->adam_b2 >= 0 && p->adam_b2 < 1) ||
      !(p->adam_eps > 0))
    return fail(RS_EINVAL, "invalid Adam hyper-parameters");
  return RS_OK;
}

rs_status create_impl(const rs_eprop_params* prm, void* stream, rs_eprop** out, const Arena* alloc = nullptr) {
  TRY(validate(prm));
  if (!fwd_fits((int)prm->n_in, (int)prm->n_rec, (int)prm->n_out))
    return fail(RS_EINVAL, "n_in %u and n_rec %u need more LDS than a forward workgroup has", prm->n_in, prm->n_rec);
  rs_eprop* n = new rs_eprop();
  *out = n;
  if (alloc) {
    n->arena.afn = alloc->afn;
    n->arena.ffn = alloc->ffn;
    n->arena.user = alloc->user;
  }
  n->p = *prm;
  n->stream = (hipStream_t)stream;
  n->B = (int)prm->batch;
  n->alpha = std::exp(-(double)prm->dt_ms / (double)prm->tau_mem_ms);
  n->rho = prm->alif ? std::exp(-(double)prm->dt_ms / (double)prm->tau_adapt_ms) : 0.0;
  n->beta = prm->alif ? (double)prm->beta : 0.0;
  hipStream_t s = n->stream;
  const int B = n->B;
  const uint64_t seed = prm->seed;

  auto setup = [&](ProjDev& P, int n_pre, int n_post, int rec, int id, float p, uint32_t cap_req) -> rs_status {
    P.n_pre = n_pre;
    P.n_post = n_post;
    P.recurrent = rec;
    P.proj_id = id;
    P.words = (n_post + 31) / 32;
    int mx = 0;
    TRY(count_rows(n->arena, s, seed, P, threshold(p), &mx));
    int cap = cap_req ? (int)cap_req : 2 * mx;
    cap = std::min(cap, n_post);
    cap = std::max(cap, 1);
    if (mx > cap) return fail(RS_EINVAL, "projection %d: longest row %d exceeds capacity %d", id, mx, cap);
    P.cap = cap;
    return RS_OK;
  };
  TRY(setup(n->in, prm->n_in, prm->n_rec, 0, 0, prm->p_in, prm->cap_in));
  TRY(setup(n->rec, prm->n_rec, prm->n_rec, 1, 1, prm->p_rec, prm->cap_rec));
  const bool il = eprop_interleaved(B, prm->alif != 0);
  TRY(alloc_proj(n->arena, n->in, B, prm->alif, prm->deepr_mask & 1, il));
  TRY(alloc_proj(n->arena, n->rec, B, prm->alif, prm->deepr_mask & 2, il));
  Arena& ar = n->arena;
  const size_t NR = prm->n_rec, NI = prm->n_in, K = prm->n_out;
  TRY(ar.alloc(&n->V, B * NR));
  TRY(ar.alloc(&n->A, B * NR));
  TRY(ar.alloc(&n->Y, B * K));
  TRY(ar.alloc(&n->xbar, NI * B));
  TRY(ar.alloc(&n->zbar, NR * B));
  // default block length: the e-prop kernel's launch (for batches of 32 and
  // more, the update interval in equal blocks of at most 32 steps); batches
  // the narrow kernel serves (B % 4 != 0) take a whole update interval of up
  // to 32 steps, one block per interval
  if (prm->trace_block)
    n->K = n->K0 = (int)prm->trace_block;
  else if (B % 4 != 0 && prm->update_interval >= 1 && prm->update_interval <= 32)
    n->K = n->K0 = (int)prm->update_interval;
  else
    eprop_default_schedule((int)B, prm->update_interval, &n->K, &n->K0);
  {
    // a segment per block of an interval, plus one
    const uint32_t U = prm->update_interval, Kb = (uint32_t)n->K, K0 = (uint32_t)n->K0;
    const uint32_t nb = U ? (U <= K0 ? 1 : 1 + (U - K0 + Kb - 1) / Kb) : 1;
    n->Q = U ? (int)std::min<uint32_t>(std::max<uint32_t>(nb + 1, 2), RING_MAX) : 2;
  }
  const size_t QS = (size_t)n->Q;
  if (eprop_tc_path((int)B)) {
    n->tr_es = 2;
    TRY(ar.alloc(&n->x0T, QS * NI * B * 2));
    TRY(ar.alloc(&n->z0T, QS * NR * B * 2));
    n->xbitsT = (uint32_t*)n->x0T + 1;
    n->zbitsT = (uint32_t*)n->z0T + 1;
  } else {
    TRY(ar.alloc(&n->x0T, QS * NI * B));
    TRY(ar.alloc(&n->z0T, QS * NR * B));
    TRY(ar.alloc(&n->xbitsT, QS * NI * B));
    TRY(ar.alloc(&n->zbitsT, QS * NR * B));
  }
  n->nslot = n->Q * n->K;
  const size_t NS = (size_t)n->nslot;
  TRY(ar.alloc(&n->psiT, NR * NS * B));
  TRY(ar.alloc(&n->LT, NR * NS * B));
  TRY(ar.alloc(&n->deltaT, K * NS * B));
  {
    const size_t KB = (size_t)n->K * B;
    TRY(ar.alloc(&n->stg[0], QS * KB * NR));                   // psi
    const size_t dims[HANDOFF_ARRAYS] = {NR, NI, NR, NI, NR};  // psi, x0, z0, xbits, zbits
    for (int q = 1; q < HANDOFF_ARRAYS; ++q) TRY(ar.alloc(&n->stg[q], QS * B * dims[q]));
    TRY(ar.alloc(&n->u_stg, QS * KB * K));
  }
  // A small network's kernels are short and latency-bound: overlapping its
  // forward pass with its eligibility work gains less than the 10-30 us each
  // cross-stream wait costs, so all of its work stays on the caller's stream.
  {
    const double syn = (double)prm->p_in * NI * NR + (double)prm->p_rec * NR * (NR - 1);
    n->single = syn * B <= (double)(1u << 21);
  }
  if (n->single) {
    n->side = n->side2 = n->stream;
  } else {
    HIP_OK(hipStreamCreateWithFlags(&n->side, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&n->side2, hipStreamNonBlocking));
  }
  // Events between the library's own kernels on its streams order them on
  // the device only: no system-scope fence (a write-back of the caches) at
  // each record.  The joins with the caller's work at the ends of a call keep it.
  const unsigned dev_ev = hipEventDisableTiming | hipEventDisableSystemFence;
  HIP_OK(hipEventCreateWithFlags(&n->ev_upd, dev_ev));
  HIP_OK(hipEventCreateWithFlags(&n->ev_rw, dev_ev));
  HIP_OK(hipEventCreateWithFlags(&n->ev_fwd, dev_ev));
  HIP_OK(hipEventCreateWithFlags(&n->ev_post, dev_ev));
  HIP_OK(hipEventCreateWithFlags(&n->ev_loop, dev_ev));
  for (int q = 0; q < n->Q; ++q) HIP_OK(hipEventCreateWithFlags(&n->ev_ep[q], dev_ev));
  HIP_OK(hipEventCreateWithFlags(&n->ev_join, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&n->ev_back, hipEventDisableTiming));
  TRY(ar.alloc(&n->z, B * NR));
  TRY(ar.alloc(&n->Wout, K * NR));
  TRY(ar.alloc(&n->bout, K));
  TRY(ar.alloc(&n->Gout, K * NR));
  TRY(ar.alloc(&n->Gb, K));
  TRY(ar.alloc(&n->Mout, K * NR));
  TRY(ar.alloc(&n->Vout, K * NR));
  TRY(ar.alloc(&n->Mb, K));
  TRY(ar.alloc(&n->Vb, K));
  TRY(ar.alloc(&n->counters, 2));
  TRY(ar.alloc(&n->cv.cnt, NR * COL_GROUPS_MAX));
  TRY(ar.alloc(&n->cv.off, NR * COL_GROUPS_MAX + 1));
  TRY(ar.alloc(&n->cv.col, (size_t)n->in.n_pre * n->in.cap + (size_t)n->rec.n_pre * n->rec.cap));
  n->cv.n_col = (int)((size_t)n->in.n_pre * n->in.cap + (size_t)n->rec.n_pre * n->rec.cap);
  if (B > 128 && B % 4 == 0) {
    const size_t gx = (size_t)((B + 127) / 128) * n->cv.n_col;
    TRY(ar.alloc(&n->cv.gx, gx));
    launch_fill_zero(s, n->cv.gx, gx * 4);
  }
  TRY(ar.alloc(&n->rw_stats, 4));
  TRY(ar.alloc(&n->zcount, (size_t)B * NR));

  for (ProjDev* P : {&n->in, &n->rec}) {  // padding slots start defined
    launch_fill_zero(s, P->ind, (size_t)P->n_pre * P->cap * 4);
    launch_fill_zero(s, P->w, (size_t)P->n_pre * P->cap * 4);
    if (P->conn) launch_fill_zero(s, P->conn, (size_t)P->n_pre * P->words * 4);
    if (P->sign) launch_fill_zero(s, P->sign, (size_t)P->n_pre * P->words * 4);
  }
  launch_fixed_rows(s, seed, n->in, threshold(prm->p_in), (double)prm->sigma_in, true);
  launch_fixed_rows(s, seed, n->rec, threshold(prm->p_rec), (double)prm->sigma_rec, true);
  launch_dense_init(s, seed, 2, (int)K, (int)NR, (double)prm->sigma_out, n->Wout);
  if (prm->deepr_mask & 1) launch_deepr_bits_init(s, seed, n->in);
  if (prm->deepr_mask & 2) launch_deepr_bits_init(s, seed, n->rec);
  launch_columns(s, n->in, n->rec, n->cv);
  zero_proj_state(s, n->in, B);
  zero_proj_state(s, n->rec, B);
  for (double* q : {n->V, n->A}) launch_fill_zero(s, q, B * NR * 8);
  launch_fill_zero(s, n->zbar, B * NR * 4);
  for (float* q : {n->psiT, n->LT}) launch_fill_zero(s, q, B * NR * NS * 4);
  launch_fill_zero(s, n->x0T, QS * B * NI * 4 * n->tr_es);
  launch_fill_zero(s, n->z0T, QS * B * NR * 4 * n->tr_es);
  if (n->tr_es == 1) {
    launch_fill_zero(s, n->xbitsT, QS * B * NI * 4);
    launch_fill_zero(s, n->zbitsT, QS * B * NR * 4);
  }
  launch_fill_zero(s, n->deltaT, B * K * NS * 4);
  launch_fill_zero(s, n->xbar, B * NI * 4);
  launch_fill_zero(s, n->Y, B * K * 8);
  launch_fill_zero(s, n->z, B * NR);
  for (float* q : {n->Gout, n->Mout, n->Vout}) launch_fill_zero(s, q, K * NR * 4);
  for (float* q : {n->bout, n->Gb, n->Mb, n->Vb}) launch_fill_zero(s, q, K * 4);
  launch_fill_zero(s, n->counters, 16);
  launch_fill_zero(s, n->rw_stats, 32);
  launch_fill_zero(s, n->zcount, (size_t)B * NR * 4);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  return RS_OK;
}

void reset_state(rs_eprop* n, hipStream_t s) {
  const size_t B = n->B, NR = n->p.n_rec, NI = n->p.n_in, K = n->p.n_out;
  launch_fill_zero(s, n->V, B * NR * 8);
  launch_fill_zero(s, n->A, B * NR * 8);
  launch_fill_zero(s, n->Y, B * K * 8);
  launch_fill_zero(s, n->xbar, B * NI * 4);
  launch_fill_zero(s, n->zbar, B * NR * 4);
  for (ProjDev* P : {&n->in, &n->rec}) {
    const size_t m = (size_t)P->n_pre * P->cap * B * 4;
    launch_fill_zero(s, P->ebar, (size_t)P->n_pre * P->cap * P->erec * 4);
    if (P->eps) launch_fill_zero(s, P->eps, m);
  }
}

// Bias corrections of Adam update k, rounded to float as the kernels use them.
float adam_inv_c(double b, uint32_t k) { return (float)(1.0 / (1.0 - std::pow(b, (double)k))); }

UpdateArgs update_args(const rs_eprop* n, uint32_t k) {
  UpdateArgs u{};
  u.B = n->B;
  u.lr = n->p.lr;
  u.b1 = n->p.adam_b1;
  u.b2 = n->p.adam_b2;
  u.eps = n->p.adam_eps;
  u.inv_c1 = adam_inv_c((double)n->p.adam_b1, k);
  u.inv_c2 = adam_inv_c((double)n->p.adam_b2, k);
  u.l1 = n->p.l1;
  u.l1_in = (n->p.deepr_mask & 1) != 0;
  u.l1_rec = (n->p.deepr_mask & 2) != 0;
  u.in = n->in;
  u.rec = n->rec;
  u.Wout = n->Wout; u.bout = n->bout; u.Gout = n->Gout; u.Gb = n->Gb;
  u.Mout = n->Mout; u.Vout = n->Vout; u.Mb = n->Mb; u.Vb = n->Vb;
  u.n_out_elems = (int)(n->p.n_out * n->p.n_rec);
  u.n_b = (int)n->p.n_out;
  return u;
}

void fold_gradients(rs_eprop* n, hipStream_t s);

void do_update(rs_eprop* n, hipStream_t s) {
  n->adam_k += 1;
  n->timer.begin(s, 2);
  fold_gradients(n, s);
  launch_update(s, update_args(n, n->adam_k));
  n->timer.end(s);
}

// The column view follows the rows after every rewire or restore; it is timed
// with the rewire phase.
void rebuild_columns(rs_eprop* n, hipStream_t s) {
  if (n->B % 4 != 0) return;  // only the target-major e-prop kernel (B % 4 == 0) reads the column view
  n->timer.begin(s, 3);
  launch_columns(s, n->in, n->rec, n->cv);
  n->timer.end(s);
}

void do_rewire(rs_eprop* n, int proj, hipStream_t s) {
  ProjDev& P = proj == 0 ? n->in : n->rec;
  n->timer.begin(s, 3);
  launch_deepr(s, n->p.seed, P, n->B, n->step, n->rw_stats);
  n->timer.end(s);
}

// Order stream `to` after the work enqueued so far on stream `from`.
void order(hipEvent_t ev, hipStream_t from, hipStream_t to) {
  if (from == to) return;
  (void)hipEventRecord(ev, from);
  (void)hipStreamWaitEvent(to, ev, 0);
}

// Staging array q (psi, x0, z0, xbits, zbits) of ring segment h.
uint32_t* stg_seg(const rs_eprop* n, int q, int h) {
  const size_t B = n->B, NR = n->p.n_rec, NI = n->p.n_in;
  const size_t per = q == 0 ? (size_t)n->K * B * NR : B * (q == 1 || q == 3 ? NI : NR);
  return n->stg[q] + (size_t)h * per;
}

// Arguments of one block's launches: steps t0 .. t0 + nsteps - 1 (absolute
// step numbers), ring segment h.  Shared by the one-network path and the
// multi-network launches, so both compute the same thing.
FwdArgs block_fwd_args(const rs_eprop* n, int h, uint64_t t0, int nsteps) {
  FwdArgs f{};
  f.n_in = (int)n->p.n_in; f.n_rec = (int)n->p.n_rec; f.n_out = (int)n->p.n_out; f.B = n->B;
  f.alpha = n->alpha; f.rho = n->rho; f.v_thr = n->p.v_thr; f.beta = n->beta;
  f.psi_scale = 0.3 / (double)n->p.v_thr;
  f.alpha_f = (float)n->alpha;
  f.V = n->V; f.A = n->A;
  f.xbar = n->xbar; f.zbar = n->zbar;
  f.psi = (float*)stg_seg(n, 0, h); f.x0 = (float*)stg_seg(n, 1, h); f.z0 = (float*)stg_seg(n, 2, h);
  f.xbits = stg_seg(n, 3, h); f.zbits = stg_seg(n, 4, h); f.z = n->z;
  f.u = n->u_stg + (size_t)h * n->K * n->B * n->p.n_out;
  f.len_in = n->in.len; f.ind_in = n->in.ind; f.w_in = n->in.w; f.cap_in = n->in.cap;
  f.len_rec = n->rec.len; f.ind_rec = n->rec.ind; f.w_rec = n->rec.w; f.cap_rec = n->rec.cap;
  f.Wout = n->Wout;
  f.x_off = n->x_off; f.x_idx = n->x_idx; f.n_idx = n->n_idx;
  if (n->poisson) {
    f.x_thr = n->x_thr; f.x_thr_stride = n->x_thr_stride; f.x_list = n->x_list;
    f.seed = n->p.seed; f.step0 = t0;
  }
  f.t0 = (int)(t0 % n->p.sample_steps); f.sample_steps = (int)n->p.sample_steps; f.nsteps = nsteps;
  f.counters = n->counters;
  // small networks keep their rows on chip for the block; a large one's
  // forward workgroups leave LDS to the e-prop launch beside them
  f.rows_lds = n->single ? 1 : 0;
  f.zcount = n->zcount;
  return f;
}

HandoffArrays block_handoff_args(const rs_eprop* n, int h, int nsteps) {
  HandoffArrays ho{};
  const size_t NI = n->p.n_in, NR = n->p.n_rec, B = n->B;
  const size_t es = n->tr_es;
  uint32_t* dst[HANDOFF_ARRAYS] = {(uint32_t*)n->psiT, (uint32_t*)(n->x0T + h * NI * B * es),
                                   (uint32_t*)(n->z0T + h * NR * B * es), n->xbitsT + h * NI * B * es,
                                   n->zbitsT + h * NR * B * es};
  const int dims[HANDOFF_ARRAYS] = {(int)NR, (int)NI, (int)NR, (int)NI, (int)NR};
  for (int q = 0; q < HANDOFF_ARRAYS; ++q) {
    ho.src[q] = stg_seg(n, q, h);
    ho.dst[q] = dst[q];
    ho.n[q] = dims[q];
    ho.steps[q] = q == 0 ? nsteps : 1;  // psi per step into the ring, the rest once per block
    ho.slot0[q] = q == 0 ? h * n->K : 0;
    ho.nslot[q] = q == 0 ? n->nslot : 1;
    ho.es[q] = q == 0 ? 1 : n->tr_es;
  }
  return ho;
}

ReadoutArgs block_readout_args(const rs_eprop* n, int h, int nsteps) {
  ReadoutArgs ro{};
  ro.n_rec = (int)n->p.n_rec; ro.n_out = (int)n->p.n_out; ro.B = n->B; ro.nsteps = nsteps;
  ro.slot0 = h * n->K; ro.nslot = n->nslot;
  ro.alpha = n->alpha;
  ro.u = n->u_stg + (size_t)h * n->K * n->B * n->p.n_out;
  ro.Y = n->Y; ro.Wout = n->Wout; ro.bout = n->bout; ro.labels = n->labels;
  ro.deltaT = n->deltaT; ro.LT = n->LT;
  return ro;
}

EpropArgs block_eprop_args(const rs_eprop* n, int h, int nsteps) {
  const size_t NI = n->p.n_in, NR = n->p.n_rec, B = n->B;
  EpropArgs a{};
  a.n_in = (int)NI; a.n_rec = (int)NR; a.n_out = (int)n->p.n_out; a.B = n->B;
  a.alif = n->p.alif ? 1 : 0;
  a.alpha = (float)n->alpha; a.rho = (float)n->rho; a.beta = (float)n->beta;
  a.one_m_rho = (float)(1.0 - n->rho);
  a.in = n->in; a.rec = n->rec;
  const size_t es = n->tr_es;
  a.x0 = n->x0T + h * NI * B * es; a.z0 = n->z0T + h * NR * B * es;
  a.xbits = n->xbitsT + h * NI * B * es; a.zbits = n->zbitsT + h * NR * B * es;
  a.tr_es = n->tr_es;
  a.tofs = 0;
  a.psiT = n->psiT; a.LT = n->LT; a.deltaT = n->deltaT;
  a.slot0 = h * n->K; a.nsteps = nsteps; a.nslot = n->nslot;
  a.Gout = n->Gout; a.Gb = n->Gb;
  a.col_off = n->cv.off; a.col = n->cv.col;
  a.gx = n->cv.gx; a.n_col = n->cv.n_col;
  return a;
}

// Bring every chunk's gradient into G: before the update, and before G is
// read or written or rows move outside it.
void fold_gradients(rs_eprop* n, hipStream_t s) {
  if (n->cv.gx) launch_gx_fold(s, block_eprop_args(n, 0, 0));
}

// Run the open block (steps accumulated since the last flush): one forward
// launch for all its steps on the caller's stream, writing ring segment
// blk_seg; the block's hand-off transpose and readout on the second side
// stream; then the e-prop launch on the side stream.  The forward pass of the
// next block (next segment) overlaps both; a segment is reused only after
// the e-prop launch that read it has finished.
void flush_block(rs_eprop* n) {
  if (n->blk_n == 0) return;
  hipStream_t s = n->stream, e = n->side, p = n->side2;
  const int h = n->blk_seg;
  if (n->ep_pending[h]) {
    (void)hipStreamWaitEvent(s, n->ev_ep[h], 0);
    n->ep_pending[h] = false;
  }
  n->timer.begin(s, 0);
  launch_fwd(s, block_fwd_args(n, h, n->blk_t0, n->blk_n));
  n->timer.end(s);
  // the transpose, readout state, softmax error and (when learning) the
  // learning signal of the block, beside the next block's forward pass: they
  // read this segment only, and the readouts of successive blocks stay in
  // order on their stream
  order(n->ev_fwd, s, p);
  n->timer.begin(p, 0);
  launch_handoff_transpose(p, block_handoff_args(n, h, n->blk_n), n->B);
  launch_readout(p, block_readout_args(n, h, n->blk_n), n->blk_learn);
  n->timer.end(p);
  n->last_slot = h * n->K + n->blk_n - 1;
  order(n->ev_post, p, e);
  if (n->blk_learn) {
    n->timer.begin(e, 1);
    launch_eprop(e, block_eprop_args(n, h, n->blk_n));
    n->timer.end(e);
  }
  // The forward launch that next writes this segment comes Q blocks later.
  // Inside a call with automatic updates, the join at the next update comes
  // first when fewer than Q blocks remain to it; that join then orders the
  // forward stream after this launch and no event is needed.
  bool covered = false;
  if (n->auto_upd) {
    const uint64_t U = n->p.update_interval, rem = (U - n->step % U) % U;
    covered = (rem + (uint64_t)n->K - 1) / (uint64_t)n->K < (uint64_t)n->Q;
  }
  if (e != s && !covered) {
    (void)hipEventRecord(n->ev_ep[h], e);
    n->ep_pending[h] = true;
  }
  n->last_seg = h;
  n->last_blk_n = n->blk_n;
  n->blk_seg = (n->blk_seg + 1) % n->Q;
  n->blk_n = 0;
}

// One timestep joins the open block; a full block, an update/rewire or a
// sample boundary runs it.
void do_step(rs_eprop* n, uint32_t flags) {
  hipStream_t s = n->stream, e = n->side;
  const bool learn = (flags & RS_LEARN) != 0;
  if (n->blk_n > 0 && learn != n->blk_learn) flush_block(n);
  if (n->blk_n == 0) {
    n->blk_learn = learn;
    n->blk_t0 = n->step;
  }
  n->blk_n += 1;
  n->step += 1;
  // under automatic updates an interval's first block is K0 steps
  const uint64_t U = n->p.update_interval;
  const bool first = n->auto_upd && U && n->blk_t0 % U == 0;
  if (n->blk_n == (first ? n->K0 : n->K)) flush_block(n);
  const bool upd = (flags & RS_AUTO_UPDATE) && n->p.update_interval && n->step % n->p.update_interval == 0;
  const bool rst = (flags & RS_AUTO_RESET) && n->step % n->p.sample_steps == 0;
  if (upd || rst) {
    // the side stream follows the last forward launch: every flush ends with
    // that wait, and the open block was flushed here or at its last step
    flush_block(n);
    if (upd) {
      do_update(n, e);
      if (n->p.deepr_mask == 3) {
        // the two projections' rewires share nothing but the summed counts:
        // the input projection's runs on a third stream beside the other
        order(n->ev_upd, e, n->side2);
        do_rewire(n, 0, n->side2);
        do_rewire(n, 1, e);
        order(n->ev_rw, n->side2, e);
      } else {
        if (n->p.deepr_mask & 1) do_rewire(n, 0, e);
        if (n->p.deepr_mask & 2) do_rewire(n, 1, e);
      }
    }
    if (rst) {
      n->timer.begin(e, 4);
      reset_state(n, e);
      n->timer.end(e);
    }
    order(n->ev_loop, e, s);
    for (bool& p : n->ep_pending) p = false;  // covered by that wait
    // only the e-prop launches, later on this stream, read the column view:
    // the next forward block runs while it is rebuilt
    if (upd && n->p.deepr_mask) rebuild_columns(n, e);
  }
}

struct VarRef {
  void* ptr;
  size_t bytes;
  size_t rows = 0, pitch = 0;  // strided ring slot: rows of bytes/rows, pitch apart
  int il = -1;                 // >= 0: word il of every pair of an interleaved array of 2 bytes/4 32-bit words
};

bool var_ref(rs_eprop* n, int32_t var, VarRef* r, bool for_write) {
  const size_t B = n->B, NR = n->p.n_rec, NI = n->p.n_in, K = n->p.n_out;
  const size_t slot_off = (size_t)n->last_slot * B * 4, pitch = (size_t)n->nslot * B * 4;
  const int pj = var / 0x100 - 1, f = var % 0x100;
  if (var < 0x100) {
    switch (var) {
      case RS_V: *r = {n->V, B * NR * 8}; return true;
      case RS_A: *r = {n->A, B * NR * 8}; return true;
      case RS_Y: *r = {n->Y, B * K * 8}; return true;
      case RS_XBAR: *r = {n->xbar, NI * B * 4}; return true;
      case RS_ZBAR: *r = {n->zbar, NR * B * 4}; return true;
      case RS_PSI: *r = {(char*)n->psiT + slot_off, NR * B * 4, NR, pitch}; return !for_write;
      case RS_LSIG: *r = {(char*)n->LT + slot_off, NR * B * 4, NR, pitch}; return !for_write;
      case RS_DELTA: *r = {(char*)n->deltaT + slot_off, K * B * 4, K, pitch}; return !for_write;
      case RS_Z: *r = {n->z, B * NR}; return !for_write;
      case RS_WOUT: *r = {n->Wout, K * NR * 4}; return true;
      case RS_BOUT: *r = {n->bout, K * 4}; return true;
      case RS_GOUT: *r = {n->Gout, K * NR * 4}; return true;
      case RS_GB: *r = {n->Gb, K * 4}; return true;
      case RS_MOUT: *r = {n->Mout, K * NR * 4}; return true;
      case RS_VOUT: *r = {n->Vout, K * NR * 4}; return true;
      case RS_MB: *r = {n->Mb, K * 4}; return true;
      case RS_VB: *r = {n->Vb, K * 4}; return true;
      case RS_ZCOUNT: *r = {n->zcount, B * NR * 4}; return true;
      case RS_ZBITS:
        if (n->tr_es == 2) {  // the second word of each (trace, spike word) pair
          *r = {n->z0T + (size_t)n->last_seg * NR * B * 2, NR * B * 4};
          r->il = 1;
        } else {
          *r = {n->zbitsT + (size_t)n->last_seg * NR * B, NR * B * 4};
        }
        return !for_write;
      default: return false;
    }
  }
  if (pj < 0 || pj > 1) return false;
  ProjDev& P = pj == 0 ? n->in : n->rec;
  const size_t ns = (size_t)P.n_pre * P.cap;
  switch (f) {
    case RS_P_LEN: *r = {P.len, (size_t)P.n_pre * 4}; return true;
    case RS_P_IND: *r = {P.ind, ns * 4}; return true;
    case RS_P_W: *r = {P.w, ns * 4}; return true;
    case RS_P_M: *r = {P.m, ns * 4}; return true;
    case RS_P_V: *r = {P.v, ns * 4}; return true;
    case RS_P_G: *r = {P.G, ns * 4}; return true;
    case RS_P_EPS:
      if ((size_t)P.erec == 2 * B) {  // the second float of each interleaved pair
        *r = {P.ebar, ns * B * 4};
        r->il = 1;
        return true;
      }
      *r = {P.eps, ns * B * 4};
      return P.eps != nullptr;
    case RS_P_EBAR:
      *r = {P.ebar, ns * B * 4};
      if ((size_t)P.erec == 2 * B) r->il = 0;
      return true;
    case RS_P_CONN: *r = {P.conn, (size_t)P.n_pre * P.words * 4}; return P.conn != nullptr;
    case RS_P_SIGN: *r = {P.sign, (size_t)P.n_pre * P.words * 4}; return P.sign != nullptr;
    case RS_P_DORMANT: *r = {P.dormant, (size_t)P.n_pre * 4}; return true;
    default: return false;
  }
}

}  // namespace

// Error reporting for the library's other source files.
rs_status rs_internal_fail(rs_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return fail(code, "%s", buf);
}

// =========================================================================== C-ABI
extern "C" {

const char* rs_last_error(void) { return g_err.c_str(); }

rs_status rs_eprop_create(const rs_eprop_params* params, void* hip_stream, rs_eprop** out) {
  if (!out) return fail(RS_EINVAL, "out is NULL");
  *out = nullptr;
  rs_eprop* n = nullptr;
  rs_status st = create_impl(params, hip_stream, &n);
  if (st != RS_OK) {
    if (n) rs_eprop_destroy(n);
    return st;
  }
  *out = n;
  return RS_OK;
}

rs_status rs_eprop_set_input(rs_eprop* n, const int32_t* off_dev, const int32_t* idx_dev, size_t n_idx,
                             const int32_t* labels_dev) {
  ENTER(n);
  if (!off_dev || !idx_dev || !labels_dev) return fail(RS_EINVAL, "input pointers must not be NULL");
  if (n_idx > (size_t)INT32_MAX) return fail(RS_EINVAL, "index array larger than 2^31 entries");
  n->x_off = off_dev;
  n->x_idx = idx_dev;
  n->n_idx = (long long)n_idx;
  n->labels = labels_dev;
  n->poisson = false;
  return RS_OK;
}

rs_status rs_eprop_set_input_poisson(rs_eprop* n, const double* rate_hz, size_t n_rates, const int32_t* labels_dev) {
  ENTER(n);
  if (!rate_hz || !labels_dev) return fail(RS_EINVAL, "rate table and labels must not be NULL");
  const size_t NI = n->p.n_in, B = n->B;
  if (n_rates != NI && n_rates != B * NI) return fail(RS_EINVAL, "n_rates must be n_in or batch * n_in");
  if ((size_t)n->K * B * NI > (size_t)INT32_MAX) return fail(RS_EINVAL, "trace_block * batch * n_in exceeds 2^31");
  std::vector<uint64_t> thr(n_rates);
  for (size_t q = 0; q < n_rates; ++q) {
    if (std::isnan(rate_hz[q])) return fail(RS_EINVAL, "rate %zu is NaN", q);
    thr[q] = threshold(rate_hz[q] * (double)n->p.dt_ms / 1000.0);
  }
  if (!n->x_thr) {
    TRY(n->arena.alloc(&n->x_thr, B * NI));
    TRY(n->arena.alloc(&n->x_list, (size_t)n->K * B * NI));
  }
  // blocks already queued read the table: the copy follows them on the stream
  flush_block(n);
  order(n->ev_join, n->side, n->stream);
  HIP_OK(hipMemcpyAsync(n->x_thr, thr.data(), n_rates * 8, hipMemcpyHostToDevice, n->stream));
  HIP_OK(hipStreamSynchronize(n->stream));
  n->x_thr_stride = n_rates == NI ? 0 : (int)NI;
  n->labels = labels_dev;
  n->x_off = nullptr;
  n->x_idx = nullptr;
  n->n_idx = 0;
  n->poisson = true;
  return RS_OK;
}

rs_status rs_eprop_step(rs_eprop* n, uint32_t n_steps, uint32_t flags) {
  ENTER(n);
  if (!n->x_off && !n->poisson) return fail(RS_ESTATE, "no input attached (rs_eprop_set_input*)");
  if (flags & ~(RS_LEARN | RS_AUTO_UPDATE | RS_AUTO_RESET)) return fail(RS_EINVAL, "unknown step flags");
  order(n->ev_join, n->stream, n->side);  // side stream follows earlier caller work
  n->auto_upd = (flags & RS_AUTO_UPDATE) && n->p.update_interval > 0;
  for (uint32_t q = 0; q < n_steps; ++q) do_step(n, flags);
  flush_block(n);
  n->auto_upd = false;
  order(n->ev_back, n->side, n->stream);  // caller's stream covers all of it
  for (bool& p : n->ep_pending) p = false;
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_eprop_update(rs_eprop* n) {
  ENTER(n);
  do_update(n, n->stream);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_eprop_rewire(rs_eprop* n, uint32_t proj, rs_rewire_stats* st) {
  ENTER(n);
  if (proj > 1 || !((n->p.deepr_mask >> proj) & 1u))
    return fail(RS_EINVAL, "projection %u is not rewired by DEEP R", proj);
  long long before[4] = {0, 0, 0, 0}, after[4];
  if (st) {  // the counters accumulate over the object's life; report this call's share
    HIP_OK(hipMemcpyAsync(before, n->rw_stats, sizeof before, hipMemcpyDeviceToHost, n->stream));
    HIP_OK(hipStreamSynchronize(n->stream));
  }
  fold_gradients(n, n->stream);
  do_rewire(n, (int)proj, n->stream);
  rebuild_columns(n, n->stream);
  HIP_OK(hipGetLastError());
  if (st) {
    HIP_OK(hipMemcpyAsync(after, n->rw_stats, sizeof after, hipMemcpyDeviceToHost, n->stream));
    HIP_OK(hipStreamSynchronize(n->stream));
    st->eliminated = after[0] - before[0];
    st->formed = after[1] - before[1];
    st->attempts = after[2] - before[2];
    st->blocked = after[3] - before[3];
  }
  return RS_OK;
}

rs_status rs_eprop_reset(rs_eprop* n) {
  ENTER(n);
  reset_state(n, n->stream);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_eprop_get(rs_eprop* n, int32_t var, void* host, size_t bytes) {
  ENTER(n);
  if (!host) return fail(RS_EINVAL, "NULL argument");
  VarRef r;
  if (!var_ref(n, var, &r, false)) return fail(RS_EINVAL, "unknown or absent variable 0x%x", var);
  if (bytes != r.bytes) return fail(RS_ECAPACITY, "variable 0x%x has %zu bytes, buffer %zu", var, r.bytes, bytes);
  if (var % 0x100 == RS_P_G && var >= 0x100) fold_gradients(n, n->stream);
  if (r.il >= 0) {  // one word of each pair: interleaved eligibility state, or the last block's spike words
    const size_t cnt = bytes / 4;
    std::vector<uint32_t> both(2 * cnt);
    HIP_OK(hipMemcpyAsync(both.data(), r.ptr, 2 * bytes, hipMemcpyDeviceToHost, n->stream));
    HIP_OK(hipStreamSynchronize(n->stream));
    uint32_t* out = (uint32_t*)host;
    for (size_t k = 0; k < cnt; ++k) out[k] = both[2 * k + r.il];
    return RS_OK;
  }
  if (r.rows) {
    const size_t w = bytes / r.rows;
    HIP_OK(hipMemcpy2DAsync(host, w, r.ptr, r.pitch, w, r.rows, hipMemcpyDeviceToHost, n->stream));
  } else {
    HIP_OK(hipMemcpyAsync(host, r.ptr, bytes, hipMemcpyDeviceToHost, n->stream));
  }
  HIP_OK(hipStreamSynchronize(n->stream));
  return RS_OK;
}

rs_status rs_eprop_set(rs_eprop* n, int32_t var, const void* host, size_t bytes) {
  ENTER(n);
  if (!host) return fail(RS_EINVAL, "NULL argument");
  VarRef r;
  if (!var_ref(n, var, &r, true)) return fail(RS_EINVAL, "unknown or read-only variable 0x%x", var);
  if (bytes != r.bytes) return fail(RS_ECAPACITY, "variable 0x%x has %zu bytes, buffer %zu", var, r.bytes, bytes);
  const int pj = var / 0x100 - 1, f = var % 0x100;
  if (pj >= 0 && (f == RS_P_LEN || f == RS_P_IND)) {
    // every slot below a row's length must hold a valid target: check the
    // new lengths against the current indices, or the new indices against
    // the current lengths
    const ProjDev& P = pj == 0 ? n->in : n->rec;
    std::vector<int32_t> len((size_t)P.n_pre), ind((size_t)P.n_pre * P.cap);
    HIP_OK(hipStreamSynchronize(n->stream));
    if (f == RS_P_LEN) {
      memcpy(len.data(), host, bytes);
      HIP_OK(hipMemcpy(ind.data(), P.ind, ind.size() * 4, hipMemcpyDeviceToHost));
    } else {
      memcpy(ind.data(), host, bytes);
      HIP_OK(hipMemcpy(len.data(), P.len, len.size() * 4, hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < P.n_pre; ++i) {
      if (len[i] < 0 || len[i] > P.cap) return fail(RS_EINVAL, "row %d length %d outside 0..%d", i, len[i], P.cap);
      for (int k = 0; k < len[i]; ++k) {
        const int32_t j = ind[(size_t)i * P.cap + k];
        if (j < 0 || j >= P.n_post) return fail(RS_EINVAL, "row %d slot %d target %d outside 0..%d", i, k, j, P.n_post - 1);
      }
    }
  }
  HIP_OK(hipStreamSynchronize(n->stream));
  // the chunks' parts go into G first: a new G replaces them too, and new
  // rows must not inherit them at slots the update no longer visits
  fold_gradients(n, n->stream);
  if (r.il >= 0) {  // replace one word of each pair of the interleaved eligibility state
    const size_t cnt = bytes / 4;
    std::vector<uint32_t> both(2 * cnt);
    HIP_OK(hipMemcpyAsync(both.data(), r.ptr, 2 * bytes, hipMemcpyDeviceToHost, n->stream));
    HIP_OK(hipStreamSynchronize(n->stream));
    const uint32_t* in = (const uint32_t*)host;
    for (size_t k = 0; k < cnt; ++k) both[2 * k + r.il] = in[k];
    HIP_OK(hipMemcpyAsync(r.ptr, both.data(), 2 * bytes, hipMemcpyHostToDevice, n->stream));
    HIP_OK(hipStreamSynchronize(n->stream));
    return RS_OK;
  }
  HIP_OK(hipMemcpyAsync(r.ptr, host, bytes, hipMemcpyHostToDevice, n->stream));
  if (pj >= 0 && (f == RS_P_LEN || f == RS_P_IND)) rebuild_columns(n, n->stream);
  HIP_OK(hipStreamSynchronize(n->stream));
  return RS_OK;
}

rs_status rs_eprop_info_get(rs_eprop* n, rs_eprop_info* o) {
  ENTER(n);
  if (!o) return fail(RS_EINVAL, "NULL argument");
  unsigned long long c[2];
  long long r[2];
  HIP_OK(hipMemcpyAsync(c, n->counters, sizeof c, hipMemcpyDeviceToHost, n->stream));
  HIP_OK(hipMemcpyAsync(r, n->rw_stats, sizeof r, hipMemcpyDeviceToHost, n->stream));
  HIP_OK(hipStreamSynchronize(n->stream));
  memset(o, 0, sizeof *o);
  o->cap_in = (uint32_t)n->in.cap;
  o->cap_rec = (uint32_t)n->rec.cap;
  o->words_in = (uint32_t)n->in.words;
  o->words_rec = (uint32_t)n->rec.words;
  o->step = n->step;
  o->adam_step = n->adam_k;
  o->last_block = (uint32_t)n->last_blk_n;
  o->synaptic_events = c[0];
  o->spikes = c[1];
  o->device_bytes = n->arena.bytes;
  o->eliminated = (uint64_t)r[0];
  o->formed = (uint64_t)r[1];
  o->trace_block = (uint32_t)n->K;
  o->first_block = (uint32_t)n->K0;
  return RS_OK;
}

rs_status rs_eprop_timing(rs_eprop* n, int32_t phase_mask) {
  ENTER(n);
  if (phase_mask < 0 || phase_mask >= (1 << RS_NUM_PHASES)) return fail(RS_EINVAL, "phase_mask out of range");
  n->timer.mask = phase_mask;
  return RS_OK;
}

rs_status rs_eprop_phase_times(rs_eprop* n, double* ms, uint64_t* count) {
  ENTER(n);
  if (!ms || !count) return fail(RS_EINVAL, "NULL argument");
  n->timer.collect();
  for (int q = 0; q < RS_NUM_PHASES; ++q) {
    ms[q] = n->timer.ms[q];
    count[q] = n->timer.count[q];
    n->timer.ms[q] = 0;
    n->timer.count[q] = 0;
  }
  return RS_OK;
}

void rs_eprop_destroy(rs_eprop* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  if (!n->single) {
    if (n->side) (void)hipStreamSynchronize(n->side);
    if (n->side2) (void)hipStreamSynchronize(n->side2);
  }
  n->timer.destroy();
  for (hipEvent_t ev : {n->ev_fwd, n->ev_post, n->ev_join, n->ev_back, n->ev_upd, n->ev_rw, n->ev_loop})
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : n->ev_ep)
    if (ev) (void)hipEventDestroy(ev);
  if (!n->single) {
    if (n->side) (void)hipStreamDestroy(n->side);
    if (n->side2) (void)hipStreamDestroy(n->side2);
  }
  n->arena.release();
  delete_custom(n->custom);
  delete n;
}

}  // extern "C"

// =========================================================================== topomap
// Largest weight magnitude of a topographic map: the simulation sums a step's
// deliveries onto one target in 64-bit fixed point (2^-36 resolution), which
// holds in-degree 4096 at this bound.
constexpr float TOPO_W_MAX = 1e4f;

struct rs_topo {
  rs_topo_params p;
  hipStream_t stream = nullptr;
  Arena arena;
  TopoDev t{};
  uint64_t* T_d2 = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // simulation (rs_topo_sim_init)
  bool sim = false;
  rs_topo_model m{};
  TopoSimDev sd{};
  uint64_t step = 0;
  uint64_t* step_dev = nullptr;
  unsigned long long* ticks = nullptr;  // [TOPO_PHASES] phase timers
  // GRAPH_INTERVALS whole rewiring intervals (simulation + rewire launches)
  // recorded once and replayed; the kernels read the step count from step_dev
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct rs_custom_state* custom = nullptr;  // scratch of custom connectivity updates
  // lateral projection (target -> target, rs_topo_add_lateral)
  bool lateral = false;
  rs_topo_params pl{};
  TopoDev tl{};
  uint64_t* T_d2_l = nullptr;
  int32_t kernel = RS_TOPO_KERNEL_AUTO;  // requested simulation kernel
  bool tiled = false;                    // the simulation runs on the tiled kernel
  bool dead = false;  // a device error occurred: every later call fails with RS_EDEVICE
};

namespace {
constexpr uint64_t GRAPH_INTERVALS = 64;

// One simulation launch on the map's kernel.
void topo_launch_sim(rs_topo* t, hipStream_t s, uint64_t t0, int n) {
  if (t->tiled) {
    ProjDev none{};
    launch_topo_tiles(s, t->p.seed, t->t.P, t->lateral ? t->tl.P : none, t->sd, t0, n);
  } else {
    launch_topo_sim(s, t->p.seed, t->t.P, t->sd, t0, n);
  }
}

// Choose the simulation kernel: the one-workgroup kernel for maps of up to
// 4096 neurons without a lateral projection (unless the tiled one is asked
// for), the tiled kernel otherwise, if the device keeps all of its tiles
// resident.
rs_status topo_pick_kernel(rs_topo* t, int32_t kind) {
  const int N = (int)(t->p.L * t->p.L);
  bool tiled = kind == RS_TOPO_KERNEL_TILED || (kind == RS_TOPO_KERNEL_AUTO && (t->lateral || !topo_sim_fits(N)));
  if (!tiled && (t->lateral || !topo_sim_fits(N)))
    return fail(RS_EINVAL, "the one-workgroup kernel needs L*L <= 4096 and no lateral projection");
  if (tiled) {
    if (N > TOPO_TILES_MAX_N) return fail(RS_EINVAL, "the tiled kernel needs L*L <= %d", TOPO_TILES_MAX_N);
    const int need = topo_tiles_grid(N), have = topo_tiles_resident(N, t->lateral);
    if (need > have) return fail(RS_EINVAL, "the tiled kernel needs %d resident workgroups, the device keeps %d",
                                 need, have);
  }
  t->tiled = tiled;
  return RS_OK;
}

// The rewires after a rewiring interval: feed-forward, then lateral.
void topo_launch_rewires(rs_topo* t, hipStream_t s, uint64_t step) {
  if (t->lateral) launch_topo_rewire_pair(s, t->p.seed, t->t, t->tl, step);
  else launch_topo_rewire(s, t->p.seed, t->t, step);
}

void topo_drop_graph(rs_topo* t) {
  if (t->gexec) (void)hipGraphExecDestroy(t->gexec);
  if (t->graph) (void)hipGraphDestroy(t->graph);
  t->gexec = nullptr;
  t->graph = nullptr;
}

rs_status topo_build_graph(rs_topo* t) {
  topo_drop_graph(t);  // a failed earlier attempt may have left a graph without its instance
  const int R = (int)t->m.rewire_steps;
  topo_sim_attrs();
  topo_rewire_attrs();
  if (!t->cap_stream) HIP_OK(hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking));
  HIP_OK(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeThreadLocal));
  for (uint64_t g = 0; g < GRAPH_INTERVALS; ++g) {
    topo_launch_sim(t, t->cap_stream, STEP_FROM_DEVICE, R);
    topo_launch_rewires(t, t->cap_stream, STEP_FROM_DEVICE);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(t->cap_stream, &g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(RS_EDEVICE, "capturing the rewiring-interval graph failed: %s", hipGetErrorString(e));
  }
  t->graph = g;
  HIP_OK(hipGraphInstantiate(&t->gexec, t->graph, nullptr, nullptr, 0));
  return RS_OK;
}
}  // namespace


namespace {

rs_status topo_check_params(const rs_topo_params* p) {
  if (p->L < 2 || p->L > 128) return fail(RS_EINVAL, "L must be in 2..128");
  if (p->cap < 1 || p->cap > 1024 || p->cap > p->L * p->L) return fail(RS_EINVAL, "cap must be in 1..min(1024, L*L)");
  if (p->n_attempts > 4096) return fail(RS_EINVAL, "n_attempts must be <= 4096");
  if (!(p->p_form >= 0) || !(p->sigma_form > 0) || !(p->p_elim_dep >= 0) || !(p->p_elim_pot >= 0))
    return fail(RS_EINVAL, "probabilities must be >= 0 and sigma_form > 0");
  if (!(std::fabs(p->g_new) <= TOPO_W_MAX) || !(std::fabs(p->g_init) <= TOPO_W_MAX))
    return fail(RS_EINVAL, "g_new and g_init must lie within +-1e4");
  return RS_OK;
}

// Allocate and build one projection between L x L sheets (rows by the
// pairwise-Bernoulli rule with the formation probability) with its rewiring
// state; `seed` keys the build draws together with p->proj_id.
rs_status topo_proj_build(rs_topo* t, const rs_topo_params* p, uint64_t seed, TopoDev& td, uint64_t** T_d2_out) {
  hipStream_t s = t->stream;
  const int L = (int)p->L, N = L * L;
  ProjDev& P = td.P;
  P.n_pre = N;
  P.n_post = N;
  P.cap = (int)p->cap;
  P.words = (N + 31) / 32;
  P.recurrent = 0;
  P.proj_id = (int)p->proj_id;
  Arena& ar = t->arena;
  TRY(ar.alloc(&P.len, (size_t)N));
  TRY(ar.alloc(&P.ind, (size_t)N * P.cap));
  TRY(ar.alloc(&P.w, (size_t)N * P.cap));
  const int half = L / 2, n_d2 = 2 * half * half + 1;
  std::vector<uint64_t> T(n_d2);
  for (int d2 = 0; d2 < n_d2; ++d2)
    T[d2] = threshold((double)p->p_form * std::exp(-(double)d2 / (2.0 * (double)p->sigma_form * (double)p->sigma_form)));
  TRY(ar.alloc(T_d2_out, (size_t)n_d2));
  TRY(ar.alloc(&td.bits, (size_t)N * P.words));
  TRY(ar.alloc(&td.kcount, (size_t)N));
  TRY(ar.alloc(&td.rowlist, (size_t)std::max<uint32_t>(p->n_attempts, 1)));
  TRY(ar.alloc(&td.nrows, 1));
  TRY(ar.alloc(&td.stats, 4));
  TRY(ar.alloc(&td.col_dirty, 1));
  HIP_OK(hipMemcpyAsync(*T_d2_out, T.data(), n_d2 * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  td.T_d2 = *T_d2_out;
  td.L = L;
  td.n_attempts = (int)p->n_attempts;
  td.g_theta = p->g_theta;
  td.g_new = p->g_new;
  td.T_dep = threshold(p->p_elim_dep);
  td.T_pot = threshold(p->p_elim_pot);
  launch_fill_zero(s, P.ind, (size_t)N * P.cap * 4);
  launch_fill_zero(s, P.w, (size_t)N * P.cap * 4);
  launch_gauss_rows(s, seed, P, L, td.T_d2, p->g_init, true);
  launch_fill_zero(s, td.bits, (size_t)N * P.words * 4);
  launch_fill_zero(s, td.stats, 32);
  launch_fill_zero(s, td.col_dirty, 4);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status topo_create_impl(const rs_topo_params* p, void* stream, rs_topo* t) {
  TRY(topo_check_params(p));
  t->p = *p;
  t->stream = (hipStream_t)stream;
  hipStream_t s = t->stream;
  TRY(topo_proj_build(t, p, p->seed, t->t, &t->T_d2));
  HIP_OK(hipEventCreate(&t->ev0));
  HIP_OK(hipEventCreate(&t->ev1));
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  return RS_OK;
}

}  // namespace

extern "C" {

rs_status rs_topo_create(const rs_topo_params* p, void* hip_stream, rs_topo** out) {
  if (!out || !p) return fail(RS_EINVAL, "NULL argument");
  *out = nullptr;
  rs_topo* t = new rs_topo();
  rs_status st = topo_create_impl(p, hip_stream, t);
  if (st != RS_OK) {
    (void)hipStreamSynchronize(t->stream);
    t->arena.release();
    delete t;
    return st;
  }
  *out = t;
  return RS_OK;
}

}  // extern "C"

namespace {

rs_status topo_rewire_impl(rs_topo* t, TopoDev& td, uint32_t n_attempts, uint64_t step, rs_rewire_stats* st) {
  if (step == STEP_FROM_DEVICE) return fail(RS_EINVAL, "step 2^64-1 is reserved");
  hipStream_t s = t->stream;
  launch_fill_zero(s, td.stats, 32);
  HIP_OK(hipEventRecord(t->ev0, s));
  launch_topo_rewire(s, t->p.seed, td, step);
  HIP_OK(hipEventRecord(t->ev1, s));
  t->timed = true;
  HIP_OK(hipGetLastError());
  if (st) {
    long long h[4];
    HIP_OK(hipMemcpyAsync(h, td.stats, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    st->eliminated = h[0];
    st->formed = h[1];
    st->blocked = h[2];
    st->attempts = n_attempts;
  }
  return RS_OK;
}

rs_status topo_get_rows_impl(rs_topo* t, const ProjDev& P, int32_t* len, int32_t* ind, float* w) {
  if (!len || !ind || !w) return fail(RS_EINVAL, "NULL argument");
  const size_t n = (size_t)P.n_pre * P.cap;
  HIP_OK(hipMemcpyAsync(len, P.len, (size_t)P.n_pre * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipMemcpyAsync(ind, P.ind, n * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipMemcpyAsync(w, P.w, n * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status topo_set_rows_impl(rs_topo* t, TopoDev& td, const int32_t* len, const int32_t* ind, const float* w) {
  if (!len || !ind || !w) return fail(RS_EINVAL, "NULL argument");
  const ProjDev& P = td.P;
  for (int i = 0; i < P.n_pre; ++i) {
    if (len[i] < 0 || len[i] > P.cap) return fail(RS_EINVAL, "row %d length %d outside 0..%d", i, len[i], P.cap);
    for (int k = 0; k < len[i]; ++k) {
      const int32_t j = ind[(size_t)i * P.cap + k];
      if (j < 0 || j >= P.n_post) return fail(RS_EINVAL, "row %d slot %d target %d out of range", i, k, j);
      const float wk = w[(size_t)i * P.cap + k];
      if (!(std::fabs(wk) <= TOPO_W_MAX)) return fail(RS_EINVAL, "row %d slot %d weight outside +-1e4", i, k);
    }
    std::vector<int32_t> r(ind + (size_t)i * P.cap, ind + (size_t)i * P.cap + len[i]);
    std::sort(r.begin(), r.end());
    if (std::adjacent_find(r.begin(), r.end()) != r.end()) return fail(RS_EINVAL, "row %d holds a target twice", i);
  }
  const size_t n = (size_t)P.n_pre * P.cap;
  HIP_OK(hipStreamSynchronize(t->stream));
  HIP_OK(hipMemcpyAsync(P.len, len, (size_t)P.n_pre * 4, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipMemcpyAsync(P.ind, ind, n * 4, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipMemcpyAsync(P.w, w, n * 4, hipMemcpyHostToDevice, t->stream));
  static const int one = 1;
  HIP_OK(hipMemcpyAsync(td.col_dirty, &one, 4, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status topo_get_bits_impl(rs_topo* t, const TopoDev& td, uint32_t* bits) {
  if (!bits) return fail(RS_EINVAL, "NULL argument");
  const ProjDev& P = td.P;
  HIP_OK(hipMemcpyAsync(bits, td.bits, (size_t)P.n_pre * P.words * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

// Synchronise and report a step barrier of the tiled kernel that gave up.
rs_status topo_sync_check(rs_topo* t) {
  HIP_OK(hipStreamSynchronize(t->stream));
  if (t->sim && t->tiled) {
    int e = 0;
    HIP_OK(hipMemcpyAsync(&e, t->sd.err, 4, hipMemcpyDeviceToHost, t->stream));
    HIP_OK(hipStreamSynchronize(t->stream));
    if (e) return fail(RS_EDEVICE, "a step barrier of the tiled simulation timed out (workgroups not resident)");
  }
  return RS_OK;
}

}  // namespace

extern "C" {

rs_status rs_topo_rewire(rs_topo* t, uint64_t step, rs_rewire_stats* st) {
  ENTER(t);
  return topo_rewire_impl(t, t->t, t->p.n_attempts, step, st);
}

rs_status rs_topo_get_rows(rs_topo* t, int32_t* len, int32_t* ind, float* w) {
  ENTER(t);
  return topo_get_rows_impl(t, t->t.P, len, ind, w);
}

rs_status rs_topo_set_rows(rs_topo* t, const int32_t* len, const int32_t* ind, const float* w) {
  ENTER(t);
  return topo_set_rows_impl(t, t->t, len, ind, w);
}

rs_status rs_topo_get_bits(rs_topo* t, uint32_t* bits) {
  ENTER(t);
  return topo_get_bits_impl(t, t->t, bits);
}

rs_status rs_topo_add_lateral(rs_topo* t, const rs_topo_params* lp) {
  ENTER(t);
  if (!lp) return fail(RS_EINVAL, "NULL argument");
  if (t->lateral) return fail(RS_ESTATE, "the map has a lateral projection");
  if (t->sim) return fail(RS_ESTATE, "add the lateral projection before rs_topo_sim_init");
  TRY(topo_check_params(lp));
  if (lp->L != t->p.L) return fail(RS_EINVAL, "the lateral projection joins the target sheet to itself: L %u != %u",
                                   lp->L, t->p.L);
  if (lp->proj_id == t->p.proj_id) return fail(RS_EINVAL, "the lateral projection needs its own proj_id");
  t->pl = *lp;
  TRY(topo_proj_build(t, lp, t->p.seed, t->tl, &t->T_d2_l));
  HIP_OK(hipStreamSynchronize(t->stream));
  t->lateral = true;
  return RS_OK;
}

rs_status rs_topo_lat_rewire(rs_topo* t, uint64_t step, rs_rewire_stats* st) {
  ENTER(t);
  if (!t->lateral) return fail(RS_ESTATE, "the map has no lateral projection");
  return topo_rewire_impl(t, t->tl, t->pl.n_attempts, step, st);
}

rs_status rs_topo_lat_get_rows(rs_topo* t, int32_t* len, int32_t* ind, float* w) {
  ENTER(t);
  if (!t->lateral) return fail(RS_ESTATE, "the map has no lateral projection");
  return topo_get_rows_impl(t, t->tl.P, len, ind, w);
}

rs_status rs_topo_lat_set_rows(rs_topo* t, const int32_t* len, const int32_t* ind, const float* w) {
  ENTER(t);
  if (!t->lateral) return fail(RS_ESTATE, "the map has no lateral projection");
  return topo_set_rows_impl(t, t->tl, len, ind, w);
}

rs_status rs_topo_lat_get_bits(rs_topo* t, uint32_t* bits) {
  ENTER(t);
  if (!t->lateral) return fail(RS_ESTATE, "the map has no lateral projection");
  return topo_get_bits_impl(t, t->tl, bits);
}

rs_status rs_topo_last_ms(rs_topo* t, double* ms) {
  ENTER(t);
  if (!ms) return fail(RS_EINVAL, "NULL argument");
  if (!t->timed) return fail(RS_ESTATE, "no rewire has run");
  float f = 0.f;
  HIP_OK(hipEventSynchronize(t->ev1));
  HIP_OK(hipEventElapsedTime(&f, t->ev0, t->ev1));
  *ms = f;
  return RS_OK;
}

rs_status rs_topo_sim_init(rs_topo* t, const rs_topo_model* m) {
  ENTER(t);
  if (!m) return fail(RS_EINVAL, "NULL argument");
  const int L = (int)t->p.L, N = L * L;
  TRY(topo_pick_kernel(t, t->kernel));
  if (m->stim_tile != 0 && (m->stim_tile > (uint32_t)L || L % (int)m->stim_tile))
    return fail(RS_EINVAL, "stim_tile %u must divide L = %d", m->stim_tile, L);
  if (!(m->h > 0) || !(m->C_m > 0) || !(m->tau_m > 0) || !(m->tau_s > 0) || !(m->tau_plus > 0) ||
      !(m->tau_minus > 0))
    return fail(RS_EINVAL, "h, C_m and every time constant must be > 0");
  if (m->stim_steps < 1) return fail(RS_EINVAL, "stim_steps must be >= 1");
  if (m->stim_kind != RS_STIM_BLOB && m->stim_kind != RS_STIM_BAR) return fail(RS_EINVAL, "unknown stim_kind");
  if (!(m->f_base >= 0) || !(m->f_peak >= 0) || !(m->sigma_stim > 0))
    return fail(RS_EINVAL, "rates must be >= 0 and sigma_stim > 0");
  if (m->ref_steps > (1u << 30)) return fail(RS_EINVAL, "ref_steps too large");
  // potentiation clips weights at g_max: keep it within the range the
  // fixed-point delivery sums hold
  if (!(m->g_max >= 0 && m->g_max <= TOPO_W_MAX)) return fail(RS_EINVAL, "g_max must lie in [0, 1e4]");
  if (!(m->A_plus >= 0 && m->A_plus <= TOPO_W_MAX) || !(m->A_minus >= 0 && m->A_minus <= TOPO_W_MAX))
    return fail(RS_EINVAL, "A_plus and A_minus must lie in [0, 1e4]");
  hipStream_t s = t->stream;
  TopoSimDev& d = t->sd;
  const int words = (N + 31) / 32, half = L / 2, n_d2 = 2 * half * half + 1;
  if (!t->sim) {
    Arena& ar = t->arena;
    uint64_t* T_in = nullptr;
    TRY(ar.alloc(&d.V, (size_t)N));
    TRY(ar.alloc(&d.g, (size_t)N));
    TRY(ar.alloc(&d.y, (size_t)N));
    TRY(ar.alloc(&d.x, (size_t)N));
    TRY(ar.alloc(&d.ref, (size_t)N));
    TRY(ar.alloc(&d.count, (size_t)N));
    TRY(ar.alloc(&d.zin, (size_t)words));
    TRY(ar.alloc(&d.zout, (size_t)words));
    TRY(ar.alloc(&d.col_len, (size_t)N));
    TRY(ar.alloc(&d.col_ent, (size_t)N * N));
    TRY(ar.alloc(&T_in, (size_t)n_d2));
    TRY(ar.alloc(&t->step_dev, 1));
    TRY(ar.alloc(&t->ticks, (size_t)TOPO_PHASES));
    d.T_in = T_in;
    // the tiled kernel's step exchange and barrier
    TRY(ar.alloc(&d.zin_b, (size_t)words));
    TRY(ar.alloc(&d.zout_b, (size_t)words));
    TRY(ar.alloc(&d.x_b, (size_t)N));
    TRY(ar.alloc(&d.bar, (size_t)TOPO_TILES_MAX * 16));
    TRY(ar.alloc(&d.err, 1));
    if (t->lateral) {
      TRY(ar.alloc(&d.xl, (size_t)N));
      TRY(ar.alloc(&d.xl_b, (size_t)N));
      TRY(ar.alloc(&d.col_len_l, (size_t)N));
      TRY(ar.alloc(&d.col_ent_l, (size_t)N * N));
    }
  }
  topo_drop_graph(t);  // the recorded launches carry the old constants
  t->m = *m;
  d.L = L;
  d.N = N;
  d.ref_steps = (int)m->ref_steps;
  d.stim_steps = (int)m->stim_steps;
  d.stim_kind = m->stim_kind;
  d.stim_L = m->stim_tile ? (int)m->stim_tile : L;
  d.stdp = m->stdp ? 1 : 0;
  d.V_rest = m->V_rest;
  d.E_exc = m->E_exc;
  d.V_th = m->V_th;
  d.V_reset = m->V_reset;
  d.R = m->tau_m / m->C_m;
  d.em = (float)std::exp(-(double)m->h / (double)m->tau_m);
  d.es = (float)std::exp(-(double)m->h / (double)m->tau_s);
  d.dx = (float)std::exp(-(double)m->h / (double)m->tau_plus);
  d.dy = (float)std::exp(-(double)m->h / (double)m->tau_minus);
  d.inv_dx = (float)(1.0 / (double)d.dx);
  d.A_plus = m->A_plus;
  d.A_minus = m->A_minus;
  d.g_max = m->g_max;
  d.col_dirty = t->t.col_dirty;
  d.step_dev = t->step_dev;
  t->t.step_dev = t->step_dev;
  d.col_cap = N;
  t->t.col_len = d.col_len;  // from here on the rewire edits the simulation's column view
  t->t.col_ent = d.col_ent;
  t->t.col_cap = N;
  if (t->lateral) {
    d.col_dirty_l = t->tl.col_dirty;
    t->tl.step_dev = t->step_dev;
    t->tl.col_len = d.col_len_l;
    t->tl.col_ent = d.col_ent_l;
    t->tl.col_cap = N;
  }
  // Bernoulli threshold of one step of the source's Poisson train, by the
  // integer squared distance from the stimulus (Tab. E rate profile)
  std::vector<uint64_t> T(n_d2);
  const double sg = (double)m->sigma_stim;
  for (int d2 = 0; d2 < n_d2; ++d2) {
    const double rate = (double)m->f_base + (double)m->f_peak * std::exp(-(double)d2 / (2.0 * sg * sg));
    T[d2] = threshold(rate * (double)m->h / 1000.0);
  }
  HIP_OK(hipMemcpyAsync((void*)d.T_in, T.data(), n_d2 * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  std::vector<float> vr((size_t)N, m->V_rest);
  HIP_OK(hipMemcpyAsync(d.V, vr.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
  launch_fill_zero(s, d.g, (size_t)N * 4);
  launch_fill_zero(s, d.y, (size_t)N * 4);
  launch_fill_zero(s, d.x, (size_t)N * 4);
  launch_fill_zero(s, d.ref, (size_t)N * 4);
  launch_fill_zero(s, d.count, (size_t)N * 4);
  launch_fill_zero(s, d.zin, (size_t)words * 4);
  launch_fill_zero(s, d.zout, (size_t)words * 4);
  // the column view is rebuilt by the first simulation launch (col_dirty);
  // until then a rewire's column edits find empty columns
  launch_fill_zero(s, d.col_len, (size_t)N * 4);
  launch_fill_zero(s, t->step_dev, 8);
  launch_fill_zero(s, t->ticks, 8 * TOPO_PHASES);
  launch_fill_zero(s, d.bar, (size_t)TOPO_TILES_MAX * 16 * 8);
  launch_fill_zero(s, d.err, 4);
  d.ticks = nullptr;  // timers off until rs_topo_sim_timing
  static const int one = 1;
  HIP_OK(hipMemcpyAsync(t->t.col_dirty, &one, 4, hipMemcpyHostToDevice, s));
  if (t->lateral) {
    launch_fill_zero(s, d.xl, (size_t)N * 4);
    launch_fill_zero(s, d.col_len_l, (size_t)N * 4);
    HIP_OK(hipMemcpyAsync(t->tl.col_dirty, &one, 4, hipMemcpyHostToDevice, s));
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  t->step = 0;
  t->sim = true;
  return RS_OK;
}

rs_status rs_topo_run(rs_topo* t, uint64_t n_steps) {
  ENTER(t);
  if (!t->sim) return fail(RS_ESTATE, "rs_topo_sim_init has not run");
  hipStream_t s = t->stream;
  const uint64_t R = t->m.rewire_steps;
  constexpr uint64_t MAX_CHUNK = 10000;  // steps per launch without rewiring
  launch_fill_zero(s, t->t.stats, 32);
  if (t->lateral) launch_fill_zero(s, t->tl.stats, 32);
  HIP_OK(hipEventRecord(t->ev0, s));
  uint64_t left = n_steps;
  while (left > 0) {
    if (R && t->step % R == 0 && left >= R * GRAPH_INTERVALS) {
      if (!t->gexec) TRY(topo_build_graph(t));
      HIP_OK(hipGraphLaunch(t->gexec, s));
      t->step += R * GRAPH_INTERVALS;
      left -= R * GRAPH_INTERVALS;
      continue;
    }
    uint64_t chunk = R ? R - t->step % R : MAX_CHUNK;
    if (chunk > left) chunk = left;
    if (chunk > MAX_CHUNK) chunk = MAX_CHUNK;
    topo_launch_sim(t, s, t->step, (int)chunk);
    t->step += chunk;
    left -= chunk;
    if (R && t->step % R == 0) topo_launch_rewires(t, s, t->step);
  }
  HIP_OK(hipEventRecord(t->ev1, s));
  t->timed = true;
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_topo_sim_timing(rs_topo* t, int32_t on) {
  ENTER(t);
  if (!t->sim) return fail(RS_ESTATE, "rs_topo_sim_init has not run");
  HIP_OK(hipStreamSynchronize(t->stream));
  launch_fill_zero(t->stream, t->ticks, 8 * TOPO_PHASES);
  unsigned long long* want = on ? t->ticks : nullptr;
  if (t->sd.ticks != want) {
    t->sd.ticks = want;
    topo_drop_graph(t);  // the recorded launches carry the old setting
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status rs_topo_sim_phase_ms(rs_topo* t, double* ms) {
  ENTER(t);
  if (!ms) return fail(RS_EINVAL, "NULL argument");
  if (!t->sim) return fail(RS_ESTATE, "rs_topo_sim_init has not run");
  unsigned long long h[TOPO_PHASES];
  HIP_OK(hipMemcpyAsync(h, t->ticks, sizeof h, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  int dev = 0, khz = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(RS_EDEVICE, "the device reports no wall-clock rate");
  for (int q = 0; q < TOPO_PHASES; ++q) ms[q] = (double)h[q] / (double)khz;
  return RS_OK;
}

rs_status rs_topo_lat_run_stats(rs_topo* t, rs_rewire_stats* st) {
  ENTER(t);
  if (!st) return fail(RS_EINVAL, "NULL argument");
  if (!t->lateral) return fail(RS_ESTATE, "the map has no lateral projection");
  TRY(topo_sync_check(t));
  long long h[4];
  HIP_OK(hipMemcpyAsync(h, t->tl.stats, sizeof h, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  st->eliminated = h[0];
  st->formed = h[1];
  st->blocked = h[2];
  st->attempts = 0;
  return RS_OK;
}

rs_status rs_topo_sim_kernel(rs_topo* t, int32_t kind) {
  ENTER(t);
  if (kind != RS_TOPO_KERNEL_AUTO && kind != RS_TOPO_KERNEL_ONE_WG && kind != RS_TOPO_KERNEL_TILED)
    return fail(RS_EINVAL, "unknown simulation kernel %d", kind);
  if (t->sim) {
    TRY(topo_sync_check(t));
    TRY(topo_pick_kernel(t, kind));
    topo_drop_graph(t);  // the recorded launches use the old kernel
  }
  t->kernel = kind;
  return RS_OK;
}

rs_status rs_topo_run_stats(rs_topo* t, rs_rewire_stats* st) {
  ENTER(t);
  if (!st) return fail(RS_EINVAL, "NULL argument");
  TRY(topo_sync_check(t));
  long long h[4];
  HIP_OK(hipMemcpyAsync(h, t->t.stats, sizeof h, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  st->eliminated = h[0];
  st->formed = h[1];
  st->blocked = h[2];
  st->attempts = 0;
  return RS_OK;
}

namespace {
rs_status topo_var(rs_topo* t, int32_t var, void** dev, size_t* bytes, bool* writable) {
  if (!t->sim) return fail(RS_ESTATE, "rs_topo_sim_init has not run");
  const size_t N = (size_t)t->sd.N, words = (N + 31) / 32;
  *writable = true;
  switch (var) {
    case RS_TV_V: *dev = t->sd.V; *bytes = N * 4; return RS_OK;
    case RS_TV_G: *dev = t->sd.g; *bytes = N * 4; return RS_OK;
    case RS_TV_Y: *dev = t->sd.y; *bytes = N * 4; return RS_OK;
    case RS_TV_X: *dev = t->sd.x; *bytes = N * 4; return RS_OK;
    case RS_TV_REF: *dev = t->sd.ref; *bytes = N * 4; return RS_OK;
    case RS_TV_COUNT: *dev = t->sd.count; *bytes = N * 4; return RS_OK;
    case RS_TV_ZIN: *dev = t->sd.zin; *bytes = words * 4; return RS_OK;
    case RS_TV_ZOUT: *dev = t->sd.zout; *bytes = words * 4; *writable = false; return RS_OK;
    case RS_TV_XLAT:
      if (!t->lateral) return fail(RS_EINVAL, "the map has no lateral projection");
      *dev = t->sd.xl; *bytes = N * 4; return RS_OK;
    case RS_TV_STEP: *dev = nullptr; *bytes = 8; return RS_OK;
    default: return fail(RS_EINVAL, "unknown topomap variable %d", var);
  }
}
}  // namespace

rs_status rs_topo_sim_get(rs_topo* t, int32_t var, void* host, size_t bytes) {
  ENTER(t);
  if (!host) return fail(RS_EINVAL, "NULL argument");
  void* dev = nullptr;
  size_t need = 0;
  bool wr = false;
  TRY(topo_var(t, var, &dev, &need, &wr));
  if (bytes != need) return fail(RS_EINVAL, "variable %d needs %zu bytes, got %zu", var, need, bytes);
  TRY(topo_sync_check(t));
  if (var == RS_TV_STEP) {
    std::memcpy(host, &t->step, 8);
    return RS_OK;
  }
  HIP_OK(hipMemcpyAsync(host, dev, need, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status rs_topo_sim_set(rs_topo* t, int32_t var, const void* host, size_t bytes) {
  ENTER(t);
  if (!host) return fail(RS_EINVAL, "NULL argument");
  void* dev = nullptr;
  size_t need = 0;
  bool wr = false;
  TRY(topo_var(t, var, &dev, &need, &wr));
  if (!wr) return fail(RS_EINVAL, "variable %d is read-only", var);
  if (bytes != need) return fail(RS_EINVAL, "variable %d needs %zu bytes, got %zu", var, need, bytes);
  if (var == RS_TV_REF) {
    const int32_t* r = (const int32_t*)host;
    for (int j = 0; j < t->sd.N; ++j)
      if (r[j] < 0) return fail(RS_EINVAL, "refractory count of neuron %d is negative", j);
  }
  if (var == RS_TV_ZIN && t->sd.N % 32) {
    const uint32_t last = ((const uint32_t*)host)[need / 4 - 1];
    if (last >> (t->sd.N % 32)) return fail(RS_EINVAL, "spike bits beyond the sheet are set");
  }
  HIP_OK(hipStreamSynchronize(t->stream));
  if (var == RS_TV_STEP) {
    uint64_t v;
    std::memcpy(&v, host, 8);
    if (v == STEP_FROM_DEVICE) return fail(RS_EINVAL, "step count 2^64-1 is reserved");
    std::memcpy(&t->step, host, 8);
    HIP_OK(hipMemcpyAsync(t->step_dev, &t->step, 8, hipMemcpyHostToDevice, t->stream));
    HIP_OK(hipStreamSynchronize(t->stream));
    return RS_OK;
  }
  HIP_OK(hipMemcpyAsync(dev, host, need, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

void rs_topo_destroy(rs_topo* t) {
  if (!t) return;
  (void)hipStreamSynchronize(t->stream);
  topo_drop_graph(t);
  if (t->cap_stream) (void)hipStreamDestroy(t->cap_stream);
  if (t->ev0) (void)hipEventDestroy(t->ev0);
  if (t->ev1) (void)hipEventDestroy(t->ev1);
  t->arena.release();
  delete_custom(t->custom);
  delete t;
}

rs_status rs_calib_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16) return fail(RS_EINVAL, "copy needs non-NULL pointers and bytes % 16 == 0");
  launch_copy((hipStream_t)hip_stream, dst, src, bytes);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

}  // extern "C"

// =========================================================================== batched networks
// A set of e-prop networks of different sizes trained together (the paper's
// batching of model copies, here copies of different sizes): every kernel of
// a step block runs once for all networks, over a work list of (network, tile)
// entries, and one whole training sample (its blocks, updates, DEEP R rewires
// and the reset) is recorded once as a HIP graph and replayed.  Each network
// is an ordinary rs_eprop object underneath, so it computes exactly what it
// computes alone.
namespace {

constexpr int MULTI_SCHEDULES = 5;
// e-prop schedules the tuner tries: threads per row, rows per work tile,
// persistent workgroups (0: one per tile)
constexpr int SCHED_TPR[MULTI_SCHEDULES] = {256, 64, 64, 64, 256};
constexpr int SCHED_TILE[MULTI_SCHEDULES] = {1, 4, 16, 4, 4};
constexpr int SCHED_GRID[MULTI_SCHEDULES] = {0, 0, 0, 2048, 2048};

// Bump allocator over a host image of the device tables.
struct TableImage {
  std::vector<unsigned char> host;
  template <class T>
  size_t put(const T* v, size_t n) {
    const size_t off = (host.size() + 255) & ~(size_t)255;
    host.resize(off + sizeof(T) * n);
    if (n) memcpy(host.data() + off, v, sizeof(T) * n);
    return off;
  }
  template <class T>
  size_t put(const std::vector<T>& v) { return put(v.data(), v.size()); }
};

struct MultiBlock {
  int h, nsteps;
  uint64_t t0;          // first step, from the sample's start
  bool covered;         // the next update's join orders the segment's reuse
  size_t fwd, work_fwd, ho, ho_B, work_ho, ro, work_ro, work_ls, ep;
  int n_fwd, n_ho, n_ro, n_ls;
  size_t work_ep[MULTI_SCHEDULES];
  int n_ep[MULTI_SCHEDULES];
};
struct MultiUpdate {
  uint64_t t;           // the update follows step t - 1 (from the sample's start)
  size_t up, work_up, dr, work_dr;
  int n_up, n_proj, n_rows;
};

}  // namespace

struct rs_multi {
  std::vector<rs_eprop*> inst;
  hipStream_t stream = nullptr;       // the caller's: forward pass of every block
  hipStream_t side = nullptr;         // e-prop, updates, rewiring, reset
  Arena arena;
  int n = 0, B = 1, K = 20, Q = 2;
  uint32_t U = 0, T = 0;
  bool alif = true;
  int fwd_items = 1, max_cap = 1, max_pre = 1;
  size_t fwd_lds = 0;
  uint64_t* step_dev = nullptr;       // steps done, at the start of the sample being run
  uint32_t* adam_dev = nullptr;       // updates done, at the start of the sample
  float* adam_tab = nullptr;          // [2 * (adam_kmax + 1)] bias corrections by update count
  int adam_kmax = 0;
  unsigned char* tab = nullptr;       // device tables of the recorded sample
  size_t tab_bytes = 0;
  std::vector<MultiBlock> blocks;
  std::vector<MultiUpdate> updates;
  size_t zero_ranges = 0;
  int n_zero = 0;
  unsigned long long zero_max = 0;
  bool tables_ok = false;
  int sched = 0;                      // e-prop schedule in use
  bool tuned = false;
  double sched_ms[MULTI_SCHEDULES] = {0};  // device time of one sample per schedule (tuning)
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_sched = -1;
  hipEvent_t ev_fwd = nullptr, ev_back = nullptr, ev_join = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  hipEvent_t ev_ep[RING_MAX] = {};
  uint64_t samples = 0;
  bool dead = false;
};

namespace {

void multi_drop_graph(rs_multi* m) {
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->gexec = nullptr;
  m->graph = nullptr;
  m->graph_sched = -1;
}

// Lay out one training sample exactly as the one-network path cuts it into
// blocks (cut at every update and at the sample's end) and write every
// launch's arguments and work lists into the device tables.
rs_status multi_build_tables(rs_multi* m) {
  TableImage im;
  m->blocks.clear();
  m->updates.clear();
  const int n = m->n;
  // block and update positions within one sample
  struct Op { bool upd; uint64_t t0; int nsteps; };
  std::vector<Op> ops;
  {
    uint64_t open_t0 = 0;
    int open_n = 0;
    for (uint64_t st = 1; st <= m->T; ++st) {
      if (open_n == 0) open_t0 = st - 1;
      ++open_n;
      if (open_n == m->K) { ops.push_back({false, open_t0, open_n}); open_n = 0; }
      if (st % m->U == 0 || st == m->T) {
        if (open_n) { ops.push_back({false, open_t0, open_n}); open_n = 0; }
        if (st % m->U == 0) ops.push_back({true, st, 0});
      }
    }
  }
  int blk = 0;
  for (size_t q = 0; q < ops.size(); ++q) {
    const Op& o = ops[q];
    if (o.upd) {
      MultiUpdate u{};
      u.t = o.t0;
      std::vector<UpdateArgs> ua(n);
      std::vector<int4> uw;
      std::vector<DeeprArgs> da;
      std::vector<int2> dw;
      const uint32_t k_in_sample = (uint32_t)m->updates.size() + 1;
      for (int i = 0; i < n; ++i) {
        rs_eprop* e = m->inst[i];
        ua[i] = update_args(e, 1);
        ua[i].adam_tab = m->adam_tab;
        ua[i].adam_base = m->adam_dev;
        ua[i].adam_off = (int)k_in_sample;
        ua[i].adam_kmax = m->adam_kmax;
        const int nb = update_blocks(ua[i]);
        for (int b = 0; b < nb; ++b) uw.push_back(make_int4(i, b, nb, 0));
        for (int p = 0; p < 2; ++p) {
          if (!((e->p.deepr_mask >> p) & 1u)) continue;
          DeeprArgs d{};
          d.seed = e->p.seed;
          d.P = p == 0 ? e->in : e->rec;
          d.B = e->B;
          d.step = o.t0;
          d.step_base = m->step_dev;
          d.stats = e->rw_stats;
          for (int r = 0; r < d.P.n_pre; ++r) dw.push_back(make_int2((int)da.size(), r));
          da.push_back(d);
        }
      }
      u.up = im.put(ua);
      u.work_up = im.put(uw);
      u.n_up = (int)uw.size();
      u.dr = im.put(da);
      u.work_dr = im.put(dw);
      u.n_proj = (int)da.size();
      u.n_rows = (int)dw.size();
      m->updates.push_back(u);
      continue;
    }
    MultiBlock b{};
    b.h = blk % m->Q;
    b.t0 = o.t0;
    b.nsteps = o.nsteps;
    {  // covered: fewer than Q blocks remain to the next update from this block's end
      const uint64_t end = o.t0 + (uint64_t)o.nsteps, U = m->U, rem = (U - end % U) % U;
      b.covered = (rem + (uint64_t)m->K - 1) / (uint64_t)m->K < (uint64_t)m->Q;
    }
    std::vector<FwdArgs> fa(n);
    std::vector<HandoffArrays> ha(n);
    std::vector<int> hB(n);
    std::vector<ReadoutArgs> ra(n);
    std::vector<EpropArgs> ea(n);
    std::vector<int2> fw;
    std::vector<int4> hw, rw, lw;
    std::vector<int4> ew[MULTI_SCHEDULES];
    for (int i = 0; i < n; ++i) {
      rs_eprop* e = m->inst[i];
      fa[i] = block_fwd_args(e, b.h, o.t0, o.nsteps);
      fa[i].rows_lds = 0;
      fa[i].step_base = m->step_dev;
      if (e->poisson) fa[i].step0 = o.t0;  // from the sample's start; the device adds the sample's first step
      fa[i].t0 = (int)(o.t0 % e->p.sample_steps);
      const size_t lds = fwd_plan(fa[i]);
      m->fwd_lds = std::max(m->fwd_lds, lds);
      m->fwd_items = std::max(m->fwd_items, fwd_items(fa[i].n_in, fa[i].n_rec));
      for (int bb = 0; bb < e->B; ++bb) fw.push_back(make_int2(i, bb));
      ha[i] = block_handoff_args(e, b.h, o.nsteps);
      hB[i] = e->B;
      int g[3];
      handoff_grid(ha[i], e->B, g);
      for (int z = 0; z < g[2]; ++z)
        for (int y = 0; y < g[1]; ++y)
          for (int x = 0; x < g[0]; ++x) hw.push_back(make_int4(i, x, y, z));
      ra[i] = block_readout_args(e, b.h, o.nsteps);
      for (int x = 0; x < readout_grid(ra[i]); ++x) rw.push_back(make_int4(i, x, 0, 0));
      learning_signal_grid(ra[i], g);
      for (int z = 0; z < g[2]; ++z)
        for (int y = 0; y < g[1]; ++y)
          for (int x = 0; x < g[0]; ++x) lw.push_back(make_int4(i, x, y, z));
      ea[i] = block_eprop_args(e, b.h, o.nsteps);
      const int rows = ea[i].n_in + ea[i].n_rec, chunks = narrow_readout_chunks(ea[i].n_rec);
      for (int sc = 0; sc < MULTI_SCHEDULES; ++sc) {
        for (int r = 0; r < rows; r += SCHED_TILE[sc])
          ew[sc].push_back(make_int4(i, r, std::min(SCHED_TILE[sc], rows - r), 0));
        for (int c = 0; c < chunks; ++c) ew[sc].push_back(make_int4(i, rows + c, 1, 0));
      }
    }
    b.fwd = im.put(fa);
    b.work_fwd = im.put(fw);
    b.n_fwd = (int)fw.size();
    b.ho = im.put(ha);
    b.ho_B = im.put(hB);
    b.work_ho = im.put(hw);
    b.n_ho = (int)hw.size();
    b.ro = im.put(ra);
    b.work_ro = im.put(rw);
    b.n_ro = (int)rw.size();
    b.work_ls = im.put(lw);
    b.n_ls = (int)lw.size();
    b.ep = im.put(ea);
    for (int sc = 0; sc < MULTI_SCHEDULES; ++sc) {
      b.work_ep[sc] = im.put(ew[sc]);
      b.n_ep[sc] = (int)ew[sc].size();
    }
    m->blocks.push_back(b);
    ++blk;
  }
  // the reset at the sample's end
  std::vector<ZeroRange> zr;
  for (rs_eprop* e : m->inst) {
    const size_t B = e->B, NR = e->p.n_rec, NI = e->p.n_in, K = e->p.n_out;
    zr.push_back({e->V, B * NR * 8});
    zr.push_back({e->A, B * NR * 8});
    zr.push_back({e->Y, B * K * 8});
    zr.push_back({e->xbar, B * NI * 4});
    zr.push_back({e->zbar, B * NR * 4});
    for (const ProjDev* P : {&e->in, &e->rec}) {
      const size_t bytes = (size_t)P->n_pre * P->cap * B * 4;
      zr.push_back({P->ebar, (size_t)P->n_pre * P->cap * P->erec * 4});
      if (P->eps) zr.push_back({P->eps, bytes});
    }
  }
  m->zero_max = 0;
  for (const ZeroRange& z : zr) m->zero_max = std::max(m->zero_max, z.bytes);
  m->zero_ranges = im.put(zr);
  m->n_zero = (int)zr.size();
  // upload
  multi_drop_graph(m);
  if (im.host.size() > m->tab_bytes) {
    if (m->tab) (void)hipFree(m->tab);
    m->tab = nullptr;
    m->tab_bytes = 0;
    if (hipMalloc(&m->tab, im.host.size()) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RS_ENOMEM, "device allocation of %zu bytes of launch tables failed", im.host.size());
    }
    m->tab_bytes = im.host.size();
  }
  HIP_OK(hipStreamSynchronize(m->stream));
  HIP_OK(hipStreamSynchronize(m->side));
  HIP_OK(hipMemcpy(m->tab, im.host.data(), im.host.size(), hipMemcpyHostToDevice));
  m->tables_ok = true;
  return RS_OK;
}

// Issue one training sample: the forward pass of each block on `s`, its
// e-prop launch on `e`, updates, rewiring and the reset on `e`, with the
// one-network path's event pattern between the two streams.  The same calls
// run directly or under stream capture.
void multi_issue_sample(rs_multi* m, int sched, hipStream_t s, hipStream_t e, std::vector<hipEvent_t>* ep_ev = nullptr) {
  unsigned char* T = m->tab;
  bool pending[RING_MAX] = {};
  size_t bi = 0, ui = 0;
  const size_t nb = m->blocks.size(), nu = m->updates.size();
  while (bi < nb || ui < nu) {
    const bool take_update = ui < nu && (bi >= nb || m->updates[ui].t <= m->blocks[bi].t0);
    if (!take_update) {
      const MultiBlock& b = m->blocks[bi++];
      if (pending[b.h]) {
        (void)hipStreamWaitEvent(s, m->ev_ep[b.h], 0);
        pending[b.h] = false;
      }
      launch_fwd_multi(s, (const FwdArgs*)(T + b.fwd), (const int2*)(T + b.work_fwd), b.n_fwd, m->fwd_items,
                       m->fwd_lds);
      launch_handoff_multi(s, (const HandoffArrays*)(T + b.ho), (const int*)(T + b.ho_B),
                           (const int4*)(T + b.work_ho), b.n_ho);
      launch_readout_multi(s, (const ReadoutArgs*)(T + b.ro), (const int4*)(T + b.work_ro), b.n_ro,
                           (const int4*)(T + b.work_ls), b.n_ls);
      (void)hipEventRecord(m->ev_fwd, s);
      (void)hipStreamWaitEvent(e, m->ev_fwd, 0);
      if (ep_ev) {
        hipEvent_t a = nullptr, z = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&z);
        ep_ev->push_back(a);
        ep_ev->push_back(z);
        (void)hipEventRecord(a, e);
      }
      launch_eprop_narrow_multi(e, (const EpropArgs*)(T + b.ep), (const int4*)(T + b.work_ep[sched]),
                                b.n_ep[sched], m->alif, SCHED_TPR[sched], SCHED_GRID[sched]);
      if (ep_ev) (void)hipEventRecord(ep_ev->back(), e);
      if (!b.covered) {
        (void)hipEventRecord(m->ev_ep[b.h], e);
        pending[b.h] = true;
      }
      continue;
    }
    const MultiUpdate& u = m->updates[ui++];
    launch_update_multi(e, (const UpdateArgs*)(T + u.up), (const int4*)(T + u.work_up), u.n_up);
    launch_deepr_multi(e, (const DeeprArgs*)(T + u.dr), u.n_proj, (const int2*)(T + u.work_dr), u.n_rows,
                       m->max_cap, m->max_pre);
    if (u.t == m->T)
      launch_fill_zero_ranges(e, (const ZeroRange*)(T + m->zero_ranges), m->n_zero, m->zero_max);
    (void)hipEventRecord(m->ev_back, e);
    (void)hipStreamWaitEvent(s, m->ev_back, 0);
    for (bool& p : pending) p = false;
  }
  // next sample: the device counts move on (the e stream follows the last join)
  launch_advance_counts(e, m->step_dev, m->T, m->adam_dev, (uint32_t)nu);
  (void)hipEventRecord(m->ev_back, e);
  (void)hipStreamWaitEvent(s, m->ev_back, 0);
}

rs_status multi_build_graph(rs_multi* m) {
  multi_drop_graph(m);
  hipStream_t s = m->stream;
  // capture on a stream of our own, joined to the caller's around replays
  hipStream_t cs = nullptr;
  fwd_attrs();  // launch attributes are set outside the capture
  deepr_attrs();
  HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (err == hipSuccess) {
    (void)hipEventRecord(m->ev_join, cs);
    (void)hipStreamWaitEvent(m->side, m->ev_join, 0);  // the side stream joins the capture
    multi_issue_sample(m, m->sched, cs, m->side);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(cs, &g);
    if (err == hipSuccess) {
      m->graph = g;
      err = hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0);
    }
  }
  (void)hipStreamDestroy(cs);
  (void)s;
  if (err != hipSuccess) {
    (void)hipGetLastError();
    multi_drop_graph(m);
    return fail(RS_EDEVICE, "recording the training-sample graph failed: %s", hipGetErrorString(err));
  }
  m->graph_sched = m->sched;
  return RS_OK;
}

// One sample, by graph replay or by direct launches; host counters follow.
// With ep_ms, the e-prop launches are timed (direct launches only).
rs_status multi_run_sample(rs_multi* m, int sched, bool graph, double* ep_ms = nullptr) {
  if (graph) {
    if (!m->gexec || m->graph_sched != sched) {
      m->sched = sched;
      TRY(multi_build_graph(m));
    }
    HIP_OK(hipGraphLaunch(m->gexec, m->stream));
  } else {
    order(m->ev_join, m->stream, m->side);
    std::vector<hipEvent_t> ev;
    multi_issue_sample(m, sched, m->stream, m->side, ep_ms ? &ev : nullptr);
    if (ep_ms) {
      *ep_ms = 0;
      for (size_t q = 0; q + 1 < ev.size(); q += 2) {
        float t = 0.f;
        HIP_OK(hipEventSynchronize(ev[q + 1]));
        HIP_OK(hipEventElapsedTime(&t, ev[q], ev[q + 1]));
        *ep_ms += t;
      }
      for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    }
  }
  for (rs_eprop* e : m->inst) {
    e->step += m->T;
    e->adam_k += (uint32_t)m->updates.size();
    const MultiBlock& last = m->blocks.back();
    e->last_seg = last.h;
    e->last_blk_n = last.nsteps;
    e->last_slot = last.h * e->K + last.nsteps - 1;
  }
  ++m->samples;
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status multi_validate(const rs_eprop_params* p, uint32_t n) {
  if (!p) return fail(RS_EINVAL, "params is NULL");
  if (n < 1 || n > 4096) return fail(RS_EINVAL, "the set holds 1..4096 networks");
  for (uint32_t i = 0; i < n; ++i) {
    TRY(validate(&p[i]));
    const rs_eprop_params &a = p[0], &b = p[i];
    if (b.batch % 4 == 0)
      return fail(RS_EINVAL, "network %u: batched sets take batches not divisible by 4 (the narrow kernel)", i);
    if (b.update_interval < 1 || b.sample_steps % b.update_interval != 0)
      return fail(RS_EINVAL, "network %u: sample_steps must be a multiple of update_interval >= 1", i);
    if (b.n_in != a.n_in || b.n_out != a.n_out || b.batch != a.batch || b.alif != a.alif ||
        b.dt_ms != a.dt_ms || b.tau_mem_ms != a.tau_mem_ms || b.tau_adapt_ms != a.tau_adapt_ms ||
        b.update_interval != a.update_interval || b.sample_steps != a.sample_steps ||
        b.trace_block != a.trace_block || b.adam_b1 != a.adam_b1 || b.adam_b2 != a.adam_b2)
      return fail(RS_EINVAL, "network %u differs from network 0 in n_in, n_out, batch, alif, time constants, "
                  "update interval, sample length, block length or Adam decay rates", i);
  }
  return RS_OK;
}

rs_status multi_create_impl(const rs_eprop_params* p, uint32_t n, void* stream, rs_multi* m) {
  TRY(multi_validate(p, n));
  m->stream = (hipStream_t)stream;
  m->n = (int)n;
  for (uint32_t i = 0; i < n; ++i) {
    rs_eprop* e = nullptr;
    rs_status st = create_impl(&p[i], stream, &e);
    if (st != RS_OK) {
      if (e) rs_eprop_destroy(e);
      return st;
    }
    m->inst.push_back(e);
  }
  rs_eprop* e0 = m->inst[0];
  m->B = e0->B;
  m->K = e0->K;
  m->Q = e0->Q;
  m->U = e0->p.update_interval;
  m->T = e0->p.sample_steps;
  m->alif = e0->p.alif != 0;
  for (rs_eprop* e : m->inst) {
    m->max_cap = std::max({m->max_cap, e->in.cap, e->rec.cap});
    m->max_pre = std::max({m->max_pre, e->in.n_pre, e->rec.n_pre});
  }
  HIP_OK(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
  for (hipEvent_t* ev : {&m->ev_fwd, &m->ev_back, &m->ev_join})
    HIP_OK(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  for (int q = 0; q < m->Q; ++q) HIP_OK(hipEventCreateWithFlags(&m->ev_ep[q], hipEventDisableTiming));
  HIP_OK(hipEventCreate(&m->ev_t0));
  HIP_OK(hipEventCreate(&m->ev_t1));
  // Adam bias corrections by update count, as the one-network path computes
  // them; beyond kmax both round to exactly 1
  {
    const double b1 = e0->p.adam_b1, b2 = e0->p.adam_b2;
    std::vector<float> tab = {1.0f, 1.0f};
    uint32_t k = 1;
    for (; k < (1u << 20); ++k) {
      const float c1 = adam_inv_c(b1, k), c2 = adam_inv_c(b2, k);
      tab.push_back(c1);
      tab.push_back(c2);
      if (c1 == 1.0f && c2 == 1.0f) break;
    }
    m->adam_kmax = (int)(tab.size() / 2 - 1);
    TRY(m->arena.alloc(&m->adam_tab, tab.size()));
    HIP_OK(hipMemcpyAsync(m->adam_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, m->stream));
  }
  TRY(m->arena.alloc(&m->step_dev, 1));
  TRY(m->arena.alloc(&m->adam_dev, 1));
  launch_fill_zero(m->stream, m->step_dev, 8);
  launch_fill_zero(m->stream, m->adam_dev, 4);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(m->stream));
  return RS_OK;
}

rs_status multi_index(rs_multi* m, uint32_t i) {
  if (i >= (uint32_t)m->n) return fail(RS_EINVAL, "network %u outside the set of %d", i, m->n);
  return RS_OK;
}

// The set's work on the side stream is ordered before later work on the
// caller's stream after every call; instance calls then see finished state.
void multi_join(rs_multi* m) { order(m->ev_back, m->side, m->stream); }

}  // namespace

extern "C" {

rs_status rs_multi_create(const rs_eprop_params* params, uint32_t n, void* hip_stream, rs_multi** out) {
  if (!out) return fail(RS_EINVAL, "out is NULL");
  *out = nullptr;
  rs_multi* m = new rs_multi();
  rs_status st = multi_create_impl(params, n, hip_stream, m);
  if (st != RS_OK) {
    rs_multi_destroy(m);
    return st;
  }
  *out = m;
  return RS_OK;
}

rs_status rs_multi_set_input(rs_multi* m, uint32_t i, const int32_t* off_dev, const int32_t* idx_dev,
                             size_t n_idx, const int32_t* labels_dev) {
  ENTER(m);
  TRY(multi_index(m, i));
  multi_join(m);
  TRY(rs_eprop_set_input(m->inst[i], off_dev, idx_dev, n_idx, labels_dev));
  m->tables_ok = false;
  return RS_OK;
}

rs_status rs_multi_set_input_poisson(rs_multi* m, uint32_t i, const double* rate_hz, size_t n_rates,
                                     const int32_t* labels_dev) {
  ENTER(m);
  TRY(multi_index(m, i));
  multi_join(m);
  TRY(rs_eprop_set_input_poisson(m->inst[i], rate_hz, n_rates, labels_dev));
  m->tables_ok = false;
  return RS_OK;
}

rs_status rs_multi_train(rs_multi* m, uint32_t n_samples) {
  ENTER(m);
  for (rs_eprop* e : m->inst) {
    if (!e->x_off && !e->poisson) return fail(RS_ESTATE, "a network of the set has no input attached");
    if (e->step % m->T != 0) return fail(RS_ESTATE, "the set is not at a sample boundary");
  }
  if (!m->tables_ok) TRY(multi_build_tables(m));
  for (uint32_t q = 0; q < n_samples; ++q) {
    if (!m->tuned) {
      // the tuner: the next untried schedule runs this sample (every schedule
      // computes the same results) with its e-prop launches timed on the
      // device; after the last one the fastest is kept.  Only the e-prop
      // launches are compared: their work is the same in every sample, while
      // the forward pass follows the networks' activity as they learn.
      int c = 0;
      while (c < MULTI_SCHEDULES && m->sched_ms[c] > 0) ++c;
      double ms = 0;
      TRY(multi_run_sample(m, c, false, &ms));
      m->sched_ms[c] = ms > 0 ? ms : 1e-6;
      if (c + 1 == MULTI_SCHEDULES) {
        int best = 0;
        for (int q2 = 1; q2 < MULTI_SCHEDULES; ++q2)
          if (m->sched_ms[q2] < m->sched_ms[best]) best = q2;
        m->sched = best;
        m->tuned = true;
      }
      continue;
    }
    TRY(multi_run_sample(m, m->sched, m->use_graph));
  }
  multi_join(m);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_multi_schedule_get(rs_multi* m, rs_multi_schedule* out) {
  ENTER(m);
  if (!out) return fail(RS_EINVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  out->tuned = m->tuned ? 1 : 0;
  out->schedule = (uint32_t)m->sched;
  out->threads_per_row = (uint32_t)SCHED_TPR[m->sched];
  out->rows_per_tile = (uint32_t)SCHED_TILE[m->sched];
  out->workgroups = (uint32_t)SCHED_GRID[m->sched];
  out->graph = m->use_graph ? 1 : 0;
  out->trace_block = (uint32_t)m->K;
  for (int q = 0; q < MULTI_SCHEDULES && q < RS_MULTI_SCHEDULES; ++q) out->sample_ms[q] = m->sched_ms[q];
  out->samples = m->samples;
  return RS_OK;
}

rs_status rs_multi_schedule_set(rs_multi* m, int32_t schedule, int32_t use_graph) {
  ENTER(m);
  if (schedule < -1 || schedule >= MULTI_SCHEDULES) return fail(RS_EINVAL, "schedule must be -1..%d", MULTI_SCHEDULES - 1);
  if (schedule == -1) {  // tune again over the next samples
    m->tuned = false;
    for (double& t : m->sched_ms) t = 0;
  } else {
    m->sched = schedule;
    m->tuned = true;
  }
  m->use_graph = use_graph != 0;
  return RS_OK;
}

rs_status rs_multi_get(rs_multi* m, uint32_t i, int32_t var, void* host, size_t bytes) {
  ENTER(m);
  TRY(multi_index(m, i));
  multi_join(m);
  return rs_eprop_get(m->inst[i], var, host, bytes);
}

rs_status rs_multi_set(rs_multi* m, uint32_t i, int32_t var, const void* host, size_t bytes) {
  ENTER(m);
  TRY(multi_index(m, i));
  multi_join(m);
  return rs_eprop_set(m->inst[i], var, host, bytes);
}

rs_status rs_multi_info_get(rs_multi* m, uint32_t i, rs_eprop_info* out) {
  ENTER(m);
  TRY(multi_index(m, i));
  multi_join(m);
  return rs_eprop_info_get(m->inst[i], out);
}

void rs_multi_destroy(rs_multi* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  if (m->side) (void)hipStreamSynchronize(m->side);
  multi_drop_graph(m);
  for (rs_eprop* e : m->inst) rs_eprop_destroy(e);
  for (hipEvent_t ev : {m->ev_fwd, m->ev_back, m->ev_join, m->ev_t0, m->ev_t1})
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : m->ev_ep)
    if (ev) (void)hipEventDestroy(ev);
  if (m->side) (void)hipStreamDestroy(m->side);
  if (m->tab) (void)hipFree(m->tab);
  m->arena.release();
  delete m;
}

}  // extern "C"

// =========================================================================== served inference
// Continuous batching of inference requests on trained networks: each
// request is one presentation of an input raster to one model; its neuron and
// readout state sits in a slot on the device for the request's whole life.
// Every call of rs_serve_step admits queued requests into free slots (while
// their state fits the memory budget) and runs one block of steps for every
// running request in one forward launch (a work list over the requests, each
// at its own position in its own input) and one readout launch; requests
// that reach their last step free their slot.

namespace {

double host_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServeSlot {
  int model = 0;
  bool busy = false;
  uint64_t ticket = 0;
  const int32_t *off = nullptr, *idx = nullptr;
  long long n_idx = 0;
  uint32_t n_steps = 0, done = 0, raster_steps = 0;
  double submit_s = 0, admit_s = 0;
  // device state
  double *V = nullptr, *A = nullptr, *Y = nullptr, *score = nullptr;
  float *xbar = nullptr, *zbar = nullptr, *u = nullptr;
  uint8_t* z = nullptr;
  uint32_t* zcount = nullptr;
  unsigned long long* counters = nullptr;
};

struct ServeRequest {
  uint64_t ticket;
  int model;
  const int32_t *off, *idx;
  long long n_idx;
  uint32_t n_steps, raster_steps;
  double submit_s;
};

}  // namespace

struct rs_serve {
  std::vector<rs_eprop*> models;
  std::vector<size_t> footprint;      // device bytes of one request's state, per model
  std::vector<int> first_slot;        // slots of model m: first_slot[m] .. first_slot[m+1]-1
  std::vector<ServeSlot> slots;
  std::deque<ServeRequest> queue;
  rs_serve_params p{};
  hipStream_t stream = nullptr;
  Arena arena;
  uint64_t budget = 0, used = 0;
  int K = 20, items = 1;
  size_t lds = 0;
  uint64_t next_ticket = 1;
  // per-block launch tables: device and pinned host images
  FwdArgs* fwd_dev = nullptr;
  int2* work_dev = nullptr;
  ServeReadout* ro_dev = nullptr;
  ZeroRange* zero_dev = nullptr;
  unsigned char* host_img = nullptr;  // pinned
  size_t img_bytes = 0, off_work = 0, off_ro = 0, off_zero = 0;
  int max_active = 0;
  std::vector<rs_serve_result> done;
  std::vector<double> done_scores;    // n_out_max per finished request
  int n_out_max = 1;
  uint64_t admitted = 0, rejected = 0, completed = 0, blocks = 0;
  double t0 = 0;
  bool dead = false;
};

namespace {

size_t serve_footprint(const rs_eprop* n, int K) {
  const size_t NR = n->p.n_rec, NI = n->p.n_in, NO = n->p.n_out;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al(NR * 8) * 2 + al(NO * 8) * 2 + al(NI * 4) + al(NR * 4) + al((size_t)K * NO * 4) + al(NR) + al(NR * 4) +
         al(16);
}

rs_status serve_create_impl(rs_eprop* const* models, uint32_t n_models, const rs_serve_params* prm, void* stream,
                            rs_serve* s) {
  if (!models || n_models < 1 || n_models > 64) return fail(RS_EINVAL, "1..64 models");
  if (!prm) return fail(RS_EINVAL, "params is NULL");
  if (prm->slots_per_model < 1 || prm->slots_per_model > 4096) return fail(RS_EINVAL, "slots_per_model in 1..4096");
  if (prm->block_steps < 1 || prm->block_steps > 32) return fail(RS_EINVAL, "block_steps in 1..32");
  if (prm->max_running < 1) return fail(RS_EINVAL, "max_running >= 1");
  s->p = *prm;
  s->stream = (hipStream_t)stream;
  s->K = (int)prm->block_steps;
  s->budget = prm->state_budget_bytes;
  const uint32_t n_in = models[0] ? models[0]->p.n_in : 0;
  for (uint32_t m = 0; m < n_models; ++m) {
    rs_eprop* e = models[m];
    if (!e) return fail(RS_EINVAL, "model %u is NULL", m);
    if (e->dead) return fail(RS_EDEVICE, "model %u is unusable after a device error", m);
    if (e->p.n_in != n_in) return fail(RS_EINVAL, "every model takes the same n_in");
    s->models.push_back(e);
    s->footprint.push_back(serve_footprint(e, s->K));
    s->n_out_max = std::max(s->n_out_max, (int)e->p.n_out);
    s->items = std::max(s->items, fwd_items((int)e->p.n_in, (int)e->p.n_rec));
    FwdArgs f = block_fwd_args(e, 0, 0, s->K);
    s->lds = std::max(s->lds, fwd_plan(f));
  }
  // slots: every model's state for slots_per_model requests
  Arena& ar = s->arena;
  for (uint32_t m = 0; m < n_models; ++m) {
    rs_eprop* e = s->models[m];
    const size_t NR = e->p.n_rec, NI = e->p.n_in, NO = e->p.n_out;
    s->first_slot.push_back((int)s->slots.size());
    for (uint32_t q = 0; q < prm->slots_per_model; ++q) {
      ServeSlot sl;
      sl.model = (int)m;
      TRY(ar.alloc(&sl.V, NR));
      TRY(ar.alloc(&sl.A, NR));
      TRY(ar.alloc(&sl.Y, NO));
      TRY(ar.alloc(&sl.score, NO));
      TRY(ar.alloc(&sl.xbar, NI));
      TRY(ar.alloc(&sl.zbar, NR));
      TRY(ar.alloc(&sl.u, (size_t)s->K * NO));
      TRY(ar.alloc(&sl.z, NR));
      TRY(ar.alloc(&sl.zcount, NR));
      TRY(ar.alloc(&sl.counters, 2));
      s->slots.push_back(sl);
    }
  }
  s->first_slot.push_back((int)s->slots.size());
  s->max_active = (int)std::min<size_t>(prm->max_running, s->slots.size());
  const int A = s->max_active, Z = A * 10;
  TRY(ar.alloc(&s->fwd_dev, (size_t)A));
  TRY(ar.alloc(&s->work_dev, (size_t)A));
  TRY(ar.alloc(&s->ro_dev, (size_t)A));
  TRY(ar.alloc(&s->zero_dev, (size_t)Z));
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  s->off_work = al(sizeof(FwdArgs) * A);
  s->off_ro = s->off_work + al(sizeof(int2) * A);
  s->off_zero = s->off_ro + al(sizeof(ServeReadout) * A);
  s->img_bytes = s->off_zero + al(sizeof(ZeroRange) * Z);
  HIP_OK(hipHostMalloc((void**)&s->host_img, s->img_bytes, hipHostMallocDefault));
  fwd_attrs();
  s->t0 = host_seconds();
  return RS_OK;
}

// Admit queued requests, in arrival order, into free slots of their model
// while the budget holds their state.
int serve_admit(rs_serve* s, ZeroRange* zr, int* nz) {
  int running = 0;
  for (const ServeSlot& sl : s->slots) running += sl.busy ? 1 : 0;
  int admitted = 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && running < s->max_active;) {
    const ServeRequest& r = *it;
    const size_t fp = s->footprint[r.model];
    int slot = -1;
    if (s->used + fp <= s->budget)
      for (int q = s->first_slot[r.model]; q < s->first_slot[r.model + 1]; ++q)
        if (!s->slots[q].busy) { slot = q; break; }
    if (slot < 0) { ++it; continue; }
    ServeSlot& sl = s->slots[slot];
    sl.busy = true;
    sl.ticket = r.ticket;
    sl.off = r.off;
    sl.idx = r.idx;
    sl.n_idx = r.n_idx;
    sl.n_steps = r.n_steps;
    sl.raster_steps = r.raster_steps;
    sl.done = 0;
    sl.submit_s = r.submit_s;
    sl.admit_s = host_seconds() - s->t0;
    const rs_eprop* e = s->models[sl.model];
    const size_t NR = e->p.n_rec, NI = e->p.n_in, NO = e->p.n_out;
    ZeroRange z[] = {{sl.V, NR * 8}, {sl.A, NR * 8}, {sl.Y, NO * 8}, {sl.score, NO * 8}, {sl.xbar, NI * 4},
                     {sl.zbar, NR * 4}, {sl.zcount, NR * 4}, {sl.counters, 16}};
    for (const ZeroRange& q : z) zr[(*nz)++] = q;
    s->used += fp;
    ++running;
    ++admitted;
    ++s->admitted;
    it = s->queue.erase(it);
  }
  return admitted;
}

rs_status serve_step_impl(rs_serve* s, uint32_t* n_done) {
  if (n_done) *n_done = 0;
  unsigned char* H = s->host_img;
  FwdArgs* fa = (FwdArgs*)H;
  int2* work = (int2*)(H + s->off_work);
  ServeReadout* ro = (ServeReadout*)(H + s->off_ro);
  ZeroRange* zr = (ZeroRange*)(H + s->off_zero);
  int nz = 0;
  serve_admit(s, zr, &nz);
  std::vector<int> act;
  for (int q = 0; q < (int)s->slots.size(); ++q)
    if (s->slots[q].busy) act.push_back(q);
  if (act.empty()) return RS_OK;
  unsigned long long zmax = 0;
  for (int q = 0; q < nz; ++q) zmax = std::max(zmax, zr[q].bytes);
  int n = 0;
  for (int q : act) {
    ServeSlot& sl = s->slots[q];
    rs_eprop* e = s->models[sl.model];
    const int nsteps = (int)std::min<uint32_t>((uint32_t)s->K, sl.n_steps - sl.done);
    FwdArgs f = block_fwd_args(e, 0, 0, nsteps);
    f.B = 1;
    f.V = sl.V; f.A = sl.A; f.xbar = sl.xbar; f.zbar = sl.zbar;
    f.psi = nullptr; f.x0 = nullptr; f.z0 = nullptr; f.xbits = nullptr; f.zbits = nullptr;
    f.z = sl.z; f.u = sl.u;
    f.x_off = sl.off; f.x_idx = sl.idx; f.n_idx = sl.n_idx;
    f.x_thr = nullptr; f.x_list = nullptr;
    f.t0 = (int)(sl.done % sl.raster_steps);
    f.sample_steps = (int)sl.raster_steps;
    f.rows_lds = 0;
    f.counters = sl.counters;
    f.zcount = sl.zcount;
    fwd_plan(f);
    fa[n] = f;
    work[n] = make_int2(n, 0);
    ServeReadout r{};
    r.n_out = (int)e->p.n_out;
    r.nsteps = nsteps;
    r.alpha = e->alpha;
    r.u = sl.u;
    r.Y = sl.Y;
    r.bout = e->bout;
    r.score = sl.score;
    ro[n] = r;
    ++n;
  }
  hipStream_t st = s->stream;
  // the tables are copied from pinned memory the host rewrites next block:
  // the block is waited for below before that happens
  if (nz) {
    HIP_OK(hipMemcpyAsync(s->zero_dev, zr, sizeof(ZeroRange) * nz, hipMemcpyHostToDevice, st));
    launch_fill_zero_ranges(st, s->zero_dev, nz, zmax);
  }
  HIP_OK(hipMemcpyAsync(s->fwd_dev, fa, sizeof(FwdArgs) * n, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(s->work_dev, work, sizeof(int2) * n, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(s->ro_dev, ro, sizeof(ServeReadout) * n, hipMemcpyHostToDevice, st));
  launch_fwd_multi(st, s->fwd_dev, s->work_dev, n, s->items, s->lds);
  launch_serve_readout(st, s->ro_dev, n);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(st));
  ++s->blocks;
  const double now = host_seconds() - s->t0;
  uint32_t fin = 0;
  for (int q : act) {
    ServeSlot& sl = s->slots[q];
    sl.done += (uint32_t)std::min<uint32_t>((uint32_t)s->K, sl.n_steps - sl.done);
    if (sl.done < sl.n_steps) continue;
    const rs_eprop* e = s->models[sl.model];
    const int NO = (int)e->p.n_out;
    std::vector<double> sc((size_t)NO);
    unsigned long long c[2];
    HIP_OK(hipMemcpyAsync(sc.data(), sl.score, (size_t)NO * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(c, sl.counters, 16, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    rs_serve_result r{};
    r.ticket = sl.ticket;
    r.model = (uint32_t)sl.model;
    r.steps = sl.n_steps;
    int best = 0;
    for (int k = 1; k < NO; ++k)
      if (sc[k] > sc[best]) best = k;
    r.decision = best;
    r.events = c[0];
    r.spikes = c[1];
    r.submit_s = sl.submit_s;
    r.admit_s = sl.admit_s;
    r.done_s = now;
    s->done.push_back(r);
    const size_t base = s->done_scores.size();
    s->done_scores.resize(base + (size_t)s->n_out_max, 0.0);
    std::copy(sc.begin(), sc.end(), s->done_scores.begin() + base);
    sl.busy = false;
    s->used -= s->footprint[sl.model];
    ++s->completed;
    ++fin;
  }
  if (n_done) *n_done = fin;
  return RS_OK;
}

}  // namespace

extern "C" {

rs_status rs_serve_create(rs_eprop* const* models, uint32_t n_models, const rs_serve_params* params,
                          void* hip_stream, rs_serve** out) {
  if (!out) return fail(RS_EINVAL, "out is NULL");
  *out = nullptr;
  rs_serve* s = new rs_serve();
  rs_status st = serve_create_impl(models, n_models, params, hip_stream, s);
  if (st != RS_OK) {
    rs_serve_destroy(s);
    return st;
  }
  *out = s;
  return RS_OK;
}

rs_status rs_serve_submit(rs_serve* s, uint32_t model, const int32_t* off_dev, const int32_t* idx_dev, size_t n_idx,
                          uint32_t raster_steps, uint32_t n_steps, uint64_t* ticket) {
  ENTER(s);
  if (model >= s->models.size()) return fail(RS_EINVAL, "model %u outside 0..%zu", model, s->models.size() - 1);
  if (!off_dev || !idx_dev) return fail(RS_EINVAL, "input pointers must not be NULL");
  if (n_steps < 1 || raster_steps < 1) return fail(RS_EINVAL, "n_steps and raster_steps must be >= 1");
  if (n_idx > (size_t)INT32_MAX) return fail(RS_EINVAL, "index array larger than 2^31 entries");
  if (s->footprint[model] > s->budget) {
    ++s->rejected;
    return fail(RS_ECAPACITY, "the request's state (%zu bytes) exceeds the budget", s->footprint[model]);
  }
  if (s->queue.size() >= s->p.max_queue) {
    ++s->rejected;
    return fail(RS_ECAPACITY, "queue full (%u requests)", s->p.max_queue);
  }
  ServeRequest r{s->next_ticket++, (int)model, off_dev, idx_dev, (long long)n_idx, n_steps, raster_steps,
                 host_seconds() - s->t0};
  s->queue.push_back(r);
  if (ticket) *ticket = r.ticket;
  return RS_OK;
}

rs_status rs_serve_step(rs_serve* s, uint32_t* n_done) {
  ENTER(s);
  return serve_step_impl(s, n_done);
}

rs_status rs_serve_poll(rs_serve* s, rs_serve_result* out, double* scores, uint32_t max, uint32_t* n) {
  ENTER(s);
  if (!out || !n) return fail(RS_EINVAL, "NULL argument");
  const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
  for (uint32_t q = 0; q < k; ++q) out[q] = s->done[q];
  if (scores)
    std::copy(s->done_scores.begin(), s->done_scores.begin() + (size_t)k * s->n_out_max, scores);
  s->done.erase(s->done.begin(), s->done.begin() + k);
  s->done_scores.erase(s->done_scores.begin(), s->done_scores.begin() + (size_t)k * s->n_out_max);
  *n = k;
  return RS_OK;
}

rs_status rs_serve_stats_get(rs_serve* s, rs_serve_stats* out) {
  ENTER(s);
  if (!out) return fail(RS_EINVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  out->admitted = s->admitted;
  out->rejected = s->rejected;
  out->completed = s->completed;
  out->queued = s->queue.size();
  int running = 0;
  for (const ServeSlot& sl : s->slots) running += sl.busy ? 1 : 0;
  out->running = (uint32_t)running;
  out->blocks = s->blocks;
  out->state_bytes_used = s->used;
  out->state_budget_bytes = s->budget;
  out->n_out_max = (uint32_t)s->n_out_max;
  out->clock_s = host_seconds() - s->t0;
  return RS_OK;
}

// Replay a request trace against the wall clock: request q is submitted once
// arrival_s[q] seconds have passed since the call began; blocks run while
// requests are running; the call returns when every request has finished or
// been rejected.  latency_ms[q] (arrival to completion) is -1 for rejected ones.
rs_status rs_serve_replay(rs_serve* s, const rs_serve_request* reqs, uint32_t n, double* latency_ms,
                          int32_t* decision, uint64_t* spikes) {
  ENTER(s);
  if (!reqs && n) return fail(RS_EINVAL, "NULL requests");
  for (uint32_t q = 1; q < n; ++q)
    if (reqs[q].arrival_s < reqs[q - 1].arrival_s) return fail(RS_EINVAL, "arrivals must be in order");
  std::unordered_map<uint64_t, uint32_t> of_ticket;  // ticket -> request
  for (uint32_t q = 0; q < n; ++q) {
    if (latency_ms) latency_ms[q] = -1.0;
    if (decision) decision[q] = -1;
    if (spikes) spikes[q] = 0;
  }
  const double start = host_seconds() - s->t0;
  uint32_t next = 0, finished = 0, rejected = 0;
  std::vector<rs_serve_result> res(256);
  while (finished + rejected < n) {
    const double now = host_seconds() - s->t0 - start;
    for (; next < n && reqs[next].arrival_s <= now; ++next) {
      const rs_serve_request& r = reqs[next];
      uint64_t t = 0;
      rs_status st = rs_serve_submit(s, r.model, r.off_dev, r.idx_dev, r.n_idx, r.raster_steps, r.n_steps, &t);
      if (st == RS_ECAPACITY) { ++rejected; continue; }
      TRY(st);
      of_ticket[t] = next;
    }
    uint32_t nd = 0;
    TRY(serve_step_impl(s, &nd));
    int running = 0;
    for (const ServeSlot& sl : s->slots) running += sl.busy ? 1 : 0;
    if (running == 0 && s->queue.empty() && next < n) {
      // idle until the next arrival
      while (host_seconds() - s->t0 - start < reqs[next].arrival_s) {
      }
    }
    for (;;) {
      uint32_t k = 0;
      TRY(rs_serve_poll(s, res.data(), nullptr, (uint32_t)res.size(), &k));
      for (uint32_t q = 0; q < k; ++q) {
        const auto f = of_ticket.find(res[q].ticket);
        if (f == of_ticket.end()) continue;  // submitted before this replay
        const uint32_t lo = f->second;
        if (latency_ms) latency_ms[lo] = 1e3 * (res[q].done_s - start - reqs[lo].arrival_s);
        if (decision) decision[lo] = res[q].decision;
        if (spikes) spikes[lo] = res[q].spikes;
        ++finished;
      }
      if (k < res.size()) break;
    }
  }
  return RS_OK;
}

void rs_serve_destroy(rs_serve* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->host_img) (void)hipHostFree(s->host_img);
  s->arena.release();
  delete s;
}

}  // extern "C"

// =========================================================================== composed networks
// The paper's problem statement as calls: declare populations and
// projections (each with its initialisation, learning rule and structural-
// plasticity rule), build, step, trigger the rule, read and write state.  A
// build recognises the models the kernels implement and assembles them: the
// e-prop classifier (spike source -> LIF/ALIF -> readout, with DEEP R on
// either ragged projection) and the topographic map (Poisson sheet ->
// conductance-LIF sheet with STDP and distance-dependent rewiring).
struct rs_net {
  hipStream_t stream = nullptr;
  Arena alloc;  // the caller's allocator (callbacks only; owns nothing)
  uint64_t seed = 0;
  struct Pop { int32_t kind; uint32_t n; rs_pop_params p; };
  struct Proj { uint32_t pre, post; rs_proj_desc d; };
  std::vector<Pop> pops;
  std::vector<Proj> projs;
  bool built = false;
  int model = 0;                 // 1: e-prop classifier, 2: topographic map
  int proj_map[3] = {-1, -1, -1};  // classifier: composed projection -> 0 input, 1 recurrent, 2 readout
  rs_eprop* ep = nullptr;
  rs_topo* tp = nullptr;
  bool dead = false;
};

namespace {

rs_status net_build_classifier(rs_net* n, uint32_t batch, uint32_t sample_steps, uint32_t trace_block) {
  // populations: one spike source, one LIF or ALIF population, one readout
  int src = -1, rec = -1, out = -1;
  for (int q = 0; q < (int)n->pops.size(); ++q) {
    const int k = n->pops[q].kind;
    if (k == RS_POP_SPIKE_SOURCE && src < 0) src = q;
    else if ((k == RS_POP_LIF || k == RS_POP_ALIF) && rec < 0) rec = q;
    else if (k == RS_POP_READOUT && out < 0) out = q;
    else return fail(RS_EINVAL, "population %d does not fit the e-prop classifier", q);
  }
  if (src < 0 || rec < 0 || out < 0)
    return fail(RS_EINVAL, "the e-prop classifier needs a spike source, a LIF or ALIF population and a readout");
  if (n->projs.size() != 3) return fail(RS_EINVAL, "the e-prop classifier has three projections");
  rs_eprop_params p{};
  const rs_pop_params& rp = n->pops[rec].p;
  p.n_in = n->pops[src].n;
  p.n_rec = n->pops[rec].n;
  p.n_out = n->pops[out].n;
  p.batch = batch;
  p.alif = n->pops[rec].kind == RS_POP_ALIF;
  p.dt_ms = rp.dt_ms;
  p.tau_mem_ms = rp.tau_mem_ms;
  p.tau_adapt_ms = p.alif ? rp.tau_adapt_ms : 2000.0f;
  p.v_thr = rp.v_thr;
  p.beta = p.alif ? rp.beta : 0.0f;
  p.sample_steps = sample_steps;
  p.trace_block = trace_block;
  p.seed = n->seed;
  bool have[3] = {false, false, false};
  for (int q = 0; q < 3; ++q) {
    const rs_net::Proj& pr = n->projs[q];
    const rs_proj_desc& d = pr.d;
    int role = -1;
    if ((int)pr.pre == src && (int)pr.post == rec) role = 0;
    else if ((int)pr.pre == rec && (int)pr.post == rec) role = 1;
    else if ((int)pr.pre == rec && (int)pr.post == out) role = 2;
    if (role < 0 || have[role]) return fail(RS_EINVAL, "projection %d does not fit the e-prop classifier", q);
    have[role] = true;
    n->proj_map[q] = role;
    if (d.learn != RS_LEARN_EPROP) return fail(RS_EINVAL, "projection %d: the classifier learns by e-prop", q);
    if (q == 0) {  // one optimiser and update interval for the whole network
      p.lr = d.lr;
      p.adam_b1 = d.adam_b1;
      p.adam_b2 = d.adam_b2;
      p.adam_eps = d.adam_eps;
      p.update_interval = d.update_interval;
    } else if (!(d.lr == p.lr && d.adam_b1 == p.adam_b1 && d.adam_b2 == p.adam_b2 && d.adam_eps == p.adam_eps &&
                 d.update_interval == p.update_interval)) {
      return fail(RS_EINVAL, "the projections share one optimiser and update interval");
    }
    if (role == 2) {
      if (d.init != RS_INIT_DENSE || d.rewire != RS_REWIRE_NONE)
        return fail(RS_EINVAL, "the readout projection is dense, without rewiring");
      p.sigma_out = d.sigma_w;
      continue;
    }
    if (d.init != RS_INIT_FIXED_PROB) return fail(RS_EINVAL, "projection %d: fixed-probability rows", q);
    if (d.rewire != RS_REWIRE_NONE && d.rewire != RS_REWIRE_DEEPR)
      return fail(RS_EINVAL, "projection %d: the classifier rewires by DEEP R", q);
    (role == 0 ? p.p_in : p.p_rec) = d.p;
    (role == 0 ? p.sigma_in : p.sigma_rec) = d.sigma_w;
    (role == 0 ? p.cap_in : p.cap_rec) = d.cap;
    if (d.rewire == RS_REWIRE_DEEPR) {
      if (p.deepr_mask && d.l1 != p.l1) return fail(RS_EINVAL, "the DEEP R projections share one L1 strength");
      p.deepr_mask |= 1u << role;
      p.l1 = d.l1;
    }
  }
  rs_eprop* e = nullptr;
  rs_status st = create_impl(&p, n->stream, &e, &n->alloc);
  if (st != RS_OK) {
    if (e) rs_eprop_destroy(e);
    return st;
  }
  n->ep = e;
  n->model = 1;
  return RS_OK;
}

// The map's projection parameters from a descriptor.
rs_topo_params topo_params_of(const rs_proj_desc& d, uint32_t L, uint32_t proj_id, uint64_t seed) {
  rs_topo_params tp{};
  tp.L = L;
  tp.cap = d.cap;
  tp.n_attempts = d.rewire == RS_REWIRE_TOPO ? d.n_attempts : 0;
  tp.proj_id = proj_id;
  tp.p_form = d.p_form;
  tp.sigma_form = d.sigma_form;
  tp.g_theta = d.g_theta;
  tp.p_elim_dep = d.p_elim_dep;
  tp.p_elim_pot = d.p_elim_pot;
  tp.g_new = d.g_new;
  tp.g_init = d.g_init;
  tp.seed = seed;
  return tp;
}

rs_status net_build_topomap(rs_net* n) {
  if (n->pops.size() != 2 || (n->projs.size() != 1 && n->projs.size() != 2))
    return fail(RS_EINVAL, "the topographic map has two sheets, a feed-forward and optionally a lateral projection");
  const rs_net::Pop &a = n->pops[0], &b = n->pops[1];
  if (a.kind != RS_POP_POISSON_SHEET || b.kind != RS_POP_COND_LIF_SHEET || a.p.L != b.p.L || a.n != a.p.L * a.p.L ||
      b.n != a.n)
    return fail(RS_EINVAL, "the topographic map projects a Poisson sheet onto a conductance-LIF sheet of one size");
  const rs_proj_desc& d = n->projs[0].d;
  if (n->projs[0].pre != 0 || n->projs[0].post != 1 || d.init != RS_INIT_GAUSS_TORUS)
    return fail(RS_EINVAL, "the sheet projection has Gaussian pairwise-Bernoulli rows");
  if (d.learn != RS_LEARN_NONE && d.learn != RS_LEARN_STDP) return fail(RS_EINVAL, "the map learns by STDP or not");
  if (d.rewire != RS_REWIRE_NONE && d.rewire != RS_REWIRE_TOPO) return fail(RS_EINVAL, "the map rewires topographically");
  const rs_proj_desc* dl = nullptr;
  if (n->projs.size() == 2) {
    dl = &n->projs[1].d;
    if (n->projs[1].pre != 1 || n->projs[1].post != 1 || dl->init != RS_INIT_GAUSS_TORUS)
      return fail(RS_EINVAL, "the lateral projection joins the target sheet to itself by Gaussian rows");
    if (dl->learn != d.learn) return fail(RS_EINVAL, "both projections of the map learn by STDP or neither");
    if (dl->rewire != d.rewire || (d.rewire == RS_REWIRE_TOPO && dl->update_interval != d.update_interval))
      return fail(RS_EINVAL, "both projections of the map rewire at the same interval or neither");
  }
  rs_topo_params tp = topo_params_of(d, a.p.L, 0, n->seed);
  rs_topo_model m = b.p.model;  // neuron and synapse of the target sheet
  const rs_topo_model& sm = a.p.model;  // stimulus of the source sheet
  m.f_base = sm.f_base;
  m.f_peak = sm.f_peak;
  m.sigma_stim = sm.sigma_stim;
  m.stim_steps = sm.stim_steps;
  m.stim_kind = sm.stim_kind;
  m.stim_tile = sm.stim_tile;
  m.stdp = d.learn == RS_LEARN_STDP;
  m.rewire_steps = d.rewire == RS_REWIRE_TOPO ? d.update_interval : 0;
  rs_topo* t = new rs_topo();
  t->arena.afn = n->alloc.afn;
  t->arena.ffn = n->alloc.ffn;
  t->arena.user = n->alloc.user;
  rs_status st = topo_create_impl(&tp, n->stream, t);
  if (st == RS_OK && dl) {
    const rs_topo_params tl = topo_params_of(*dl, a.p.L, 1, n->seed);
    st = rs_topo_add_lateral(t, &tl);
  }
  if (st == RS_OK) st = rs_topo_sim_init(t, &m);
  if (st != RS_OK) {
    rs_topo_destroy(t);
    return st;
  }
  n->tp = t;
  n->model = 2;
  return RS_OK;
}

}  // namespace

extern "C" {

rs_status rs_create(void* hip_stream, rs_alloc_fn alloc_fn, rs_free_fn free_fn, void* user, uint64_t seed,
                    rs_net** out) {
  if (!out) return fail(RS_EINVAL, "out is NULL");
  *out = nullptr;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(RS_EINVAL, "give both allocator functions or neither");
  rs_net* n = new rs_net();
  n->stream = (hipStream_t)hip_stream;
  n->alloc.afn = alloc_fn;
  n->alloc.ffn = free_fn;
  n->alloc.user = user;
  n->seed = seed;
  *out = n;
  return RS_OK;
}

rs_status rs_add_pop(rs_net* n, int32_t kind, uint32_t size, const rs_pop_params* p, uint32_t* pop) {
  ENTER(n);
  if (n->built) return fail(RS_ESTATE, "the network is built");
  if (!p) return fail(RS_EINVAL, "params is NULL");
  if (kind < RS_POP_SPIKE_SOURCE || kind > RS_POP_COND_LIF_SHEET) return fail(RS_EINVAL, "unknown population kind");
  if (size < 1) return fail(RS_EINVAL, "a population has at least one neuron");
  n->pops.push_back({kind, size, *p});
  if (pop) *pop = (uint32_t)n->pops.size() - 1;
  return RS_OK;
}

rs_status rs_add_proj(rs_net* n, uint32_t pre, uint32_t post, const rs_proj_desc* d, uint32_t* proj) {
  ENTER(n);
  if (n->built) return fail(RS_ESTATE, "the network is built");
  if (!d) return fail(RS_EINVAL, "descriptor is NULL");
  if (pre >= n->pops.size() || post >= n->pops.size()) return fail(RS_EINVAL, "unknown population");
  n->projs.push_back({pre, post, *d});
  if (proj) *proj = (uint32_t)n->projs.size() - 1;
  return RS_OK;
}

rs_status rs_build(rs_net* n, uint32_t batch, uint32_t sample_steps, uint32_t trace_block) {
  ENTER(n);
  if (n->built) return fail(RS_ESTATE, "the network is built");
  bool sheet = false;
  for (const auto& q : n->pops) sheet |= q.kind == RS_POP_POISSON_SHEET || q.kind == RS_POP_COND_LIF_SHEET;
  TRY(sheet ? net_build_topomap(n) : net_build_classifier(n, batch, sample_steps, trace_block));
  n->built = true;
  return RS_OK;
}

rs_status rs_eprop_of(rs_net* n, rs_eprop** out) {
  ENTER(n);
  if (!out) return fail(RS_EINVAL, "NULL argument");
  if (!n->ep) return fail(RS_ESTATE, "not an e-prop classifier, or not built");
  *out = n->ep;
  return RS_OK;
}

rs_status rs_topo_of(rs_net* n, rs_topo** out) {
  ENTER(n);
  if (!out) return fail(RS_EINVAL, "NULL argument");
  if (!n->tp) return fail(RS_ESTATE, "not a topographic map, or not built");
  *out = n->tp;
  return RS_OK;
}

rs_status rs_step(rs_net* n, uint32_t n_steps, uint32_t flags) {
  ENTER(n);
  if (n->ep) return rs_eprop_step(n->ep, n_steps, flags);
  if (n->tp) return rs_topo_run(n->tp, n_steps);
  return fail(RS_ESTATE, "the network is not built");
}

rs_status rs_update(rs_net* n) {
  ENTER(n);
  if (!n->ep) return fail(RS_ESTATE, "only an e-prop classifier has a parameter update");
  return rs_eprop_update(n->ep);
}

rs_status rs_rewire(rs_net* n, uint32_t proj, rs_rewire_stats* st) {
  ENTER(n);
  if (proj >= n->projs.size()) return fail(RS_EINVAL, "unknown projection %u", proj);
  if (n->ep) {
    const int role = n->proj_map[proj];
    if (role > 1) return fail(RS_EINVAL, "projection %u is not rewired", proj);
    return rs_eprop_rewire(n->ep, (uint32_t)role, st);
  }
  if (n->tp) {
    uint64_t step = 0;
    TRY(rs_topo_sim_get(n->tp, RS_TV_STEP, &step, 8));
    return proj == 1 ? rs_topo_lat_rewire(n->tp, step, st) : rs_topo_rewire(n->tp, step, st);
  }
  return fail(RS_ESTATE, "the network is not built");
}

rs_status rs_get_rows(rs_net* n, uint32_t proj, int32_t* len, int32_t* ind, float* w, size_t cap_elems,
                      size_t* needed) {
  ENTER(n);
  if (proj >= n->projs.size()) return fail(RS_EINVAL, "unknown projection %u", proj);
  if (!len || !ind || !w) return fail(RS_EINVAL, "NULL argument");
  if (n->tp) {
    const ProjDev& P = proj == 1 ? n->tp->tl.P : n->tp->t.P;
    const size_t need = (size_t)P.n_pre * P.cap;
    if (needed) *needed = need;
    if (cap_elems < need) return fail(RS_ECAPACITY, "row buffers need %zu elements", need);
    return proj == 1 ? rs_topo_lat_get_rows(n->tp, len, ind, w) : rs_topo_get_rows(n->tp, len, ind, w);
  }
  if (!n->ep) return fail(RS_ESTATE, "the network is not built");
  const int role = n->proj_map[proj];
  if (role > 1) return fail(RS_EINVAL, "projection %u is dense, not ragged", proj);
  const ProjDev& P = role == 0 ? n->ep->in : n->ep->rec;
  const size_t need = (size_t)P.n_pre * P.cap;
  if (needed) *needed = need;
  if (cap_elems < need) return fail(RS_ECAPACITY, "row buffers need %zu elements", need);
  TRY(rs_eprop_get(n->ep, RS_PROJ(role, RS_P_LEN), len, (size_t)P.n_pre * 4));
  TRY(rs_eprop_get(n->ep, RS_PROJ(role, RS_P_IND), ind, need * 4));
  return rs_eprop_get(n->ep, RS_PROJ(role, RS_P_W), w, need * 4);
}

rs_status rs_get_var(rs_net* n, int32_t var, void* host, size_t bytes) {
  ENTER(n);
  if (n->ep) return rs_eprop_get(n->ep, var, host, bytes);
  if (n->tp) return rs_topo_sim_get(n->tp, var, host, bytes);
  return fail(RS_ESTATE, "the network is not built");
}

rs_status rs_set_var(rs_net* n, int32_t var, const void* host, size_t bytes) {
  ENTER(n);
  if (n->ep) return rs_eprop_set(n->ep, var, host, bytes);
  if (n->tp) return rs_topo_sim_set(n->tp, var, host, bytes);
  return fail(RS_ESTATE, "the network is not built");
}

rs_status rs_sync(rs_net* n) {
  ENTER(n);
  if (n->ep) {
    order(n->ep->ev_back, n->ep->side, n->ep->stream);
    HIP_OK(hipStreamSynchronize(n->ep->stream));
  } else {
    HIP_OK(hipStreamSynchronize(n->stream));
  }
  return RS_OK;
}

uint64_t rs_step_counter(const rs_net* n) {
  if (!n) return 0;
  if (n->ep) return n->ep->step;
  if (n->tp) return n->tp->step;
  return 0;
}

void rs_destroy(rs_net* n) {
  if (!n) return;
  if (n->ep) rs_eprop_destroy(n->ep);
  if (n->tp) rs_topo_destroy(n->tp);
  delete n;
}

}  // extern "C"

// =========================================================================== custom connectivity updates
// A rule's host part runs here on the host (the paper's host_update_code,
// with the counter-based generator's host implementation), its row parts on
// the device (rs_custom.hpp).  A caller's host function may inspect and
// change the rule's per-row variable between the two.

namespace {

struct CustomScratch {
  long long* stats = nullptr;     // [4]
  uint32_t* pre_var = nullptr;    // [n_pre] the rule's per-row variable on the device
  size_t n_pre = 0;
};

rs_status custom_scratch(Arena& ar, CustomScratch& cs, size_t n_pre) {
  if (!cs.stats) TRY(ar.alloc(&cs.stats, 4));
  if (cs.n_pre < n_pre) {
    TRY(ar.alloc(&cs.pre_var, n_pre));
    cs.n_pre = n_pre;
  }
  return RS_OK;
}

// DEEP R's distribution of the dormant total over the rows, on the host: the
// device kernel's rounds and fallback, the same draws.
int64_t host_deepr_distribute(uint64_t seed, const ProjDev& P, uint64_t step, const std::vector<int>& len,
                              const std::vector<int>& dormant, std::vector<uint32_t>& asg, int64_t* unplaced) {
  int limit = P.n_post - (P.recurrent ? 1 : 0);
  limit = std::min(limit, P.cap);
  asg.assign((size_t)P.n_pre, 0u);
  int64_t pending = 0;
  for (int d : dormant) pending += d;
  std::vector<int> cnt((size_t)P.n_pre);
  for (int round = 0; pending > 0 && round < MAX_ROUNDS; ++round) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t a = 0; a < pending; ++a)
      ++cnt[host_below(host_draw_u32(seed, TAG_DR_ROW, (uint32_t)P.proj_id, step, (uint64_t)a, (uint64_t)round, 0),
                       (uint32_t)P.n_pre)];
    int64_t rej = 0;
    for (int r = 0; r < P.n_pre; ++r) {
      const int room = std::max(limit - len[r] - (int)asg[r], 0);
      const int acc = std::min(cnt[r], room);
      asg[r] += (uint32_t)acc;
      rej += cnt[r] - acc;
    }
    pending = rej;
  }
  for (int r = 0; r < P.n_pre && pending > 0; ++r) {
    const int room = limit - len[r] - (int)asg[r];
    if (room <= 0) continue;
    const int take = (int)std::min<int64_t>(pending, room);
    asg[r] += (uint32_t)take;
    pending -= take;
  }
  *unplaced = pending;
  int64_t placed = 0;
  for (uint32_t a : asg) placed += a;
  return placed;
}

rs_status run_host_fn(rs_host_update_fn fn, void* user, const ProjDev& P, int32_t rule, uint64_t seed, uint64_t step,
                      const std::vector<int>& len, std::vector<uint32_t>& var) {
  if (!fn) return RS_OK;
  rs_custom_host h{};
  h.n_pre = P.n_pre;
  h.n_post = P.n_post;
  h.cap = P.cap;
  h.recurrent = P.recurrent;
  h.len = len.data();
  h.pre_var = var.data();
  h.seed = seed;
  h.step = step;
  h.proj_id = (uint32_t)P.proj_id;
  h.rule = rule;
  fn(user, &h);
  return RS_OK;
}

// One custom update of projection P (rows, records and bitfields on the
// device), on stream s.  Fills the host stats (synchronising).
rs_status custom_update(Arena& ar, CustomScratch& cs, hipStream_t s, uint64_t seed, ProjDev P, int B, int32_t rule,
                        uint64_t step, rs_host_update_fn fn, void* user, const TopoDev* topo, rs_rewire_stats* st) {
  TRY(custom_scratch(ar, cs, (size_t)P.n_pre));
  launch_fill_zero(s, cs.stats, 32);
  if (topo) launch_fill_zero(s, topo->stats, 32);
  std::vector<int> len((size_t)P.n_pre);
  std::vector<uint32_t> var((size_t)P.n_pre, 0u);
  int64_t placed = 0, unplaced = 0;
  auto pull_len = [&]() -> rs_status {
    HIP_OK(hipMemcpyAsync(len.data(), P.len, len.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return RS_OK;
  };
  auto push_var = [&]() -> rs_status {
    HIP_OK(hipMemcpyAsync(cs.pre_var, var.data(), var.size() * 4, hipMemcpyHostToDevice, s));
    return RS_OK;
  };
  switch (rule) {
    case RS_RULE_ADD_DIAGONAL:
      launch_add_diagonal(s, P, B, cs.stats);
      break;
    case RS_RULE_REMOVE_RANDOM: {
      // host part: each row picks a random target to try and remove
      TRY(pull_len());
      for (int i = 0; i < P.n_pre; ++i)
        var[i] = host_below(host_draw_u32(seed, TAG_CUSTOM, (uint32_t)P.proj_id, step, (uint64_t)i, 0, 0),
                            (uint32_t)P.n_post);
      TRY(run_host_fn(fn, user, P, rule, seed, step, len, var));
      TRY(push_var());
      launch_remove_post(s, P, cs.pre_var, B, cs.stats);
      break;
    }
    case RS_RULE_DEEPR: {
      if (!P.conn || !P.sign) return fail(RS_EINVAL, "DEEP R needs the projection's connectivity and sign bits");
      launch_deepr_elim_rule(s, P, B, cs.stats);
      // host part: sum the dormant counts, spread them over the rows
      std::vector<int> dormant((size_t)P.n_pre);
      HIP_OK(hipMemcpyAsync(dormant.data(), P.dormant, dormant.size() * 4, hipMemcpyDeviceToHost, s));
      TRY(pull_len());
      placed = host_deepr_distribute(seed, P, step, len, dormant, var, &unplaced);
      TRY(run_host_fn(fn, user, P, rule, seed, step, len, var));
      const int limit = std::min(P.n_post - (P.recurrent ? 1 : 0), P.cap);
      for (int r = 0; r < P.n_pre; ++r)
        if ((int64_t)len[r] + var[r] > limit) return fail(RS_EINVAL, "row %d assigned beyond its room", r);
      HIP_OK(hipMemcpyAsync(P.assigned, var.data(), var.size() * 4, hipMemcpyHostToDevice, s));
      launch_deepr_form_rule(s, seed, P, B, step, cs.stats);
      break;
    }
    case RS_RULE_TOPO: {
      if (!topo) return fail(RS_EINVAL, "the topographic rule needs a topographic map");
      // host part: the attempts go to rows drawn uniformly, with replacement
      TRY(pull_len());
      for (int a = 0; a < topo->n_attempts; ++a)
        ++var[host_below(host_draw_u32(seed, TAG_TP_ROW, (uint32_t)P.proj_id, step, (uint64_t)a, 0, 0),
                         (uint32_t)P.n_pre)];
      TRY(run_host_fn(fn, user, P, rule, seed, step, len, var));
      TRY(push_var());
      TopoDev t = *topo;
      t.stats = cs.stats;  // removed, added from the row kernel; blocked beside them
      launch_topo_rule(s, seed, t, step, (const int*)cs.pre_var, cs.stats);
      break;
    }
    default:
      return fail(RS_EINVAL, "unknown rule %d", rule);
  }
  HIP_OK(hipGetLastError());
  if (st) {
    long long h[4];
    HIP_OK(hipMemcpyAsync(h, cs.stats, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    st->eliminated = h[0];
    st->formed = h[1];
    st->blocked = rule == RS_RULE_TOPO ? h[2] : unplaced;
    st->attempts = rule == RS_RULE_TOPO ? topo->n_attempts : rule == RS_RULE_DEEPR ? placed : 0;
  }
  return RS_OK;
}

}  // namespace

struct rs_custom_state {
  CustomScratch cs;
};
void delete_custom(rs_custom_state* c) { delete c; }

extern "C" {

rs_status rs_eprop_custom_update(rs_eprop* n, uint32_t proj, int32_t rule, uint64_t step, rs_host_update_fn fn,
                                 void* user, rs_rewire_stats* st) {
  ENTER(n);
  if (proj > 1) return fail(RS_EINVAL, "projection %u: 0 input, 1 recurrent", proj);
  if (rule == RS_RULE_TOPO) return fail(RS_EINVAL, "the topographic rule runs on a topographic map");
  if (step == STEP_FROM_DEVICE) return fail(RS_EINVAL, "step 2^64-1 is reserved");
  // the update follows everything queued on the network
  order(n->ev_join, n->side, n->stream);
  for (bool& p : n->ep_pending) p = false;
  if (!n->custom) n->custom = new rs_custom_state();
  fold_gradients(n, n->stream);
  TRY(custom_update(n->arena, n->custom->cs, n->stream, n->p.seed, proj == 0 ? n->in : n->rec, n->B, rule, step, fn,
                    user, nullptr, st));
  rebuild_columns(n, n->stream);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

rs_status rs_topo_custom_update(rs_topo* t, int32_t rule, uint64_t step, rs_host_update_fn fn, void* user,
                                rs_rewire_stats* st) {
  ENTER(t);
  if (rule == RS_RULE_DEEPR) return fail(RS_EINVAL, "DEEP R runs on an e-prop projection");
  if (step == STEP_FROM_DEVICE) return fail(RS_EINVAL, "step 2^64-1 is reserved");
  if (!t->custom) t->custom = new rs_custom_state();
  TopoDev td = t->t;
  td.col_len = nullptr;  // the rules do not edit an attached simulation's column view ...
  TRY(custom_update(t->arena, t->custom->cs, t->stream, t->p.seed, t->t.P, 1, rule, step, fn, user, &td, st));
  static const int one = 1;  // ... which the next simulation launch rebuilds
  HIP_OK(hipMemcpyAsync(t->t.col_dirty, &one, 4, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

}  // extern "C"
