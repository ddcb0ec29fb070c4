// Host engine behind the C-ABI of include/ragsnn.h: argument validation,
// device memory plan, build sequence, timestep loop and snapshot access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ragsnn.h"
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

// Device allocation list owned by one object.
struct Arena {
  std::vector<void*> ptrs;
  uint64_t bytes = 0;
  template <class T>
  rs_status alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) return RS_OK;
    void* q = nullptr;
    size_t b = (n * sizeof(T) + 255) & ~(size_t)255;
    if (hipMalloc(&q, b) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RS_ENOMEM, "device allocation of %zu bytes failed", b);
    }
    ptrs.push_back(q);
    bytes += b;
    *p = (T*)q;
    return RS_OK;
  }
  void release() {
    for (void* q : ptrs) (void)hipFree(q);
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
    (void)hipEventCreate(&e);
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
  float *x0T = nullptr, *z0T = nullptr;
  uint32_t *xbitsT = nullptr, *zbitsT = nullptr;
  // the forward kernel's coalesced staging of one block, [tau][B][n]
  uint32_t *stg[HANDOFF_ARRAYS] = {};                 // psi [K][B][NR]; x0, z0, xbits, zbits [B][n]
  float *u_stg = nullptr;                             // readout drive [Q segments][K][B][n_out]
  int K = 8, Q = 2, nslot = 16;
  int blk_seg = 0, blk_n = 0, last_slot = 0;
  int last_seg = 0, last_blk_n = 0;                   // the most recently run block
  uint64_t blk_t0 = 0;
  bool blk_learn = false;
  hipStream_t side = nullptr;                         // e-prop / update / rewire stream
  hipStream_t side2 = nullptr;                        // input-projection rewire, beside the recurrent one
  bool single = false;                                // small network: everything on the caller's stream
  bool auto_upd = false;                              // inside a step call with RS_AUTO_UPDATE
  hipEvent_t ev_fwd = nullptr, ev_ep[RING_MAX] = {}, ev_join = nullptr, ev_back = nullptr;
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
  bool dead = false;  // a device error occurred: every later call fails with RS_EDEVICE
};

namespace {

rs_status alloc_proj(Arena& ar, ProjDev& P, int B, bool alif, bool deepr) {
  const size_t n = (size_t)P.n_pre * P.cap;
  TRY(ar.alloc(&P.len, (size_t)P.n_pre));
  TRY(ar.alloc(&P.ind, n));
  TRY(ar.alloc(&P.w, n));
  TRY(ar.alloc(&P.m, n));
  TRY(ar.alloc(&P.v, n));
  TRY(ar.alloc(&P.G, n));
  TRY(ar.alloc(&P.ebar, n * B));
  if (alif) TRY(ar.alloc(&P.eps, n * B));
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
  launch_fill_zero(s, P.ebar, n * B * 4);
  if (P.eps) launch_fill_zero(s, P.eps, n * B * 4);
  launch_fill_zero(s, P.dormant, (size_t)P.n_pre * 4);
  launch_fill_zero(s, P.assigned, (size_t)P.n_pre * 4);
}

// Count rows on the device, return the longest.
rs_status count_rows(hipStream_t s, uint64_t seed, ProjDev& P, uint64_t T, int* max_len) {
  int* d_len = nullptr;
  HIP_OK(hipMalloc(&d_len, sizeof(int) * P.n_pre));
  ProjDev tmp = P;
  tmp.len = d_len;
  tmp.cap = 0;
  launch_fixed_rows(s, seed, tmp, T, 0.0, false);
  std::vector<int> h(P.n_pre);
  hipError_t e = hipMemcpyAsync(h.data(), d_len, sizeof(int) * P.n_pre, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_len);
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

rs_status create_impl(const rs_eprop_params* prm, void* stream, rs_eprop** out) {
  TRY(validate(prm));
  if (!fwd_fits((int)prm->n_in, (int)prm->n_rec, (int)prm->n_out))
    return fail(RS_EINVAL, "n_in %u and n_rec %u need more LDS than a forward workgroup has", prm->n_in, prm->n_rec);
  rs_eprop* n = new rs_eprop();
  *out = n;
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
    TRY(count_rows(s, seed, P, threshold(p), &mx));
    int cap = cap_req ? (int)cap_req : 2 * mx;
    cap = std::min(cap, n_post);
    cap = std::max(cap, 1);
    if (mx > cap) return fail(RS_EINVAL, "projection %d: longest row %d exceeds capacity %d", id, mx, cap);
    P.cap = cap;
    return RS_OK;
  };
  TRY(setup(n->in, prm->n_in, prm->n_rec, 0, 0, prm->p_in, prm->cap_in));
  TRY(setup(n->rec, prm->n_rec, prm->n_rec, 1, 1, prm->p_rec, prm->cap_rec));
  TRY(alloc_proj(n->arena, n->in, B, prm->alif, prm->deepr_mask & 1));
  TRY(alloc_proj(n->arena, n->rec, B, prm->alif, prm->deepr_mask & 2));
  Arena& ar = n->arena;
  const size_t NR = prm->n_rec, NI = prm->n_in, K = prm->n_out;
  TRY(ar.alloc(&n->V, B * NR));
  TRY(ar.alloc(&n->A, B * NR));
  TRY(ar.alloc(&n->Y, B * K));
  TRY(ar.alloc(&n->xbar, NI * B));
  TRY(ar.alloc(&n->zbar, NR * B));
  // default block length: 20 steps, the target-major e-prop kernel's launch;
  // batches the narrow kernel serves (B % 4 != 0) take a whole update
  // interval of up to 32 steps, one block per interval
  if (prm->trace_block)
    n->K = (int)prm->trace_block;
  else if (B % 4 != 0 && prm->update_interval >= 1 && prm->update_interval <= 32)
    n->K = (int)prm->update_interval;
  else
    n->K = 20;
  {
    const uint32_t U = prm->update_interval, Kb = (uint32_t)n->K;
    n->Q = U ? (int)std::min<uint32_t>(std::max<uint32_t>((U + Kb - 1) / Kb + 1, 2), RING_MAX) : 2;
  }
  const size_t QS = (size_t)n->Q;
  TRY(ar.alloc(&n->x0T, QS * NI * B));
  TRY(ar.alloc(&n->z0T, QS * NR * B));
  TRY(ar.alloc(&n->xbitsT, QS * NI * B));
  TRY(ar.alloc(&n->zbitsT, QS * NR * B));
  n->nslot = n->Q * n->K;
  const size_t NS = (size_t)n->nslot;
  TRY(ar.alloc(&n->psiT, NR * NS * B));
  TRY(ar.alloc(&n->LT, NR * NS * B));
  TRY(ar.alloc(&n->deltaT, K * NS * B));
  {
    const size_t KB = (size_t)n->K * B;
    TRY(ar.alloc(&n->stg[0], KB * NR));                   // psi
    const size_t dims[HANDOFF_ARRAYS] = {NR, NI, NR, NI, NR};  // psi, x0, z0, xbits, zbits
    for (int q = 1; q < HANDOFF_ARRAYS; ++q) TRY(ar.alloc(&n->stg[q], (size_t)B * dims[q]));
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
  HIP_OK(hipEventCreateWithFlags(&n->ev_upd, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&n->ev_rw, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&n->ev_fwd, hipEventDisableTiming));
  for (int q = 0; q < n->Q; ++q) HIP_OK(hipEventCreateWithFlags(&n->ev_ep[q], hipEventDisableTiming));
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
  launch_fill_zero(s, n->x0T, QS * B * NI * 4);
  launch_fill_zero(s, n->z0T, QS * B * NR * 4);
  launch_fill_zero(s, n->xbitsT, QS * B * NI * 4);
  launch_fill_zero(s, n->zbitsT, QS * B * NR * 4);
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
    launch_fill_zero(s, P->ebar, m);
    if (P->eps) launch_fill_zero(s, P->eps, m);
  }
}

void do_update(rs_eprop* n, hipStream_t s) {
  n->adam_k += 1;
  UpdateArgs u{};
  u.B = n->B;
  u.lr = n->p.lr;
  u.b1 = n->p.adam_b1;
  u.b2 = n->p.adam_b2;
  u.eps = n->p.adam_eps;
  u.inv_c1 = (float)(1.0 / (1.0 - std::pow((double)n->p.adam_b1, (double)n->adam_k)));
  u.inv_c2 = (float)(1.0 / (1.0 - std::pow((double)n->p.adam_b2, (double)n->adam_k)));
  u.l1 = n->p.l1;
  u.l1_in = (n->p.deepr_mask & 1) != 0;
  u.l1_rec = (n->p.deepr_mask & 2) != 0;
  u.in = n->in;
  u.rec = n->rec;
  u.Wout = n->Wout; u.bout = n->bout; u.Gout = n->Gout; u.Gb = n->Gb;
  u.Mout = n->Mout; u.Vout = n->Vout; u.Mb = n->Mb; u.Vb = n->Vb;
  u.n_out_elems = (int)(n->p.n_out * n->p.n_rec);
  u.n_b = (int)n->p.n_out;
  n->timer.begin(s, 2);
  launch_update(s, u);
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

// Run the open block (steps accumulated since the last flush): one forward
// launch for all its steps on the caller's stream, writing ring segment
// blk_seg, then the e-prop launch on the side stream.  The forward pass of
// the next block (next segment) overlaps this e-prop launch; a segment is
// reused only after the e-prop launch that read it has finished.
void flush_block(rs_eprop* n) {
  if (n->blk_n == 0) return;
  hipStream_t s = n->stream, e = n->side;
  const int h = n->blk_seg;
  if (n->ep_pending[h]) {
    (void)hipStreamWaitEvent(s, n->ev_ep[h], 0);
    n->ep_pending[h] = false;
  }
  FwdArgs f{};
  f.n_in = (int)n->p.n_in; f.n_rec = (int)n->p.n_rec; f.n_out = (int)n->p.n_out; f.B = n->B;
  f.alpha = n->alpha; f.rho = n->rho; f.v_thr = n->p.v_thr; f.beta = n->beta;
  f.psi_scale = 0.3 / (double)n->p.v_thr;
  f.alpha_f = (float)n->alpha;
  f.V = n->V; f.A = n->A;
  f.xbar = n->xbar; f.zbar = n->zbar;
  f.psi = (float*)n->stg[0]; f.x0 = (float*)n->stg[1]; f.z0 = (float*)n->stg[2];
  f.xbits = n->stg[3]; f.zbits = n->stg[4]; f.z = n->z;
  f.u = n->u_stg + (size_t)h * n->K * n->B * n->p.n_out;
  f.len_in = n->in.len; f.ind_in = n->in.ind; f.w_in = n->in.w; f.cap_in = n->in.cap;
  f.len_rec = n->rec.len; f.ind_rec = n->rec.ind; f.w_rec = n->rec.w; f.cap_rec = n->rec.cap;
  f.Wout = n->Wout;
  f.x_off = n->x_off; f.x_idx = n->x_idx; f.n_idx = n->n_idx;
  if (n->poisson) {
    f.x_thr = n->x_thr; f.x_thr_stride = n->x_thr_stride; f.x_list = n->x_list;
    f.seed = n->p.seed; f.step0 = n->blk_t0;
  }
  f.t0 = (int)(n->blk_t0 % n->p.sample_steps); f.sample_steps = (int)n->p.sample_steps; f.nsteps = n->blk_n;
  f.counters = n->counters;
  // small networks keep their rows on chip for the block; a large one's
  // forward workgroups leave LDS to the e-prop launch beside them
  f.rows_lds = n->single ? 1 : 0;
  f.zcount = n->zcount;
  n->timer.begin(s, 0);
  launch_fwd(s, f);
  HandoffArrays ho{};
  const size_t NI = n->p.n_in, NR = n->p.n_rec, B = n->B;
  uint32_t* dst[HANDOFF_ARRAYS] = {(uint32_t*)n->psiT, (uint32_t*)(n->x0T + h * NI * B),
                                   (uint32_t*)(n->z0T + h * NR * B), n->xbitsT + h * NI * B,
                                   n->zbitsT + h * NR * B};
  const int dims[HANDOFF_ARRAYS] = {(int)NR, (int)NI, (int)NR, (int)NI, (int)NR};
  for (int q = 0; q < HANDOFF_ARRAYS; ++q) {
    ho.src[q] = n->stg[q];
    ho.dst[q] = dst[q];
    ho.n[q] = dims[q];
    ho.steps[q] = q == 0 ? n->blk_n : 1;  // psi per step into the ring, the rest once per block
    ho.slot0[q] = q == 0 ? h * n->K : 0;
    ho.nslot[q] = q == 0 ? n->nslot : 1;
  }
  launch_handoff_transpose(s, ho, n->B);
  // readout state, softmax error and (when learning) the learning signal of
  // the block, still on the forward stream: the e-prop stream, which carries
  // the longer work, starts with the eligibility launch itself
  ReadoutArgs ro{};
  ro.n_rec = f.n_rec; ro.n_out = f.n_out; ro.B = n->B; ro.nsteps = n->blk_n;
  ro.slot0 = h * n->K; ro.nslot = n->nslot;
  ro.alpha = n->alpha;
  ro.u = f.u; ro.Y = n->Y; ro.Wout = n->Wout; ro.bout = n->bout; ro.labels = n->labels;
  ro.deltaT = n->deltaT; ro.LT = n->LT;
  launch_readout(s, ro, n->blk_learn);
  n->timer.end(s);
  n->last_slot = h * n->K + n->blk_n - 1;
  order(n->ev_fwd, s, e);
  if (n->blk_learn) {
    EpropArgs a{};
    a.n_in = f.n_in; a.n_rec = f.n_rec; a.n_out = f.n_out; a.B = n->B;
    a.alif = n->p.alif ? 1 : 0;
    a.alpha = (float)n->alpha; a.rho = (float)n->rho; a.beta = (float)n->beta;
    a.one_m_rho = (float)(1.0 - n->rho);
    a.in = n->in; a.rec = n->rec;
    a.x0 = n->x0T + h * NI * B; a.z0 = n->z0T + h * NR * B;
    a.xbits = n->xbitsT + h * NI * B; a.zbits = n->zbitsT + h * NR * B;
    a.tofs = 0;
    a.psiT = n->psiT; a.LT = n->LT; a.deltaT = n->deltaT;
    a.slot0 = h * n->K; a.nsteps = n->blk_n; a.nslot = n->nslot;
    a.Gout = n->Gout; a.Gb = n->Gb;
    a.col_off = n->cv.off; a.col = n->cv.col;
    n->timer.begin(e, 1);
    launch_eprop(e, a);
    n->timer.end(e);
  }
  // the next forward launch into this segment waits for everything above,
  // unless a join at an update or at the end of the call covers it first
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
  if (n->blk_n == n->K) flush_block(n);
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
    order(n->ev_back, e, s);
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
      case RS_ZBITS: *r = {n->zbitsT + (size_t)n->last_seg * NR * B, NR * B * 4}; return !for_write;
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
    case RS_P_EPS: *r = {P.eps, ns * B * 4}; return P.eps != nullptr;
    case RS_P_EBAR: *r = {P.ebar, ns * B * 4}; return true;
    case RS_P_CONN: *r = {P.conn, (size_t)P.n_pre * P.words * 4}; return P.conn != nullptr;
    case RS_P_SIGN: *r = {P.sign, (size_t)P.n_pre * P.words * 4}; return P.sign != nullptr;
    case RS_P_DORMANT: *r = {P.dormant, (size_t)P.n_pre * 4}; return true;
    default: return false;
  }
}

}  // namespace

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
  for (hipEvent_t ev : {n->ev_fwd, n->ev_join, n->ev_back, n->ev_upd, n->ev_rw})
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : n->ev_ep)
    if (ev) (void)hipEventDestroy(ev);
  if (!n->single) {
    if (n->side) (void)hipStreamDestroy(n->side);
    if (n->side2) (void)hipStreamDestroy(n->side2);
  }
  n->arena.release();
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
  bool dead = false;  // a device error occurred: every later call fails with RS_EDEVICE
};

namespace {
constexpr uint64_t GRAPH_INTERVALS = 64;

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
    launch_topo_sim(t->cap_stream, t->p.seed, t->t.P, t->sd, STEP_FROM_DEVICE, R);
    launch_topo_rewire(t->cap_stream, t->p.seed, t->t, STEP_FROM_DEVICE);
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

rs_status topo_create_impl(const rs_topo_params* p, void* stream, rs_topo* t) {
  if (p->L < 2 || p->L > 128) return fail(RS_EINVAL, "L must be in 2..128");
  if (p->cap < 1 || p->cap > 1024 || p->cap > p->L * p->L) return fail(RS_EINVAL, "cap must be in 1..min(1024, L*L)");
  if (p->n_attempts > 4096) return fail(RS_EINVAL, "n_attempts must be <= 4096");
  if (!(p->p_form >= 0) || !(p->sigma_form > 0) || !(p->p_elim_dep >= 0) || !(p->p_elim_pot >= 0))
    return fail(RS_EINVAL, "probabilities must be >= 0 and sigma_form > 0");
  if (!(std::fabs(p->g_new) <= TOPO_W_MAX) || !(std::fabs(p->g_init) <= TOPO_W_MAX))
    return fail(RS_EINVAL, "g_new and g_init must lie within +-1e4");
  t->p = *p;
  t->stream = (hipStream_t)stream;
  hipStream_t s = t->stream;
  const int L = (int)p->L, N = L * L;
  ProjDev& P = t->t.P;
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
  TRY(ar.alloc(&t->T_d2, (size_t)n_d2));
  TRY(ar.alloc(&t->t.bits, (size_t)N * P.words));
  TRY(ar.alloc(&t->t.kcount, (size_t)N));
  TRY(ar.alloc(&t->t.rowlist, (size_t)std::max<uint32_t>(p->n_attempts, 1)));
  TRY(ar.alloc(&t->t.nrows, 1));
  TRY(ar.alloc(&t->t.stats, 4));
  TRY(ar.alloc(&t->t.col_dirty, 1));
  HIP_OK(hipMemcpyAsync(t->T_d2, T.data(), n_d2 * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  t->t.T_d2 = t->T_d2;
  t->t.L = L;
  t->t.n_attempts = (int)p->n_attempts;
  t->t.g_theta = p->g_theta;
  t->t.g_new = p->g_new;
  t->t.T_dep = threshold(p->p_elim_dep);
  t->t.T_pot = threshold(p->p_elim_pot);
  launch_fill_zero(s, P.ind, (size_t)N * P.cap * 4);
  launch_fill_zero(s, P.w, (size_t)N * P.cap * 4);
  launch_gauss_rows(s, p->seed, P, L, t->T_d2, p->g_init, true);
  launch_fill_zero(s, t->t.bits, (size_t)N * P.words * 4);
  launch_fill_zero(s, t->t.stats, 32);
  launch_fill_zero(s, t->t.col_dirty, 4);
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

rs_status rs_topo_rewire(rs_topo* t, uint64_t step, rs_rewire_stats* st) {
  ENTER(t);
  if (step == STEP_FROM_DEVICE) return fail(RS_EINVAL, "step 2^64-1 is reserved");
  hipStream_t s = t->stream;
  launch_fill_zero(s, t->t.stats, 32);
  HIP_OK(hipEventRecord(t->ev0, s));
  launch_topo_rewire(s, t->p.seed, t->t, step);
  HIP_OK(hipEventRecord(t->ev1, s));
  t->timed = true;
  HIP_OK(hipGetLastError());
  if (st) {
    long long h[4];
    HIP_OK(hipMemcpyAsync(h, t->t.stats, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    st->eliminated = h[0];
    st->formed = h[1];
    st->blocked = h[2];
    st->attempts = t->p.n_attempts;
  }
  return RS_OK;
}

rs_status rs_topo_get_rows(rs_topo* t, int32_t* len, int32_t* ind, float* w) {
  ENTER(t);
  if (!len || !ind || !w) return fail(RS_EINVAL, "NULL argument");
  const ProjDev& P = t->t.P;
  const size_t n = (size_t)P.n_pre * P.cap;
  HIP_OK(hipMemcpyAsync(len, P.len, (size_t)P.n_pre * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipMemcpyAsync(ind, P.ind, n * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipMemcpyAsync(w, P.w, n * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status rs_topo_set_rows(rs_topo* t, const int32_t* len, const int32_t* ind, const float* w) {
  ENTER(t);
  if (!len || !ind || !w) return fail(RS_EINVAL, "NULL argument");
  const ProjDev& P = t->t.P;
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
  HIP_OK(hipMemcpyAsync(t->t.col_dirty, &one, 4, hipMemcpyHostToDevice, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
}

rs_status rs_topo_get_bits(rs_topo* t, uint32_t* bits) {
  ENTER(t);
  if (!bits) return fail(RS_EINVAL, "NULL argument");
  const ProjDev& P = t->t.P;
  HIP_OK(hipMemcpyAsync(bits, t->t.bits, (size_t)P.n_pre * P.words * 4, hipMemcpyDeviceToHost, t->stream));
  HIP_OK(hipStreamSynchronize(t->stream));
  return RS_OK;
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
  if (!topo_sim_fits(N)) return fail(RS_EINVAL, "the simulation needs L*L <= 4096 (L = %d)", L);
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
  }
  topo_drop_graph(t);  // the recorded launches carry the old constants
  t->m = *m;
  d.L = L;
  d.N = N;
  d.ref_steps = (int)m->ref_steps;
  d.stim_steps = (int)m->stim_steps;
  d.stim_kind = m->stim_kind;
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
  d.ticks = nullptr;  // timers off until rs_topo_sim_timing
  static const int one = 1;
  HIP_OK(hipMemcpyAsync(t->t.col_dirty, &one, 4, hipMemcpyHostToDevice, s));
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
    launch_topo_sim(s, t->p.seed, t->t.P, t->sd, t->step, (int)chunk);
    t->step += chunk;
    left -= chunk;
    if (R && t->step % R == 0) launch_topo_rewire(s, t->p.seed, t->t, t->step);
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

rs_status rs_topo_run_stats(rs_topo* t, rs_rewire_stats* st) {
  ENTER(t);
  if (!st) return fail(RS_EINVAL, "NULL argument");
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
  HIP_OK(hipStreamSynchronize(t->stream));
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
  delete t;
}

rs_status rs_calib_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16) return fail(RS_EINVAL, "copy needs non-NULL pointers and bytes % 16 == 0");
  launch_copy((hipStream_t)hip_stream, dst, src, bytes);
  HIP_OK(hipGetLastError());
  return RS_OK;
}

}  // extern "C"
