// DEEP R rewiring of caller-owned ragged rows without any device allocation,
// for callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid it).  The rewire kernels' scratch memory (per-row
// dormant and activation counts, the counters) lives in one file-scope device
// array of fixed size, shared by every call on a device.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/ragsnn.h"
#include "rs_kernels.hpp"

namespace {

constexpr int NOALLOC_MAX_PRE = 8192;  // rows per projection
// dormant[max], assigned[max] (int32), then 4 int64 counters
constexpr size_t SCRATCH_BYTES = (size_t)NOALLOC_MAX_PRE * 8 + 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::once_flag g_once[MAX_DEVICES];
void* g_scratch[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};

}  // namespace

rs_status rs_internal_fail(rs_status code, const char* fmt, ...);

extern "C" rs_status rs_deepr_rewire_noalloc(const rs_deepr_rows* r, uint64_t seed, uint32_t proj_id, uint64_t step,
                                             void* hip_stream, rs_rewire_stats* stats) {
  if (!r) return rs_internal_fail(RS_EINVAL, "rows are NULL");
  if (r->n_pre < 1 || r->n_pre > NOALLOC_MAX_PRE)
    return rs_internal_fail(RS_EINVAL, "n_pre %d outside 1..%d (the scratch holds %d rows)", r->n_pre,
                            NOALLOC_MAX_PRE, NOALLOC_MAX_PRE);
  if (r->n_post < 1 || r->cap < 1 || r->cap > r->n_post || r->batch < 1 || r->words != (r->n_post + 31) / 32)
    return rs_internal_fail(RS_EINVAL, "inconsistent sizes (n_post, cap, batch, words)");
  if (!r->len || !r->ind || !r->w || !r->m || !r->v || !r->G || !r->ebar || !r->conn || !r->sign)
    return rs_internal_fail(RS_EINVAL, "row arrays must not be NULL (eps may be)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    (void)hipGetLastError();
    return rs_internal_fail(RS_EDEVICE, "no current device");
  }
  // the array's address on this device, looked up once with the device current
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  if (!g_scratch[dev])
    return rs_internal_fail(RS_EDEVICE, "scratch address: %s", hipGetErrorString(g_scratch_err[dev]));
  unsigned char* base = (unsigned char*)g_scratch[dev];
  rs::ProjDev P{};
  P.n_pre = r->n_pre;
  P.n_post = r->n_post;
  P.cap = r->cap;
  P.words = r->words;
  P.recurrent = r->recurrent ? 1 : 0;
  P.proj_id = (int)proj_id;
  P.len = r->len;
  P.ind = r->ind;
  P.w = r->w;
  P.m = r->m;
  P.v = r->v;
  P.G = r->G;
  P.eps = r->eps;
  P.ebar = r->ebar;
  P.erec = (int)r->batch;  // the caller's ebar and eps are separate arrays
  P.conn = r->conn;
  P.sign = r->sign;
  P.dormant = (int*)base;                           // written for every row by the elimination
  P.assigned = (int*)(base + NOALLOC_MAX_PRE * 4);  // written for every row by the distribution
  long long* counters = (long long*)(base + (size_t)NOALLOC_MAX_PRE * 8);
  hipStream_t s = (hipStream_t)hip_stream;
  rs::launch_fill_zero(s, counters, 32);  // a kernel: the counters start at zero
  rs::launch_deepr(s, seed, P, r->batch, step, counters);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && stats) {
    long long h[4];
    e = hipMemcpyAsync(h, counters, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      stats->eliminated = h[0];
      stats->formed = h[1];
      stats->attempts = h[2];
      stats->blocked = h[3];
    }
  }
  if (e != hipSuccess) return rs_internal_fail(RS_EDEVICE, "DEEP R launch: %s", hipGetErrorString(e));
  return RS_OK;
}
