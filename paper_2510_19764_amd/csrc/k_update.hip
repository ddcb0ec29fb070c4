// Parameter update after an e-prop interval: gradient averaged over the batch,
// L1 term with the sign bit for DEEP R projections (Sec. 2.1.2, "L1
// regularisation"), one Adam step (Kingma & Ba defaults), gradient cleared.
// One thread per slot of the padded row arrays; slots past a row's length are
// skipped, the dense readout follows in the same grid.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int UPD_NT = 256;

struct AdamC {
  float inv_c1, inv_c2;  // bias corrections 1 / (1 - b^k) of this update
};

__device__ __forceinline__ void adam(float& w, float& m, float& v, float g, const UpdateArgs& a, AdamC c) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * g * g;
  const float mhat = m * c.inv_c1, vhat = v * c.inv_c2;
  w -= a.lr * mhat / (sqrtf(vhat) + a.eps);
}

// The update's bias corrections: passed by value, or (a recorded launch
// replayed) looked up by the device's update count in a table the host filled
// with the same values.
__device__ __forceinline__ AdamC adam_c(const UpdateArgs& a) {
  if (!a.adam_tab) return {a.inv_c1, a.inv_c2};
  uint32_t k = *a.adam_base + (uint32_t)a.adam_off;
  k = k < (uint32_t)a.adam_kmax ? k : (uint32_t)a.adam_kmax;
  return {a.adam_tab[2 * k], a.adam_tab[2 * k + 1]};
}

__device__ __forceinline__ void update_slot(const ProjDev& P, int64_t q, bool l1, const UpdateArgs& a, AdamC c) {
  const int i = (int)(q / P.cap), k = (int)(q % P.cap);
  if (k >= P.len[i]) return;
  float g = P.G[q] / (float)a.B;
  if (l1) {
    const int j = P.ind[q];
    g += get_bit(P.sign, P.words, i, j) ? -a.l1 : a.l1;
  }
  float w = P.w[q], m = P.m[q], v = P.v[q];
  adam(w, m, v, g, a, c);
  P.w[q] = w;
  P.m[q] = m;
  P.v[q] = v;
  P.G[q] = 0.0f;
}

__device__ __forceinline__ void update_body(const UpdateArgs& a, const int blk, const int nblk) {
  const AdamC c = adam_c(a);
  const int64_t n_in = (int64_t)a.in.n_pre * a.in.cap, n_rec = (int64_t)a.rec.n_pre * a.rec.cap;
  const int64_t total = n_in + n_rec + a.n_out_elems + a.n_b;
  const int64_t stride = (int64_t)nblk * UPD_NT;
  for (int64_t q = (int64_t)blk * UPD_NT + threadIdx.x; q < total; q += stride) {
    if (q < n_in) {
      update_slot(a.in, q, a.l1_in, a, c);
    } else if (q < n_in + n_rec) {
      update_slot(a.rec, q - n_in, a.l1_rec, a, c);
    } else if (q < n_in + n_rec + a.n_out_elems) {
      const int64_t r = q - n_in - n_rec;
      float w = a.Wout[r], m = a.Mout[r], v = a.Vout[r];
      adam(w, m, v, a.Gout[r] / (float)a.B, a, c);
      a.Wout[r] = w;
      a.Mout[r] = m;
      a.Vout[r] = v;
      a.Gout[r] = 0.0f;
    } else {
      const int64_t r = q - n_in - n_rec - a.n_out_elems;
      float w = a.bout[r], m = a.Mb[r], v = a.Vb[r];
      adam(w, m, v, a.Gb[r] / (float)a.B, a, c);
      a.bout[r] = w;
      a.Mb[r] = m;
      a.Vb[r] = v;
      a.Gb[r] = 0.0f;
    }
  }
}

__global__ void __launch_bounds__(UPD_NT) k_update(UpdateArgs a) { update_body(a, blockIdx.x, gridDim.x); }

// Several networks: workgroup g is block work[g].y of work[g].z blocks of
// network work[g].x.
__global__ void __launch_bounds__(UPD_NT) k_update_multi(const UpdateArgs* __restrict__ A,
                                                         const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  const UpdateArgs a = A[w.x];
  update_body(a, w.y, w.z);
}

int update_blocks(const UpdateArgs& a) {
  const int64_t total = (int64_t)a.in.n_pre * a.in.cap + (int64_t)a.rec.n_pre * a.rec.cap + a.n_out_elems + a.n_b;
  int64_t blocks = (total + UPD_NT - 1) / UPD_NT;
  return (int)(blocks > 4096 ? 4096 : blocks);
}

void launch_update_multi(hipStream_t s, const UpdateArgs* A, const int4* work, int n_work) {
  if (n_work > 0) hipLaunchKernelGGL(k_update_multi, dim3(n_work), dim3(UPD_NT), 0, s, A, work);
}

void launch_update(hipStream_t s, const UpdateArgs& a) {
  hipLaunchKernelGGL(k_update, dim3((unsigned)update_blocks(a)), dim3(UPD_NT), 0, s, a);
}

}  // namespace rs
