// Parameter update after an e-prop interval: gradient averaged over the batch,
// L1 term with the sign bit for DEEP R projections (Sec. 2.1.2, "L1
// regularisation"), one Adam step (Kingma & Ba defaults), gradient cleared.
// One thread per slot of the padded row arrays; slots past a row's length are
// skipped, the dense readout follows in the same grid.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

__device__ __forceinline__ void adam(float& w, float& m, float& v, float g, const UpdateArgs& a) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * g * g;
  const float mhat = m * a.inv_c1, vhat = v * a.inv_c2;
  w -= a.lr * mhat / (sqrtf(vhat) + a.eps);
}

__device__ __forceinline__ void update_slot(const ProjDev& P, int64_t q, bool l1, const UpdateArgs& a) {
  const int i = (int)(q / P.cap), k = (int)(q % P.cap);
  if (k >= P.len[i]) return;
  float g = P.G[q] / (float)a.B;
  if (l1) {
    const int j = P.ind[q];
    g += get_bit(P.sign, P.words, i, j) ? -a.l1 : a.l1;
  }
  float w = P.w[q], m = P.m[q], v = P.v[q];
  adam(w, m, v, g, a);
  P.w[q] = w;
  P.m[q] = m;
  P.v[q] = v;
  P.G[q] = 0.0f;
}

__global__ void k_update(UpdateArgs a) {
  const int64_t n_in = (int64_t)a.in.n_pre * a.in.cap, n_rec = (int64_t)a.rec.n_pre * a.rec.cap;
  const int64_t total = n_in + n_rec + a.n_out_elems + a.n_b;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    if (q < n_in) {
      update_slot(a.in, q, a.l1_in, a);
    } else if (q < n_in + n_rec) {
      update_slot(a.rec, q - n_in, a.l1_rec, a);
    } else if (q < n_in + n_rec + a.n_out_elems) {
      const int64_t r = q - n_in - n_rec;
      float w = a.Wout[r], m = a.Mout[r], v = a.Vout[r];
      adam(w, m, v, a.Gout[r] / (float)a.B, a);
      a.Wout[r] = w;
      a.Mout[r] = m;
      a.Vout[r] = v;
      a.Gout[r] = 0.0f;
    } else {
      const int64_t r = q - n_in - n_rec - a.n_out_elems;
      float w = a.bout[r], m = a.Mb[r], v = a.Vb[r];
      adam(w, m, v, a.Gb[r] / (float)a.B, a);
      a.bout[r] = w;
      a.Mb[r] = m;
      a.Vb[r] = v;
      a.Gb[r] = 0.0f;
    }
  }
}

void launch_update(hipStream_t s, const UpdateArgs& a) {
  const int64_t total = (int64_t)a.in.n_pre * a.in.cap + (int64_t)a.rec.n_pre * a.rec.cap + a.n_out_elems + a.n_b;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace rs
