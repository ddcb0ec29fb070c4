// Readout of served inference requests (paper, recurrent classifier section,
// without learning): one wave per running request takes its leaky readout
// through the block's steps,
//   y_k <- alpha y_k + u_k + b_k   (double),   pi = softmax(y),
// and adds every step's pi to the request's score sum_t pi_k^t, whose argmax
// is the request's decision.  The softmax is computed as the training
// readout computes it.
#include "rs_device.hpp"
#include "rs_kernels.hpp"

namespace rs {

constexpr int SR_KMAX = 4;  // n_out <= 4 * WAVE

__global__ void __launch_bounds__(256) k_serve_readout(const ServeReadout* __restrict__ R, int n) {
  const int w = blockIdx.x * 4 + wave_id(), lane = lane_id();
  if (w >= n) return;
  const ServeReadout a = R[w];
  double y[SR_KMAX], sc[SR_KMAX];
  float bias[SR_KMAX];
#pragma unroll
  for (int q = 0; q < SR_KMAX; ++q) {
    const int k = q * WAVE + lane;
    y[q] = k < a.n_out ? a.Y[k] : 0.0;
    sc[q] = k < a.n_out ? a.score[k] : 0.0;
    bias[q] = k < a.n_out ? a.bout[k] : 0.0f;
  }
  for (int tau = 0; tau < a.nsteps; ++tau) {
    const float* u = a.u + (int64_t)tau * a.n_out;
    float m = -INFINITY;
#pragma unroll
    for (int q = 0; q < SR_KMAX; ++q) {
      const int k = q * WAVE + lane;
      if (k < a.n_out) {
        y[q] = a.alpha * y[q] + (double)u[k] + (double)bias[q];
        m = fmaxf(m, (float)y[q]);
      }
    }
    m = wave_max(m);
    float den = 0.0f;
#pragma unroll
    for (int q = 0; q < SR_KMAX; ++q)
      if (q * WAVE + lane < a.n_out) den += expf((float)y[q] - m);
    den = wave_sum(den);
#pragma unroll
    for (int q = 0; q < SR_KMAX; ++q)
      if (q * WAVE + lane < a.n_out) sc[q] += (double)(expf((float)y[q] - m) / den);
  }
#pragma unroll
  for (int q = 0; q < SR_KMAX; ++q) {
    const int k = q * WAVE + lane;
    if (k < a.n_out) {
      a.Y[k] = y[q];
      a.score[k] = sc[q];
    }
  }
}

void launch_serve_readout(hipStream_t s, const ServeReadout* R, int n) {
  if (n > 0) hipLaunchKernelGGL(k_serve_readout, dim3((n + 3) / 4), dim3(256), 0, s, R, n);
}

}  // namespace rs
