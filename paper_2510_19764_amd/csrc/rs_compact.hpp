// Wave-parallel removal from a ragged row (paper Sec. 2.1: the last synapse of
// a row moves into a removed slot and the row shrinks by one).
//
// Applied sequentially, with the moved synapse examined again, that rule ends
// in a closed-form arrangement: with n' = n - |R| survivors, the removed slots
// below n' (ascending) receive the surviving slots at or above n' (descending),
// one to one, and nothing else moves.  One wave computes that pairing with two
// ballot/prefix passes; the caller then moves the records of each pair.
#pragma once
#include "rs_device.hpp"

namespace rs {

// remf[k] (LDS, k < n) flags removal.  Fills holes[q] / tail[q] (LDS) with the
// destination / source slot of pair q.  Returns the number of pairs; *n_keep
// receives n'.  Must be called by every lane of exactly one wave.
__device__ __forceinline__ int wave_compaction_plan(int n, const uint8_t* remf, int* holes, int* tail,
                                                    int* n_keep) {
  const int lane = lane_id();
  int R = 0;
  for (int c = 0; c < n; c += WAVE) {
    const int k = c + lane;
    R += __popcll(ballot(k < n && remf[k]));
  }
  const int n2 = n - R;
  int h = 0;
  for (int c = 0; c < n2; c += WAVE) {
    const int k = c + lane;
    const bool is_hole = k < n2 && remf[k];
    const uint64_t m = ballot(is_hole);
    if (is_hole) holes[h + __popcll(m & lanemask_lt())] = k;
    h += __popcll(m);
  }
  int t = 0;
  for (int c = 0; c < n - n2; c += WAVE) {
    const int k = n - 1 - (c + lane);
    const bool is_surv = k >= n2 && !remf[k];
    const uint64_t m = ballot(is_surv);
    if (is_surv) tail[t + __popcll(m & lanemask_lt())] = k;
    t += __popcll(m);
  }
  __syncthreads();
  *n_keep = n2;
  return h;  // == t
}

}  // namespace rs
