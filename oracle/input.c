/*
 * Oracle Poisson input source (test infrastructure only).
 *
 * The topographic-map model drives its source layer with Poisson spike trains
 * (Tab. A and B, "Input"), and the tiny e-prop network takes Poisson input
 * neurons with fixed rates.  In discrete time with step dt a Poisson train of
 * rate f fires in a step with probability p = f*dt; here that is a Bernoulli
 * trial per (step, instance, channel) on the counter-based generator:
 *
 *   channel i of instance b spikes at step t  <=>  u32(INPUT; t, b, i, 0) < thr_i
 *   thr_i = floor(p_i * 2^32),  p_i = rate_i * dt_ms / 1000  (p >= 1: every step)
 *
 * where u32 is the top half of Philox4x64-10 output word 0 under key
 * (seed, INPUT).  The draws depend only on (seed, t, b, i), so every instance
 * and step is independent of the others and of the order of evaluation.
 */
#include "oracle.h"

uint64_t orc_rate_threshold(double rate_hz, double dt_ms)
{
    return orc_threshold(rate_hz * dt_ms / 1000.0);
}

int64_t orc_poisson_input(uint64_t seed, uint64_t step, int32_t B, int32_t n_in,
                          const uint64_t *thr, int32_t per_instance,
                          int32_t *x_idx, int32_t *x_off)
{
    int64_t n = 0;
    for (int32_t b = 0; b < B; ++b) {
        x_off[b] = (int32_t)n;
        const uint64_t *tb = thr + (per_instance ? (int64_t)b * n_in : 0);
        for (int32_t i = 0; i < n_in; ++i) {
            const uint32_t u = orc_u32(seed, ORC_TAG_INPUT, 0, step, (uint64_t)b, (uint64_t)i, 0);
            if ((uint64_t)u < tb[i]) x_idx[n++] = i;
        }
    }
    x_off[B] = (int32_t)n;
    return n;
}
