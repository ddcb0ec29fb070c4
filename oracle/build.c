/*
 * Oracle network construction (test infrastructure only).
 *
 * - Fixed-probability connectivity: every (pre, post) pair is connected with
 *   probability p (paper, recurrent classifier model; no autapses in the
 *   recurrent projection since its input sum runs over i != j).
 * - Pairwise-Bernoulli Gaussian connectivity for the topographic map: a pair is
 *   connected with the formation probability p_form exp(-d^2 / 2 sigma^2) of
 *   Tab. B, d being the distance on an L x L grid with periodic boundaries
 *   (Tab. A; initialisation rule described in the topographic-map section).
 * - DEEP R bitfields (Sec. 2.1.2, Fig. 2A): clear all connectivity bits,
 *   randomise all sign bits, then for every existing synapse set its
 *   connectivity bit and force its sign bit to the sign of its weight.
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "oracle.h"

int32_t orc_fixed_prob_rows(uint64_t seed, orc_proj *P, double p, double sigma)
{
    uint64_t T = orc_threshold(p);
    int32_t max_len = 0;
    for (int32_t i = 0; i < P->n_pre; ++i) {
        int32_t n = 0;
        for (int32_t j = 0; j < P->n_post; ++j) {
            if (P->recurrent && j == i) continue;
            uint32_t u = orc_u32(seed, ORC_TAG_CONN, P->proj_id, 0, i, j, 0);
            if ((uint64_t)u < T) {
                if (P->ind) {
                    P->ind[(int64_t)i * P->cap + n] = j;
                    P->w[(int64_t)i * P->cap + n] =
                        (double)(float)(sigma * orc_normal(seed, ORC_TAG_WINIT, P->proj_id, 0, i, j, 0));
                }
                ++n;
            }
        }
        P->len[i] = n;
        if (n > max_len) max_len = n;
    }
    return max_len;
}

int32_t orc_torus_d2(int32_t L, int32_t i, int32_t j)
{
    int32_t xi = i % L, yi = i / L, xj = j % L, yj = j / L;
    int32_t dx = abs(xi - xj), dy = abs(yi - yj);
    if (L - dx < dx) dx = L - dx;
    if (L - dy < dy) dy = L - dy;
    return dx * dx + dy * dy;
}

int32_t orc_gauss_rows(uint64_t seed, orc_proj *P, int32_t L, double p_form, double sigma,
                       double g_init)
{
    int32_t max_len = 0;
    for (int32_t i = 0; i < P->n_pre; ++i) {
        int32_t n = 0;
        for (int32_t j = 0; j < P->n_post; ++j) {
            double d2 = (double)orc_torus_d2(L, i, j);
            uint64_t T = orc_threshold(p_form * exp(-d2 / (2.0 * sigma * sigma)));
            uint32_t u = orc_u32(seed, ORC_TAG_CONN, P->proj_id, 0, i, j, 0);
            if ((uint64_t)u < T) {
                if (P->ind && n < P->cap) {
                    P->ind[(int64_t)i * P->cap + n] = j;
                    P->w[(int64_t)i * P->cap + n] = (double)(float)g_init;
                }
                ++n;
            }
        }
        P->len[i] = (P->ind && n > P->cap) ? P->cap : n;
        if (n > max_len) max_len = n;
    }
    return max_len;
}

void orc_dense_init(uint64_t seed, int32_t proj_id, int32_t rows, int32_t cols, double sigma,
                    double *W)
{
    for (int32_t k = 0; k < rows; ++k)
        for (int32_t j = 0; j < cols; ++j)
            W[(int64_t)k * cols + j] =
                (double)(float)(sigma * orc_normal(seed, ORC_TAG_WINIT, proj_id, 0, k, j, 0));
}

static void set_bit(uint32_t *bits, int32_t words, int32_t i, int32_t j, int on)
{
    uint32_t *wd = &bits[(int64_t)i * words + (j >> 5)];
    if (on) *wd |= (1u << (j & 31));
    else *wd &= ~(1u << (j & 31));
}

void orc_deepr_init_bits(uint64_t seed, orc_proj *P)
{
    /* all connectivity bits cleared, every potential sign randomised */
    for (int32_t i = 0; i < P->n_pre; ++i) {
        for (int32_t wd = 0; wd < P->words; ++wd) P->conn[(int64_t)i * P->words + wd] = 0u;
        for (int32_t j = 0; j < P->n_post; ++j) {
            uint32_t u = orc_u32(seed, ORC_TAG_SIGN, P->proj_id, 0, i, j, 0);
            set_bit(P->sign, P->words, i, j, (int)(u >> 31));
        }
    }
    /* existing synapses: connectivity bit set, sign bit = weight is negative */
    for (int32_t i = 0; i < P->n_pre; ++i)
        for (int32_t k = 0; k < P->len[i]; ++k) {
            int32_t j = P->ind[(int64_t)i * P->cap + k];
            set_bit(P->conn, P->words, i, j, 1);
            set_bit(P->sign, P->words, i, j, ((float)P->w[(int64_t)i * P->cap + k]) < 0.0f);
        }
}
