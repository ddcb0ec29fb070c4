/*
 * Oracle topographic-map rewiring (test infrastructure only), paper Sec. 2.1.3,
 * Fig. 3, Tab. B and Tab. G.
 *
 * One connectivity update:
 *   1. the host distributes N_attempts attempts uniformly, with replacement,
 *      over the presynaptic rows;
 *   2. each row with k attempts sets k distinct bits of its own section of the
 *      attempt bitfield, chosen uniformly without replacement (candidates);
 *   3. elimination: every existing synapse whose target bit is set is removed
 *      with probability p_elim_dep if its weight is below g_theta, p_elim_pot
 *      otherwise, and its bit is cleared either way;
 *   4. formation: every bit still set marks an empty slot; a synapse with weight
 *      g_new is formed there with probability p_form exp(-d^2 / 2 sigma^2) and
 *      the bit is cleared.  No multapses are possible since occupied targets only
 *      ever reach step 3.
 * Readings: the uniform draw R < p is taken as u32 < floor(p 2^32) with
 * p >= 1 always succeeding; each elimination draw is keyed by the synapse's
 * slot before any removal in this update, so the removal set does not depend on
 * processing order; removal moves the row's last synapse into the freed slot and
 * examines it again; a row already at capacity cannot form (counted as blocked);
 * formation visits the surviving candidates in ascending target order.
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "oracle.h"

static int get_bit(const uint32_t *bits, int32_t words, int32_t i, int32_t j)
{
    return (int)((bits[(int64_t)i * words + (j >> 5)] >> (j & 31)) & 1u);
}

static void put_bit(uint32_t *bits, int32_t words, int32_t i, int32_t j, int on)
{
    uint32_t *wd = &bits[(int64_t)i * words + (j >> 5)];
    if (on) *wd |= (1u << (j & 31));
    else *wd &= ~(1u << (j & 31));
}

void orc_topo_rewire_with(orc_proj *P, const orc_topo_params *tp, const orc_topo_draws *d,
                          uint32_t *bits, int32_t *stats)
{
    const int32_t n_pre = P->n_pre, n_post = P->n_post, W = P->words;
    int32_t *k = (int32_t *)calloc((size_t)n_pre, sizeof(int32_t));
    int32_t *orig = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P->cap > 0 ? P->cap : 1));
    uint8_t *remove = (uint8_t *)malloc((size_t)(P->cap > 0 ? P->cap : 1));
    uint64_t T_dep = orc_threshold(tp->p_elim_dep), T_pot = orc_threshold(tp->p_elim_pot);
    float g_theta = (float)tp->g_theta;
    int32_t eliminated = 0, formed = 0, blocked = 0;

    /* 1. attempts -> rows, with replacement */
    for (int32_t a = 0; a < tp->n_attempts; ++a) k[d->attempt_row(d->ctx, a)]++;

    for (int32_t r = 0; r < n_pre; ++r) {
        if (k[r] == 0) continue;
        int64_t base = (int64_t)r * P->cap;
        /* 2. candidate targets without replacement */
        int32_t kr = k[r] < n_post ? k[r] : n_post;
        for (int32_t q = 0; q < kr; ++q) {
            int32_t j = -1;
            for (int32_t t = 0; t < ORC_MAX_TRIES; ++t) {
                int32_t c = (int32_t)d->target(d->ctx, r, q, t);
                if (!get_bit(bits, W, r, c)) { j = c; break; }
            }
            if (j < 0) {
                int32_t start = (int32_t)d->target(d->ctx, r, q, ORC_MAX_TRIES);
                for (int32_t s = 0; s < n_post; ++s) {
                    int32_t c = (start + s) % n_post;
                    if (!get_bit(bits, W, r, c)) { j = c; break; }
                }
            }
            put_bit(bits, W, r, j, 1);
        }
        /* 3. elimination attempts on existing synapses marked as candidates */
        int32_t n = P->len[r];
        for (int32_t s = 0; s < n; ++s) {
            int32_t j = P->ind[base + s];
            remove[s] = 0;
            orig[s] = s;
            if (get_bit(bits, W, r, j)) {
                uint64_t T = ((float)P->w[base + s] < g_theta) ? T_dep : T_pot;
                remove[s] = (uint64_t)d->elim_u32(d->ctx, r, s) < T;
                put_bit(bits, W, r, j, 0);
            }
        }
        int32_t s = 0;
        while (s < P->len[r]) {
            if (remove[orig[s]]) {
                int32_t last = P->len[r] - 1;
                if (s != last) {
                    P->ind[base + s] = P->ind[base + last];
                    P->w[base + s] = P->w[base + last];
                    if (P->m) P->m[base + s] = P->m[base + last];
                    if (P->v) P->v[base + s] = P->v[base + last];
                    if (P->G) P->G[base + s] = P->G[base + last];
                    orig[s] = orig[last];
                }
                P->len[r]--;
                eliminated++;
            } else {
                ++s;
            }
        }
        /* 4. formation attempts on the remaining (empty) candidates */
        for (int32_t j = 0; j < n_post; ++j) {
            if (!get_bit(bits, W, r, j)) continue;
            put_bit(bits, W, r, j, 0);
            double d2 = (double)orc_torus_d2(tp->L, r, j);
            uint64_t T = orc_threshold(tp->p_form * exp(-d2 / (2.0 * tp->sigma_form * tp->sigma_form)));
            if ((uint64_t)d->form_u32(d->ctx, r, j) < T) {
                if (P->len[r] < P->cap) {
                    int64_t slot = base + P->len[r];
                    P->ind[slot] = j;
                    P->w[slot] = (double)(float)tp->g_new;
                    if (P->m) P->m[slot] = 0.0;
                    if (P->v) P->v[slot] = 0.0;
                    if (P->G) P->G[slot] = 0.0;
                    P->len[r]++;
                    formed++;
                } else {
                    blocked++;
                }
            }
        }
    }
    stats[0] = eliminated;
    stats[1] = formed;
    stats[2] = blocked;
    stats[3] = tp->n_attempts;
    free(k);
    free(orig);
    free(remove);
}

/* ---- Philox-backed draw source ---- */
typedef struct {
    uint64_t seed, step;
    uint32_t proj;
    int32_t n_pre, n_post;
} philox_ctx;

static uint32_t ph_row(void *c, int32_t a)
{
    philox_ctx *p = (philox_ctx *)c;
    return orc_below(orc_u32(p->seed, ORC_TAG_TP_ROW, p->proj, p->step, (uint64_t)a, 0, 0), (uint32_t)p->n_pre);
}
static uint32_t ph_tgt(void *c, int32_t r, int32_t q, int32_t t)
{
    philox_ctx *p = (philox_ctx *)c;
    return orc_below(orc_u32(p->seed, ORC_TAG_TP_TGT, p->proj, p->step, (uint64_t)r, (uint64_t)q, (uint64_t)t),
                     (uint32_t)p->n_post);
}
static uint32_t ph_elim(void *c, int32_t r, int32_t s)
{
    philox_ctx *p = (philox_ctx *)c;
    return orc_u32(p->seed, ORC_TAG_TP_ELIM, p->proj, p->step, (uint64_t)r, (uint64_t)s, 0);
}
static uint32_t ph_form(void *c, int32_t r, int32_t j)
{
    philox_ctx *p = (philox_ctx *)c;
    return orc_u32(p->seed, ORC_TAG_TP_FORM, p->proj, p->step, (uint64_t)r, (uint64_t)j, 0);
}

void orc_topo_rewire(uint64_t seed, orc_proj *P, const orc_topo_params *tp, uint64_t step,
                     uint32_t *bits, int32_t *stats)
{
    philox_ctx c = {seed, step, (uint32_t)P->proj_id, P->n_pre, P->n_post};
    orc_topo_draws d = {ph_row, ph_tgt, ph_elim, ph_form, &c};
    orc_topo_rewire_with(P, tp, &d, bits, stats);
}
