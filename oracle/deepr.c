/*
 * Oracle DEEP R rewiring (test infrastructure only), paper Sec. 2.1.2 / Fig. 2.
 *
 * Elimination: every synapse whose weight sign no longer matches its sign bit
 * is removed, the row's dormant counter is incremented and its connectivity bit
 * cleared.  Removal uses the ragged-row rule of Sec. 2.1: the last synapse of
 * the row moves into the freed slot (with all its variables) and the row length
 * drops by one; the moved synapse is examined again.  A weight of exactly zero
 * is never a mismatch.
 *
 * Formation: the dormant counts are summed and redistributed uniformly over the
 * rows as activations (each activation picks a row uniformly; rows that cannot
 * take more because they are full send their excess to a redraw round).  Each
 * row then adds one synapse per activation to a random target whose
 * connectivity bit is clear (no duplicates, no autapses in recurrent
 * projections); new synapses start with weight, optimiser state, gradient and
 * eligibility traces at zero (unreferenced variables are zero-initialised,
 * Sec. 2.1).  The connection count is therefore unchanged.
 */
#include <string.h>
#include <stdlib.h>
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

/* Move the whole record of slot `from` into slot `to` of the same row. */
static void move_record(orc_proj *P, int32_t B, int64_t to, int64_t from)
{
    P->ind[to] = P->ind[from];
    P->w[to] = P->w[from];
    if (P->m) P->m[to] = P->m[from];
    if (P->v) P->v[to] = P->v[from];
    if (P->G) P->G[to] = P->G[from];
    if (P->Gabs) P->Gabs[to] = P->Gabs[from];
    if (P->eps) memcpy(&P->eps[to * B], &P->eps[from * B], sizeof(double) * B);
    if (P->ebar) memcpy(&P->ebar[to * B], &P->ebar[from * B], sizeof(double) * B);
}

static int sign_mismatch(const orc_proj *P, int32_t i, int64_t s)
{
    float w = (float)P->w[s];
    int negative = get_bit(P->sign, P->words, i, P->ind[s]);
    return (w > 0.0f && negative) || (w < 0.0f && !negative);
}

void orc_deepr_rewire(uint64_t seed, orc_proj *P, int32_t B, uint64_t step, int32_t *dormant,
                      int32_t *stats)
{
    const int32_t n_pre = P->n_pre;
    /* ---- elimination, row by row ---- */
    int64_t D = 0;
    for (int32_t i = 0; i < n_pre; ++i) {
        dormant[i] = 0;
        int64_t base = (int64_t)i * P->cap;
        int32_t k = 0;
        while (k < P->len[i]) {
            if (sign_mismatch(P, i, base + k)) {
                put_bit(P->conn, P->words, i, P->ind[base + k], 0);
                dormant[i]++;
                int32_t last = P->len[i] - 1;
                if (k != last) move_record(P, B, base + k, base + last);
                P->len[i]--;
                /* the moved synapse is examined at the same slot */
            } else {
                ++k;
            }
        }
        D += dormant[i];
    }

    /* ---- formation: distribute D activations over rows ---- */
    int32_t limit = P->n_post - (P->recurrent ? 1 : 0);
    if (limit > P->cap) limit = P->cap;
    int32_t *assigned = (int32_t *)calloc((size_t)n_pre, sizeof(int32_t));
    int32_t *cnt = (int32_t *)calloc((size_t)n_pre, sizeof(int32_t));
    int64_t pending = D;
    for (int32_t round = 0; pending > 0 && round < ORC_MAX_ROUNDS; ++round) {
        memset(cnt, 0, sizeof(int32_t) * n_pre);
        for (int64_t a = 0; a < pending; ++a) {
            uint32_t u = orc_u32(seed, ORC_TAG_DR_ROW, P->proj_id, step, (uint64_t)a, (uint64_t)round, 0);
            cnt[orc_below(u, (uint32_t)n_pre)]++;
        }
        int64_t rejected = 0;
        for (int32_t r = 0; r < n_pre; ++r) {
            int32_t room = limit - P->len[r] - assigned[r];
            if (room < 0) room = 0;
            int32_t acc = cnt[r] < room ? cnt[r] : room;
            assigned[r] += acc;
            rejected += cnt[r] - acc;
        }
        pending = rejected;
    }
    for (int32_t r = 0; r < n_pre && pending > 0; ++r) {
        int32_t room = limit - P->len[r] - assigned[r];
        if (room <= 0) continue;
        int32_t take = pending < room ? (int32_t)pending : room;
        assigned[r] += take;
        pending -= take;
    }

    /* ---- formation: each row adds its activations ---- */
    int64_t formed = 0;
    for (int32_t r = 0; r < n_pre; ++r) {
        for (int32_t k = 0; k < assigned[r]; ++k) {
            int32_t j = -1;
            for (int32_t t = 0; t < ORC_MAX_TRIES; ++t) {
                uint32_t u = orc_u32(seed, ORC_TAG_DR_TGT, P->proj_id, step, (uint64_t)r, (uint64_t)k, (uint64_t)t);
                int32_t c = (int32_t)orc_below(u, (uint32_t)P->n_post);
                if (!get_bit(P->conn, P->words, r, c) && !(P->recurrent && c == r)) { j = c; break; }
            }
            if (j < 0) { /* bounded fallback: first free target after a random start */
                uint32_t u = orc_u32(seed, ORC_TAG_DR_TGT, P->proj_id, step, (uint64_t)r, (uint64_t)k, ORC_MAX_TRIES);
                int32_t start = (int32_t)orc_below(u, (uint32_t)P->n_post);
                for (int32_t d = 0; d < P->n_post; ++d) {
                    int32_t c = (start + d) % P->n_post;
                    if (!get_bit(P->conn, P->words, r, c) && !(P->recurrent && c == r)) { j = c; break; }
                }
            }
            if (j < 0) break; /* cannot happen: the row had room */
            int64_t s = (int64_t)r * P->cap + P->len[r];
            P->ind[s] = j;
            P->w[s] = 0.0;
            if (P->m) P->m[s] = 0.0;
            if (P->v) P->v[s] = 0.0;
            if (P->G) P->G[s] = 0.0;
            if (P->Gabs) P->Gabs[s] = 0.0;
            if (P->eps) memset(&P->eps[s * B], 0, sizeof(double) * B);
            if (P->ebar) memset(&P->ebar[s * B], 0, sizeof(double) * B);
            put_bit(P->conn, P->words, r, j, 1);
            P->len[r]++;
            formed++;
        }
    }
    stats[0] = (int32_t)D;
    stats[1] = (int32_t)formed;
    free(assigned);
    free(cnt);
}
