/*
 * Oracle custom connectivity updates (test infrastructure only): the paper's
 * two worked examples of the custom connectivity-update framework (Sec. 2.1),
 * written as the sequential row loops they describe.
 *
 * add_diagonal: the row update of every presynaptic neuron adds one synapse
 * onto the postsynaptic neuron with the same index, weight 1.0; variables the
 * update does not set start at zero.  A row without room is left as it is
 * (the ragged structure cannot grow past its capacity); a projection that
 * records connectivity in a bitfield skips a target already connected.
 *
 * remove_random: the host update picks one random postsynaptic index per row;
 * the row update walks the row's synapses in slot order and removes the first
 * one onto that index (the last synapse of the row moves into its slot and
 * the row shrinks by one), then stops.
 */
#include <string.h>
#include "oracle.h"

static void clear_record(orc_proj *P, int32_t B, int64_t s)
{
    if (P->m) P->m[s] = 0.0;
    if (P->v) P->v[s] = 0.0;
    if (P->G) P->G[s] = 0.0;
    if (P->Gabs) P->Gabs[s] = 0.0;
    if (P->eps) memset(&P->eps[s * B], 0, sizeof(double) * B);
    if (P->ebar) memset(&P->ebar[s * B], 0, sizeof(double) * B);
}

static void copy_record(orc_proj *P, int32_t B, int64_t to, int64_t from)
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

int32_t orc_add_diagonal(orc_proj *P, int32_t B)
{
    int32_t added = 0;
    for (int32_t i = 0; i < P->n_pre && i < P->n_post; ++i) {
        if (P->len[i] >= P->cap) continue;
        if (P->conn && ((P->conn[(int64_t)i * P->words + (i >> 5)] >> (i & 31)) & 1u)) continue;
        int64_t s = (int64_t)i * P->cap + P->len[i];
        P->ind[s] = i;
        P->w[s] = 1.0;
        clear_record(P, B, s);
        if (P->conn) P->conn[(int64_t)i * P->words + (i >> 5)] |= 1u << (i & 31);
        P->len[i]++;
        added++;
    }
    return added;
}

void orc_remove_random_targets(uint64_t seed, const orc_proj *P, uint64_t step, uint32_t *post_ind)
{
    for (int32_t i = 0; i < P->n_pre; ++i)
        post_ind[i] = orc_below(orc_u32(seed, ORC_TAG_CUSTOM, (uint32_t)P->proj_id, step, (uint64_t)i, 0, 0),
                                (uint32_t)P->n_post);
}

int32_t orc_remove_targets(orc_proj *P, int32_t B, const uint32_t *post_ind)
{
    int32_t removed = 0;
    for (int32_t i = 0; i < P->n_pre; ++i) {
        int64_t base = (int64_t)i * P->cap;
        for (int32_t k = 0; k < P->len[i]; ++k) {
            if ((uint32_t)P->ind[base + k] != post_ind[i]) continue;
            int32_t j = P->ind[base + k];
            if (P->conn) P->conn[(int64_t)i * P->words + (j >> 5)] &= ~(1u << (j & 31));
            int32_t last = P->len[i] - 1;
            if (k != last) copy_record(P, B, base + k, base + last);
            P->len[i]--;
            removed++;
            break;
        }
    }
    return removed;
}
