/*
 * Oracle parameter update (test infrastructure only).
 *
 * After each update interval the accumulated e-prop gradients are averaged over
 * the batch; for projections rewired by DEEP R a constant L1 term is added with
 * the sign recorded in the sign bitfield, pushing weights towards zero (paper,
 * Sec. 2.1.2, "L1 regularisation"); all parameters then take one Adam step with
 * the default hyper-parameters of Kingma & Ba (results section: "Adam optimizer
 * with default parameters"), and the accumulators are cleared.
 */
#include <math.h>
#include "oracle.h"

static void adam(double *w, double *m, double *v, double g, double lr, double b1, double b2,
                 double eps, double c1, double c2)
{
    *m = b1 * *m + (1.0 - b1) * g;
    *v = b2 * *v + (1.0 - b2) * g * g;
    double mhat = *m / c1, vhat = *v / c2;
    *w -= lr * mhat / (sqrt(vhat) + eps);
}

static void update_proj(orc_proj *P, int32_t B, int32_t with_l1, double l1, double lr, double b1,
                        double b2, double eps, double c1, double c2)
{
    for (int32_t i = 0; i < P->n_pre; ++i)
        for (int32_t k = 0; k < P->len[i]; ++k) {
            int64_t s = (int64_t)i * P->cap + k;
            double g = P->G[s] / (double)B;
            if (with_l1) {
                int32_t j = P->ind[s];
                int negative = (P->sign[(int64_t)i * P->words + (j >> 5)] >> (j & 31)) & 1u;
                g += negative ? -l1 : l1;
            }
            adam(&P->w[s], &P->m[s], &P->v[s], g, lr, b1, b2, eps, c1, c2);
            P->G[s] = 0.0;
            if (P->Gabs) P->Gabs[s] = 0.0;
        }
}

void orc_adam_update(orc_net *N, int32_t k, double lr, double b1, double b2, double eps,
                     double l1, int32_t deepr_mask)
{
    double c1 = 1.0 - pow(b1, (double)k), c2 = 1.0 - pow(b2, (double)k);
    int32_t B = N->batch;
    update_proj(N->in, B, (deepr_mask & 1) != 0, l1, lr, b1, b2, eps, c1, c2);
    update_proj(N->rec, B, (deepr_mask & 2) != 0, l1, lr, b1, b2, eps, c1, c2);
    int64_t nout = (int64_t)N->n_out * N->n_rec;
    for (int64_t q = 0; q < nout; ++q) {
        adam(&N->Wout[q], &N->Mout[q], &N->Vout[q], N->Gout[q] / (double)B, lr, b1, b2, eps, c1, c2);
        N->Gout[q] = 0.0;
        if (N->Goutabs) N->Goutabs[q] = 0.0;
    }
    for (int32_t q = 0; q < N->n_out; ++q) {
        adam(&N->bout[q], &N->Mb[q], &N->Vb[q], N->Gb[q] / (double)B, lr, b1, b2, eps, c1, c2);
        N->Gb[q] = 0.0;
        if (N->Gbabs) N->Gbabs[q] = 0.0;
    }
}
