/*
 * Oracle e-prop classifier step (test infrastructure only).
 *
 * Follows the recurrent-classifier section of the paper:
 *   ALIF neuron   v_j <- alpha (v_j - z_j v_thr) + sum_i W_rec z_i + sum_i W_in x_i
 *                 a_j <- rho a_j + z_j,   z_j = H(v_j - (v_thr + beta a_j))
 *   LIF           beta = rho = 0
 *   readout       y_k <- alpha y_k + sum_j W_out[k][j] z_j + b_k
 *   surrogate     psi_j = (0.3 / v_thr) max(0, 1 - |v_j - (v_thr + beta a_j)| / v_thr)
 *   eligibility   (eq. eprop_elig_1/2, eprop_elig_lif)
 *                 e    = psi_j (zbar_i - beta eps_ji)       [LIF: e = psi_j zbar_i]
 *                 eps <- psi_j zbar_i + (rho - psi_j beta) eps_ji
 *                 ebar <- alpha ebar + e
 *   gradients     dW_ji += L_j ebar_ji,  L_j = sum_k W_out[k][j] (pi_k - pi*_k)
 *                 dW_out[k][j] += (pi_k - pi*_k) zbar_j,  db_k += (pi_k - pi*_k)
 * Readings where the printed equations are ambiguous:
 *   - zbar_i in the eligibility update is the filtered presynaptic activity of
 *     spikes up to the previous step (the spikes that shaped v_j this step);
 *     the parenthesis of eq. eprop_elig_2 is read as psi (zbar - beta eps).
 *   - low-pass filters are F <- alpha F + x (no (1 - alpha) factor), which
 *     makes the readout delta rule the exact gradient of the leaky readout.
 *   - the learning signal pairs pi computed from y after this step's spikes
 *     with ebar including this step's e, i.e. the loss is summed over steps.
 *   - z = 1 when v >= threshold; recurrent rows never contain autapses.
 * All sums over the batch are plain sums; the update divides by B.
 *
 * Loops over independent items (batch instances, rows, readout units) carry
 * OpenMP pragmas for the multi-core timing build; every value is computed by
 * the same operations in the same order in either build, so the two agree
 * bit for bit.  The parity build compiles without OpenMP.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void orc_eprop_spikes(const orc_net *N, uint8_t *z_out, double *margin_out)
{
    for (int32_t b = 0; b < N->batch; ++b)
        for (int32_t j = 0; j < N->n_rec; ++j) {
            int64_t q = (int64_t)b * N->n_rec + j;
            double A = N->v_thr + N->beta * N->a[q];
            z_out[q] = N->v[q] >= A ? 1 : 0;
            if (margin_out) margin_out[q] = N->v[q] - A;
        }
}

void orc_eprop_reset(orc_net *N)
{
    int64_t B = N->batch;
    memset(N->v, 0, sizeof(double) * B * N->n_rec);
    memset(N->a, 0, sizeof(double) * B * N->n_rec);
    memset(N->y, 0, sizeof(double) * B * N->n_out);
    memset(N->xbar, 0, sizeof(double) * B * N->n_in);
    memset(N->zbar, 0, sizeof(double) * B * N->n_rec);
    orc_proj *projs[2] = {N->in, N->rec};
    for (int p = 0; p < 2; ++p) {
        orc_proj *P = projs[p];
        int64_t n = (int64_t)P->n_pre * P->cap * B;
        if (P->eps) memset(P->eps, 0, sizeof(double) * n);
        if (P->ebar) memset(P->ebar, 0, sizeof(double) * n);
    }
}

/* Per-synapse eligibility update for one projection, presynaptic trace pre[B][n_pre]. */
static void eligibility(const orc_net *N, orc_proj *P, const double *pre)
{
    int32_t B = N->batch;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < P->n_pre; ++i)
        for (int32_t k = 0; k < P->len[i]; ++k) {
            int64_t s = (int64_t)i * P->cap + k;
            int32_t j = P->ind[s];
            for (int32_t b = 0; b < B; ++b) {
                double psi = N->psi[(int64_t)b * N->n_rec + j];
                double p = pre[(int64_t)b * P->n_pre + i];
                double e;
                if (N->alif) {
                    double eps = P->eps[s * B + b];
                    e = psi * (p - N->beta * eps);
                    P->eps[s * B + b] = psi * p + (N->rho - psi * N->beta) * eps;
                } else {
                    e = psi * p;
                }
                P->ebar[s * B + b] = N->alpha * P->ebar[s * B + b] + e;
            }
        }
}

/* dW_ji += sum_b L_j ebar_ji */
static void accumulate_grad(const orc_net *N, orc_proj *P)
{
    int32_t B = N->batch;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < P->n_pre; ++i)
        for (int32_t k = 0; k < P->len[i]; ++k) {
            int64_t s = (int64_t)i * P->cap + k;
            int32_t j = P->ind[s];
            double g = 0.0, ga = 0.0;
            for (int32_t b = 0; b < B; ++b) {
                double L = N->L[(int64_t)b * N->n_rec + j], eb = P->ebar[s * B + b];
                g += L * eb;
                if (N->Labs) ga += fabs(eb) * (2.0 * fabs(L) + N->Labs[(int64_t)b * N->n_rec + j]);
            }
            P->G[s] += g;
            if (P->Gabs) P->Gabs[s] += ga;
        }
}

void orc_eprop_step(orc_net *N, const int32_t *x_idx, const int32_t *x_off,
                    const int32_t *labels, const uint8_t *z_force, int32_t learn)
{
    const int32_t B = N->batch, NR = N->n_rec, NI = N->n_in, K = N->n_out;

    /* 1. spikes and surrogate derivative from the state at the start of the step */
#pragma omp parallel for schedule(static)
    for (int32_t b = 0; b < B; ++b)
        for (int32_t j = 0; j < NR; ++j) {
            int64_t q = (int64_t)b * NR + j;
            double A = N->v_thr + N->beta * N->a[q];
            N->z[q] = z_force ? z_force[q] : (N->v[q] >= A ? 1 : 0);
            double h = 1.0 - fabs(N->v[q] - A) / N->v_thr;
            N->psi[q] = (0.3 / N->v_thr) * (h > 0.0 ? h : 0.0);
        }

    /* 2. eligibility traces with the presynaptic traces of the previous step */
    if (learn) {
        eligibility(N, N->in, N->xbar);
        eligibility(N, N->rec, N->zbar);
    }

    /* 3.-7. per batch instance; the instances are independent */
#pragma omp parallel
    {
        double *I = (double *)calloc((size_t)NR, sizeof(double));
        uint8_t *x = (uint8_t *)calloc((size_t)NI, 1);
#pragma omp for schedule(static)
        for (int32_t b = 0; b < B; ++b) {
            const int32_t *xs = x_idx + x_off[b];
            int32_t nx = x_off[b + 1] - x_off[b];
            uint8_t *zb = N->z + (int64_t)b * NR;
            memset(I, 0, sizeof(double) * NR);
            memset(x, 0, (size_t)NI);
            /* 3. propagation through the ragged rows of spiking sources */
            for (int32_t q = 0; q < nx; ++q) {
                int32_t i = xs[q];
                x[i] = 1;
                for (int32_t k = 0; k < N->in->len[i]; ++k) {
                    int64_t s = (int64_t)i * N->in->cap + k;
                    I[N->in->ind[s]] += N->in->w[s];
                }
            }
            for (int32_t i = 0; i < NR; ++i) {
                if (!zb[i]) continue;
                for (int32_t k = 0; k < N->rec->len[i]; ++k) {
                    int64_t s = (int64_t)i * N->rec->cap + k;
                    I[N->rec->ind[s]] += N->rec->w[s];
                }
            }
            /* 4. neuron update with subtractive reset */
            for (int32_t j = 0; j < NR; ++j) {
                int64_t q = (int64_t)b * NR + j;
                N->v[q] = N->alpha * (N->v[q] - zb[j] * N->v_thr) + I[j];
                N->a[q] = N->rho * N->a[q] + zb[j];
            }
            /* 5. presynaptic traces */
            for (int32_t i = 0; i < NI; ++i)
                N->xbar[(int64_t)b * NI + i] = N->alpha_trace * N->xbar[(int64_t)b * NI + i] + x[i];
            for (int32_t j = 0; j < NR; ++j)
                N->zbar[(int64_t)b * NR + j] = N->alpha_trace * N->zbar[(int64_t)b * NR + j] + zb[j];
            /* 6. leaky readout, softmax, output error */
            double *yb = N->y + (int64_t)b * K;
            double ymax = -INFINITY;
            for (int32_t k = 0; k < K; ++k) {
                double s = 0.0;
                for (int32_t j = 0; j < NR; ++j) s += N->Wout[(int64_t)k * NR + j] * zb[j];
                yb[k] = N->alpha * yb[k] + s + N->bout[k];
                if (yb[k] > ymax) ymax = yb[k];
            }
            double den = 0.0;
            for (int32_t k = 0; k < K; ++k) den += exp(yb[k] - ymax);
            for (int32_t k = 0; k < K; ++k) {
                double pi = exp(yb[k] - ymax) / den;
                N->delta[(int64_t)b * K + k] = pi - (k == labels[b] ? 1.0 : 0.0);
            }
            /* 7. learning signal through B = W_out^T */
            for (int32_t j = 0; j < NR; ++j) {
                double l = 0.0, la = 0.0;
                for (int32_t k = 0; k < K; ++k) {
                    double d = N->delta[(int64_t)b * K + k], pi = d + (k == labels[b] ? 1.0 : 0.0);
                    l += N->Wout[(int64_t)k * NR + j] * d;
                    la += fabs(N->Wout[(int64_t)k * NR + j]) * (fabs(d) + pi);
                }
                N->L[(int64_t)b * NR + j] = l;
                if (N->Labs) N->Labs[(int64_t)b * NR + j] = la;
            }
        }
        free(I);
        free(x);
    }
    /* 8. readout delta rule, summed over the instances in their order */
    if (learn) {
#pragma omp parallel for schedule(static)
        for (int32_t k = 0; k < K; ++k) {
            for (int32_t b = 0; b < B; ++b) {
                double d = N->delta[(int64_t)b * K + k];
                double pi = d + (k == labels[b] ? 1.0 : 0.0);
                for (int32_t j = 0; j < NR; ++j) {
                    double zb_ = N->zbar[(int64_t)b * NR + j];
                    N->Gout[(int64_t)k * NR + j] += d * zb_;
                    if (N->Goutabs) N->Goutabs[(int64_t)k * NR + j] += fabs(zb_) * (2.0 * fabs(d) + pi);
                }
                N->Gb[k] += d;
                if (N->Gbabs) N->Gbabs[k] += fabs(d) + pi;
            }
        }
    }
    /* 9. recurrent and input weight gradients */
    if (learn) {
        accumulate_grad(N, N->in);
        accumulate_grad(N, N->rec);
    }
}
