/*
 * Oracle topographic-map simulation step (test infrastructure only).
 *
 * The model of the topographic-map section, Tab. A-F, on one feed-forward
 * ragged projection from an L x L Poisson source sheet to an L x L sheet of
 * conductance-based LIF neurons, with time step h (Tab. H):
 *
 *   neuron (Tab. B, D)   tau_m dV/dt = V_rest - V + (g / g_leak)(E_exc - V),
 *                        g_leak = C_m / tau_m; spike when V >= V_theta, then V
 *                        is held at V_reset for tau_ref; tau_s dg/dt = -g plus
 *                        g_syn for every presynaptic spike, delivered t_d later
 *   input (Tab. B, E)    Poisson trains of rate f_base + f_peak exp(-d^2/2 s^2)
 *                        around a stimulus position redrawn every t_stim
 *   STDP (Tab. B, F)     all-to-all additive pairing: a postsynaptic spike adds
 *                        A_+ x_pre, a presynaptic spike subtracts A_- y_post,
 *                        dx/dt = -x/tau_+ + pre spikes, dy/dt = -y/tau_- + post
 *                        spikes, g_syn clipped to [0, g_max]
 *
 * Readings where the tables leave the discrete-time form open:
 *   - exponential Euler with the synaptic current g (E_exc - V) held over the
 *     step: V <- V_rest + R I + (V - V_rest - R I) exp(-h/tau_m), R = tau_m/C_m;
 *   - the delay t_d equals h: spikes the source draws at step t are delivered
 *     at step t+1, and their STDP and trace effects happen at delivery;
 *   - one step: decay x and y by exp(-h/tau); deliver (add the synapse's
 *     conductance to g of its target, then depress it by A_- y_target; the
 *     delivering neuron's x += 1); integrate every neuron and emit spikes; g
 *     decays by exp(-h/tau_s); potentiate every synapse onto a neuron that
 *     spiked by A_+ x_source, then y += 1 for it; draw this step's input.
 *     A pair at lag k steps then changes the weight by exactly A_+ exp(-k h /
 *     tau_+) (pre first, k >= 0) or -A_- exp(-k h / tau_-) (post first, k >= 1);
 *   - refractoriness: the tau_ref/h steps after a spike hold V = V_reset and
 *     emit nothing; g still receives deliveries and decays;
 *   - the stimulus position is an integer cell, so every rate depends on an
 *     integer squared torus distance: "blob" (the paper's) uses the distance to
 *     a centre drawn uniformly each epoch of t_stim; "bar" uses the distance
 *     along one axis to a line whose orientation (rows or columns) and position
 *     are drawn each epoch;
 *   - epoch e's draws: x = below(u32(STIM; e, 0), L), y = below(u32(STIM; e, 1),
 *     L), orientation = u32(STIM; e, 2) & 1; input channel i spikes at step t
 *     when its uniform 32-bit draw is below floor(f h 2^32).  The tables leave
 *     the random stream open; one generator call serves eight channels: the
 *     draw of channel i is output word (i mod 8)/2 of Philox4x64-10 under key
 *     (seed, TP_INPUT) at counter (t, floor(i/8), 0, 0), its upper half for even
 *     i and its lower half for odd i;
 *   - scaled maps (L = s L_0): the correlated input is replicated in each
 *     L_0 x L_0 square, so the s^2 stimulus locations sit at the same offset in
 *     every square: the position is drawn in [0, L_0) and a channel's distance
 *     is measured on the L_0 torus from its coordinates modulo L_0, which is its
 *     distance to the nearest of the s^2 replicated locations (stim_tile = L_0;
 *     0 means the whole sheet is one square).
 *
 * Lateral projection (Tab. A "feed-forward and lateral connections"): target ->
 * target rows with their own conductances, STDP and rewiring, read as a
 * second projection of the same kind onto the same targets:
 *   - a target spike of step t is delivered at t+1, as source spikes are: it
 *     adds the lateral weight to g of each lateral target and depresses that
 *     weight by A_- y_target; the spiking neuron's lateral pre trace xl += 1;
 *   - xl decays with tau_+ like x; potentiation of a lateral synapse onto a
 *     target that spiked adds A_+ xl_pre; the post trace y is shared;
 *   - within a step the feed-forward deliveries come first, then the lateral
 *     ones, both before the neuron update (the conductance sum is exact in the
 *     GPU's fixed point, so the order only moves the oracle's last bits);
 *   - autapses are allowed: at distance zero the lateral formation probability
 *     is p_form-lat, and the map's connection-change counts at zero distance
 *     are autapses.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

uint32_t orc_topo_input_u32(uint64_t seed, uint64_t t, int32_t i)
{
    uint64_t ctr[4] = {t, (uint64_t)(i / 8), 0, 0}, o[4];
    orc_philox4x64_10(seed, (uint64_t)ORC_TAG_TP_INPUT, ctr, o);
    const uint64_t w = o[(i % 8) / 2];
    return (i % 2) ? (uint32_t)w : (uint32_t)(w >> 32);
}

static int32_t axis_d(int32_t L, int32_t a, int32_t b)
{
    int32_t d = abs(a - b);
    return d < L - d ? d : L - d;
}

/* Side of the square the stimulus is replicated over. */
static int32_t stim_side(const orc_topo_model *M)
{
    return M->stim_tile > 0 ? M->stim_tile : M->L;
}

void orc_topo_stimulus(uint64_t seed, const orc_topo_model *M, uint64_t step, int32_t *cx,
                       int32_t *cy, int32_t *orient)
{
    const uint64_t e = step / (uint64_t)M->stim_steps;
    const uint32_t Ls = (uint32_t)stim_side(M);
    *cx = (int32_t)orc_below(orc_u32(seed, ORC_TAG_STIM, 0, e, 0, 0, 0), Ls);
    *cy = (int32_t)orc_below(orc_u32(seed, ORC_TAG_STIM, 0, e, 1, 0, 0), Ls);
    *orient = (int32_t)(orc_u32(seed, ORC_TAG_STIM, 0, e, 2, 0, 0) & 1u);
}

int32_t orc_topo_stim_d2(const orc_topo_model *M, int32_t i, int32_t cx, int32_t cy, int32_t orient)
{
    const int32_t Ls = stim_side(M);
    const int32_t dx = axis_d(Ls, (i % M->L) % Ls, cx), dy = axis_d(Ls, (i / M->L) % Ls, cy);
    if (M->stim_kind == ORC_STIM_BAR) return orient ? dy * dy : dx * dx;
    return dx * dx + dy * dy;
}

double orc_topo_rate(const orc_topo_model *M, int32_t d2)
{
    return M->f_base + M->f_peak * exp(-(double)d2 / (2.0 * M->sigma_stim * M->sigma_stim));
}

/* Deliver the spikes flagged in z through the rows of Q: conductance, then
 * depression by A_- y_target, then the presynaptic trace. */
static void deliver(const orc_topo_model *M, orc_proj *Q, const uint8_t *z, double *pre_trace,
                    orc_topo_state *S)
{
    for (int32_t i = 0; i < Q->n_pre; ++i) {
        if (!z[i]) continue;
        for (int32_t s = 0; s < Q->len[i]; ++s) {
            const int64_t k = (int64_t)i * Q->cap + s;
            const int32_t j = Q->ind[k];
            S->g[j] += Q->w[k];
            if (M->stdp) {
                const double w = Q->w[k] - M->A_minus * S->y[j];
                Q->w[k] = w > 0.0 ? w : 0.0;
            }
        }
        pre_trace[i] += 1.0;
    }
}

/* Potentiate every synapse of Q onto a target that spiked by A_+ times its
 * presynaptic trace, capped at g_max. */
static void potentiate(const orc_topo_model *M, orc_proj *Q, const double *pre_trace,
                       const orc_topo_state *S)
{
    for (int32_t i = 0; i < Q->n_pre; ++i)
        for (int32_t s = 0; s < Q->len[i]; ++s) {
            const int64_t k = (int64_t)i * Q->cap + s;
            if (!S->zout[Q->ind[k]]) continue;
            const double w = Q->w[k] + M->A_plus * pre_trace[i];
            Q->w[k] = w < M->g_max ? w : M->g_max;
        }
}

void orc_topo_sim_step(uint64_t seed, const orc_topo_model *M, orc_proj *P, orc_topo_state *S,
                       uint64_t t)
{
    orc_topo_sim_step_lat(seed, M, P, NULL, S, t);
}

void orc_topo_sim_step_lat(uint64_t seed, const orc_topo_model *M, orc_proj *P, orc_proj *PL,
                           orc_topo_state *S, uint64_t t)
{
    const int32_t N = M->L * M->L;
    const double dx_ = exp(-M->h / M->tau_plus), dy_ = exp(-M->h / M->tau_minus);
    const double em = exp(-M->h / M->tau_m), es = exp(-M->h / M->tau_s);
    const double R = M->tau_m / M->C_m;

    /* traces decay */
    for (int32_t i = 0; i < N; ++i) S->x[i] *= dx_;
    for (int32_t j = 0; j < N; ++j) S->y[j] *= dy_;
    if (PL)
        for (int32_t i = 0; i < N; ++i) S->xl[i] *= dx_;

    /* delivery of the spikes of the step before (delay one step), with
     * depression: the source's, then the targets' own through the lateral rows */
    deliver(M, P, S->zin, S->x, S);
    if (PL) deliver(M, PL, S->zout, S->xl, S);

    /* neurons: exponential Euler, threshold, reset, refractoriness */
    for (int32_t j = 0; j < N; ++j) {
        S->zout[j] = 0;
        if (S->ref[j] > 0) {
            S->ref[j] -= 1;
            S->V[j] = M->V_reset;
        } else {
            const double I = S->g[j] * (M->E_exc - S->V[j]);
            S->V[j] = M->V_rest + R * I + (S->V[j] - M->V_rest - R * I) * em;
            if (S->V[j] >= M->V_th) {
                S->zout[j] = 1;
                S->V[j] = M->V_reset;
                S->ref[j] = M->ref_steps;
                S->count[j] += 1;
            }
        }
        S->g[j] *= es;
    }

    /* potentiation of every synapse onto a neuron that spiked, then y */
    if (M->stdp) {
        potentiate(M, P, S->x, S);
        if (PL) potentiate(M, PL, S->xl, S);
    }
    for (int32_t j = 0; j < N; ++j) S->y[j] += S->zout[j];

    /* this step's input spikes, delivered next step */
    int32_t cx, cy, orient;
    orc_topo_stimulus(seed, M, t, &cx, &cy, &orient);
    for (int32_t i = 0; i < N; ++i) {
        const double p = orc_topo_rate(M, orc_topo_stim_d2(M, i, cx, cy, orient)) * M->h / 1000.0;
        const uint32_t u = orc_topo_input_u32(seed, t, i);
        S->zin[i] = (uint64_t)u < orc_threshold(p) ? 1 : 0;
    }
}

void orc_topo_run(uint64_t seed, const orc_topo_model *M, orc_proj *P, const orc_topo_params *tp,
                  orc_topo_state *S, uint64_t t0, uint64_t n_steps, uint32_t *bits, int32_t *stats)
{
    orc_topo_run_lat(seed, M, P, tp, NULL, NULL, S, t0, n_steps, bits, NULL, stats, NULL);
}

void orc_topo_run_lat(uint64_t seed, const orc_topo_model *M, orc_proj *P, const orc_topo_params *tp,
                      orc_proj *PL, const orc_topo_params *tpl, orc_topo_state *S, uint64_t t0,
                      uint64_t n_steps, uint32_t *bits, uint32_t *bits_l, int32_t *stats,
                      int32_t *stats_l)
{
    for (uint64_t t = t0; t < t0 + n_steps; ++t) {
        orc_topo_sim_step_lat(seed, M, P, PL, S, t);
        if (M->rewire_steps > 0 && (t + 1) % (uint64_t)M->rewire_steps == 0) {
            int32_t st[4];
            orc_topo_rewire(seed, P, tp, t + 1, bits, st);
            if (stats)
                for (int q = 0; q < 4; ++q) stats[q] += st[q];
            if (PL) {
                orc_topo_rewire(seed, PL, tpl, t + 1, bits_l, st);
                if (stats_l)
                    for (int q = 0; q < 4; ++q) stats_l[q] += st[q];
            }
        }
    }
}
