/*
 * Reference CPU oracle for ragged-row spiking networks with e-prop, DEEP R and
 * topographic-map rewiring (Knight, Senk, Nowotny et al., "A flexible framework
 * for structural plasticity in GPU-accelerated sparse spiking neural networks").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a deliberately plain, slow,
 * single-threaded fp64 re-statement of the paper's method.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library, and never
 * includes anything from it.
 *
 * Conventions
 *   - Floating point state is double.  Weights handed in from a float32 device
 *     snapshot are widened exactly; decisions that the method takes on weights
 *     (sign mismatch, w < g_theta) are taken in float32, the precision the
 *     weights are stored in.
 *   - Ragged rows (paper, Sec. 2.1 and Fig. 1): len[n_pre], and for slot k of
 *     row i the flat index i*cap + k into ind / w / m / v / G.  Per-batch
 *     synapse traces are stored per slot: eps[(i*cap + k)*B + b].
 *   - Bitfields (paper, Sec. 2.1.2, Fig. 2 and Sec. 2.1.3, Fig. 3): one section
 *     of ceil(n_post/32) 32-bit words per presynaptic row; bit j%32 of word
 *     j/32 stands for target j.
 *   - Random draws: Philox4x64-10 (Salmon et al., SC'11), key = (seed,
 *     tag | proj<<8), counter = (c0, c1, c2, c3).  A 32-bit draw is the top
 *     half of output word 0; an integer below n is (u32*n)>>32; a Bernoulli
 *     trial with probability p succeeds when u32 < floor(p*2^32) (computed in
 *     double; p >= 1 always succeeds).
 */
#ifndef RAGSNN_ORACLE_H
#define RAGSNN_ORACLE_H
#include <stdint.h>

/* Random stream tags (key word 1 = tag | proj << 8). */
enum {
    ORC_TAG_CONN = 1,    /* connectivity Bernoulli trial, counter (0, i, j, 0) */
    ORC_TAG_WINIT = 2,   /* initial weight normal draw,   counter (0, i, j, 0) */
    ORC_TAG_SIGN = 3,    /* DEEP R sign bit,              counter (0, i, j, 0) */
    ORC_TAG_DR_ROW = 4,  /* DEEP R activation -> row,     counter (step, a, round, 0) */
    ORC_TAG_DR_TGT = 5,  /* DEEP R new target,            counter (step, r, k, try) */
    ORC_TAG_TP_ROW = 6,  /* topomap attempt -> row,       counter (step, a, 0, 0) */
    ORC_TAG_TP_TGT = 7,  /* topomap candidate target,     counter (step, r, q, try) */
    ORC_TAG_TP_ELIM = 8, /* topomap elimination draw,     counter (step, r, s, 0) */
    ORC_TAG_TP_FORM = 9, /* topomap formation draw,       counter (step, r, j, 0) */
    ORC_TAG_INPUT = 10,  /* Poisson input spike,          counter (step, b, i, 0) */
    ORC_TAG_STIM = 11,   /* topomap stimulus position,    counter (epoch, k, 0, 0) */
    ORC_TAG_TP_INPUT = 12, /* topomap source spikes,      counter (step, i/8, 0, 0), 8 per call */
    ORC_TAG_CUSTOM = 13  /* custom update draws,          counter (step, i, 0, 0) */
};

/* Draws per (row, activation) before the bounded fallback scan takes over. */
#define ORC_MAX_TRIES 64
/* Distribution rounds before the deterministic fallback assignment. */
#define ORC_MAX_ROUNDS 64

/* Threads of the multi-core timing build (1 in the parity build). */
int32_t orc_threads(void);

/* ---- counter-based generator --------------------------------------------- */
void orc_philox4x64_10(uint64_t key0, uint64_t key1, const uint64_t ctr[4], uint64_t out[4]);
uint32_t orc_u32(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1,
                 uint64_t c2, uint64_t c3);
uint32_t orc_below(uint32_t u, uint32_t n);
uint64_t orc_threshold(double p);
double orc_normal(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1,
                  uint64_t c2, uint64_t c3);

/* ---- Poisson input -------------------------------------------------------- */
/* Bernoulli threshold of one step of a Poisson train: floor(rate*dt*2^32). */
uint64_t orc_rate_threshold(double rate_hz, double dt_ms);
/* Input spikes of step `step` for every instance: channel i of instance b
 * fires when u32(INPUT; step, b, i, 0) < thr[i] (thr[b*n_in + i] with
 * per_instance).  Writes ascending channel lists, x_off[B+1] delimiting each
 * instance's list in x_idx (capacity B*n_in); returns the spike count. */
int64_t orc_poisson_input(uint64_t seed, uint64_t step, int32_t B, int32_t n_in,
                          const uint64_t *thr, int32_t per_instance,
                          int32_t *x_idx, int32_t *x_off);

/* ---- one ragged projection ----------------------------------------------- */
typedef struct orc_proj {
    int32_t n_pre, n_post, cap;
    int32_t recurrent; /* 1: targets may not equal the row index (no autapses) */
    int32_t proj_id;   /* random stream id */
    int32_t *len;      /* [n_pre] */
    int32_t *ind;      /* [n_pre*cap] */
    double *w, *m, *v, *G; /* [n_pre*cap]; m, v, G may be NULL when not trained */
    double *eps, *ebar;    /* [n_pre*cap*B]; eps NULL for LIF, both NULL untrained */
    uint32_t *conn, *sign; /* [n_pre*words] or NULL */
    int32_t words;         /* ceil(n_post/32) */
    /* Error-bound bookkeeping for tests, no part of the method (may be NULL):
     * Gabs[s] accumulates, beside G, the first-order error scale of its terms
     * L_j ebar_ji when L is known to r (|L| + Labs) and ebar to r |ebar|:
     * sum_b |ebar| (2 |L| + Labs), so that a test can bound G per element by
     * r (|G| + Gabs) despite cancellation.  Needs the net's Labs; cleared,
     * moved and zeroed together with G. */
    double *Gabs;
} orc_proj;

/* ---- e-prop classifier (input -> LIF/ALIF recurrent -> leaky readout) ---- */
typedef struct orc_net {
    int32_t n_in, n_rec, n_out, batch;
    int32_t alif;           /* 0: LIF (beta = rho = 0) */
    double alpha, rho, v_thr, beta;
    double alpha_trace;     /* decay of the presynaptic traces xbar, zbar: alpha, or
                               alpha as a float implementation stores it */
    orc_proj *in, *rec;
    double *v, *a;          /* [B][n_rec] */
    double *y;              /* [B][n_out] */
    double *xbar;           /* [B][n_in]   input spike trace  */
    double *zbar;           /* [B][n_rec]  recurrent spike trace */
    double *Wout, *bout;    /* [n_out][n_rec], [n_out] */
    double *Gout, *Gb;      /* [n_out][n_rec], [n_out] accumulated over b and t */
    double *Mout, *Vout, *Mb, *Vb; /* Adam moments of the readout */
    /* per-step outputs, overwritten by every step */
    double *psi, *L;        /* [B][n_rec] */
    uint8_t *z;             /* [B][n_rec] spikes emitted this step */
    double *delta;          /* [B][n_out] pi - onehot(label) */
    /* Error-bound bookkeeping for tests (each may be NULL): first-order
     * error scales of the sums with cancellation when delta_k = pi_k -
     * [k = label] is known to r (|delta_k| + pi_k) (pi rounds relative to
     * itself) and zbar to r |zbar|.  Labs[B][n_rec] = sum_k |W_out[k][j]|
     * (|delta_k| + pi_k) of the last step; beside Gout and Gb, Goutabs
     * accumulates |zbar_j| (2 |delta_k| + pi_k) and Gbabs |delta_k| + pi_k. */
    double *Labs, *Goutabs, *Gbabs;
} orc_net;

/* Build: fixed-probability rows (paper, classifier model section).  Row i
 * connects to j (ascending) when the CONN draw passes p; j == i is skipped for
 * recurrent projections.  With ind == NULL only len[] is filled.  Weights are
 * sigma * N(0,1).  Returns the largest row length. */
int32_t orc_fixed_prob_rows(uint64_t seed, orc_proj *P, double p, double sigma);
/* Build: pairwise-Bernoulli rows with Gaussian distance-dependent probability
 * on an L x L torus (paper, topographic-map model, Tab. B / Tab. G). */
int32_t orc_gauss_rows(uint64_t seed, orc_proj *P, int32_t L, double p_form, double sigma,
                       double g_init);
/* Dense readout init, W[k][j] = sigma * N(0,1). */
void orc_dense_init(uint64_t seed, int32_t proj_id, int32_t rows, int32_t cols, double sigma,
                    double *W);
/* DEEP R bitfield init (paper, Sec. 2.1.2, Fig. 2A). */
void orc_deepr_init_bits(uint64_t seed, orc_proj *P);

/* One timestep of the e-prop network for every batch instance.  x_off has B+1
 * entries delimiting each instance's input spike list in x_idx.  When z_force
 * is not NULL it replaces the spikes the oracle would emit ([B][n_rec]).
 * learn = 0 skips eligibility and gradients. */
void orc_eprop_step(orc_net *N, const int32_t *x_idx, const int32_t *x_off,
                    const int32_t *labels, const uint8_t *z_force, int32_t learn);
/* Spikes the network would emit from its current state, without stepping. */
void orc_eprop_spikes(const orc_net *N, uint8_t *z_out, double *margin_out);
/* Reset neuron, readout and trace state at a sample boundary. */
void orc_eprop_reset(orc_net *N);

/* Parameter update: gradient averaged over the batch, L1 term for DEEP R
 * projections, then Adam (Kingma & Ba) with update counter k >= 1. */
void orc_adam_update(orc_net *N, int32_t k, double lr, double b1, double b2, double eps,
                     double l1, int32_t deepr_mask);

/* DEEP R rewiring of one projection (paper, Sec. 2.1.2): elimination of
 * sign-mismatched synapses, then formation of the same number elsewhere.
 * stats[0] = eliminated, stats[1] = formed. */
void orc_deepr_rewire(uint64_t seed, orc_proj *P, int32_t batch, uint64_t step,
                      int32_t *dormant, int32_t *stats);

/* Custom connectivity updates: the paper's worked examples (Sec. 2.1).
 * add_diagonal adds synapse i -> i (weight 1) to every row i < n_post with
 * room (and, with a bitfield, not yet connected); returns the count.
 * remove_random's host part draws post_ind[i] = below(u32(CUSTOM; step, i, 0,
 * 0), n_post); its row part removes each row's first synapse (slot order)
 * onto post_ind[i] by moving the row's last synapse into its slot; returns
 * the count removed. */
int32_t orc_add_diagonal(orc_proj *P, int32_t batch);
void orc_remove_random_targets(uint64_t seed, const orc_proj *P, uint64_t step, uint32_t *post_ind);
int32_t orc_remove_targets(orc_proj *P, int32_t batch, const uint32_t *post_ind);

/* Topographic-map rewiring (paper, Sec. 2.1.3, Fig. 3, Tab. B and G). */
typedef struct orc_topo_params {
    int32_t L;             /* sheet side; pre and post sheets are L x L */
    int32_t n_attempts;
    double p_form, sigma_form, g_theta, p_elim_dep, p_elim_pot, g_new;
} orc_topo_params;
/* Draw source; the default uses Philox, tests may script the outcomes. */
typedef struct orc_topo_draws {
    uint32_t (*attempt_row)(void *ctx, int32_t a);
    uint32_t (*target)(void *ctx, int32_t r, int32_t q, int32_t try_);
    uint32_t (*elim_u32)(void *ctx, int32_t r, int32_t s);
    uint32_t (*form_u32)(void *ctx, int32_t r, int32_t j);
    void *ctx;
} orc_topo_draws;
/* stats[0] = eliminated, [1] = formed, [2] = blocked (row full), [3] = attempts.
 * bits is the attempt bitfield ([n_pre*words]) and must be all zero on entry;
 * it is all zero again on return. */
void orc_topo_rewire_with(orc_proj *P, const orc_topo_params *tp, const orc_topo_draws *d,
                          uint32_t *bits, int32_t *stats);
void orc_topo_rewire(uint64_t seed, orc_proj *P, const orc_topo_params *tp, uint64_t step,
                     uint32_t *bits, int32_t *stats);
/* Squared torus distance between node i of one sheet and node j of the other. */
int32_t orc_torus_d2(int32_t L, int32_t i, int32_t j);

/* Topographic-map simulation (paper, topographic-map model, Tab. A-F, H). */
enum { ORC_STIM_BLOB = 0, ORC_STIM_BAR = 1 };
typedef struct orc_topo_model {
    int32_t L;
    double h;                                  /* time step, ms */
    double C_m, tau_m, V_rest, E_exc, V_th, V_reset, tau_s;   /* nF, ms, mV, ms */
    int32_t ref_steps;                         /* tau_ref / h */
    double f_base, f_peak, sigma_stim;         /* Hz, Hz, cells */
    int32_t stim_steps, stim_kind;             /* t_stim / h; ORC_STIM_* */
    int32_t stdp;                              /* 0: weights fixed */
    double g_max, A_plus, A_minus, tau_plus, tau_minus;      /* uS, uS, uS, ms, ms */
    int32_t rewire_steps;                      /* t_rewiring / h; 0: no rewiring */
    int32_t stim_tile;                         /* side L_0 of the replicated stimulus square; 0: L */
} orc_topo_model;
/* State of both sheets, L*L entries each. */
typedef struct orc_topo_state {
    double *V, *g, *y;   /* target sheet: membrane (mV), conductance (uS), post trace */
    int32_t *ref;        /* remaining refractory steps */
    int32_t *count;      /* spikes emitted so far */
    uint8_t *zout;       /* spikes of the last step */
    double *x;           /* source sheet: pre trace */
    uint8_t *zin;        /* spikes drawn last step, delivered next step */
    double *xl;          /* target sheet: lateral pre trace (used with a lateral projection) */
} orc_topo_state;
/* Uniform 32-bit draw of source channel i at step t (eight channels per
 * generator call: word (i%8)/2, upper half for even i). */
uint32_t orc_topo_input_u32(uint64_t seed, uint64_t t, int32_t i);
/* Stimulus position of the epoch containing `step`. */
void orc_topo_stimulus(uint64_t seed, const orc_topo_model *M, uint64_t step, int32_t *cx,
                       int32_t *cy, int32_t *orient);
/* Squared distance of source node i from the stimulus (blob: point, bar: line). */
int32_t orc_topo_stim_d2(const orc_topo_model *M, int32_t i, int32_t cx, int32_t cy, int32_t orient);
/* Firing rate (Hz) at squared stimulus distance d2. */
double orc_topo_rate(const orc_topo_model *M, int32_t d2);
/* One step t of the model (weights change only with stdp). */
void orc_topo_sim_step(uint64_t seed, const orc_topo_model *M, orc_proj *P, orc_topo_state *S,
                       uint64_t t);
/* One step with a lateral projection PL (target -> target rows; NULL: none). */
void orc_topo_sim_step_lat(uint64_t seed, const orc_topo_model *M, orc_proj *P, orc_proj *PL,
                           orc_topo_state *S, uint64_t t);
/* Steps t0 .. t0+n-1; after step t with (t+1) % rewire_steps == 0 a topomap
 * rewire keyed by t+1.  stats (may be NULL) accumulates the rewire stats. */
void orc_topo_run(uint64_t seed, const orc_topo_model *M, orc_proj *P, const orc_topo_params *tp,
                  orc_topo_state *S, uint64_t t0, uint64_t n_steps, uint32_t *bits, int32_t *stats);
/* The same with a lateral projection, rewired after the feed-forward one at
 * the same steps with its own parameters (its draws keyed by its proj_id). */
void orc_topo_run_lat(uint64_t seed, const orc_topo_model *M, orc_proj *P, const orc_topo_params *tp,
                      orc_proj *PL, const orc_topo_params *tpl, orc_topo_state *S, uint64_t t0,
                      uint64_t n_steps, uint32_t *bits, uint32_t *bits_l, int32_t *stats,
                      int32_t *stats_l);

#endif
