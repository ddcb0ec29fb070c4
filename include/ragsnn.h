/*
 * ragsnn -- MI355X (gfx950) engine for sparse spiking networks stored as ragged
 * rows, trained with e-prop and rewired with DEEP R, plus topographic-map
 * rewiring.  Method: Knight, Senk, Nowotny et al., "A flexible framework for
 * structural plasticity in GPU-accelerated sparse spiking neural networks"
 * (arXiv 2510.19764).
 *
 * Conventions for every call
 *   - Return value: RS_OK (0) or a negative rs_status.  Arguments are validated
 *     before anything is enqueued, so a call that fails with RS_EINVAL,
 *     RS_ECAPACITY or RS_ESTATE leaves the object unchanged.  RS_EDEVICE reports
 *     a HIP runtime error; it is sticky: every later call on that object
 *     returns RS_EDEVICE without enqueuing work (destroy still releases it).
 *     rs_last_error() describes the most recent failure of the calling thread.
 *   - Ownership: the library allocates and owns all device state of an object
 *     (released by its destroy call).  Buffers passed in belong to the caller;
 *     "device" pointers must stay valid for as long as the call's work may run
 *     on the object's stream, "host" pointers only for the duration of the call.
 *   - Streams: every object is bound to the HIP stream given at creation
 *     (NULL = the default stream).  Calls order their work after earlier work
 *     on it, and later work on it after theirs, and return without waiting,
 *     except where a call is documented as synchronising.
 *   - Threads: an object must not be used by two threads at once.
 *   - Randomness: every random decision is a Philox4x64-10 draw keyed by
 *     (seed, stream tag, projection) with a counter of (step, row, slot/target,
 *     retry), so results depend only on the seed and the call sequence.
 */
#ifndef RAGSNN_H
#define RAGSNN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rs_status;
#define RS_OK 0
#define RS_EINVAL (-1)     /* invalid argument, size or shape */
#define RS_ENOMEM (-2)     /* device allocation failed */
#define RS_ECAPACITY (-3)  /* caller buffer too small */
#define RS_ESTATE (-4)     /* call not valid in the object's current state */
#define RS_EDEVICE (-5)    /* HIP runtime error */

/* Message describing the last failed call on this thread ("" if none). */
const char* rs_last_error(void);

/* Device allocator a caller may hand to rs_create (for example one bound to
 * a framework's caching allocator): returns `bytes` of device memory on the
 * current device, or NULL; the free function releases such a block.  `user`
 * is passed through. */
typedef void* (*rs_alloc_fn)(size_t bytes, void* user);
typedef void (*rs_free_fn)(void* ptr, void* user);

/* Counts returned by a rewiring call. */
typedef struct rs_rewire_stats {
  int64_t eliminated;  /* synapses removed */
  int64_t formed;      /* synapses added */
  int64_t blocked;     /* topomap: formations skipped because the row was full;
                          DEEP R: activations for which no row had room (0 while
                          the rows' capacity exceeds the synapse count) */
  int64_t attempts;    /* topomap: rewiring attempts; DEEP R: activations
                          distributed over the rows (the dormant total D less
                          `blocked`) */
} rs_rewire_stats;

/* ==========================================================================
 * e-prop classifier: Poisson/raster input -> recurrent LIF or ALIF -> leaky
 * readout (paper, "Recurrent classifier" section), input and recurrent weights
 * stored as ragged rows (Sec. 2.1, Fig. 1) with DEEP R rewiring (Sec. 2.1.2).
 * ========================================================================== */
typedef struct rs_eprop rs_eprop;

typedef struct rs_eprop_params {
  uint32_t n_in;        /* input channels, 1..8192 */
  uint32_t n_rec;       /* recurrent neurons, 1..8192 */
  uint32_t n_out;       /* readout units, 1..256 */
  uint32_t batch;       /* batch instances simulated together, 1..65536 */
  int32_t alif;         /* 1: ALIF neurons, 0: LIF (beta = rho = 0) */
  float dt_ms, tau_mem_ms, tau_adapt_ms, v_thr, beta;
  float p_in, p_rec;    /* fixed connection probabilities */
  float sigma_in, sigma_rec, sigma_out;  /* initial weight standard deviations */
  uint32_t cap_in, cap_rec;  /* row capacities; 0 = twice the longest initial row */
  uint32_t deepr_mask;  /* bit 0: rewire the input projection, bit 1: recurrent */
  float l1;             /* DEEP R L1 strength added to the batch-mean gradient */
  float lr, adam_b1, adam_b2, adam_eps;
  uint32_t update_interval;  /* steps between automatic update + rewire (0 = never) */
  uint32_t sample_steps;     /* steps per presented sample; state resets after each */
  uint64_t seed;
  uint32_t trace_block;      /* steps whose eligibility updates the library applies
                                together, 1..32; 0 = 20, or update_interval when
                                batch % 4 != 0 and update_interval <= 32.  Neuron
                                state, traces and eps/ebar do not depend on it, the
                                gradient only by float rounding of its sum */
  uint32_t reserved;         /* must be 0 */
} rs_eprop_params;

/* Step flags */
#define RS_LEARN 1u        /* eligibility traces and gradient accumulation */
#define RS_AUTO_UPDATE 2u  /* update + DEEP R rewire whenever step % update_interval == 0 */
#define RS_AUTO_RESET 4u   /* reset neuron/trace state whenever step % sample_steps == 0 */

/* Create and build a network on `hip_device` (the caller's current device).
 * Builds the fixed-probability rows (weights sigma*N(0,1)), the dense readout
 * (bias 0) and, for projections in deepr_mask, the DEEP R connectivity and
 * sign bitfields (Sec. 2.1.2: signs of all potential synapses random, then
 * matched to the initial weights of existing ones).  Synchronises the stream.
 * `hip_stream` is a hipStream_t or NULL.  Networks with more than 2^21 expected
 * synapse-instances (p * n_pre * n_post summed over projections, times batch)
 * also own two internal streams, so that a block's forward pass overlaps the
 * previous block's eligibility work; every call still orders its work after
 * earlier work on `hip_stream` and the stream after its own.  Smaller networks
 * run every kernel on `hip_stream`.  Errors: RS_EINVAL (bad parameters, or a
 * network whose per-instance neuron state does not fit one workgroup's LDS:
 * about 16 * n_rec + 4.25 * n_in bytes must stay within 149 KB), RS_ENOMEM,
 * RS_EDEVICE.  *out is NULL on failure. */
rs_status rs_eprop_create(const rs_eprop_params* params, void* hip_stream, rs_eprop** out);

/* Attach the input of one sample batch: a compressed raster of
 * params->sample_steps steps.  Device pointers: off int32[sample_steps*batch+1],
 * idx int32[n_idx] with the channels of instance b at step t in
 * idx[off[t*batch+b] .. off[t*batch+b+1]), labels int32[batch] in [0, n_out).
 * Step t of the simulation reads raster step t % sample_steps.  The library
 * keeps the pointers (no copy, no host round trip).  Any content is memory
 * safe: offsets are clamped to [0, n_idx], channels outside [0, n_in) are
 * ignored and a label outside [0, n_out) gives an all-zero target.
 * Errors: RS_EINVAL (NULL pointer). */
rs_status rs_eprop_set_input(rs_eprop* net, const int32_t* off_dev, const int32_t* idx_dev, size_t n_idx,
                             const int32_t* labels_dev);

/* Attach a Poisson input source instead of a raster (the topographic-map
 * model's input layer, Tab. A and B, and Poisson input neurons in general):
 * in every step each input channel fires with probability rate * dt, drawn on
 * the counter-based generator.  Channel i of instance b fires at step t (the
 * object's step count, so successive samples draw fresh spikes) when the
 * 32-bit draw of stream INPUT (tag 10, proj 0) at counter (t, b, i, 0) is
 * below floor(p * 2^32), p = rate_hz * dt_ms / 1000 computed in double (p <= 0:
 * never, p >= 1: every step).  rate_hz is a host array, copied, of n_in
 * entries (one table for every instance) or batch * n_in entries ([b][i]);
 * labels_dev int32[batch] as for rs_eprop_set_input, kept by pointer.
 * Synchronises the stream.  A later rs_eprop_set_input returns to a raster.
 * Errors: RS_EINVAL (NULL pointer, n_rates neither n_in nor batch * n_in, a
 * NaN rate, trace_block * batch * n_in above 2^31), RS_ENOMEM. */
rs_status rs_eprop_set_input_poisson(rs_eprop* net, const double* rate_hz, size_t n_rates,
                                     const int32_t* labels_dev);

/* Advance n_steps timesteps.  Each step: spikes and surrogate derivatives from
 * the current state, eligibility traces (eq. eprop_elig_1/2 or eprop_elig_lif),
 * propagation of input and recurrent spikes through the ragged rows, neuron
 * update with subtractive reset, presynaptic traces, leaky readout, softmax
 * error and learning signal, and gradient accumulation (RS_LEARN).  With
 * RS_AUTO_UPDATE, rs_eprop_update and DEEP R rewiring of the deepr_mask
 * projections follow every update_interval-th step; with RS_AUTO_RESET the
 * state resets after every sample_steps-th step.  Errors: RS_ESTATE (no input
 * attached). */
rs_status rs_eprop_step(rs_eprop* net, uint32_t n_steps, uint32_t flags);

/* Parameter update: gradient / batch, + l1 * (sign of the potential
 * connection) for DEEP R projections (Sec. 2.1.2, L1 regularisation), then one
 * Adam step (update counter += 1) for input, recurrent and readout weights and
 * readout biases; gradients are cleared. */
rs_status rs_eprop_update(rs_eprop* net);

/* DEEP R rewiring of projection `proj` (0 = input, 1 = recurrent), Sec. 2.1.2:
 * eliminate synapses whose weight sign differs from their sign bit, then form
 * the same number at random free targets (weight and all synapse state zero).
 * Random counter step = the object's current step count.  With stats != NULL
 * the call synchronises and fills it.  Errors: RS_EINVAL (proj not in
 * deepr_mask). */
rs_status rs_eprop_rewire(rs_eprop* net, uint32_t proj, rs_rewire_stats* stats);

/* Zero neuron, readout and eligibility-trace state (sample boundary). */
rs_status rs_eprop_reset(rs_eprop* net);

/* Variable identifiers for rs_eprop_get / rs_eprop_set.  Membrane, adaptation
 * and readout state is double (it is small, and its rounding would otherwise
 * drift the surrogate derivative); the presynaptic traces are float, updated
 * as F <- fma(alpha, F, spike) so that the e-prop kernels can rebuild every
 * step's value exactly from a block's start value and spike bits; synapse
 * state is float.  Network variables (element type, layout): */
#define RS_V 0x01      /* double[batch][n_rec]  membrane voltage */
#define RS_A 0x02      /* double[batch][n_rec]  adaptation */
#define RS_Y 0x03      /* double[batch][n_out]  readout */
#define RS_XBAR 0x04   /* float[batch][n_in]    filtered input spikes */
#define RS_ZBAR 0x05   /* float[batch][n_rec]   filtered recurrent spikes */
#define RS_PSI 0x06    /* float[n_rec][batch]   surrogate derivative of the last step */
#define RS_LSIG 0x07   /* float[n_rec][batch]   learning signal of the last step */
#define RS_DELTA 0x08  /* float[n_out][batch]   softmax - one-hot of the last step */
#define RS_Z 0x09      /* uint8[batch][n_rec]   spikes emitted by the last step */
#define RS_WOUT 0x0A   /* float[n_out][n_rec] */
#define RS_BOUT 0x0B   /* float[n_out] */
#define RS_GOUT 0x0C   /* float[n_out][n_rec]   accumulated readout gradient */
#define RS_GB 0x0D     /* float[n_out] */
#define RS_MOUT 0x0E   /* float[n_out][n_rec]   Adam moments */
#define RS_VOUT 0x0F
#define RS_MB 0x10     /* float[n_out] */
#define RS_VB 0x11
#define RS_ZCOUNT 0x12 /* uint32[batch][n_rec]  spikes per neuron since creation or the
                          last rs_eprop_set of this variable */
#define RS_ZBITS 0x13  /* uint32[n_rec][batch]  spike raster of the last block of steps run
                          (rs_eprop_info.last_block steps, the end of the last step call):
                          bit t = the block's t-th step; read-only */
/* Projection variables: RS_PROJ(p, field), p = 0 input, 1 recurrent;
 * cap = row capacity (rs_eprop_info), words = ceil(n_post/32). */
#define RS_PROJ(p, f) (0x100 * ((p) + 1) + (f))
#define RS_P_LEN 0x01     /* int32[n_pre] row lengths */
#define RS_P_IND 0x02     /* int32[n_pre][cap] postsynaptic indices */
#define RS_P_W 0x03       /* float[n_pre][cap] weights */
#define RS_P_M 0x04       /* float[n_pre][cap] Adam first moment */
#define RS_P_V 0x05       /* float[n_pre][cap] Adam second moment */
#define RS_P_G 0x06       /* float[n_pre][cap] accumulated gradient */
#define RS_P_EPS 0x07     /* float[n_pre][cap][batch] ALIF eligibility vector */
#define RS_P_EBAR 0x08    /* float[n_pre][cap][batch] filtered eligibility trace */
#define RS_P_CONN 0x09    /* uint32[n_pre][words] DEEP R connectivity bits */
#define RS_P_SIGN 0x0A    /* uint32[n_pre][words] DEEP R sign bits (1 = negative) */
#define RS_P_DORMANT 0x0B /* int32[n_pre] eliminated per row by the last rewire */

/* Copy a variable to host memory (`bytes` must equal its full size).
 * Synchronises the stream.  Errors: RS_EINVAL (unknown variable),
 * RS_ECAPACITY (bytes differs from the size). */
rs_status rs_eprop_get(rs_eprop* net, int32_t var, void* host, size_t bytes);
/* Overwrite a variable from host memory (snapshot restore).  Slots beyond a
 * row's length are ignored by every kernel.  Synchronises the stream. */
rs_status rs_eprop_set(rs_eprop* net, int32_t var, const void* host, size_t bytes);

typedef struct rs_eprop_info {
  uint32_t cap_in, cap_rec;       /* row capacities */
  uint32_t words_in, words_rec;   /* bitfield words per row */
  uint64_t step;                  /* timesteps done */
  uint32_t adam_step;             /* Adam updates done */
  uint32_t last_block;            /* steps in the block RS_ZBITS covers */
  uint64_t synaptic_events;       /* spikes x row lengths propagated so far */
  uint64_t spikes;                /* recurrent spikes emitted so far */
  uint64_t device_bytes;          /* device memory held */
  uint64_t eliminated, formed;    /* DEEP R synapses removed / created so far, both projections */
  uint32_t trace_block;           /* steps per eligibility block (trace_block, or the default chosen) */
  uint32_t first_block;           /* steps of an update interval's first block under RS_AUTO_UPDATE
                                     (trace_block when it was given) */
} rs_eprop_info;
/* Synchronises the stream. */
rs_status rs_eprop_info_get(rs_eprop* net, rs_eprop_info* out);

/* Per-phase device timers (the paper's kernel timers, Sec. 2.1): HIP events
 * bracket every kernel launch of the phases selected by `phase_mask` (bit p
 * for phase p; 0 switches timing off).  Phases: 0 forward (neurons,
 * propagation, readout), 1 e-prop eligibility and gradients, 2 update,
 * 3 rewiring, 4 state reset. */
#define RS_NUM_PHASES 5
rs_status rs_eprop_timing(rs_eprop* net, int32_t phase_mask);
/* Synchronises; ms[p] = total milliseconds and count[p] = launches since the
 * last call (both arrays of RS_NUM_PHASES), then clears the totals. */
rs_status rs_eprop_phase_times(rs_eprop* net, double* ms, uint64_t* count);

void rs_eprop_destroy(rs_eprop* net);

/* ==========================================================================
 * Batched networks: a set of e-prop classifiers of different sizes trained
 * together, in the manner of the paper's batching of model copies (several
 * instances of a model simulated in one kernel launch), here copies that
 * differ in size and connection density.  Every kernel of a block of steps
 * runs once for the whole set over a work list of (network, tile) entries;
 * one whole training sample (its blocks of steps, the Adam updates, the DEEP R
 * rewiring and the reset) is recorded once as a HIP graph and replayed.  Each
 * network computes exactly what an rs_eprop object with the same parameters
 * computes alone (bit for bit), whatever the schedule.
 * ========================================================================== */
typedef struct rs_multi rs_multi;

/* Create the set from params[0 .. n-1] (n in 1..4096), built as
 * rs_eprop_create builds each.  The networks may differ in n_rec, connection
 * probabilities, weight spreads, capacities, DEEP R mask, L1 strength,
 * learning rate and seed; they share n_in, n_out, batch, alif, dt and the time
 * constants, update_interval, sample_steps, trace_block and the Adam decay
 * rates.  The batch must not be a multiple of 4, and sample_steps a multiple
 * of update_interval.  Synchronises.  Errors: RS_EINVAL, RS_ENOMEM,
 * RS_EDEVICE. */
rs_status rs_multi_create(const rs_eprop_params* params, uint32_t n, void* hip_stream, rs_multi** out);
/* Input of network i, as rs_eprop_set_input / rs_eprop_set_input_poisson. */
rs_status rs_multi_set_input(rs_multi* m, uint32_t i, const int32_t* off_dev, const int32_t* idx_dev,
                             size_t n_idx, const int32_t* labels_dev);
rs_status rs_multi_set_input_poisson(rs_multi* m, uint32_t i, const double* rate_hz, size_t n_rates,
                                     const int32_t* labels_dev);
/* Train every network of the set over n_samples whole samples: for each, what
 * rs_eprop_step(net, sample_steps, RS_LEARN | RS_AUTO_UPDATE | RS_AUTO_RESET)
 * does.  Until the schedule is tuned, each sample runs with the next untried
 * e-prop schedule by direct launches, its e-prop launches timed on the device;
 * after the last the fastest is kept, and later samples replay the recorded
 * graph.
 * Errors: RS_ESTATE (an input is missing, or the set is not at a sample
 * boundary), RS_EDEVICE. */
rs_status rs_multi_train(rs_multi* m, uint32_t n_samples);

#define RS_MULTI_SCHEDULES 8
typedef struct rs_multi_schedule {
  uint32_t tuned;            /* 1 once every schedule has been timed */
  uint32_t schedule;         /* the schedule in use */
  uint32_t threads_per_row;  /* e-prop: threads sharing one row's synapses (64 or 256) */
  uint32_t rows_per_tile;    /* e-prop: rows per work-list entry */
  uint32_t workgroups;       /* e-prop: persistent workgroups, 0 = one per entry */
  uint32_t graph;            /* 1: samples replay the recorded graph */
  uint32_t trace_block;      /* steps per block */
  uint32_t reserved;
  double sample_ms[RS_MULTI_SCHEDULES];  /* device time of the e-prop launches of the tuning sample run
                                            with each schedule */
  uint64_t samples;          /* samples trained */
} rs_multi_schedule;
rs_status rs_multi_schedule_get(rs_multi* m, rs_multi_schedule* out);
/* Fix the e-prop schedule (0..4), or -1 to tune again over the next samples;
 * use_graph 0 runs samples by direct launches instead of graph replay. */
rs_status rs_multi_schedule_set(rs_multi* m, int32_t schedule, int32_t use_graph);
/* Variables and counters of network i, as rs_eprop_get / rs_eprop_set /
 * rs_eprop_info_get (synchronising). */
rs_status rs_multi_get(rs_multi* m, uint32_t i, int32_t var, void* host, size_t bytes);
rs_status rs_multi_set(rs_multi* m, uint32_t i, int32_t var, const void* host, size_t bytes);
rs_status rs_multi_info_get(rs_multi* m, uint32_t i, rs_eprop_info* out);
void rs_multi_destroy(rs_multi* m);

/* ==========================================================================
 * Served inference: classification requests on trained networks (the
 * recurrent classifier without learning: input, spikes, propagation, neuron
 * update and leaky readout), with continuous batching.  A request presents an
 * input raster to one model for n_steps steps; its decision is the argmax
 * over readout units k of the summed softmax sum_t pi_k^t.  Each running
 * request holds its neuron and readout state in a slot on the device; every
 * rs_serve_step admits queued requests (in arrival order, skipping those
 * whose model has no free slot) while their state fits the memory budget,
 * then runs one block of steps for every running request in one forward and
 * one readout launch.  A request's result depends only on its model and
 * input, not on the others running beside it.
 * ========================================================================== */
typedef struct rs_serve rs_serve;
typedef struct rs_serve_params {
  uint32_t slots_per_model;      /* state slots allocated per model, 1..4096 */
  uint32_t block_steps;          /* steps per block, 1..32 */
  uint32_t max_running;          /* requests running at once (1: one request per launch) */
  uint32_t max_queue;            /* queued requests beyond which submissions are rejected */
  uint64_t state_budget_bytes;   /* device bytes the running requests' state may take */
} rs_serve_params;
typedef struct rs_serve_result {
  uint64_t ticket;
  uint32_t model, steps;
  int32_t decision;              /* argmax_k sum_t pi_k^t */
  uint32_t reserved;
  uint64_t spikes, events;       /* recurrent spikes, synaptic events of the request */
  double submit_s, admit_s, done_s;  /* host clock, seconds since the server's creation */
} rs_serve_result;
typedef struct rs_serve_stats {
  uint64_t admitted, rejected, completed, blocks;
  uint64_t queued;
  uint32_t running, n_out_max;
  uint64_t state_bytes_used, state_budget_bytes;
  double clock_s;
} rs_serve_stats;
/* Create a server for the models (trained networks, kept by pointer: they
 * must outlive the server and not be stepped while it runs; weights and rows
 * are read in place).  Every model takes the same n_in.  Errors: RS_EINVAL,
 * RS_ENOMEM, RS_EDEVICE. */
rs_status rs_serve_create(rs_eprop* const* models, uint32_t n_models, const rs_serve_params* params,
                          void* hip_stream, rs_serve** out);
/* Queue a request: model index, the input raster (device pointers, B = 1
 * layout of rs_eprop_set_input with raster_steps steps, read cyclically), the
 * presentation length.  Errors: RS_ECAPACITY (rejected: queue full, or the
 * request's state exceeds the budget), RS_EINVAL. */
rs_status rs_serve_submit(rs_serve* s, uint32_t model, const int32_t* off_dev, const int32_t* idx_dev, size_t n_idx,
                          uint32_t raster_steps, uint32_t n_steps, uint64_t* ticket);
/* Admit, run one block for every running request and synchronise; *n_done =
 * requests that finished in it. */
rs_status rs_serve_step(rs_serve* s, uint32_t* n_done);
/* Take up to max finished results (in completion order); scores (NULL or
 * [max][n_out_max] doubles) receives each one's sum_t pi. */
rs_status rs_serve_poll(rs_serve* s, rs_serve_result* out, double* scores, uint32_t max, uint32_t* n);
rs_status rs_serve_stats_get(rs_serve* s, rs_serve_stats* out);
/* One request of a trace: arrival time in seconds from the replay's start. */
typedef struct rs_serve_request {
  double arrival_s;
  uint32_t model, n_steps, raster_steps, reserved;
  const int32_t* off_dev;
  const int32_t* idx_dev;
  size_t n_idx;
} rs_serve_request;
/* Replay a trace (arrivals ascending) against the host's wall clock: each
 * request is submitted once its arrival time has passed, blocks run while
 * requests run, and the call returns when every request has finished or
 * been rejected.  Per request (arrays of n, each may be NULL): latency from
 * arrival to completion in ms (-1 if rejected), decision, spikes. */
rs_status rs_serve_replay(rs_serve* s, const rs_serve_request* reqs, uint32_t n, double* latency_ms,
                          int32_t* decision, uint64_t* spikes);
void rs_serve_destroy(rs_serve* s);

/* ==========================================================================
 * Topographic-map projection (Sec. 2.1.3, Fig. 3; model in Tab. A-H): two
 * L x L sheets with periodic boundaries, rows capped at `cap` synapses.
 * ========================================================================== */
typedef struct rs_topo rs_topo;

typedef struct rs_topo_params {
  uint32_t L;            /* sheet side; n_pre = n_post = L*L, L <= 1024 */
  uint32_t cap;          /* row capacity, 1..1024 */
  uint32_t n_attempts;   /* rewiring attempts per update */
  uint32_t proj_id;      /* random stream id */
  float p_form, sigma_form;   /* formation: p_form exp(-d^2 / 2 sigma^2) */
  float g_theta;              /* weights below it use p_elim_dep */
  float p_elim_dep, p_elim_pot;
  float g_new;                /* weight of newly formed synapses, |g_new| <= 1e4 */
  float g_init;               /* weight of initial synapses, |g_init| <= 1e4 */
  uint64_t seed;
} rs_topo_params;

/* Create and build rows by the pairwise-Bernoulli rule with the formation
 * probability (topographic-map section).  Rows longer than cap keep their
 * first cap targets.  Synchronises.  Errors: RS_EINVAL, RS_ENOMEM, RS_EDEVICE. */
rs_status rs_topo_create(const rs_topo_params* params, void* hip_stream, rs_topo** out);
/* One connectivity update (Sec. 2.1.3): attempts distributed over rows with
 * replacement, candidate targets set without replacement in the row's bitfield
 * section, elimination of candidate synapses with weight-dependent probability,
 * formation at the remaining candidates with distance-dependent probability,
 * all bits cleared.  `step` keys the random draws.  With stats != NULL the call
 * synchronises and fills it. */
rs_status rs_topo_rewire(rs_topo* t, uint64_t step, rs_rewire_stats* stats);
/* Row access, host buffers: len int32[n_pre], ind int32[n_pre][cap],
 * w float[n_pre][cap].  Synchronise.  Errors: RS_EINVAL (len beyond cap,
 * index out of range, a target twice in one row or |w| > 1e4 on set). */
rs_status rs_topo_get_rows(rs_topo* t, int32_t* len, int32_t* ind, float* w);
rs_status rs_topo_set_rows(rs_topo* t, const int32_t* len, const int32_t* ind, const float* w);
/* The attempt bitfield uint32[n_pre][ceil(n_post/32)] (all zero between updates). */
rs_status rs_topo_get_bits(rs_topo* t, uint32_t* bits);
/* Device timing in milliseconds of the last rs_topo_rewire or rs_topo_run
 * (all kernels). */
rs_status rs_topo_last_ms(rs_topo* t, double* ms);
void rs_topo_destroy(rs_topo* t);

/* --------------------------------------------------------------------------
 * Topographic-map simulation (topographic-map model, Tab. A-F, H): the source
 * sheet fires Poisson trains around a stimulus position, the projection's
 * weights are conductances (uS) onto conductance-based LIF targets, STDP
 * changes them, and the rewiring above runs every rewire_steps steps.
 *
 * One step t: decay the STDP traces x (source) and y (target) by
 * exp(-h/tau_plus), exp(-h/tau_minus); deliver the source spikes drawn at t-1
 * (delay one step): each synapse adds its weight to its target's conductance
 * g and, with stdp, loses A_minus*y_target (floored at 0), and x_source += 1;
 * every target not refractory integrates by exponential Euler with the current
 * g*(E_exc - V) held over the step, V <- V_rest + R*I + (V - V_rest - R*I) *
 * exp(-h/tau_m), R = tau_m/C_m, and spikes when V >= V_th (V <- V_reset, then
 * ref_steps steps held at V_reset); g decays by exp(-h/tau_s); with stdp every
 * synapse onto a target that spiked gains A_plus*x_source (capped at g_max),
 * and y += 1 for it; finally the source draws step t's spikes: channel i fires
 * when its 32-bit draw is below floor(p*2^32), p = (f_base + f_peak*exp(-d2 /
 * (2*sigma_stim^2))) * h / 1000, with d2 the squared torus distance of i from
 * the stimulus (blob: a cell; bar: a row or column of cells, distance along
 * the other axis) whose position is redrawn every stim_steps steps.  Draws:
 * one Philox4x64-10 call under key (seed, TP_INPUT = 12) at counter
 * (t, c, 0, 0) serves channels 8c .. 8c+7; channel 8c + b takes 32-bit half
 * b of the call's output (word b/2; the upper half for even b, the lower half
 * for odd b).
 * -------------------------------------------------------------------------- */
enum { RS_STIM_BLOB = 0, RS_STIM_BAR = 1 };

typedef struct rs_topo_model {
  float h;                               /* time step, ms (Tab. H) */
  float C_m, tau_m, V_rest, E_exc;       /* nF, ms, mV, mV (Tab. D) */
  float V_th, V_reset, tau_s;            /* mV, mV, ms */
  uint32_t ref_steps;                    /* tau_ref / h */
  float f_base, f_peak, sigma_stim;      /* Hz, Hz, cells (Tab. E) */
  uint32_t stim_steps;                   /* t_stim / h, >= 1 */
  int32_t stim_kind;                     /* RS_STIM_BLOB or RS_STIM_BAR */
  int32_t stdp;                          /* 0: weights fixed */
  float g_max, A_plus, A_minus;          /* uS (Tab. F) */
  float tau_plus, tau_minus;             /* ms */
  uint32_t rewire_steps;                 /* t_rewiring / h; 0: no rewiring */
  uint32_t stim_tile;                    /* scaled maps: the input is replicated in every stim_tile x
                                            stim_tile square (the s^2 stimulus locations of the scaling
                                            paragraph, one drawn position at the same offset in each);
                                            0 = one square, the whole sheet.  Must divide L. */
} rs_topo_model;

/* Lateral projection (Tab. A "feed-forward and lateral connections"; Tab. G
 * p_form-lat, sigma_form-lat): target -> target rows built and rewired like
 * the feed-forward projection, with `lp` giving its capacity, attempts,
 * formation and elimination parameters and its proj_id (which must differ
 * from the map's; the map's seed keys its draws).  Autapses are allowed.  In
 * the simulation a target spike of step t is delivered at t+1 through these
 * rows after the source spikes: each synapse adds its weight to its target's
 * g and, with stdp, loses A_minus*y_target; the spiking neuron's lateral trace
 * xl (decay exp(-h/tau_plus)) gains 1; a target that spikes potentiates its
 * lateral synapses by A_plus*xl_pre, capped at g_max.  rs_topo_run rewires the
 * lateral projection after the feed-forward one at the same steps.  Call
 * before rs_topo_sim_init.  Synchronises.  Errors: RS_EINVAL (parameters, L
 * different from the map's, equal proj_id), RS_ESTATE (already added, or the
 * simulation is attached), RS_ENOMEM, RS_EDEVICE. */
rs_status rs_topo_add_lateral(rs_topo* t, const rs_topo_params* lp);
/* The rs_topo_rewire / get_rows / set_rows / get_bits / run_stats calls for
 * the lateral projection (n_pre = n_post = L*L).  Errors: RS_ESTATE without
 * a lateral projection, else as the feed-forward calls. */
rs_status rs_topo_lat_rewire(rs_topo* t, uint64_t step, rs_rewire_stats* stats);
rs_status rs_topo_lat_get_rows(rs_topo* t, int32_t* len, int32_t* ind, float* w);
rs_status rs_topo_lat_set_rows(rs_topo* t, const int32_t* len, const int32_t* ind, const float* w);
rs_status rs_topo_lat_get_bits(rs_topo* t, uint32_t* bits);
rs_status rs_topo_lat_run_stats(rs_topo* t, rs_rewire_stats* stats);

/* Simulation kernels.  ONE_WG: one workgroup holds both sheets (L*L <= 4096,
 * no lateral projection).  TILED: one workgroup per 256 targets with a
 * device-wide barrier per step (L*L <= 16384, every tile resident at once;
 * a barrier that waits longer than a few seconds gives up, and the next
 * synchronising call reports RS_EDEVICE).  AUTO (default): ONE_WG where it
 * applies, else TILED.  Both compute the model above; they round the traces
 * differently in the last bits (the one-workgroup kernel folds the decay of x
 * into potentiation). */
enum { RS_TOPO_KERNEL_AUTO = 0, RS_TOPO_KERNEL_ONE_WG = 1, RS_TOPO_KERNEL_TILED = 2 };
/* Choose the kernel (before or after rs_topo_sim_init).  Errors: RS_EINVAL
 * (unknown kind, or a kind the map does not fit). */
rs_status rs_topo_sim_kernel(rs_topo* t, int32_t kind);

/* Attach the simulation to a topographic map and reset its state: V = V_rest,
 * everything else zero, step counter 0.  Needs L*L <= 16384 (4096 for the
 * one-workgroup kernel).  Synchronises.
 * Errors: RS_EINVAL (sizes, non-positive time constants or steps, stim_tile),
 * RS_ENOMEM. */
rs_status rs_topo_sim_init(rs_topo* t, const rs_topo_model* m);
/* Run n_steps steps from the step counter on, with a rewire (keyed by the
 * step count reached) after every step count divisible by rewire_steps.
 * Asynchronous on the map's stream.  Runs of 64 whole rewiring intervals are
 * replayed from a HIP graph recorded at their first use (and again after
 * rs_topo_sim_init); the results equal those of step-by-step calls bit for
 * bit.  Rewire statistics accumulate from the call's start
 * (rs_topo_run_stats).  The step count 2^64-1 is reserved.
 * Errors: RS_ESTATE before rs_topo_sim_init, RS_EDEVICE if recording fails. */
rs_status rs_topo_run(rs_topo* t, uint64_t n_steps);
/* Summed rewire statistics of the last rs_topo_run.  Synchronises. */
rs_status rs_topo_run_stats(rs_topo* t, rs_rewire_stats* stats);
/* Per-phase timers of the simulation kernel, in the manner of the paper's
 * Fig. 10 split: one thread reads the device wall clock at each phase
 * boundary.  on != 0 enables them, 0 disables them; either way the
 * accumulated times restart from zero.  Timing changes no result.
 * Synchronises.  Errors: RS_ESTATE before rs_topo_sim_init. */
rs_status rs_topo_sim_timing(rs_topo* t, int32_t on);
/* Milliseconds accumulated per phase since the last rs_topo_sim_timing:
 * ms[0] delivery with the source draws, ms[1] neuron update, ms[2]
 * potentiation, ms[3] launch prologue (state loads and any column rebuild).
 * On the tiled kernel (timed on its first workgroup) ms[0] is the delivery,
 * ms[1] the neuron update with the publishing of the tile's spikes and
 * traces, and ms[3] also holds the source draws and the step-barrier waits.
 * The rewire kernels and launch gaps make up the rest of rs_topo_last_ms.
 * Synchronises.  Errors: RS_ESTATE before rs_topo_sim_init, RS_EDEVICE. */
rs_status rs_topo_sim_phase_ms(rs_topo* t, double ms[4]);
/* Simulation variables, host buffers of exactly the stated size.  Synchronise. */
enum {
  RS_TV_V = 0,      /* float[L*L] target membrane potential, mV */
  RS_TV_G = 1,      /* float[L*L] target conductance, uS */
  RS_TV_Y = 2,      /* float[L*L] target STDP trace */
  RS_TV_X = 3,      /* float[L*L] source STDP trace */
  RS_TV_REF = 4,    /* int32[L*L] remaining refractory steps */
  RS_TV_COUNT = 5,  /* uint32[L*L] target spikes since init */
  RS_TV_ZIN = 6,    /* uint32[ceil(L*L/32)] source spikes drawn at the last step (delivered next) */
  RS_TV_ZOUT = 7,   /* uint32[ceil(L*L/32)] target spikes of the last step (read-only) */
  RS_TV_STEP = 8,   /* uint64[1] step counter */
  RS_TV_XLAT = 9    /* float[L*L] target lateral STDP trace (with a lateral projection) */
};
rs_status rs_topo_sim_get(rs_topo* t, int32_t var, void* host, size_t bytes);
rs_status rs_topo_sim_set(rs_topo* t, int32_t var, const void* host, size_t bytes);

/* ==========================================================================
 * DEEP R on caller-owned rows without device allocation
 * ========================================================================== */
/* A ragged projection in caller-owned device memory, laid out as the
 * RS_PROJ(p, f) variables of rs_eprop_get: len int32[n_pre]; ind, w, m, v, G
 * [n_pre][cap]; eps (or NULL), ebar [n_pre][cap][batch]; conn, sign
 * uint32[n_pre][words], words = ceil(n_post / 32). */
typedef struct rs_deepr_rows {
  int32_t n_pre, n_post, cap, words, recurrent, batch;
  int32_t *len, *ind;
  float *w, *m, *v, *G, *eps, *ebar;
  uint32_t *conn, *sign;
} rs_deepr_rows;
/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid allocation): DEEP R rewiring
 * (Sec. 2.1.2) of the rows in place, exactly as rs_eprop_rewire rewires a
 * projection with the same seed, projection id (0 input, 1 recurrent) and
 * step.  Its scratch (per-row dormant and activation counts, counters) is one
 * fixed device array of the library, so n_pre is at most 8192; it is never
 * allocated, and calls that overlap on one device race for it.  Runs on
 * hip_stream; with stats != NULL it synchronises and fills them as
 * rs_eprop_rewire does.  Errors: RS_EINVAL (sizes, NULL arrays, n_pre above
 * 8192), RS_EDEVICE. */
rs_status rs_deepr_rewire_noalloc(const rs_deepr_rows* rows, uint64_t seed, uint32_t proj_id, uint64_t step,
                                  void* hip_stream, rs_rewire_stats* stats);

/* ==========================================================================
 * Custom connectivity updates (Sec. 2.1): a rule's host part runs on the
 * host, its row parts on the device in parallel over the rows, each visiting
 * its row's synapses (removing some, with the ragged rule: the row's last
 * synapse moves into the freed slot) and appending new ones.  The rules here
 * are written on the library's C++ row-update interface (rs_custom.hpp),
 * which new rules compiled into the library use too:
 *   RS_RULE_ADD_DIAGONAL   every row i < n_post adds a synapse onto target i,
 *                          weight 1 (skipped where a connectivity bitfield
 *                          shows it present); no host part
 *   RS_RULE_REMOVE_RANDOM  host part: row i picks target below(u32(CUSTOM = 13;
 *                          step, i, 0, 0), n_post); row part: the first synapse
 *                          onto it (slot order) is removed
 *   RS_RULE_DEEPR          DEEP R (Sec. 2.1.2) as elimination row part, the
 *                          dormant total spread over the rows on the host, and
 *                          formation row part: the same rows, records and bits
 *                          as rs_eprop_rewire at the same step
 *   RS_RULE_TOPO           the topographic rewiring (Sec. 2.1.3): attempts
 *                          spread over rows on the host, the row part as
 *                          rs_topo_rewire's: the same rows and weights
 * New synapses' other variables (optimiser state, gradient, traces) start at
 * zero.  A host function, when given, runs after the rule's host part and may
 * change its per-row variable (REMOVE_RANDOM: the target per row; DEEPR: the
 * activations per row, which must fit each row's room; TOPO: the attempts
 * per row) before the row part reads it.
 * ========================================================================== */
enum { RS_RULE_ADD_DIAGONAL = 1, RS_RULE_REMOVE_RANDOM = 2, RS_RULE_DEEPR = 3, RS_RULE_TOPO = 4 };
typedef struct rs_custom_host {
  int32_t n_pre, n_post, cap, recurrent;
  const int32_t* len;   /* row lengths when the host part runs (read-only) */
  uint32_t* pre_var;    /* the rule's per-row variable [n_pre] */
  uint64_t seed, step;
  uint32_t proj_id;
  int32_t rule;
} rs_custom_host;
typedef void (*rs_host_update_fn)(void* user, rs_custom_host* host);
/* Run `rule` on projection proj (0 input, 1 recurrent) of an e-prop network
 * (after the work queued on it), draws keyed by `step`.  Synchronises; with
 * stats: eliminated = removed, formed = added, attempts = DEEP R's
 * activations placed, blocked = activations without room.  Errors: RS_EINVAL
 * (unknown rule, DEEP R without bitfields, a host function's assignment
 * beyond a row's room). */
rs_status rs_eprop_custom_update(rs_eprop* net, uint32_t proj, int32_t rule, uint64_t step, rs_host_update_fn fn,
                                 void* user, rs_rewire_stats* stats);
/* The same on a topographic map's projection (RS_RULE_TOPO: stats as
 * rs_topo_rewire's).  An attached simulation rebuilds its column view at its
 * next launch. */
rs_status rs_topo_custom_update(rs_topo* t, int32_t rule, uint64_t step, rs_host_update_fn fn, void* user,
                                rs_rewire_stats* stats);

/* ==========================================================================
 * Composed networks: the paper's problem statement (Sec. 2.1) as calls --
 * declare populations and projections with their initialisation, learning
 * rule and structural-plasticity rule, build, step, trigger the rule, read and
 * write state.  rs_build recognises the models the kernels implement:
 *   - the e-prop classifier: a spike source, a LIF or ALIF population and a
 *     readout; source -> recurrent and recurrent -> recurrent fixed-probability
 *     projections (DEEP R on either), recurrent -> readout dense; all learn by
 *     e-prop with one Adam optimiser and update interval;
 *   - the topographic map: a Poisson sheet projecting onto a conductance-LIF
 *     sheet of the same size by Gaussian pairwise-Bernoulli rows, STDP or
 *     fixed weights, topographic rewiring or none; optionally a second,
 *     lateral projection from the conductance-LIF sheet onto itself (Gaussian
 *     rows, the same learning and rewiring interval, rs_topo_add_lateral).
 * Any other composition is refused at build with RS_EINVAL naming the misfit.
 * With an allocator (both functions non-NULL) every device buffer of the
 * built network comes from it and returns to it at rs_destroy.
 * ========================================================================== */
typedef struct rs_net rs_net;
enum {
  RS_POP_SPIKE_SOURCE = 0,   /* input channels: a raster or Poisson rates attached by rs_eprop_set_input* */
  RS_POP_LIF = 1,            /* leaky integrate-and-fire, subtractive reset */
  RS_POP_ALIF = 2,           /* adaptive LIF */
  RS_POP_READOUT = 3,        /* leaky readout units */
  RS_POP_POISSON_SHEET = 4,  /* L x L Poisson source around a moving stimulus */
  RS_POP_COND_LIF_SHEET = 5  /* L x L conductance-based LIF with refractoriness */
};
typedef struct rs_pop_params {
  float dt_ms, tau_mem_ms, tau_adapt_ms, v_thr, beta;  /* LIF, ALIF */
  uint32_t L;                                          /* sheets: side, n = L * L */
  rs_topo_model model;  /* COND_LIF_SHEET: neuron and synapse fields; POISSON_SHEET: stimulus fields */
} rs_pop_params;
enum { RS_INIT_FIXED_PROB = 0, RS_INIT_GAUSS_TORUS = 1, RS_INIT_DENSE = 2 };
enum { RS_LEARN_NONE = 0, RS_LEARN_EPROP = 1, RS_LEARN_STDP = 2 };
enum { RS_REWIRE_NONE = 0, RS_REWIRE_DEEPR = 1, RS_REWIRE_TOPO = 2 };
typedef struct rs_proj_desc {
  int32_t init;                 /* RS_INIT_* */
  float p, sigma_w;             /* FIXED_PROB: probability, weights sigma_w N(0,1); DENSE: sigma_w N(0,1) */
  float p_form, sigma_form, g_init;  /* GAUSS_TORUS: p_form exp(-d^2 / 2 sigma_form^2), weight g_init */
  uint32_t cap;                 /* row capacity, 0 = twice the longest initial row */
  int32_t learn;                /* RS_LEARN_* (STDP parameters: the target sheet's model) */
  float lr, adam_b1, adam_b2, adam_eps;  /* EPROP */
  int32_t rewire;               /* RS_REWIRE_* */
  float l1;                     /* DEEPR */
  uint32_t n_attempts;          /* TOPO */
  float g_theta, p_elim_dep, p_elim_pot, g_new;  /* TOPO */
  uint32_t update_interval;     /* EPROP: steps between updates (and DEEP R); TOPO: steps between rewires */
} rs_proj_desc;
rs_status rs_create(void* hip_stream, rs_alloc_fn alloc_fn, rs_free_fn free_fn, void* user, uint64_t seed,
                    rs_net** out);
rs_status rs_add_pop(rs_net* net, int32_t kind, uint32_t n, const rs_pop_params* params, uint32_t* pop);
rs_status rs_add_proj(rs_net* net, uint32_t pre, uint32_t post, const rs_proj_desc* desc, uint32_t* proj);
/* Build (the classifier: `batch` instances, samples of sample_steps steps,
 * trace_block as in rs_eprop_params; the map ignores the three).
 * Synchronises.  Errors: RS_EINVAL (a composition no model implements, or
 * invalid parameters), RS_ENOMEM, RS_EDEVICE, RS_ESTATE (built before). */
rs_status rs_build(rs_net* net, uint32_t batch, uint32_t sample_steps, uint32_t trace_block);
/* The built model's own object, for the calls specific to it (input, timers,
 * snapshots); owned by the network. */
rs_status rs_eprop_of(rs_net* net, rs_eprop** out);
rs_status rs_topo_of(rs_net* net, rs_topo** out);
/* Step: rs_eprop_step with `flags`, or rs_topo_run (flags ignored). */
rs_status rs_step(rs_net* net, uint32_t n_steps, uint32_t flags);
rs_status rs_update(rs_net* net);
/* Trigger the projection's structural-plasticity rule now (DEEP R, or one
 * topographic rewire keyed by the step count). */
rs_status rs_rewire(rs_net* net, uint32_t proj, rs_rewire_stats* stats);
/* Rows of a ragged projection: len int32[n_pre], ind int32[n_pre][cap],
 * w float[n_pre][cap]; *needed = n_pre * cap.  Errors: RS_ECAPACITY when
 * cap_elems is smaller. */
rs_status rs_get_rows(rs_net* net, uint32_t proj, int32_t* len, int32_t* ind, float* w, size_t cap_elems,
                      size_t* needed);
/* Variables: the classifier's RS_* ids (rs_eprop_get/set), the map's RS_TV_* ids. */
rs_status rs_get_var(rs_net* net, int32_t var, void* host, size_t bytes);
rs_status rs_set_var(rs_net* net, int32_t var, const void* host, size_t bytes);
rs_status rs_sync(rs_net* net);
uint64_t rs_step_counter(const rs_net* net);
void rs_destroy(rs_net* net);

/* ==========================================================================
 * Calibration
 * ========================================================================== */
/* Plain streaming copy of `bytes` (multiple of 16) from src to dst (device
 * pointers) on `hip_stream`; used to calibrate hardware byte counters. */
rs_status rs_calib_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
