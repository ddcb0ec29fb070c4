// Internal launch interface between the host engine and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

// Device view of one ragged projection.
struct ProjDev {
  int n_pre, n_post, cap, words, recurrent, proj_id;
  int* len;          // [n_pre]
  int* ind;          // [n_pre*cap]
  float* w;          // [n_pre*cap]
  float* m;          // Adam moments / gradient, may be null
  float* v;
  float* G;
  float* eps;        // [n_pre*cap*B], null for LIF / untrained / interleaved
  float* ebar;       // [n_pre*cap*B], or [n_pre*cap*B][2] interleaved; null if untrained
  // floats per slot in ebar: B, or 2B when ebar holds ebar and eps of each
  // instance side by side (the transfer-coefficient kernel's ALIF layout, eps
  // null); record moves copy erec floats of ebar (and B of eps if present)
  int erec;
  uint32_t* conn;    // [n_pre*words] DEEP R connectivity bits, may be null
  uint32_t* sign;    // [n_pre*words] DEEP R sign bits, may be null
  int* dormant;      // [n_pre] eliminated per row by the last rewire
  int* assigned;     // [n_pre] activations per row of the last formation
};

// Column view of the two projections onto the recurrent layer, for the
// target-major e-prop kernel: col[off[j*G+g] .. off[j*G+g+1]) holds (r, slot)
// of every synapse onto target j from a row r with r % G == g, where G is the
// kernel's number of source groups (at most COL_GROUPS_MAX) and r = i for input
// rows and n_in + i for recurrent rows.  Rebuilt whenever rows change.
constexpr int COL_GROUPS_MAX = 8;
struct ColumnView {
  int* cnt;          // [n_rec*COL_GROUPS_MAX] counts, then the fill cursor
  int* off;          // [n_rec*COL_GROUPS_MAX + 1]
  int2* col;         // [n_in*cap_in + n_rec*cap_rec]
  // the transfer-coefficient e-prop kernel with more than 128 instances:
  // each instance chunk's gradient accumulates by list position until a fold
  // (before the update, or before G is read or written or rows move) adds
  // the chunks to G in chunk order and clears them; zero otherwise
  float* gx;         // [ceil(B/128)][n_in*cap_in + n_rec*cap_rec]
  int n_col;         // n_in*cap_in + n_rec*cap_rec
};

// ---------------------------------------------------------------- build
void launch_fixed_rows(hipStream_t s, uint64_t seed, const ProjDev& P, uint64_t T, double sigma, bool fill);
void launch_gauss_rows(hipStream_t s, uint64_t seed, const ProjDev& P, int L, const uint64_t* T_d2,
                       float g_init, bool fill);
void launch_dense_init(hipStream_t s, uint64_t seed, int proj_id, int rows, int cols, double sigma, float* W);
void launch_deepr_bits_init(hipStream_t s, uint64_t seed, const ProjDev& P);
void launch_fill_zero(hipStream_t s, void* p, size_t bytes);

// ---------------------------------------------------------------- e-prop step
struct FwdArgs {
  int n_in, n_rec, n_out, B;
  double alpha, rho, v_thr, beta;            // neuron recurrences are evaluated in double
  double psi_scale;                          // 0.3 / v_thr
  float alpha_f;                             // trace decay: F <- fma(alpha_f, F, spike) in float
  double* V; double* A;                      // [B][n_rec]
  float* xbar; float* zbar;                  // [B][n_in], [B][n_rec] presynaptic traces
  // hand-off, instance-major staging (coalesced writes); psi, x0, z0, xbits
  // and zbits may be null (inference: no eligibility work follows)
  float* psi;                                // [tau][B][n_rec] surrogate derivative of each step
  float* u;                                  // [tau][B][n_out] readout drive sum_j W_out[k][j] z_j
  float* x0; float* z0;                      // [B][n] traces at the start of the block
  uint32_t* xbits; uint32_t* zbits;          // [B][n] spikes of the block, bit tau = step tau
  uint8_t* z;                                // [B][n_rec]
  const int* len_in; const int* ind_in; const float* w_in; int cap_in;
  const int* len_rec; const int* ind_rec; const float* w_rec; int cap_rec;
  const float* Wout;                         // [n_out][n_rec]
  const int* x_off; const int* x_idx; long long n_idx;
  int t0, sample_steps, nsteps;              // steps t0 .. t0+nsteps-1 (raster step t % sample_steps)
  // Poisson source (x_thr != null, raster unused): channel i of instance b
  // fires at step step0 + tau when draw_u32(seed, INPUT; step0+tau, b, i, 0)
  // < x_thr[b * x_thr_stride + i]; the block's lists go to x_list [K][B][n_in]
  const uint64_t* x_thr; int x_thr_stride; int* x_list;
  uint64_t seed, step0;
  const uint64_t* step_base;                 // null, or a device step count added to step0 (replayed launches)
  int wout_lds;                              // 1: stage W_out in LDS for the block
  int rows_lds;                              // 1: stage both projections' rows in LDS if they fit
  int xcap;                                  // LDS capacity for the block's input spike lists
  unsigned long long* counters;              // [0] synaptic events, [1] spikes
  uint32_t* zcount;                          // [B][n_rec] spikes per neuron, accumulated
};
// One launch runs `nsteps` consecutive steps into the staging buffers.
void launch_fwd(hipStream_t s, const FwdArgs& a);
// LDS plan of one network's forward launch (xcap, wout_lds set in `a`); returns the bytes it needs.
size_t fwd_plan(FwdArgs& a);
// Items per thread a network needs (1, 2, 4 or 8).
int fwd_items(int n_in, int n_rec);
// Several networks in one launch: A[work[g].x] runs batch instance work[g].y;
// `items` covers every network, `lds` is the largest plan.
void launch_fwd_multi(hipStream_t s, const FwdArgs* A, const int2* work, int n_work, int items, size_t lds);
// Whether one forward workgroup's LDS holds a network of this size.
bool fwd_fits(int n_in, int n_rec, int n_out);

// Readout over a block: y, softmax error delta into the ring, and (if asked)
// the learning signal L = W_out^T delta into the ring.
struct ReadoutArgs {
  int n_rec, n_out, B, nsteps, slot0, nslot;
  double alpha;
  const float* u;                            // staging [tau][B][n_out]
  double* Y;                                 // [B][n_out] readout state
  const float* Wout; const float* bout;      // [n_out][n_rec], [n_out]
  const int* labels;                         // [B]
  float* deltaT; float* LT;                  // rings [n_out][nslot][B], [n_rec][nslot][B]
};
void launch_readout(hipStream_t s, const ReadoutArgs& a, bool learning_signal);
// Several networks: work lists of (network, x, y, z) tiles of each kernel's grid.
void launch_readout_multi(hipStream_t s, const ReadoutArgs* A, const int4* ro_work, int n_ro,
                          const int4* ls_work, int n_ls);
int readout_grid(const ReadoutArgs& a);                 // k_readout workgroups
void learning_signal_grid(const ReadoutArgs& a, int g[3]);

// Move staged hand-off arrays ([step][B][n], 32-bit words) into neuron-major
// layout ([n][nslot][B], step tau to slot slot0 + tau).
constexpr int HANDOFF_ARRAYS = 5;  // psi (per step); x0, z0, xbits, zbits (per block)
struct HandoffArrays {
  const uint32_t* src[HANDOFF_ARRAYS];
  uint32_t* dst[HANDOFF_ARRAYS];
  int n[HANDOFF_ARRAYS], steps[HANDOFF_ARRAYS], slot0[HANDOFF_ARRAYS], nslot[HANDOFF_ARRAYS];
  int es[HANDOFF_ARRAYS];  // words between consecutive elements of dst: 1, or 2 in a pair array
};
void launch_handoff_transpose(hipStream_t s, const HandoffArrays& h, int B);
void handoff_grid(const HandoffArrays& h, int B, int g[3]);
void launch_handoff_multi(hipStream_t s, const HandoffArrays* H, const int* Bs, const int4* work, int n_work);

struct EpropArgs {
  int n_in, n_rec, n_out, B, alif;
  float alpha, rho, beta;   // eligibility arithmetic is float; state is float
  float one_m_rho;          // 1 - rho, so the slow eps decay carries no rounding bias
  ProjDev in, rec;
  // presynaptic traces of the block, rebuilt step by step with
  // F <- fma(alpha, F, spike) from the block's start values and spike bits
  // ([n][B]; bit t of a word = step t of the block)
  const float* x0; const float* z0;
  const uint32_t* xbits; const uint32_t* zbits;
  int tr_es;                // 2: x0/xbits (z0/zbits) are one [n][B][2] array of (trace, word) pairs; else 1
  int tofs;                 // steps of the block before this launch's first step
  // ring [n][nslot][B]; this launch applies steps slot0 .. slot0+nsteps-1
  const float* psiT; const float* LT; const float* deltaT;
  int slot0, nsteps, nslot;
  float* Gout; float* Gb;
  const int* col_off; const int2* col;   // ColumnView (B % 4 == 0)
  float* gx; int n_col;                  // ColumnView's per-chunk gradients (B > 128)
};
void launch_eprop(hipStream_t s, const EpropArgs& a);
// Whether a network of batch B runs the transfer-coefficient e-prop kernel,
// which reads the block-start traces and spike words as (trace, word) pairs.
bool eprop_tc_path(int B);
// Whether a network of batch B keeps ebar and eps interleaved (ALIF under the
// transfer-coefficient kernel, which reads a synapse's state as one record).
bool eprop_interleaved(int B, bool alif);
// Add the per-chunk gradients (a.gx, B > 128) to G in chunk order and clear
// them; reads the column view that the e-prop launches used.
void launch_gx_fold(hipStream_t s, const EpropArgs& a);
// Default steps per eligibility block (one e-prop launch) for batch B.
int eprop_default_block(int B, uint32_t update_interval);
// Default block lengths when automatic updates run every update_interval
// steps: the first block of an interval K0 steps, the others at most K.
void eprop_default_schedule(int B, uint32_t update_interval, int* K, int* K0);
// Narrow e-prop kernel over several networks, persistent over a work list of
// row tiles (network, first row, rows; rows >= n_in + n_rec are readout
// chunks): `grid` workgroups (0: one per work item), `tpr` threads per row (64
// or 256).
void launch_eprop_narrow_multi(hipStream_t s, const EpropArgs* A, const int4* work, int n_work, bool alif,
                               int tpr, int grid);
int narrow_readout_chunks(int n_rec);
void launch_columns(hipStream_t s, const ProjDev& in, const ProjDev& rec, const ColumnView& cv);

// ---------------------------------------------------------------- update
struct UpdateArgs {
  int B;
  float lr, b1, b2, eps, inv_c1, inv_c2, l1;
  int l1_in, l1_rec;
  ProjDev in, rec;
  float* Wout; float* bout; float* Gout; float* Gb; float* Mout; float* Vout; float* Mb; float* Vb;
  int n_out_elems, n_b;
  // replayed launches: the bias corrections of update k = *adam_base + adam_off
  // come from adam_tab[2 min(k, adam_kmax)], [.. + 1] (inv_c1, inv_c2); null: the fields above
  const float* adam_tab; const uint32_t* adam_base; int adam_off, adam_kmax;
};
void launch_update(hipStream_t s, const UpdateArgs& a);
int update_blocks(const UpdateArgs& a);
// work[g] = (network, block, blocks of that network)
void launch_update_multi(hipStream_t s, const UpdateArgs* A, const int4* work, int n_work);

// ---------------------------------------------------------------- DEEP R
// stats: int64[4] device counters, incremented: 0 eliminated (= D, the dormant
// total), 1 formed, 2 activations distributed to rows, 3 activations no row had
// room for
void launch_deepr(hipStream_t s, uint64_t seed, const ProjDev& P, int B, uint64_t step,
                  long long* stats);
struct DeeprArgs {
  uint64_t seed;
  ProjDev P;
  int B;
  uint64_t step;               // random step, plus *step_base when step_base is set
  const uint64_t* step_base;
  long long* stats;            // int64[4] as above
};
// DEEP R of n_proj projections; rows[g] = (projection, row) over all their rows.
void launch_deepr_multi(hipStream_t s, const DeeprArgs* D, int n_proj, const int2* rows, int n_rows, int max_cap,
                        int max_pre);

// ---------------------------------------------------------------- topomap
struct TopoDev {
  ProjDev P;
  int L, n_attempts;
  float g_theta, g_new;
  uint64_t T_dep, T_pot;
  const uint64_t* T_d2;   // [2*(L/2)^2 + 1]
  uint32_t* bits;         // [n_pre*words]
  int* kcount;            // [n_pre]
  int* rowlist;           // [max(n_attempts,1)]
  int* nrows;             // [1]
  long long* stats;       // [4]
  int* col_dirty;         // [1] set to 1 when a rewire changes any row; may be null
  const uint64_t* step_dev;  // [1] step count, read when a launch passes STEP_FROM_DEVICE
  // column view of an attached simulation, edited by the rewire; null without one
  int* col_len;           // [n_post]
  int* col_ent;           // [n_post][col_cap]
  int col_cap;
};
// Step argument telling a topographic-map kernel to read the step count from
// device memory (launches recorded once in a graph and replayed).
constexpr uint64_t STEP_FROM_DEVICE = ~0ull;
void launch_topo_rewire(hipStream_t s, uint64_t seed, const TopoDev& t, uint64_t step);
// Two projections' rewires (the same step), in one launch where both fit it.
void launch_topo_rewire_pair(hipStream_t s, uint64_t seed, const TopoDev& a, const TopoDev& b, uint64_t step);

// Topographic-map simulation state and constants (model of Tab. B, D-F).
struct TopoSimDev {
  int L, N, ref_steps, stim_steps, stim_kind, stdp;
  int stim_L;             // side of the square the stimulus is replicated over (L: one square)
  float V_rest, E_exc, V_th, V_reset, R, em, es, dx, dy, inv_dx, A_plus, A_minus, g_max;
  const uint64_t* T_in;   // [2*(L/2)^2 + 1] input Bernoulli threshold by squared stimulus distance
  float *V, *g, *y, *x;   // [N]
  int* ref;               // [N]
  uint32_t* count;        // [N]
  uint32_t *zin, *zout;   // [ceil(N/32)] bits
  int *col_len, *col_ent; // [N], [N][col_cap]: column j's slot indices, -1 for removed synapses
  int col_cap;            // N: no target can have more synapses than there are rows
  int* col_dirty;         // [1]
  uint64_t* step_dev;     // [1] step count: read for t0 == STEP_FROM_DEVICE, written at the end
  unsigned long long* ticks;  // [TOPO_PHASES] wall-clock ticks per phase, or null (timers off)
  // lateral projection (target -> target), tiled kernel only
  float* xl;                    // [N] lateral pre trace
  int *col_len_l, *col_ent_l;   // its column view, [N], [N][col_cap]
  int* col_dirty_l;             // [1]
  // tiled kernel: second buffer of the per-step exchange (the first is zin,
  // zout, x, xl), the step barrier's per-tile flags and the barrier-timeout flag
  uint32_t *zin_b, *zout_b;     // [ceil(N/32)]
  float *x_b, *xl_b;            // [N]
  unsigned long long* bar;      // [TOPO_TILES_MAX * 16]: tile g's count at bar[16 g]
  int* err;                     // [1]
};
// Phases of the simulation's timers: delivery with the source draws, neuron
// update, potentiation, launch prologue (state loads and any column rebuild).
constexpr int TOPO_PHASES = 4;
bool topo_sim_fits(int N);
size_t topo_sim_lds_bytes(int N);
void launch_topo_sim(hipStream_t s, uint64_t seed, const ProjDev& P, const TopoSimDev& sd, uint64_t t0,
                     int n_steps);
// Tiled simulation: one workgroup per TOPO_TILE targets, a device-wide step
// barrier; PL.n_pre == 0 means no lateral projection.
constexpr int TOPO_TILE = 256;
constexpr int TOPO_TILES_MAX_N = 16384;
constexpr int TOPO_TILES_MAX = TOPO_TILES_MAX_N / TOPO_TILE;  // 64: one polling lane per tile
size_t topo_tiles_lds_bytes(int N, bool lateral);
int topo_tiles_grid(int N);
// Workgroups of the tiled kernel the device keeps resident at once (0 on error).
int topo_tiles_resident(int N, bool lateral);
void launch_topo_tiles(hipStream_t s, uint64_t seed, const ProjDev& P, const ProjDev& PL, const TopoSimDev& sd,
                       uint64_t t0, int n_steps);
// Set the kernels' launch attributes ahead of a stream capture (idempotent).
void topo_sim_attrs();
void topo_rewire_attrs();
void fwd_attrs();
void deepr_attrs();

// ---------------------------------------------------------------- custom connectivity updates
// Rules on the row-update interface (rs_custom.hpp, k_custom.hip); stats
// int64: [0] removed, [1] added (incremented).
void launch_add_diagonal(hipStream_t s, const ProjDev& P, int B, long long* stats);
void launch_remove_post(hipStream_t s, const ProjDev& P, const uint32_t* post_ind, int B, long long* stats);
void launch_deepr_elim_rule(hipStream_t s, const ProjDev& P, int B, long long* stats);  // writes P.dormant
void launch_deepr_form_rule(hipStream_t s, uint64_t seed, const ProjDev& P, int B, uint64_t step,
                            long long* stats);  // reads P.assigned
void launch_topo_rule(hipStream_t s, uint64_t seed, const TopoDev& t, uint64_t step, const int* kcount,
                      long long* stats);  // stats = t.stats ([2] blocked)

// ---------------------------------------------------------------- served inference
// Readout of one running request over a block of steps.
struct ServeReadout {
  int n_out, nsteps;
  double alpha;
  const float* u;      // [nsteps][n_out] readout drive of the block
  double* Y;           // [n_out] readout state
  const float* bout;   // [n_out]
  double* score;       // [n_out] sum over the request's steps of softmax(y)
};
void launch_serve_readout(hipStream_t s, const ServeReadout* R, int n);

// ---------------------------------------------------------------- misc
void launch_copy(hipStream_t s, void* dst, const void* src, size_t bytes);
// Zero a list of device ranges in one launch (a kernel, so it can be recorded
// in a graph): ranges[q] = {pointer, bytes}, bytes a multiple of 4.
struct ZeroRange { void* p; unsigned long long bytes; };
void launch_fill_zero_ranges(hipStream_t s, const ZeroRange* ranges, int n, unsigned long long max_bytes);
// Add `steps` to a device step count and `updates` to an update count (one thread).
void launch_advance_counts(hipStream_t s, uint64_t* step, uint64_t steps, uint32_t* updates, uint32_t n_upd);

}  // namespace rs
