/*
 * qtree: quantization-tree transition estimation and backward dynamic
 * programming on one AMD Instinct MI355X (gfx950).
 *
 * Method: Pages & Wilbertz, "GPGPUs in computational finance: Massive
 * parallel computing for American style options" (arXiv:1101.3228).
 *   - Sec. 2: grids Gamma_k of N_k points, Voronoi cells C_i(Gamma_k), the
 *     nearest neighbour projection, transition weights
 *     pi^k_ij = P(X_{k+1} in C_j(Gamma_{k+1}) | X_k in C_i(Gamma_k)) (eq. defPi,
 *     read from layer k to k+1), and the quantized backward dynamic
 *     programming V_k = max(phi_k, sum_j pi^k_ij V_{k+1}(j)).
 *   - Sec. 3: the AR(1) proposition X_{k+1} = A_k X_k + T_k eps_k and the
 *     Monte Carlo estimate of pi^k_ij by counters p^k_ij (Algorithm I,
 *     parallel over paths as Algorithm II).
 *   - Sec. 4: the time-layer parallel estimate that samples (X_k, eps_k)
 *     directly from the marginal of X_k (Algorithm III).
 *
 * Conventions for every call:
 *   - Host pointers are marked "host", device pointers "device".  Device
 *     buffers are owned by the caller (for instance torch tensors); the
 *     library never frees them.  No call allocates device memory except
 *     where its comment says so.
 *   - Arrays are row-major and the layers are concatenated:
 *       grid   : float[sum_k N_k][d], layers k = 0..n
 *       counts : int32[sum_{k<n} N_k N_{k+1}], block k is N_k x N_{k+1}
 *       phi, V : double[n_pay][sum_k N_k]
 *   - Layer 0 is the start point: N_0 = 1 and grid layer 0 = {x_0}.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it unless their comment says otherwise.
 *   - Errors are returned, never raised; qtree_status_string() names them and
 *     qtree_last_error() gives the detail of the last failure on this thread.
 *     Argument checks run on the host before any device work: on an error
 *     return no device work was queued and outputs are untouched.
 *   - Results are bitwise deterministic: counts depend only on (model, grid,
 *     m0, M, seed, contract_id, mode), never on the launch configuration.
 */
#ifndef QTREE_H
#define QTREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QTREE_OK = 0,
  QTREE_EINVAL = 1,      /* bad argument: shape, pointer, non-finite or unsorted grid */
  QTREE_ENOMEM = 2,      /* workspace too small */
  QTREE_EOVERFLOW = 3,   /* a count could exceed int32 (M >= 2^31) or m0 + M > 2^32 */
  QTREE_EDEVICE = 4,     /* a HIP runtime call failed (detail in qtree_last_error) */
  QTREE_EUNSUPPORTED = 5 /* valid request the library does not implement */
} qtree_status;

typedef enum {
  QTREE_LAYERWISE = 0, /* Algorithm III: M pairs (X_k, X_{k+1}) per layer, layers in parallel */
  QTREE_PATHWISE = 1   /* Algorithm I/II: M paths X_0 -> X_n, one thread per path */
} qtree_mode;

/* AR(1) model of the Proposition in Sec. 3, FP32, host arrays:
 *   X_{k+1} = A_k X_k + b_k + T_k eps_k,  eps_k ~ N(0, I_d)   (k = 0..n-1)
 *   X_k     = mu_k + L_k z,               z ~ N(0, I_d)        (k = 0..n)
 * A, T: [n][d][d]; b: [n][d]; mu: [n+1][d]; L: [n+1][d][d]; x0: [d].
 * The marginal form (mu, L) is what the time-layer parallel mode samples. */
typedef struct {
  int32_t d; /* state dimension, 1..3 */
  int32_t n; /* number of transitions; layers 0..n */
  const float *A, *b, *T;
  const float *mu, *L;
  const float *x0;
} qtree_model;

typedef struct qtree_plan qtree_plan; /* opaque host object */

const char *qtree_status_string(qtree_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char *qtree_last_error(void);
/* Library version string. */
const char *qtree_version(void);

/* Bytes of device workspace a plan for this shape needs (d in 1..3,
 * N: host [n+1]) when its counting scratch is to hold `batch_samples`
 * LAYERWISE samples per layer per pass (0: 2^22).  Larger M runs in several
 * passes; a plan uses all the scratch its workspace has room for.  For d = 2
 * it includes the bucket tables of the cell search, 64 bytes per bucket and
 * about 64 buckets per grid point (8 MB for a layer of 2000 points).  Pure
 * host arithmetic. */
qtree_status qtree_workspace_size(int32_t d, int32_t n, const int32_t *N, uint64_t batch_samples,
                                  size_t *bytes);

/* Validate a model and its grids on the host and upload the per-layer tables
 * the kernels read (model coefficients, grid points, 1-D cell midpoints or
 * d >= 2 half norms) into `workspace` (device, >= qtree_workspace_size bytes,
 * owned by the caller and referenced by the plan until it is destroyed).
 * grid: host float[sum N_k][d]; 1-D grids must be strictly increasing, all
 * values finite; N[0] == 1.  Blocks until the upload has finished.
 * *out receives a host object released by qtree_plan_destroy. */
qtree_status qtree_plan_create(const qtree_model *model, const float *grid, const int32_t *N,
                               void *workspace, size_t workspace_bytes, qtree_plan **out);
void qtree_plan_destroy(qtree_plan *plan);
/* Tracing: when `event_after_keys` (a hipEvent_t) is not NULL, LAYERWISE
 * two-pass calls record it on their stream right after each sampling pass
 * (before the histogram pass), so callers can time the two kernels apart. */
qtree_status qtree_plan_trace(qtree_plan *plan, void *event_after_keys);
/* LAYERWISE samples per layer one counting pass holds (0: one-pass atomics only). */
int64_t qtree_plan_batch_samples(const qtree_plan *plan);
/* The 1-D cell search of the LAYERWISE forward and the stratified counts
 * (host query, no device work): *guide_k = the largest number of midpoints
 * that one bucket of a layer's guide table adds (the search is the bucket's
 * first cell plus that many comparisons), or -1 when some layer has no such
 * table within the bound of 4 or the tables do not fit in LDS (then every
 * layer is searched by the breadth-first binary search); *guide_buckets =
 * the largest table (0 with -1).  d >= 2 plans report -1.  Either pointer
 * may be NULL.  EINVAL if plan is NULL. */
qtree_status qtree_plan_cell_search(const qtree_plan *plan, int32_t *guide_k,
                                    int32_t *guide_buckets);
/* The d = 2 bucket geometry of layer k (see QTREE_TUNE_BUCKETS): a point x
 * is in bucket (floor((x_0 - lo[0]) scale[0]), floor((x_1 - lo[1]) scale[1]))
 * (FP32 arithmetic) of the B[0] x B[1] buckets; B = {0, 0} when the layer
 * has no tables (d != 2, or one point).  lo, scale: host float[2]; B: host
 * int32[2].  Reads the layer's record back from the device (blocking). */
qtree_status qtree_plan_buckets(const qtree_plan *plan, int32_t k, float *lo, float *scale,
                                int32_t *B);
/* The candidate count of every bucket of layer k, row-major (bucket (i, j)
 * at i B[1] + j; 0xFFFF: more than 31 candidates, the full scan decides):
 * counts, host uint16[B[0] B[1]] (nothing written when the layer has no
 * tables).  Blocking. */
qtree_status qtree_plan_bucket_counts(const qtree_plan *plan, int32_t k, uint16_t *counts);
/* Shape queries (host). */
int32_t qtree_plan_dim(const qtree_plan *plan);
int32_t qtree_plan_layers(const qtree_plan *plan);
int64_t qtree_plan_count_entries(const qtree_plan *plan); /* sum_{k<n} N_k N_{k+1} */
int64_t qtree_plan_points(const qtree_plan *plan);        /* sum_k N_k */

/* Launch tuning of a plan (results never depend on it).
 *   QTREE_TUNE_CHUNK   : samples per workgroup in LAYERWISE mode (0 = automatic;
 *                        otherwise rounded up to an even number >= 2).
 *   QTREE_TUNE_XCD_MAP : 1 (default) deals the chunks of one layer to one XCD,
 *                        0 uses the plain block order.
 *   QTREE_TUNE_COUNT   : LAYERWISE counting: 0 automatic (two-pass when every
 *                        count block has at most 4096 tiles of 4096 entries and
 *                        the per-chunk sort fits in LDS),
 *                        1 one pass with a device-scope atomic per sample,
 *                        2 two-pass (per-chunk keys grouped by tile, then one
 *                        LDS histogram per tile; uses the workspace scratch).
 *   QTREE_TUNE_GROUPS  : two-pass only: the layers are split into this many
 *                        groups (1..8; 0 = automatic, the default: 4 for
 *                        d = 1, 1 for d >= 2); the histogram pass of a
 *                        group runs on a stream of the plan, concurrently with
 *                        the sampling pass of the next group.  The call still
 *                        completes in order on `stream` (which waits for it).
 *                        A plan used with groups > 1 must not be used from
 *                        two host threads at once.
 *   QTREE_TUNE_ND_SAMPLES : d >= 2 two-pass sampling: samples per lane that
 *                        share each grid record read from LDS, 8 or 4 (default
 *                        8; 4 for a d = 2 plan that has bucket tables).
 *   QTREE_TUNE_TAIL    : with layer groups, the last group's share of the
 *                        layers in percent of each other group's (10..100,
 *                        default 100: equal groups); its histogram pass is
 *                        the one no sampling pass overlaps.
 *   QTREE_TUNE_BUCKETS : d = 2: 1 (default) finds cells through the plan's
 *                        bucket tables (each bucket of a layer's reachable box
 *                        lists every point that can be the FP32 argmin in it,
 *                        the key's rounding included, so the cell is the full
 *                        scan's), 0 scans every point (the brute-force search
 *                        of Sec. 4); used by the LAYERWISE two-pass forward
 *                        and qtree_cells.
 */
typedef enum {
  QTREE_TUNE_CHUNK = 0,
  QTREE_TUNE_XCD_MAP = 1,
  QTREE_TUNE_COUNT = 2,
  QTREE_TUNE_GROUPS = 3,
  QTREE_TUNE_ND_SAMPLES = 4,
  QTREE_TUNE_TAIL = 5,
  QTREE_TUNE_BUCKETS = 6
} qtree_tune_key;
qtree_status qtree_plan_tune(qtree_plan *plan, int32_t key, int64_t value);
/* Current value of a tuning key (-1 for a NULL plan or an unknown key). */
int64_t qtree_plan_get_tune(const qtree_plan *plan, int32_t key);
/* Autotuner of a plan's LAYERWISE forward: times, with HIP events on
 * `stream`, one forward of M samples per layer (seed `seed`, contract 0,
 * written to `counts`, device int32 [entries]) under each candidate --
 * d = 1: one layer group, or 2, 4, 6, 8 groups with the last at 100, 50 or 33
 * percent of the others; d >= 2: 8 or 4 samples per lane, 1 or 2 groups --
 * three runs each (the fastest counts) after one warm-up, and sets the
 * fastest (QTREE_TUNE_GROUPS, _TAIL,
 * _ND_SAMPLES).  *best_ms (may be NULL) receives its time.  Blocks the
 * host until the timings are in.  Counts never depend on the choice. */
qtree_status qtree_plan_autotune(qtree_plan *plan, uint64_t M, uint64_t seed, int32_t *counts,
                                 void *stream, double *best_ms);

/* Monte Carlo transition counts p^k_ij (Sec. 3 Algorithm I/II, Sec. 4
 * Algorithm III) over samples m = m0 .. m0+M-1.
 *   LAYERWISE: sample m of layer k draws z, eps from Philox4x32-10 with key
 *     (seed lo, seed hi) and counter (block(m), k, contract_id, 0), sets
 *     X_k = mu_k + L_k z, X_{k+1} = A_k X_k + b_k + T_k eps and adds one to
 *     counts[k][cell_k(X_k)][cell_{k+1}(X_{k+1})].
 *   PATHWISE: path m starts at x0 in cell 0 of layer 0 and for k = 0..n-1
 *     steps X_{k+1} = A_k X_k + b_k + T_k eps_k (counter (m, k>>s, contract_id, 1))
 *     and adds one to counts[k][i][j] for the cells i, j it leaves and enters.
 * cell_k is the Voronoi cell of Gamma_k: in 1-D the number of FP32 midpoints
 * (x_r + x_{r+1})/2 strictly below the point; in d >= 2 the lowest index
 * minimising the FP32 half-norm form |g|^2/2 - <x, g> of the squared distance.
 * counts: device int32[qtree_plan_count_entries], zeroed and overwritten.
 * Requires M < 2^31 and m0 + M <= 2^32.  Asynchronous on `stream`. */
qtree_status qtree_transitions(const qtree_plan *plan, uint64_t m0, uint64_t M, uint64_t seed,
                               uint32_t contract_id, qtree_mode mode, int32_t *counts,
                               void *stream);

/* As qtree_transitions but adds to `counts` instead of overwriting them:
 * counts over [m0, m0+M) accumulate onto earlier calls, so a run can be split
 * into sample chunks (and resumed) with totals identical to one call. */
qtree_status qtree_transitions_add(const qtree_plan *plan, uint64_t m0, uint64_t M, uint64_t seed,
                                   uint32_t contract_id, qtree_mode mode, int32_t *counts,
                                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the counts
 * of qtree_transitions, bit for bit, with the LAYERWISE two-pass key scratch
 * taken from a fixed device array of the library (QTREE_FIXED_SCRATCH_BYTES
 * per device, held until the process ends) instead of the plan's workspace,
 * so a plan created with batch_samples = 0 still counts in two passes.  The
 * call allocates nothing (no hipMalloc, no stream or event creation: one
 * layer group on `stream`); samples run in as many passes as the array
 * holds.  The array keeps the last call's contents and is shared by every
 * call on the device: calls that overlap in time on one device (different
 * streams or host threads) race and must be serialised by the caller.  The
 * current device must be the plan's.  EUNSUPPORTED (nothing launched) when
 * one chunk of every layer does not fit the array (n (8192 + 4 (tiles + 1))
 * bytes, tiles = the largest layer's ceil(N_k N_{k+1} / 4096)); other errors
 * as qtree_transitions.  PATHWISE calls and plans tuned to one-pass counting
 * use no scratch. */
#define QTREE_FIXED_SCRATCH_BYTES (64u << 20)
qtree_status qtree_transitions_fixed_scratch(const qtree_plan *plan, uint64_t m0, uint64_t M,
                                             uint64_t seed, uint32_t contract_id,
                                             qtree_mode mode, int32_t *counts, void *stream);

/* Quantized backward dynamic programming (Sec. 2), FP64, for n_pay obstacle
 * vectors sharing one set of counts:
 *   V_n = phi_n;  V_k(i) = max(phi_k(i), sum_j c_ij V_{k+1}(j) / p_i),
 *   p_i = sum_j c_ij; a row no sample reached (p_i = 0) has continuation 0.
 * counts: device int32 (as written by qtree_transitions); phi: device
 * double[n_pay][sum N_k] (use -inf for k < n to price a European claim);
 * V: device double[n_pay][sum N_k] output (all layers); 1 <= n_pay <= 2^20,
 * one launch per layer for all payoffs.  If V0_host is not
 * NULL the call copies V_0 of every payoff there and synchronises `stream`
 * before returning; otherwise it is asynchronous. */
qtree_status qtree_bdp(const qtree_plan *plan, const int32_t *counts, const double *phi,
                       int32_t n_pay, double *V, double *V0_host, void *stream);

/* The estimated transition weights pi^k_ij = c_ij / p_i (eq. defPi read
 * from layer k to k+1; Sec. 3: the counters p^k_ij normalised by their row
 * totals), FP64, with the range of the nonzero columns of every row, in a
 * caller-owned device buffer `pi` of qtree_pi_workspace_size bytes
 * (256-byte aligned).  A row that no sample reached gets zero weights (its
 * continuation value is 0, as in qtree_bdp).  Computed once per count set;
 * qtree_bdp_many reads it.  counts: device int32 as written by
 * qtree_transitions.  Asynchronous. */
qtree_status qtree_pi_workspace_size(const qtree_plan *plan, size_t *bytes);
qtree_status qtree_pi(const qtree_plan *plan, const int32_t *counts, void *pi, size_t pi_bytes,
                      void *stream);

/* One contract's obstacle, the parameters of qtree_payoff in one record:
 * kind bit 0 put on S^1 (0) or call on max_a S^a (1), bit 1 European; sigma
 * [d] used; mix: row-major d x d in the first d*d entries, used when
 * has_mix != 0 (else y = x). */
typedef struct {
  double S0, K, r, Tm;
  double sigma[3];
  double mix[9];
  int32_t kind;
  int32_t has_mix;
} qtree_payoff_spec;

/* Quantized BDP (Sec. 2) of n_q contracts on one tree, FP64:
 *   V_n = phi_n,  V_k(i) = max(phi_k(i), sum_j pi^k_ij V_{k+1}(j)),
 * with phi_k the obstacle of qtree_payoff computed from the contract's
 * record where it is needed (never stored), and pi from qtree_pi; one
 * launch prices every contract (64 per workgroup, their value vectors
 * resident on chip through all layers).  specs: device
 * qtree_payoff_spec[n_q] (not validated: non-finite parameters give
 * non-finite prices); V0: device double[n_q] output, V_0 of each contract.
 * Layers of at most 256 points (EUNSUPPORTED beyond).  The prices equal
 * those of qtree_payoff + qtree_bdp up to the rounding of the weights
 * (relative ~1e-15).  Asynchronous. */
qtree_status qtree_bdp_many(const qtree_plan *plan, const void *pi, size_t pi_bytes, int64_t n_q,
                            const qtree_payoff_spec *specs, double *V0, void *stream);

/* The same for many trees in one launch (a tree per number of layers, for
 * instance): tree t (plans[t], its weights pi[t] of pi_bytes[t] bytes from
 * qtree_pi) prices contracts q_begin[t] .. q_begin[t+1] - 1 of specs / V0
 * (q_begin: host int64[n_trees + 1], nondecreasing).  All trees share one
 * dimension; layers of at most 256 points.  The call copies a table of the
 * trees (80 bytes each) into `workspace` (device, >= 80 n_trees bytes,
 * 16-byte aligned), in use until the launch ends.  Workgroups take the trees
 * with the most layers first.  V0 equals qtree_bdp_many tree by tree, bit
 * for bit.  Asynchronous. */
qtree_status qtree_bdp_many_trees(int32_t n_trees, const qtree_plan *const *plans,
                                  const void *const *pi, const size_t *pi_bytes,
                                  const int64_t *q_begin, const qtree_payoff_spec *specs,
                                  double *V0, void *workspace, size_t workspace_bytes,
                                  void *stream);

/* Discounted obstacle on the plan's grid points, FP64, device output
 * phi: double[sum N_k]:  phi_k(x) = exp(-r t_k) payoff(S_{t_k}(x)),
 * t_k = k Tm / n, S^a_t(x) = S0 exp((r - sigma_a^2/2) t + sigma_a y_a) with
 * the Brownian factors y = mix x (Sec. 2: obstacle of the optimal stopping
 * problem on a Brownian state).  mix: host double[d][d] row-major, or NULL
 * for the identity; sqrt(T) I prices maturity T on the grid of a unit-time
 * Brownian motion, sqrt(T) chol(R) adds a correlation R to independent
 * factors.  kind bit 0: 0 put on S^1, 1 call on max_a S^a; bit 1: European
 * (phi_k = -inf for k < n).  sigma: host double[d].  Asynchronous. */
qtree_status qtree_payoff(const qtree_plan *plan, int32_t kind, double S0, double K, double r,
                          double Tm, const double *sigma, const double *mix, double *phi,
                          void *stream);
/* The same for n_pay contracts in one launch per 16 contracts: host arrays
 * kind, S0, K, r, Tm [n_pay], sigma [n_pay][d] and mix [n_pay][d][d] (or
 * NULL); phi: device double[n_pay][sum N_k]. */
qtree_status qtree_payoff_batch(const qtree_plan *plan, int32_t n_pay, const int32_t *kind,
                                const double *S0, const double *K, const double *r,
                                const double *Tm, const double *sigma, const double *mix,
                                double *phi, void *stream);

/* Forward on the sum of the factors, the obstacle of the swing contract on
 * the Gaussian factor model (Sec. 3: S_t = s0 exp(sum_a sigma_a X^a_t -
 * mu_t / 2)), FP64, device output v: double[sum N_k]:
 *   v_k(x) = exp(-r t_k) (S0 exp(s_k(x) - w . mu_k - var_k / 2) - K),
 *   s_k(x) = w . x,  w = mix' sigma,  var_k = |L_k' w|^2,
 * with the plan's marginal X_k = mu_k + L_k z, so that E S_k = S0 (no
 * positive part).  sigma: host double[d]; mix: host double[d][d] or NULL
 * (identity).  t_k = k Tm / n.  Asynchronous. */
qtree_status qtree_payoff_forward(const qtree_plan *plan, double S0, double K, double r,
                                  double Tm, const double *sigma, const double *mix, double *v,
                                  void *stream);

/* Swing option on the tree (Sec. 2: the stochastic control problem with
 * volume constraints, whose optimal control is bang-bang), FP64.  Dates
 * k = 0..n-1, q_k in {0, 1}, sum_k q_k in [Qmin, Qmax] (0 <= Qmin <= Qmax
 * <= n, Qmax <= 2046).  State: the volume c consumed before date k;
 *   P_n(c) = 0 for Qmin <= c <= Qmax, -inf otherwise,
 *   P_k(i, c) = max over x in {0, 1} with c + x <= Qmax and
 *               c + x + (n - k - 1) >= Qmin of x v_k(i) + cont_k(i, c + x),
 *   cont_k(i, c') = sum_j c_ij P_{k+1}(j, c') / p_i (0 for a row no sample
 *   reached), -inf where no x is feasible.
 * counts: as written by qtree_transitions; v: device double[sum N_k]
 * (layer n unused), e.g. from qtree_payoff_forward; P: device
 * double[sum N_k][Qmax + 1] output (grid point major: the volume levels
 * of a point are contiguous; all layers).  If P0_host is not NULL the call
 * copies P_0(0, 0) there and synchronises `stream`.  One launch per layer. */
qtree_status qtree_swing(const qtree_plan *plan, const int32_t *counts, const double *v,
                         int32_t Qmin, int32_t Qmax, double *P, double *P0_host, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many contracts with uneven n and N_k priced together.
 * Each contract names a plan (model + grids, created as above), the samples
 * per layer M (LAYERWISE, from sample 0), its seed and Philox contract id,
 * its count buffer, its obstacles phi [n_pay][points] and its value buffer V
 * [n_pay][points] (all device).  qtree_batch_plan builds a device work list
 * of (contract, layer, chunk range) units sorted longest first; a run then
 * issues, per scratch group, two sampling launches (the d >= 2 units, then
 * the 1-D units) with one workgroup per chunk of the list, in list order (the
 * costly units are dispatched first), and one histogram launch, and then
 * one BDP launch in which each workgroup walks all layers of one contract for
 * up to 16 of its payoffs.  Counts and values are bit-for-bit / 1e-9 the
 * ones of qtree_transitions + qtree_bdp per contract (same Philox counters).
 * qtree_batch_plan allocates the batch's device tables and its key scratch
 * (`scratch_bytes`, 0 = 4 GiB; contracts are grouped so that each group
 * fits) -- the only call besides the tuner that allocates device memory.
 * An allocation that fails returns ENOMEM (nothing is kept); for tests of
 * that path, QTREE_FAULT_ALLOC=k (k >= 1) in the environment makes the k-th
 * device allocation of a qtree_batch_plan call fail that way.
 * flags bit 0: capture the run sequence into a hipGraph after the first run
 * and replay it from then on (needs a non-NULL stream).
 *
 * Autotuner.  A run's launch configuration (never its results) is a code:
 * bit 0 set = 4 instead of 8 samples per lane share each grid read in the
 * d >= 2 sampling launch; bit 1 = the 1-D sampling launch runs on a second
 * stream beside the d >= 2 one instead of after it; bits 8-15 = at most that
 * many workgroups per CU for the d >= 2 launch (0: its occupancy limit).
 * With a tuner, the first run of a batch whose shape signature the tuner
 * does not know times the forward launches of every candidate configuration
 * (both sample counts, serial and overlapped launches when the batch has
 * both kinds, the occupancy limit and one workgroup per CU below it) with
 * HIP events on the run's stream, after one warm-up, and keeps the fastest;
 * that run blocks the host until the timings are in.  The tuner caches
 * (signature, code, milliseconds) in a text file (path given, else
 * $QTREE_TUNE_CACHE, else memory only), so later batches of the same shape
 * skip the timing.  Without a tuner the default code 0 is used.
 * ---------------------------------------------------------------------- */
typedef struct {
  const qtree_plan *plan;
  uint64_t M;
  uint64_t seed;
  uint32_t contract_id;
  int32_t *counts;
  const double *phi;
  int32_t n_pay;
  double *V;
} qtree_contract;

typedef struct qtree_tuner qtree_tuner;
typedef struct qtree_batch qtree_batch;

qtree_status qtree_tuner_create(const char *cache_path, qtree_tuner **out);
void qtree_tuner_destroy(qtree_tuner *tuner);
/* Cached configuration code for a batch signature, -1 if none. */
int32_t qtree_tuner_lookup(const qtree_tuner *tuner, const char *signature);

qtree_status qtree_batch_plan(const qtree_contract *contracts, int32_t n, qtree_tuner *tuner,
                              size_t scratch_bytes, uint32_t flags, qtree_batch **out);
/* Run the batch on `stream`; if V0_host (double[sum n_pay], contracts in
 * order) is not NULL, copy every V_0 there and synchronise. */
qtree_status qtree_batch_run(qtree_batch *batch, double *V0_host, void *stream);
/* Work units, histogram tiles, scratch groups, and the workgroups per CU of
 * the 1-D and of the d >= 2 sampling launch under the current configuration
 * (any pointer may be NULL). */
qtree_status qtree_batch_info(const qtree_batch *batch, int64_t *units, int64_t *tiles,
                              int32_t *groups, int32_t *per_cu_1d, int32_t *per_cu_nd);
/* The configuration code in use, the forward time the tuner measured for it
 * (ms; 0 if not measured) and how many candidates this batch timed (0 when
 * the code came from the cache or from qtree_batch_set_config). */
qtree_status qtree_batch_tuning(const qtree_batch *batch, int32_t *config, double *ms,
                                int32_t *timed);
/* Use configuration `config` from now on (the tuner is skipped; a captured
 * graph is dropped and captured again on the next run).  EINVAL for an
 * unknown code. */
qtree_status qtree_batch_set_config(qtree_batch *batch, int32_t config);
const char *qtree_batch_signature(const qtree_batch *batch);
void qtree_batch_destroy(qtree_batch *batch);

/* Per-sample diagnostics, computed by the same device code as the forward
 * kernels, so tests can compare intermediate results one by one.
 * qtree_box_muller: z0/z1[i] = Box-Muller transform of the Philox words
 *   (ra[i], rb[i]) (device arrays of `count` elements).
 * qtree_layer_samples: X_k and X_{k+1} of LAYERWISE samples m0..m0+count-1
 *   of layer k (0 <= k < n), device float[count][d] each.
 * qtree_cells: Voronoi cell in layer k (0 <= k <= n) of `count` device points
 *   x (float[count][d]); cell: device int32[count].  d >= 2: the forward's
 *   search -- with bucket tables (d = 2, QTREE_TUNE_BUCKETS on) each point's
 *   bucket list, else the tiled scan over the layer's records staged in LDS,
 *   eight points per lane (the brute-force search of Sec. 4); d = 1: the
 *   binary search over the layer's sorted midpoints.
 * All asynchronous on `stream`. */
qtree_status qtree_box_muller(const uint32_t *ra, const uint32_t *rb, int64_t count, float *z0,
                              float *z1, void *stream);
qtree_status qtree_layer_samples(const qtree_plan *plan, int32_t k, uint64_t m0, int64_t count,
                                 uint64_t seed, uint32_t contract_id, float *x, float *y,
                                 void *stream);
qtree_status qtree_cells(const qtree_plan *plan, int32_t k, const float *x, int64_t count,
                         int32_t *cell, void *stream);

/* The quarter-disc experiment of the generator comparison (Sec. 3, Table
 * rngs) on the library's Philox4x32-10: for repetitions rep0 .. rep0+reps-1
 * adds to inside[rep - rep0] (device uint64, caller-zeroed) the number of
 * the npts points (npts even, <= 2^33) of that repetition with
 * u^2 + v^2 <= 1, point h of block i being u = (r_{2h} >> 8) 2^-24,
 * v = (r_{2h+1} >> 8) 2^-24 of Philox(counter (i, rep, 0, 3), key = seed).
 * The estimate is 4 inside / npts.  Asynchronous. */
qtree_status qtree_pi_quarter_disc(uint64_t seed, uint32_t rep0, int32_t reps, uint64_t npts,
                                   uint64_t *inside, void *stream);

/* Stratified time-layer counts (d = 1; a variance reduction of Algorithm
 * III's estimate, not in the paper).  For every layer k < n and every cell i
 * of Gamma_k, M_i samples of X_k are drawn from its marginal N(mu_k, L_k^2)
 * conditioned on the cell: M_i = M (alloc 0, equal allocation) or
 * max(1, rint(M (e_{i+1} - e_i))) in FP64 (alloc 1, proportional allocation;
 * qtree_strat_row returns M_i, -1 for a bad request).  Sample t of row i
 * takes Philox counter (t, k, contract_id, 4 + 256 i), u = (k52 + 1/2) 2^-52
 * with k52 = (r0 >> 12) 2^32 + r1, p = e_i + u (e_{i+1} - e_i) (kept inside
 * [2^-1074, 1 - 2^-53]) for the marginal probabilities e below the cell
 * edges (e_0 = 0, e_{r+1} = erfc(-a / sqrt 2) / 2 at a = (m_r - mu_k) / L_k
 * for the FP32 midpoints m_r, e_N = 1, computed at plan creation), z =
 * Phi^-1(p) by Wichura's algorithm AS 241 in FP64, X_k = fma(L_k, (float)z,
 * mu_k); eps = the first Box-Muller normal of words (2, 3); X_{k+1} =
 * fma(T_k, eps, fma(A_k, X_k, b_k)) and its cell j in Gamma_{k+1} by the
 * tree's rule.  counts[k][i][j] = the number of row-i samples in cell j:
 * row i sums to M_i, so pi^k_ij = counts / M_i and qtree_bdp applies
 * unchanged.  counts: device int32[entries], overwritten entirely.
 * workspace: device, at least qtree_strat_workspace_size(plan, M, alloc)
 * bytes (the work list: tiles of 4 rows cut into segments of at most 65536
 * samples; 0 for a bad request), caller-owned, in use until the call's work
 * on `stream` ends.
 * Errors (before any device work): EUNSUPPORTED (d != 1, N above 8192),
 * EOVERFLOW (M outside 1 .. 2^31 - 1), EINVAL (NULL, alloc not 0 or 1,
 * L_k <= 0 on a layer with N_k > 1), ENOMEM (workspace too small).
 * Asynchronous on `stream`.
 * qtree_strat_samples: (X_k, X_{k+1}) of samples t0 .. t0+count-1 of row i
 * of layer k (t0 + count <= M_i), device float[count] each (a diagnostic). */
size_t qtree_strat_workspace_size(const qtree_plan *plan, uint64_t M, int32_t alloc);
qtree_status qtree_transitions_stratified(const qtree_plan *plan, uint64_t M, int32_t alloc,
                                          uint64_t seed, uint32_t contract_id, int32_t *counts,
                                          void *workspace, size_t workspace_bytes,
                                          void *stream);
int64_t qtree_strat_row(const qtree_plan *plan, int32_t k, int32_t i, uint64_t M, int32_t alloc);
qtree_status qtree_strat_samples(const qtree_plan *plan, int32_t k, int32_t i, uint64_t M,
                                 int32_t alloc, uint64_t t0, int64_t count, uint64_t seed,
                                 uint32_t contract_id, float *x, float *y, void *stream);

/* Banded stratified counts (d = 1; not in the paper): the counts of
 * qtree_transitions_stratified keeping, of row i of layer k, only the band
 * of columns its samples can reach, packed row after row, instead of the
 * dense N_k x N_{k+1} blocks.  Rows r = sum_{l<k} N_l + i, r < R = sum_{k<n}
 * N_k.  The band of a row comes from the plan: X_k lies in cell i (the end
 * cells reach mu_k - 38.5 L_k and mu_k + 8.3 L_k, the quantiles of the
 * clamped probabilities) and eps within +-5.769 (the largest Box-Muller
 * normal), so X_{k+1} = A_k X_k + b_k + T_k eps lies in an interval whose
 * cells of layer k+1, widened for FP32 rounding, form the band.
 * qtree_strat_band (host query): *values = the packed length; row_off
 *   (host int64[R + 1] or NULL): row r's columns row_lo[r] + w,
 *   w < row_off[r + 1] - row_off[r], are stored at band[row_off[r] + w];
 *   row_lo (host int32[R] or NULL).  EUNSUPPORTED for d != 1.
 * qtree_transitions_stratified_banded: as qtree_transitions_stratified
 *   with band: device int32[values], overwritten entirely; *overflow
 *   (device uint32, zeroed by the call) receives the number of samples
 *   that fell outside their row's band (0 unless the band is wrong; those
 *   samples are not stored).  Same workspace and errors.  Asynchronous.
 * qtree_bdp_banded: qtree_bdp on banded counts (the row total is the sum of
 *   the band).  EUNSUPPORTED for d != 1. */
qtree_status qtree_strat_band(const qtree_plan *plan, int64_t *values, int64_t *row_off,
                              int32_t *row_lo);
qtree_status qtree_transitions_stratified_banded(const qtree_plan *plan, uint64_t M,
                                                 int32_t alloc, uint64_t seed,
                                                 uint32_t contract_id, int32_t *band,
                                                 uint32_t *overflow, void *workspace,
                                                 size_t workspace_bytes, void *stream);
qtree_status qtree_bdp_banded(const qtree_plan *plan, const int32_t *band, const double *phi,
                              int32_t n_pay, double *V, double *V0_host, void *stream);

/* Grid optimization (Sec. 2, eq. Qerr): `steps` randomized Lloyd steps that
 * lower the quadratic quantization error E min_i |X - x_i|^2 of X = L z,
 * z ~ N(0, I_d).  A step draws M samples (sample m of step t: Philox counter
 * (m, fresh ? t : 0, 0, 2), key = seed; z_0, z_1 from Box-Muller of words
 * (0, 1), z_2 from words (2, 3); X_r = sum_c L[r][c] z_c as a chain of fused
 * multiply-adds from 0), assigns each to its cell by the tree's rule (d = 1:
 * the number of FP32 midpoints strictly below; d >= 2: the lowest-index
 * minimum of |g|^2/2 - <X, g>), and moves every point to the mean of its
 * cell's samples (a cell without samples keeps its point).  Cell sums are
 * exact integers (rint(x 2^24) per coordinate), so the result does not
 * depend on the order of summation; new point = (sum 2^-24) / count in
 * FP64, rounded to FP32.
 *   d: 1..3; N: 1..8192 (d = 1) or 1..2048 (d = 2, 3).
 *   L: host float[d][d], row-major; every row's absolute sum <= 64 / 5.77.
 *   grid0: host float[N][d], the start grid, coordinates within [-64, 64]
 *     (d = 1: strictly increasing).
 *   grid: device float[N][d], receives the result (written from grid0 first).
 *   M: samples per step, 1 .. 2^31 - 1.  steps >= 1.
 *   fresh: nonzero draws new samples every step; zero reuses the samples of
 *     step 0 (Lloyd's method on a fixed empirical measure: the distortion
 *     does not increase).
 *   distortion: device double[steps] or NULL: entry t = the mean squared
 *     distance of step t's samples to their cell's point before the move.
 *   workspace: device, qtree_lloyd_workspace_size(d, N) bytes, caller-owned.
 * Errors (before any device work): EINVAL (bad d, NULL, non-finite or
 * unsorted grid0, steps < 1), EOVERFLOW (M, L or grid0 out of range),
 * ENOMEM (workspace too small), EUNSUPPORTED (N above the limit).
 * Asynchronous on `stream` (grid0 is copied before the call returns). */
size_t qtree_lloyd_workspace_size(int32_t d, int32_t N);
qtree_status qtree_lloyd(int32_t d, int32_t N, const float *L, const float *grid0, float *grid,
                         uint64_t M, int32_t steps, uint64_t seed, int32_t fresh,
                         double *distortion, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Grids for marginals of any law (Sec. 2: optimal grids where they are
 * known, otherwise sub-optimal grids matching the first two moments of X_k;
 * the Lloyd condition of eq. Qerr on an empirical measure).  A sample is
 * admissible when every coordinate is finite and within [-64, 64]; the
 * others are skipped (and counted by qtree_lloyd_samples).
 *
 * qtree_lloyd_samples: `steps` Lloyd steps as in qtree_lloyd, but step t
 *   takes the window of `batch` samples (t batch + j) mod M, j < batch, of
 *   the caller's set x (device float[M][d], row-major, M <= 2^40), and moves
 *   each point to its cell's sample mean (gamma = 1) or the fraction gamma
 *   of the way there, new = g + gamma (mean - g) in FP64 rounded once
 *   (0 < gamma < 1: the batch form of the competitive-learning step).
 *   grid0: host float[N][d] (limits as qtree_lloyd); grid: device output;
 *   batch: 1 .. 2^31 - 1; distortion: device double[steps] or NULL, entry t
 *   = mean of |x - g|^2 over the window's admissible samples before the move
 *   (0 if none); rejected: device int64 or NULL, the inadmissible samples
 *   met over all steps; workspace: qtree_lloyd_workspace_size(d, N) bytes.
 *   Errors as qtree_lloyd, and EINVAL for gamma outside (0, 1] or M = 0.
 *   Asynchronous on `stream`.
 * qtree_sample_moments: exact integer moment sums of the admissible samples
 *   of x (device float[M][d], M <= 2^31): sums (device int64[1 + d + d d])
 *   = count, s1[r] = sum rint(x_r 2^24), s2[r][c] = sum rint(x_r x_c 2^16)
 *   (the product exact in FP64); order independent.  Asynchronous.
 * qtree_moment_grid: from such sums, mean = s1 2^-24 / count, covariance
 *   = s2 2^-16 / count - mean mean', its lower Cholesky factor (column by
 *   column; a non-positive pivot gives a zero column) in FP64, and
 *   grid[i] = mean + chol base[i] (FP64, rounded once).  base, grid: device
 *   float[N][d]; moments: device double[d + 2 d d] (mean, covariance,
 *   factor) or NULL.  A zero count gives a zero mean and factor.
 *   Asynchronous. */
qtree_status qtree_lloyd_samples(int32_t d, int32_t N, const float *grid0, float *grid,
                                 const float *x, uint64_t M, uint64_t batch, int32_t steps,
                                 double gamma, double *distortion, int64_t *rejected,
                                 void *workspace, size_t workspace_bytes, void *stream);
qtree_status qtree_sample_moments(int32_t d, const float *x, uint64_t M, int64_t *sums,
                                  void *stream);
qtree_status qtree_moment_grid(int32_t d, const int64_t *sums, const float *base, int32_t N,
                               float *grid, double *moments, void *stream);

/* Host helpers for inputs (FP64, host memory, no device work). */
/* 1-D quadratic-optimal quantizer of N(0,1) with N points (Sec. 2,
 * eq. Qerr): stationary grid of Lloyd's method, out: double[N], ascending. */
qtree_status qtree_gauss_quantizer(int32_t N, double *out);

#ifdef __cplusplus
}
#endif
#endif /* QTREE_H */
