/*
 * Oracle for the quantization-tree forward step and its backward dynamic
 * programming (Pages & Wilbertz, "GPGPUs in computational finance: Massive
 * parallel computing for American style options", arXiv:1101.3228).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial-per-sample CPU
 * implementation written from the paper's definitions.  Only tests/, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source, header, table or constant generator with the GPU
 * library: every constant below is retyped from its mathematical definition.
 *
 * Layouts (all host memory, row-major):
 *   grid   : float[sum_k N_k][d], layers concatenated k = 0..n
 *   counts : int32[sum_{k<n} N_k*N_{k+1}], counts[k] is the N_k x N_{k+1}
 *            block of layer k -> k+1, blocks concatenated k = 0..n-1
 *   model  : A,T [n][d][d]; b [n][d]; mu [n+1][d]; L [n+1][d][d]; x0 [d]
 *            X_{k+1} = A_k X_k + b_k + T_k eps_k   (Proposition, Sec. 3)
 *            X_k    ~ mu_k + L_k z               (marginal, Algorithm III)
 */
#ifndef QTREE_ORACLE_H
#define QTREE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t d, n;
  const float *A, *b, *T;
  const float *mu, *L;
  const float *x0;
} oracle_model;

enum { ORACLE_LAYERWISE = 0, ORACLE_PATHWISE = 1 };

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* ln(K * 2^-24) for K in [1, 2^24]. */
float oracle_ln_u24(uint32_t K);
/* sin and cos of 2*pi*J*2^-24 for J in [0, 2^24). */
void oracle_sincos_2pi_u24(uint32_t J, float *s, float *c);
/* Box-Muller pair from two Philox words. */
void oracle_box_muller(uint32_t ra, uint32_t rb, float *z0, float *z1);
/* LAYERWISE sample m of layer k: X_k and X_{k+1} (Algorithm III). */
void oracle_layer_pair(const oracle_model *mdl, int32_t k, uint64_t m, uint64_t seed,
                       uint32_t contract, float *xk, float *xk1);
/* PATHWISE innovation eps_k of path m (Algorithm I / II). */
void oracle_path_noise(int32_t d, int32_t k, uint64_t m, uint64_t seed, uint32_t contract,
                       float *eps);
/* Voronoi cell of x in a grid of N points (nearest neighbour projection). */
int32_t oracle_cell(const float *grid_k, int32_t N, int32_t d, const float *x);
/* Transition counts over samples (or paths) m0 .. m0+M-1; counts overwritten.
   Returns 0 on success, nonzero on invalid arguments. */
int oracle_transitions(const oracle_model *mdl, const float *grid, const int32_t *N,
                       uint64_t m0, uint64_t M, uint64_t seed, uint32_t contract,
                       int32_t mode, int32_t *counts, int32_t nthreads);
/* Backward dynamic programming on the tree, FP64.  phi: [n_pay][sum N_k];
   V_all (optional): [n_pay][sum N_k]; V0: [n_pay].  Returns the number of
   empty source rows (p_i = 0) met, summed over payoffs. */
int64_t oracle_bdp(const int32_t *counts, const int32_t *N, int32_t n, const double *phi,
                   int32_t n_pay, double *V_all, double *V0);
/* Discounted obstacle phi_k(x) = exp(-r t_k) * payoff(S_{t_k}(x)), t_k = k*Tm/n.
   The Brownian factors are y = mix x (mix: [d][d] row-major, FP64; NULL is
   the identity), y_a = sum_b mix[a][b] x_b summed in order of b.
   kind bit 0 clear: put (K - S)^+ on S = S0 exp((r - sigma^2/2) t + sigma y_0).
   kind bit 0 set  : call on the max of d assets S^a = S0 exp((r - sigma_a^2/2) t + sigma_a y_a).
   kind bit 1 set  : European, phi_k = -inf for k < n (the max in the BDP then
                     always takes the continuation value). */
void oracle_payoff(int32_t kind, int32_t d, int32_t n, const int32_t *N, const float *grid,
                   double S0, double K, double r, double Tm, const double *sigma,
                   const double *mix, double *phi);

/* Forward on the sum of the factors (obstacle of the swing contract on the
   2-factor model, Sec. 3): with y = mix x (mix NULL: identity) and
   s_k = sum_a sigma_a y_a,
     v_k(x) = exp(-r t_k) (S0 exp(s_k - sigma' mix mu_k - var_k / 2) - K),
   var_k = |L_k' mix' sigma|^2 the variance of s_k under the marginal law
   X_k = mu_k + L_k z, so that E S_k = S0.  mu: [n+1][d], L: [n+1][d][d]
   (FP32 model inputs), t_k = k Tm / n.  No positive part. */
void oracle_forward_payoff(int32_t d, int32_t n, const int32_t *N, const float *grid,
                           const float *mu, const float *L, double S0, double K, double r,
                           double Tm, const double *sigma, const double *mix, double *v);

/* Swing option on the tree (Sec. 2: the stochastic control problem with a
   bang-bang control): exercise dates k = 0..n-1, q_k in {0, 1}, total
   consumption in [Qmin, Qmax] (0 <= Qmin <= Qmax <= n).  The state is the
   consumption c used before date k; x in {0, 1} is feasible at (k, c) when
   c + x <= Qmax and c + x + (n - k - 1) >= Qmin.
     P_n(c)   = 0 for Qmin <= c <= Qmax, -inf otherwise,
     P_k(i,c) = max over feasible x of  x v_k(i) + cont_k(i, c + x),
     cont_k(i, c') = sum_j c_ij P_{k+1}(j, c') / p_i   (0 for an empty row),
   -inf where no x is feasible.  v: [sum N_k] (layer n unused).  P_all
   (optional): [Qmax + 1][sum N_k].  Returns P_0(0, 0). */
double oracle_swing(const int32_t *counts, const int32_t *N, int32_t n, const double *v,
                    int32_t Qmin, int32_t Qmax, double *P_all);

/* Bulk helpers for tests. */
void oracle_ln_u24_bulk(uint32_t K0, int64_t count, float *out);
void oracle_sincos_bulk(uint32_t J0, int64_t count, float *s, float *c);
void oracle_box_muller_bulk(const uint32_t *ra, const uint32_t *rb, int64_t count, float *z0,
                            float *z1);
void oracle_philox_bulk(const uint32_t *ctr, const uint32_t key[2], int64_t count,
                        uint32_t *out);
void oracle_layer_pairs_bulk(const oracle_model *mdl, int32_t k, uint64_t m0, int64_t count,
                             uint64_t seed, uint32_t contract, float *xk, float *xk1);
double oracle_pi_estimate(uint64_t seed, uint32_t rep, uint64_t npts);
/* Cells of count points x[count][d] in one grid of N points. */
void oracle_cells_bulk(const float *grid_k, int32_t N, int32_t d, const float *x, int64_t count,
                       int32_t *out);
/* Counts of the single layer k -> k+1 (Algorithm III) over samples
   m0..m0+M-1; counts_k: int32[N_k][N_{k+1}], overwritten. */
int oracle_layer_counts(const oracle_model *mdl, const float *grid, const int32_t *N, int32_t k,
                        uint64_t m0, uint64_t M, uint64_t seed, uint32_t contract,
                        int32_t *counts_k, int32_t nthreads);

/* Randomized Lloyd iteration for eq. Qerr of X = L z (Sec. 2): `iters`
   steps of M samples each over grid[N][d] (in: start, out: result);
   distortion[iters] (optional) = the mean squared distance before each
   step.  Returns 0, or -1 when memory runs out. */
void oracle_lloyd_sample(int32_t d, const float *L, uint64_t seed, int32_t fresh, int32_t it,
                         uint64_t m, float *x);
int oracle_lloyd(int32_t d, int32_t N, const float *L, float *grid, uint64_t M, int32_t iters,
                 uint64_t seed, int32_t fresh, double *distortion);

/* Grids from samples of a marginal of any law (Sec. 2: grids matching the
   first two moments of X_k when no optimal grid is available; the Lloyd
   stationarity condition of eq. Qerr on an empirical measure).  A sample is
   admissible when every coordinate is finite and within [-64, 64]; the
   others are skipped and counted.
   oracle_sample_moments: exact integer sums s1[c] = sum rint(x_c 2^24),
     s2[r d + c] = sum rint(x_r x_c 2^16) over the admissible samples of
     x[M][d]; returns their number.
   oracle_moment_map: mean, covariance and lower Cholesky factor (FP64) from
     those sums, and grid[i] = mean + chol base[i] (FP64, rounded once);
     moments[d + 2 d d] = mean, covariance, factor.
   oracle_lloyd_empirical: `steps` steps over windows of `batch` samples
     (step t takes samples (t batch + j) mod M, j < batch): cells by the
     tree's rule, exact cell sums, new point = mean (gamma == 1) or
     g + gamma (mean - g) (0 < gamma < 1), a cell without samples keeps its
     point; distortion[t] = mean squared distance of the window's admissible
     samples before the move; rejected = inadmissible samples met. */
int64_t oracle_sample_moments(int32_t d, const float *x, int64_t M, int64_t *s1, int64_t *s2);
void oracle_moment_map(int32_t d, int64_t count, const int64_t *s1, const int64_t *s2,
                       const float *base, int32_t N, float *grid, double *moments);
int oracle_lloyd_empirical(int32_t d, int32_t N, float *grid, const float *x, int64_t M,
                           int64_t batch, int32_t steps, double gamma, double *distortion,
                           int64_t *rejected);

/* Stratified time-layer estimate (d = 1, not in the paper): ln in FP64, the
   normal quantile (AS 241), the cell-edge probabilities of a layer, the
   samples of a row (equal or proportional allocation), one stratified pair,
   and the counts (row i sums to its sample count). */
double oracle_ln64(double x);
double oracle_ppnd16(double p);
void oracle_strat_edges(const float *g, int32_t N, float mu, float L, double *e);
int64_t oracle_strat_row(const double *e, int32_t i, uint64_t M, int32_t alloc);
void oracle_strat_pair(const oracle_model *mdl, int32_t k, const double *e, int32_t i,
                       uint64_t t, uint64_t seed, uint32_t contract, float *x, float *y);
int oracle_transitions_stratified(const oracle_model *mdl, const float *grid, const int32_t *N,
                                  uint64_t M, int32_t alloc, uint64_t seed, uint32_t contract,
                                  int32_t *counts);

#ifdef __cplusplus
}
#endif
#endif
