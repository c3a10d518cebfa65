/*
 * Driver for an AddressSanitizer + UndefinedBehaviorSanitizer build of the
 * oracle (tests/test_oracle_sanitize.py compiles it with oracle/oracle.c and
 * runs it on the CPU).  It calls every oracle entry point on small inputs of
 * each dimension and mode, checks the invariants that need no reference
 * (every layer's counts sum to the sample count, pathwise flow
 * conservation, a row-stochastic BDP is bounded by the payoff range), and
 * exits 0.  Any out-of-bounds access, leak, signed overflow or misaligned
 * access aborts the run with a sanitizer report.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      exit(1);                                                     \
    }                                                              \
  } while (0)

/* Brownian model X_k = W_{k/n} in d dimensions (independent factors). */
typedef struct {
  float *A, *b, *T, *mu, *L, *x0;
  oracle_model m;
} bm;

static void bm_make(bm *s, int d, int n) {
  s->A = calloc((size_t)n * d * d, sizeof(float));
  s->b = calloc((size_t)n * d, sizeof(float));
  s->T = calloc((size_t)n * d * d, sizeof(float));
  s->mu = calloc((size_t)(n + 1) * d, sizeof(float));
  s->L = calloc((size_t)(n + 1) * d * d, sizeof(float));
  s->x0 = calloc((size_t)d, sizeof(float));
  for (int k = 0; k <= n; ++k)
    for (int c = 0; c < d; ++c) {
      if (k < n) {
        s->A[(size_t)k * d * d + c * d + c] = 1.0f;
        s->T[(size_t)k * d * d + c * d + c] = sqrtf(1.0f / n);
      }
      s->L[(size_t)k * d * d + c * d + c] = sqrtf((float)k / n);
    }
  oracle_model m = {d, n, s->A, s->b, s->T, s->mu, s->L, s->x0};
  s->m = m;
}

static void bm_free(bm *s) {
  free(s->A); free(s->b); free(s->T); free(s->mu); free(s->L); free(s->x0);
}

/* Layer grids: layer 0 = {0}; layer k = sqrt(k/n) times a fixed sorted set
   of points per axis (a product grid for d >= 2). */
static float *grid_make(int d, int n, int side, int32_t *N, int64_t *points) {
  int per = 1;
  for (int c = 0; c < d; ++c) per *= side;
  N[0] = 1;
  for (int k = 1; k <= n; ++k) N[k] = per;
  *points = 1 + (int64_t)n * per;
  float *g = calloc((size_t)*points * d, sizeof(float));
  for (int k = 1; k <= n; ++k) {
    float s = sqrtf((float)k / n);
    for (int p = 0; p < per; ++p) {
      int q = p;
      for (int c = d - 1; c >= 0; --c) {
        int a = q % side;
        q /= side;
        g[((size_t)1 + (size_t)(k - 1) * per + p) * d + c] = s * (-2.0f + 4.0f * a / (side - 1));
      }
    }
  }
  return g;
}

static int64_t sum_block(const int32_t *c, int64_t len) {
  int64_t s = 0;
  for (int64_t i = 0; i < len; ++i) s += c[i];
  return s;
}

static void run_dim(int d) {
  const int n = 4, side = d == 1 ? 9 : (d == 2 ? 4 : 3);
  const uint64_t M = 3001;
  bm s;
  bm_make(&s, d, n);
  int32_t N[5];
  int64_t P;
  float *g = grid_make(d, n, side, N, &P);
  int64_t entries = 0, off[5];
  for (int k = 0; k < n; ++k) {
    off[k] = entries;
    entries += (int64_t)N[k] * N[k + 1];
  }
  int32_t *c = calloc((size_t)entries, sizeof(int32_t));
  int32_t *c2 = calloc((size_t)entries, sizeof(int32_t));
  for (int mode = 0; mode <= 1; ++mode)
    for (int th = 1; th <= 3; th += 2) {
      CHECK(oracle_transitions(&s.m, g, N, 5, M, 77, 2, mode, c, th) == 0);
      for (int k = 0; k < n; ++k) CHECK(sum_block(c + off[k], (int64_t)N[k] * N[k + 1]) == (int64_t)M);
      if (mode == ORACLE_PATHWISE)
        for (int k = 0; k + 1 < n; ++k)
          for (int j = 0; j < N[k + 1]; ++j) {
            int64_t in = 0, out = 0;
            for (int i = 0; i < N[k]; ++i) in += c[off[k] + (int64_t)i * N[k + 1] + j];
            for (int l = 0; l < N[k + 2]; ++l) out += c[off[k + 1] + (int64_t)j * N[k + 2] + l];
            CHECK(in == out);
          }
    }
  CHECK(oracle_transitions(&s.m, g, N, 5, M, 77, 2, ORACLE_LAYERWISE, c, 1) == 0);
  for (int k = 0; k < n; ++k) {
    CHECK(oracle_layer_counts(&s.m, g, N, k, 5, M, 77, 2, c2, 3) == 0);
    CHECK(memcmp(c2, c + off[k], sizeof(int32_t) * (size_t)N[k] * N[k + 1]) == 0);
  }
  CHECK(oracle_layer_counts(&s.m, g, N, n, 0, 10, 1, 0, c2, 1) != 0);
  CHECK(oracle_transitions(&s.m, g, N, 0, 1ull << 31, 1, 0, 0, c, 1) != 0);

  /* cells of the samples of one layer */
  float *x = calloc((size_t)M * d, sizeof(float)), *y = calloc((size_t)M * d, sizeof(float));
  int32_t *cell = calloc((size_t)M, sizeof(int32_t));
  oracle_layer_pairs_bulk(&s.m, 2, 0, (int64_t)M, 77, 2, x, y);
  oracle_cells_bulk(g + ((size_t)1 + (size_t)N[1]) * d, N[2], d, x, (int64_t)M, cell);
  for (uint64_t m = 0; m < M; ++m) CHECK(cell[m] >= 0 && cell[m] < N[2]);

  /* obstacles and the backward step */
  double *phi = calloc((size_t)2 * P, sizeof(double)), *V = calloc((size_t)2 * P, sizeof(double));
  double V0[2], sigma[3] = {0.2, 0.3, 0.25}, mix[9] = {1, 0, 0, 0.3, 0.95, 0, 0.1, 0.2, 0.97};
  oracle_payoff(d == 1 ? 0 : 1, d, n, N, g, 100.0, 100.0, 0.05, 1.0, sigma, NULL, phi);
  oracle_payoff((d == 1 ? 0 : 1) | 2, d, n, N, g, 100.0, 100.0, 0.05, 1.0, sigma, mix, phi + P);
  (void)oracle_bdp(c, N, n, phi, 2, V, V0);
  double lo = 0.0, hi = 0.0;
  for (int64_t t = 0; t < P; ++t) hi = phi[t] > hi ? phi[t] : hi;
  CHECK(V0[0] >= lo && V0[0] <= hi);
  CHECK(V0[0] >= V0[1] - 1e-12 || d > 1);

  /* swing obstacle and BDP */
  double *v = calloc((size_t)P, sizeof(double));
  double *Pall = calloc((size_t)(n + 1) * P, sizeof(double));
  oracle_forward_payoff(d, n, N, g, s.mu, s.L, 20.0, 20.0, 0.0, 1.0, sigma, NULL, v);
  double p0 = oracle_swing(c, N, n, v, 1, 3, Pall);
  CHECK(isfinite(p0));

  /* grid optimisation on the last layer's grid */
  float Lm[9] = {1, 0, 0, 0.3f, 0.95f, 0, 0.1f, 0.2f, 0.97f};
  float *gl = calloc((size_t)N[n] * d, sizeof(float));
  memcpy(gl, g + ((size_t)P - N[n]) * d, sizeof(float) * (size_t)N[n] * d);
  double dist[3];
  CHECK(oracle_lloyd(d, N[n], Lm, gl, 2000, 3, 5, 1, dist) == 0);
  for (int t = 0; t < 3; ++t) CHECK(dist[t] >= 0.0);

  /* grids from samples: moment matching, then Lloyd steps on windows (one
     inadmissible sample among them) */
  {
    const int64_t Ms = 1000;
    float *xs = calloc((size_t)Ms * d, sizeof(float));
    for (int64_t m = 0; m < Ms; ++m)
      for (int c = 0; c < d; ++c) xs[m * d + c] = (float)sin(0.37 * (double)(m * d + c + 1));
    xs[17 * d] = NAN;
    int64_t s1[3], s2[9], rej = -1;
    CHECK(oracle_sample_moments(d, xs, Ms, s1, s2) == Ms - 1);
    float *gm = calloc((size_t)N[n] * d, sizeof(float));
    double mom[3 + 18];
    oracle_moment_map(d, Ms - 1, s1, s2, gl, N[n], gm, mom);
    for (int c = 0; c < d; ++c) CHECK(mom[d + c * d + c] > 0.0);
    if (d == 1)
      for (int32_t i = 0; i + 1 < N[n]; ++i) gm[i + 1] = fmaxf(gm[i + 1], nextafterf(gm[i], 1e9f));
    double dist4[4];
    CHECK(oracle_lloyd_empirical(d, N[n], gm, xs, Ms, 370, 4, 0.5, dist4, &rej) == 0);
    CHECK(rej == 1 || rej == 2);
    free(gm);
    free(xs);
  }

  if (d == 1) {
    int32_t *cs = calloc((size_t)entries, sizeof(int32_t));
    CHECK(oracle_transitions_stratified(&s.m, g, N, 50, 1, 9, 1, cs) == 0);
    CHECK(oracle_transitions_stratified(&s.m, g, N, 50, 0, 9, 1, cs) == 0);
    for (int k = 0; k < n; ++k)
      CHECK(sum_block(cs + off[k], (int64_t)N[k] * N[k + 1]) == (int64_t)50 * N[k]);
    free(cs);
    CHECK(fabs(oracle_ppnd16(0.975) - 1.959963984540054) < 1e-12);
    CHECK(fabs(oracle_ln64(2.0) - 0.6931471805599453) < 1e-15);
  }
  free(gl); free(v); free(Pall); free(phi); free(V); free(x); free(y); free(cell);
  free(c); free(c2); free(g);
  bm_free(&s);
}

int main(void) {
  for (int d = 1; d <= 3; ++d) run_dim(d);
  uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, out[4];
  oracle_philox4x32_10(ctr, key, out);
  float z0, z1;
  oracle_box_muller(out[0], out[1], &z0, &z1);
  CHECK(isfinite(z0) && isfinite(z1));
  double pi = oracle_pi_estimate(1, 0, 20000);
  CHECK(pi > 3.0 && pi < 3.3);
  printf("oracle sanitizer run ok\n");
  return 0;
}
