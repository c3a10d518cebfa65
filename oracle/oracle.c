/*
 * Oracle: plain CPU implementation of the quantization-tree forward step
 * (transition counts between Voronoi cells of consecutive layers) and of the
 * backward dynamic programming on the tree, after Pages & Wilbertz,
 * arXiv:1101.3228.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares
 * no code with the GPU library.
 *
 * The paper fixes neither the random number generator nor the Gaussian
 * transform nor the floating point rules of the cell search; the readings
 * used here (counter-based Philox, Box-Muller with series-defined ln/sin/cos,
 * fixed FP32 operation order) are the arithmetic specification written down
 * in the design notes.  Everything is FP32 with explicit fmaf where the
 * specification says "fused"; build with -ffp-contract=off -fno-fast-math.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10, as published by Salmon et al. (SC'11): ten rounds of
   two 32x32->64 multiplies with the round keys bumped by the Weyl
   increments between rounds.                                          */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------ */
/* ln(K 2^-24), K in [1, 2^24].  K = 2^e f exactly; f is folded into
   [2/3, 4/3) by an exact halving; ln(1+t), t = f-1 (exact by Sterbenz),
   is the Mercator series truncated after t^14, evaluated by Horner with
   fused multiply-adds; ln 2 is split Cody-Waite style so that e*LN2_HI
   is exact.                                                           */
/* ------------------------------------------------------------------ */
float oracle_ln_u24(uint32_t K) {
  /* coefficients (-1)^(n+1)/n, n = 2..14, each the nearest FP32 value */
  static const float c[15] = {
      0.0f, 0.0f,
      -0x1p-1f,          /*  -1/2  */
      0x1.555556p-2f,    /*   1/3  */
      -0x1p-2f,          /*  -1/4  */
      0x1.99999ap-3f,    /*   1/5  */
      -0x1.555556p-3f,   /*  -1/6  */
      0x1.24924ap-3f,    /*   1/7  */
      -0x1p-3f,          /*  -1/8  */
      0x1.c71c72p-4f,    /*   1/9  */
      -0x1.99999ap-4f,   /* -1/10  */
      0x1.745d18p-4f,    /*  1/11  */
      -0x1.555556p-4f,   /* -1/12  */
      0x1.3b13b2p-4f,    /*  1/13  */
      -0x1.24924ap-4f,   /* -1/14  */
  };
  const float LN2_HI = 0x1.62e4p-1f;      /* floor(ln2 * 2^16) / 2^16 */
  const float LN2_LO = 0x1.7f7d1cp-20f;   /* nearest FP32 to ln2 - LN2_HI */
  float F = (float)K;                     /* exact: K < 2^25 */
  uint32_t bits = f2u(F);
  int32_t e = (int32_t)(bits >> 23) - 127;
  uint32_t mb = (bits & 0x007FFFFFu) | 0x3F800000u; /* f in [1, 2) */
  if (mb >= 0x3FAAAAABu) {                 /* f >= 4/3: halve f, bump e */
    mb -= 0x00800000u;
    e += 1;
  }
  float t = u2f(mb) - 1.0f;                /* exact */
  float P = c[14];
  for (int n = 13; n >= 2; --n) P = fmaf(P, t, c[n]);
  float w = t * t;
  float r = fmaf(w, P, t);                 /* ln(1+t) = t + t^2 P(t) */
  float ee = (float)(e - 24);
  float s = fmaf(ee, LN2_LO, r);
  return fmaf(ee, LN2_HI, s);
}

/* ------------------------------------------------------------------ */
/* sin and cos of theta = 2 pi J 2^-24.  Quadrant q = J>>22 and the
   in-quadrant fraction r (22 bits) are split in integer arithmetic; an
   exact reflection r -> 2^22 - r keeps y = r 2^-22 in [0, 1/2]; the
   Taylor series of sin(pi y/2) (to y^9) and cos(pi y/2) (to y^10) are
   evaluated by Horner in w = y^2.                                     */
/* ------------------------------------------------------------------ */
void oracle_sincos_2pi_u24(uint32_t J, float *sn, float *cs) {
  /* (-1)^k (pi/2)^(2k+1)/(2k+1)!, k = 0..4 */
  const float S0 = 0x1.921fb6p+0f, S1 = -0x1.4abbcep-1f, S2 = 0x1.466bc6p-4f,
              S3 = -0x1.32d2ccp-8f, S4 = 0x1.507834p-13f;
  /* (-1)^k (pi/2)^(2k)/(2k)!, k = 0..5 */
  const float C0 = 1.0f, C1 = -0x1.3bd3ccp+0f, C2 = 0x1.03c1f0p-2f,
              C3 = -0x1.55d3c8p-6f, C4 = 0x1.e1f506p-11f, C5 = -0x1.a6d1f2p-16f;
  uint32_t q = J >> 22;
  uint32_t r = J & 0x003FFFFFu;
  int swap = 0;
  if (r > 0x00200000u) {
    r = 0x00400000u - r;
    swap = 1;
  }
  float y = (float)r * 0x1p-22f;           /* exact */
  float w = y * y;
  float ps = fmaf(S4, w, S3);
  ps = fmaf(ps, w, S2);
  ps = fmaf(ps, w, S1);
  ps = fmaf(ps, w, S0);
  float sy = ps * y;                       /* sin(pi y / 2) */
  float pc = fmaf(C5, w, C4);
  pc = fmaf(pc, w, C3);
  pc = fmaf(pc, w, C2);
  pc = fmaf(pc, w, C1);
  float cy = fmaf(pc, w, C0);              /* cos(pi y / 2) */
  float sp = swap ? cy : sy;               /* sin and cos of the in-quadrant angle */
  float cp = swap ? sy : cy;
  switch (q) {
    case 0: *sn = sp;  *cs = cp;  break;
    case 1: *sn = cp;  *cs = -sp; break;
    case 2: *sn = -sp; *cs = -cp; break;
    default: *sn = -cp; *cs = sp; break;
  }
}

/* Box-Muller: rho = sqrt(-2 ln u_a), u_a = ((ra>>8)+1) 2^-24 in (0,1];
   angle 2 pi u_b, u_b = (rb>>8) 2^-24 in [0,1). */
void oracle_box_muller(uint32_t ra, uint32_t rb, float *z0, float *z1) {
  float l = oracle_ln_u24((ra >> 8) + 1u);
  float rho = sqrtf(-2.0f * l);
  float s, c;
  oracle_sincos_2pi_u24(rb >> 8, &s, &c);
  *z0 = rho * c;
  *z1 = rho * s;
}

static void seed_key(uint64_t seed, uint32_t key[2]) {
  key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
  key[1] = (uint32_t)(seed >> 32);
}

/* Counter words: (c0, c1, c2, c3) = (sample block, layer, contract, tag).
   Tag 0: time-layer sampling (Algorithm III), 16: its second block for d = 3;
   tag 1: pathwise innovations (Algorithm I). */
static void normals_layer(int32_t d, int32_t k, uint64_t m, uint64_t seed, uint32_t contract,
                          float *zx, float *eps) {
  uint32_t key[2], r[4];
  seed_key(seed, key);
  if (d == 1) {
    uint32_t ctr[4] = {(uint32_t)(m >> 1), (uint32_t)k, contract, 0u};
    oracle_philox4x32_10(ctr, key, r);
    if ((m & 1u) == 0) oracle_box_muller(r[0], r[1], &zx[0], &eps[0]);
    else oracle_box_muller(r[2], r[3], &zx[0], &eps[0]);
  } else if (d == 2) {
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)k, contract, 0u};
    oracle_philox4x32_10(ctr, key, r);
    oracle_box_muller(r[0], r[1], &zx[0], &zx[1]);
    oracle_box_muller(r[2], r[3], &eps[0], &eps[1]);
  } else {
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)k, contract, 0u};
    oracle_philox4x32_10(ctr, key, r);
    oracle_box_muller(r[0], r[1], &zx[0], &zx[1]);
    oracle_box_muller(r[2], r[3], &zx[2], &eps[0]);
    uint32_t ctr2[4] = {(uint32_t)m, (uint32_t)k, contract, 16u};
    oracle_philox4x32_10(ctr2, key, r);
    oracle_box_muller(r[0], r[1], &eps[1], &eps[2]);
  }
}

void oracle_path_noise(int32_t d, int32_t k, uint64_t m, uint64_t seed, uint32_t contract,
                       float *eps) {
  uint32_t key[2], r[4];
  seed_key(seed, key);
  float z[4];
  if (d == 1) {
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)k >> 2, contract, 1u};
    oracle_philox4x32_10(ctr, key, r);
    oracle_box_muller(r[0], r[1], &z[0], &z[1]);
    oracle_box_muller(r[2], r[3], &z[2], &z[3]);
    eps[0] = z[k & 3];
  } else if (d == 2) {
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)k >> 1, contract, 1u};
    oracle_philox4x32_10(ctr, key, r);
    if ((k & 1) == 0) oracle_box_muller(r[0], r[1], &eps[0], &eps[1]);
    else oracle_box_muller(r[2], r[3], &eps[0], &eps[1]);
  } else {
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)k, contract, 1u};
    oracle_philox4x32_10(ctr, key, r);
    oracle_box_muller(r[0], r[1], &eps[0], &eps[1]);
    oracle_box_muller(r[2], r[3], &eps[2], &z[0]);
  }
}

/* y = b + A x + T eps, each row a left-to-right chain of fused
   multiply-adds starting from b (Proposition, Sec. 3). */
static void ar_step(int32_t d, const float *A, const float *b, const float *T, const float *x,
                    const float *eps, float *y) {
  for (int r = 0; r < d; ++r) {
    float v = b[r];
    for (int c = 0; c < d; ++c) v = fmaf(A[r * d + c], x[c], v);
    for (int c = 0; c < d; ++c) v = fmaf(T[r * d + c], eps[c], v);
    y[r] = v;
  }
}

void oracle_layer_pair(const oracle_model *mdl, int32_t k, uint64_t m, uint64_t seed,
                       uint32_t contract, float *xk, float *xk1) {
  int d = mdl->d;
  float zx[3], eps[3];
  normals_layer(d, k, m, seed, contract, zx, eps);
  const float *mu = mdl->mu + (size_t)k * d;
  const float *L = mdl->L + (size_t)k * d * d;
  for (int r = 0; r < d; ++r) {       /* X_k = mu_k + L_k z */
    float v = mu[r];
    for (int c = 0; c < d; ++c) v = fmaf(L[r * d + c], zx[c], v);
    xk[r] = v;
  }
  ar_step(d, mdl->A + (size_t)k * d * d, mdl->b + (size_t)k * d, mdl->T + (size_t)k * d * d,
          xk, eps, xk1);
}

/* Nearest neighbour projection (Sec. 2).  d = 1: cell = number of
   midpoints m_r = (x_r + x_{r+1})/2 strictly below x, so a point on a
   midpoint goes to the lower cell.  d >= 2: the cell minimises the
   half-norm form h_p - <x, g_p> of the squared distance
   (|x - g_p|^2 = |x|^2 + 2 (h_p - <x, g_p>), h_p = |g_p|^2 / 2); the
   lowest index wins ties. */
static float half_norm(const float *g, int d) {
  float t = g[0] * g[0];
  for (int c = 1; c < d; ++c) t = fmaf(g[c], g[c], t);
  return 0.5f * t;
}

int32_t oracle_cell(const float *grid_k, int32_t N, int32_t d, const float *x) {
  if (d == 1) {
    int32_t cnt = 0;
    for (int32_t r = 0; r + 1 < N; ++r) {
      float mid = 0.5f * (grid_k[r] + grid_k[r + 1]);
      if (mid < x[0]) ++cnt;
    }
    return cnt;
  }
  int32_t best = 0;
  float bestkey = 0.0f;
  for (int32_t p = 0; p < N; ++p) {
    const float *g = grid_k + (size_t)p * d;
    float key = half_norm(g, d);
    for (int c = 0; c < d; ++c) key = fmaf(-x[c], g[c], key);
    if (p == 0 || key < bestkey) {
      bestkey = key;
      best = p;
    }
  }
  return best;
}

/* Per-layer precomputation used by the sample loops: midpoints (d = 1) or
   half norms (d >= 2) of the grid, exactly as in oracle_cell. */
typedef struct {
  const float *g;
  float *aux;
  int32_t N, d;
} layer_grid;

static void layer_grid_init(layer_grid *lg, const float *g, int32_t N, int32_t d) {
  lg->g = g; lg->N = N; lg->d = d;
  lg->aux = (float *)malloc(sizeof(float) * (size_t)(N > 0 ? N : 1));
  if (d == 1) {
    for (int32_t r = 0; r + 1 < N; ++r) lg->aux[r] = 0.5f * (g[r] + g[r + 1]);
  } else {
    for (int32_t p = 0; p < N; ++p) lg->aux[p] = half_norm(g + (size_t)p * d, d);
  }
}

static int32_t layer_cell(const layer_grid *lg, const float *x) {
  if (lg->d == 1) {
    int32_t cnt = 0;
    for (int32_t r = 0; r + 1 < lg->N; ++r)
      if (lg->aux[r] < x[0]) ++cnt;
    return cnt;
  }
  int32_t best = 0;
  float bestkey = 0.0f;
  for (int32_t p = 0; p < lg->N; ++p) {
    const float *g = lg->g + (size_t)p * lg->d;
    float key = lg->aux[p];
    for (int c = 0; c < lg->d; ++c) key = fmaf(-x[c], g[c], key);
    if (p == 0 || key < bestkey) {
      bestkey = key;
      best = p;
    }
  }
  return best;
}

typedef struct {
  const oracle_model *mdl;
  const layer_grid *lg;   /* [n+1] */
  const int64_t *coff;    /* [n] */
  const int32_t *N;
  uint64_t m0, M, seed;
  uint32_t contract;
  int32_t *counts;
  int32_t mode;
  int32_t tid, nthreads;
} job;

/* Serial Algorithm III for the layers owned by one thread (layers are
   independent, so splitting them over threads changes nothing). */
static void *run_layerwise(void *arg) {
  job *J = (job *)arg;
  const oracle_model *mdl = J->mdl;
  for (int32_t k = J->tid; k < mdl->n; k += J->nthreads) {
    int32_t *ck = J->counts + J->coff[k];
    int32_t N1 = J->N[k + 1];
    for (uint64_t m = J->m0; m < J->m0 + J->M; ++m) {
      float x[3], y[3];
      oracle_layer_pair(mdl, k, m, J->seed, J->contract, x, y);
      int32_t i = layer_cell(&J->lg[k], x);
      int32_t j = layer_cell(&J->lg[k + 1], y);
      ck[(int64_t)i * N1 + j] += 1;
    }
  }
  return NULL;
}

/* Serial Algorithm I for a slice of the paths; the increments are atomic
   integer additions so that threads may share the counters. */
static void *run_pathwise(void *arg) {
  job *J = (job *)arg;
  const oracle_model *mdl = J->mdl;
  int d = mdl->d;
  uint64_t per = (J->M + (uint64_t)J->nthreads - 1) / (uint64_t)J->nthreads;
  uint64_t lo = J->m0 + per * (uint64_t)J->tid;
  uint64_t hi = lo + per;
  if (hi > J->m0 + J->M) hi = J->m0 + J->M;
  for (uint64_t m = lo; m < hi; ++m) {
    float x[3], y[3], eps[3];
    for (int c = 0; c < d; ++c) x[c] = mdl->x0[c];
    int32_t i = 0;
    for (int32_t k = 0; k < mdl->n; ++k) {
      oracle_path_noise(d, k, m, J->seed, J->contract, eps);
      ar_step(d, mdl->A + (size_t)k * d * d, mdl->b + (size_t)k * d,
              mdl->T + (size_t)k * d * d, x, eps, y);
      int32_t j = layer_cell(&J->lg[k + 1], y);
      int32_t *slot = J->counts + J->coff[k] + (int64_t)i * J->N[k + 1] + j;
      if (J->nthreads > 1) __atomic_fetch_add(slot, 1, __ATOMIC_RELAXED);
      else *slot += 1;
      i = j;
      for (int c = 0; c < d; ++c) x[c] = y[c];
    }
  }
  return NULL;
}

int oracle_transitions(const oracle_model *mdl, const float *grid, const int32_t *N,
                       uint64_t m0, uint64_t M, uint64_t seed, uint32_t contract,
                       int32_t mode, int32_t *counts, int32_t nthreads) {
  if (!mdl || !grid || !N || !counts) return 1;
  int32_t d = mdl->d, n = mdl->n;
  if (d < 1 || d > 3 || n < 1 || N[0] != 1) return 1;
  if (M >= (1ull << 31) || m0 + M > (1ull << 32)) return 2;
  for (int32_t k = 0; k <= n; ++k)
    if (N[k] < 1) return 1;
  if (nthreads < 1) nthreads = 1;
  layer_grid *lg = (layer_grid *)malloc(sizeof(layer_grid) * (size_t)(n + 1));
  int64_t *coff = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t poff = 0, co = 0;
  for (int32_t k = 0; k <= n; ++k) {
    layer_grid_init(&lg[k], grid + poff * d, N[k], d);
    poff += N[k];
    if (k < n) {
      coff[k] = co;
      co += (int64_t)N[k] * N[k + 1];
    }
  }
  memset(counts, 0, sizeof(int32_t) * (size_t)co);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  job *jobs = (job *)malloc(sizeof(job) * (size_t)nthreads);
  for (int32_t t = 0; t < nthreads; ++t) {
    job J = {mdl, lg, coff, N, m0, M, seed, contract, counts, mode, t, nthreads};
    jobs[t] = J;
  }
  void *(*fn)(void *) = (mode == ORACLE_PATHWISE) ? run_pathwise : run_layerwise;
  if (nthreads == 1) {
    fn(&jobs[0]);
  } else {
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, &jobs[t]);
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  for (int32_t k = 0; k <= n; ++k) free(lg[k].aux);
  free(lg); free(coff); free(th); free(jobs);
  return 0;
}

/* Backward dynamic programming on the quantization tree (Sec. 2):
   V_n = phi_n;  V_k(i) = max(phi_k(i), sum_j pi_ij V_{k+1}(j)),
   pi_ij = c_ij / p_i, p_i = sum_j c_ij.  A row that no sample reached
   (p_i = 0) has continuation value 0. */
int64_t oracle_bdp(const int32_t *counts, const int32_t *N, int32_t n, const double *phi,
                   int32_t n_pay, double *V_all, double *V0) {
  int64_t total = 0;
  int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 2));
  int64_t *coff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  poff[0] = 0;
  coff[0] = 0;
  for (int32_t k = 0; k <= n; ++k) poff[k + 1] = poff[k] + N[k];
  for (int32_t k = 0; k < n; ++k) coff[k + 1] = coff[k] + (int64_t)N[k] * N[k + 1];
  int64_t P = poff[n + 1];
  double *V = (double *)malloc(sizeof(double) * (size_t)P);
  int64_t empty = 0;
  for (int32_t q = 0; q < n_pay; ++q) {
    const double *ph = phi + (size_t)q * P;
    for (int32_t i = 0; i < N[n]; ++i) V[poff[n] + i] = ph[poff[n] + i];
    for (int32_t k = n - 1; k >= 0; --k) {
      const int32_t *ck = counts + coff[k];
      for (int32_t i = 0; i < N[k]; ++i) {
        int64_t p = 0;
        double s = 0.0;
        for (int32_t j = 0; j < N[k + 1]; ++j) {
          int32_t c = ck[(int64_t)i * N[k + 1] + j];
          p += c;
          s += (double)c * V[poff[k + 1] + j];
        }
        double cont = 0.0;
        if (p > 0) cont = s / (double)p;
        else ++empty;
        double f = ph[poff[k] + i];
        V[poff[k] + i] = (f > cont) ? f : cont;
      }
    }
    if (V_all) memcpy(V_all + (size_t)q * P, V, sizeof(double) * (size_t)P);
    if (V0) V0[q] = V[0];
  }
  total = empty;
  free(V); free(poff); free(coff);
  return total;
}

void oracle_payoff(int32_t kind, int32_t d, int32_t n, const int32_t *N, const float *grid,
                   double S0, double K, double r, double Tm, const double *sigma,
                   const double *mix, double *phi) {
  int max_call = kind & 1, european = kind & 2;
  int64_t off = 0;
  for (int32_t k = 0; k <= n; ++k) {
    double t = Tm * (double)k / (double)n;
    double disc = exp(-r * t);
    for (int32_t i = 0; i < N[k]; ++i) {
      const float *x = grid + (off + i) * d;
      double y[3];
      for (int a = 0; a < d; ++a) {
        if (!mix) {
          y[a] = (double)x[a];
          continue;
        }
        y[a] = 0.0;
        for (int b = 0; b < d; ++b) y[a] += mix[a * d + b] * (double)x[b];
      }
      double v;
      if (max_call) {
        double smax = -INFINITY;
        for (int a = 0; a < d; ++a) {
          double s = S0 * exp((r - 0.5 * sigma[a] * sigma[a]) * t + sigma[a] * y[a]);
          if (s > smax) smax = s;
        }
        v = disc * fmax(smax - K, 0.0);
      } else {
        double s = S0 * exp((r - 0.5 * sigma[0] * sigma[0]) * t + sigma[0] * y[0]);
        v = disc * fmax(K - s, 0.0);
      }
      if (european && k < n) v = -INFINITY;
      phi[off + i] = v;
    }
    off += N[k];
  }
}

void oracle_forward_payoff(int32_t d, int32_t n, const int32_t *N, const float *grid,
                           const float *mu, const float *L, double S0, double K, double r,
                           double Tm, const double *sigma, const double *mix, double *v) {
  int64_t off = 0;
  for (int32_t k = 0; k <= n; ++k) {
    const double t = Tm * (double)k / (double)n;
    const double disc = exp(-r * t);
    /* w = mix' sigma: s_k = w . x */
    double w[3];
    for (int b = 0; b < d; ++b) {
      w[b] = 0.0;
      for (int a = 0; a < d; ++a) w[b] += sigma[a] * (mix ? mix[a * d + b] : (a == b ? 1.0 : 0.0));
    }
    /* var_k = |L_k' w|^2, mean term w . mu_k */
    const float *Lk = L + (size_t)k * d * d;
    double var = 0.0, wm = 0.0;
    for (int c = 0; c < d; ++c) {
      double u = 0.0;
      for (int b = 0; b < d; ++b) u += w[b] * (double)Lk[b * d + c];
      var += u * u;
    }
    for (int b = 0; b < d; ++b) wm += w[b] * (double)mu[(size_t)k * d + b];
    for (int32_t i = 0; i < N[k]; ++i) {
      const float *x = grid + (off + i) * d;
      double s = 0.0;
      for (int b = 0; b < d; ++b) s += w[b] * (double)x[b];
      v[off + i] = disc * (S0 * exp(s - wm - 0.5 * var) - K);
    }
    off += N[k];
  }
}

double oracle_swing(const int32_t *counts, const int32_t *N, int32_t n, const double *v,
                    int32_t Qmin, int32_t Qmax, double *P_all) {
  const int32_t C = Qmax + 1;
  int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 2));
  int64_t *coff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  poff[0] = 0;
  coff[0] = 0;
  for (int32_t k = 0; k <= n; ++k) poff[k + 1] = poff[k] + N[k];
  for (int32_t k = 0; k < n; ++k) coff[k + 1] = coff[k] + (int64_t)N[k] * N[k + 1];
  const int64_t P = poff[n + 1];
  double *V = (double *)malloc(sizeof(double) * (size_t)P * (size_t)C);  /* [c][P] */
  for (int32_t c = 0; c < C; ++c)
    for (int32_t i = 0; i < N[n]; ++i)
      V[(size_t)c * P + poff[n] + i] = (c >= Qmin && c <= Qmax) ? 0.0 : -INFINITY;
  double *cont = (double *)malloc(sizeof(double) * (size_t)(C + 1));
  for (int32_t k = n - 1; k >= 0; --k) {
    const int32_t *ck = counts + coff[k];
    for (int32_t i = 0; i < N[k]; ++i) {
      int64_t p = 0;
      for (int32_t j = 0; j < N[k + 1]; ++j) p += ck[(int64_t)i * N[k + 1] + j];
      for (int32_t c = 0; c < C; ++c) {
        double s = 0.0;
        for (int32_t j = 0; j < N[k + 1]; ++j) {
          const int32_t cij = ck[(int64_t)i * N[k + 1] + j];
          if (cij) s += (double)cij * V[(size_t)c * P + poff[k + 1] + j];
        }
        cont[c] = p > 0 ? s / (double)p : 0.0;
      }
      for (int32_t c = 0; c < C; ++c) {
        double best = -INFINITY;
        for (int x = 0; x <= 1; ++x) {
          if (c + x > Qmax || c + x + (n - k - 1) < Qmin) continue;
          const double val = (x ? v[poff[k] + i] : 0.0) + cont[c + x];
          if (val > best) best = val;
        }
        V[(size_t)c * P + poff[k] + i] = best;
      }
    }
  }
  const double P0 = V[0];
  if (P_all) memcpy(P_all, V, sizeof(double) * (size_t)P * (size_t)C);
  free(cont); free(V); free(poff); free(coff);
  return P0;
}

/* Bulk helpers for the exhaustive and statistical tests (plain loops). */
void oracle_ln_u24_bulk(uint32_t K0, int64_t count, float *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = oracle_ln_u24(K0 + (uint32_t)i);
}

void oracle_sincos_bulk(uint32_t J0, int64_t count, float *s, float *c) {
  for (int64_t i = 0; i < count; ++i) oracle_sincos_2pi_u24(J0 + (uint32_t)i, &s[i], &c[i]);
}

void oracle_box_muller_bulk(const uint32_t *ra, const uint32_t *rb, int64_t count, float *z0,
                            float *z1) {
  for (int64_t i = 0; i < count; ++i) oracle_box_muller(ra[i], rb[i], &z0[i], &z1[i]);
}

void oracle_philox_bulk(const uint32_t *ctr, const uint32_t key[2], int64_t count,
                        uint32_t *out) {
  for (int64_t i = 0; i < count; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Layer samples m0..m0+count-1 of layer k (Algorithm III): xk, xk1 [count][d]. */
void oracle_layer_pairs_bulk(const oracle_model *mdl, int32_t k, uint64_t m0, int64_t count,
                             uint64_t seed, uint32_t contract, float *xk, float *xk1) {
  int d = mdl->d;
  for (int64_t i = 0; i < count; ++i)
    oracle_layer_pair(mdl, k, m0 + (uint64_t)i, seed, contract, xk + i * d, xk1 + i * d);
}

/* Monte Carlo estimate of pi from npts points (u, v) of the unit square,
   u = (r0>>8) 2^-24, v = (r1>>8) 2^-24 and likewise (r2, r3), counter
   (i, rep, 0, 3): four times the fraction of points with u^2 + v^2 <= 1
   (the quarter-disc experiment of the RNG comparison in Sec. 3). */
double oracle_pi_estimate(uint64_t seed, uint32_t rep, uint64_t npts) {
  uint32_t key[2], r[4];
  seed_key(seed, key);
  uint64_t inside = 0;
  for (uint64_t i = 0; i < npts / 2; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, rep, 0u, 3u};
    oracle_philox4x32_10(ctr, key, r);
    for (int h = 0; h < 2; ++h) {
      double u = (double)(r[2 * h] >> 8) * 0x1p-24;
      double v = (double)(r[2 * h + 1] >> 8) * 0x1p-24;
      if (u * u + v * v <= 1.0) ++inside;
    }
  }
  return 4.0 * (double)inside / (double)((npts / 2) * 2);
}

/* Counts of one layer k -> k+1 of the time-layer parallel estimate over
   samples m0 .. m0+M-1 (Algorithm III restricted to one layer), for checking
   single layers of large problems.  counts_k: int32[N_k][N_{k+1}],
   overwritten.  Threads split the samples and add atomically. */
typedef struct {
  const oracle_model *mdl;
  const layer_grid *g0, *g1;
  int32_t k, N1;
  uint64_t lo, hi, seed;
  uint32_t contract;
  int32_t *ck;
} layer_job;

static void *run_one_layer(void *arg) {
  layer_job *J = (layer_job *)arg;
  for (uint64_t m = J->lo; m < J->hi; ++m) {
    float x[3], y[3];
    oracle_layer_pair(J->mdl, J->k, m, J->seed, J->contract, x, y);
    int32_t i = layer_cell(J->g0, x);
    int32_t j = layer_cell(J->g1, y);
    __atomic_fetch_add(&J->ck[(int64_t)i * J->N1 + j], 1, __ATOMIC_RELAXED);
  }
  return NULL;
}

int oracle_layer_counts(const oracle_model *mdl, const float *grid, const int32_t *N, int32_t k,
                        uint64_t m0, uint64_t M, uint64_t seed, uint32_t contract,
                        int32_t *counts_k, int32_t nthreads) {
  if (!mdl || !grid || !N || !counts_k || k < 0 || k >= mdl->n) return 1;
  if (M >= (1ull << 31) || m0 + M > (1ull << 32)) return 2;
  if (nthreads < 1) nthreads = 1;
  int d = mdl->d;
  int64_t off = 0;
  for (int32_t l = 0; l < k; ++l) off += N[l];
  layer_grid g0, g1;
  layer_grid_init(&g0, grid + off * d, N[k], d);
  layer_grid_init(&g1, grid + (off + N[k]) * d, N[k + 1], d);
  memset(counts_k, 0, sizeof(int32_t) * (size_t)N[k] * (size_t)N[k + 1]);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  layer_job *jobs = (layer_job *)malloc(sizeof(layer_job) * (size_t)nthreads);
  uint64_t per = (M + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
  for (int32_t t = 0; t < nthreads; ++t) {
    uint64_t lo = m0 + per * (uint64_t)t, hi = lo + per;
    if (lo > m0 + M) lo = m0 + M;
    if (hi > m0 + M) hi = m0 + M;
    layer_job J = {mdl, &g0, &g1, k, N[k + 1], lo, hi, seed, contract, counts_k};
    jobs[t] = J;
    pthread_create(&th[t], NULL, run_one_layer, &jobs[t]);
  }
  for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(g0.aux); free(g1.aux); free(th); free(jobs);
  return 0;
}

/* Cells of `count` points x[count][d] in one grid (plain loop over oracle_cell). */
void oracle_cells_bulk(const float *grid_k, int32_t N, int32_t d, const float *x, int64_t count,
                       int32_t *out) {
  layer_grid lg;
  layer_grid_init(&lg, grid_k, N, d);
  for (int64_t i = 0; i < count; ++i) out[i] = layer_cell(&lg, x + i * d);
  free(lg.aux);
}

/* ------------------------------------------------------------------ */
/* Grid optimization (Sec. 2, eq. Qerr): randomized Lloyd iteration for  */
/* the quadratic quantization error of X = L z, z ~ N(0, I_d).           */
/* ------------------------------------------------------------------ */
/* Sample m of iteration `it` draws one Philox block, counter
   (m, fresh ? it : 0, 0, 2), and takes z_0, z_1 from Box-Muller of
   (r0, r1) and z_2 from (r2, r3); X_r = sum_c L[r][c] z_c as a chain of
   fused multiply-adds from 0.  Each sample is assigned to its cell by the
   tree's own rule (oracle_cell).  A Lloyd step replaces every grid point
   by the mean of the samples of its cell (a cell without samples keeps its
   point): the fixed points of this map are the stationary grids of
   eq. Qerr.  The cell sums are kept exactly as integers: coordinate x
   contributes rint(x 2^24), the squared distance to the cell's point
   rint(|x - g|^2 2^16) (both in FP64), so the result does not depend on
   the order in which samples are added.  New point: (sum 2^-24) / count in
   FP64, rounded once to FP32.  distortion[it] = (sum of the squared
   distances) / M before the update of iteration it. */
static int64_t fixed_scaled(double v, double scale) { return (int64_t)rint(v * scale); }

void oracle_lloyd_sample(int32_t d, const float *L, uint64_t seed, int32_t fresh, int32_t it,
                         uint64_t m, float *x) {
  uint32_t key[2], r[4], ctr[4] = {(uint32_t)m, fresh ? (uint32_t)it : 0u, 0u, 2u};
  float z[4];
  seed_key(seed, key);
  oracle_philox4x32_10(ctr, key, r);
  oracle_box_muller(r[0], r[1], &z[0], &z[1]);
  oracle_box_muller(r[2], r[3], &z[2], &z[3]);
  for (int row = 0; row < d; ++row) {
    float v = 0.0f;
    for (int c = 0; c < d; ++c) v = fmaf(L[row * d + c], z[c], v);
    x[row] = v;
  }
}

int oracle_lloyd(int32_t d, int32_t N, const float *L, float *grid, uint64_t M, int32_t iters,
                 uint64_t seed, int32_t fresh, double *distortion) {
  int64_t *sum = (int64_t *)calloc((size_t)N * d, sizeof(int64_t));
  int64_t *cnt = (int64_t *)calloc((size_t)N, sizeof(int64_t));
  if (!sum || !cnt) { free(sum); free(cnt); return -1; }
  for (int32_t it = 0; it < iters; ++it) {
    memset(sum, 0, sizeof(int64_t) * (size_t)N * d);
    memset(cnt, 0, sizeof(int64_t) * (size_t)N);
    int64_t dist = 0;
    layer_grid lg;
    layer_grid_init(&lg, grid, N, d);
    for (uint64_t m = 0; m < M; ++m) {
      float x[3];
      oracle_lloyd_sample(d, L, seed, fresh, it, m, x);
      const int32_t i = layer_cell(&lg, x);
      const float *g = grid + (size_t)i * d;
      double d2 = 0.0;
      for (int c = 0; c < d; ++c) {
        const double dx = (double)x[c] - (double)g[c];
        d2 = d2 + dx * dx;
        sum[(size_t)i * d + c] += fixed_scaled((double)x[c], 0x1p24);
      }
      cnt[i] += 1;
      dist += fixed_scaled(d2, 0x1p16);
    }
    free(lg.aux);
    if (distortion) distortion[it] = ((double)dist * 0x1p-16) / (double)M;
    for (int32_t i = 0; i < N; ++i) {
      if (cnt[i] == 0) continue;
      for (int c = 0; c < d; ++c)
        grid[(size_t)i * d + c] =
            (float)(((double)sum[(size_t)i * d + c] * 0x1p-24) / (double)cnt[i]);
    }
  }
  free(sum);
  free(cnt);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Grids from samples of a marginal of any law.  Sec. 2 uses optimal     */
/* grids of Gaussian marginals and, otherwise, sub-optimal grids that    */
/* match the first two moments of X_k.  The moment-matching grid here    */
/* maps a standard grid `base` (for instance an N(0, I_d) quantizer) by  */
/* the sample mean and the Cholesky factor of the sample covariance.     */
/* The Lloyd map of eq. Qerr (every point to the mean of its Voronoi     */
/* cell) is applied to windows of a caller's sample set; gamma < 1 moves */
/* each point only that fraction of the way (the batch form of the       */
/* competitive-learning step toward the cell's samples).                 */
/* ------------------------------------------------------------------ */
static int sample_admissible(const float *x, int d) {
  for (int c = 0; c < d; ++c)
    if (!(fabsf(x[c]) <= 64.0f)) return 0; /* also false for NaN */
  return 1;
}

int64_t oracle_sample_moments(int32_t d, const float *x, int64_t M, int64_t *s1, int64_t *s2) {
  int64_t cnt = 0;
  for (int c = 0; c < d; ++c) s1[c] = 0;
  for (int c = 0; c < d * d; ++c) s2[c] = 0;
  for (int64_t m = 0; m < M; ++m) {
    const float *xm = x + (size_t)m * d;
    if (!sample_admissible(xm, d)) continue;
    cnt += 1;
    for (int r = 0; r < d; ++r) {
      s1[r] += fixed_scaled((double)xm[r], 0x1p24);
      for (int c = 0; c < d; ++c)
        s2[r * d + c] += fixed_scaled((double)xm[r] * (double)xm[c], 0x1p16);
    }
  }
  return cnt;
}

void oracle_moment_map(int32_t d, int64_t count, const int64_t *s1, const int64_t *s2,
                       const float *base, int32_t N, float *grid, double *moments) {
  double mean[3] = {0.0, 0.0, 0.0}, cov[9] = {0.0}, chol[9] = {0.0};
  if (count > 0) {
    for (int r = 0; r < d; ++r) mean[r] = ((double)s1[r] * 0x1p-24) / (double)count;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c)
        cov[r * d + c] = ((double)s2[r * d + c] * 0x1p-16) / (double)count - mean[r] * mean[c];
  }
  /* lower Cholesky factor, column by column; a non-positive pivot (a
     degenerate direction) gives a zero column */
  for (int r = 0; r < d; ++r) {
    for (int c = 0; c <= r; ++c) {
      double v = cov[r * d + c];
      for (int q = 0; q < c; ++q) v = v - chol[r * d + q] * chol[c * d + q];
      if (r == c) chol[r * d + c] = v > 0.0 ? sqrt(v) : 0.0;
      else chol[r * d + c] = chol[c * d + c] > 0.0 ? v / chol[c * d + c] : 0.0;
    }
  }
  for (int32_t i = 0; i < N; ++i) {
    for (int r = 0; r < d; ++r) {
      double v = mean[r];
      for (int c = 0; c <= r; ++c) v = v + chol[r * d + c] * (double)base[(size_t)i * d + c];
      grid[(size_t)i * d + r] = (float)v;
    }
  }
  if (moments) {
    for (int r = 0; r < d; ++r) moments[r] = mean[r];
    for (int c = 0; c < d * d; ++c) {
      moments[d + c] = cov[c];
      moments[d + d * d + c] = chol[c];
    }
  }
}

int oracle_lloyd_empirical(int32_t d, int32_t N, float *grid, const float *x, int64_t M,
                           int64_t batch, int32_t steps, double gamma, double *distortion,
                           int64_t *rejected) {
  int64_t *sum = (int64_t *)calloc((size_t)N * d, sizeof(int64_t));
  int64_t *cnt = (int64_t *)calloc((size_t)N, sizeof(int64_t));
  if (!sum || !cnt) { free(sum); free(cnt); return -1; }
  int64_t bad = 0;
  for (int32_t t = 0; t < steps; ++t) {
    memset(sum, 0, sizeof(int64_t) * (size_t)N * d);
    memset(cnt, 0, sizeof(int64_t) * (size_t)N);
    int64_t dist = 0, used = 0;
    layer_grid lg;
    layer_grid_init(&lg, grid, N, d);
    const int64_t start = (int64_t)(((uint64_t)t * (uint64_t)batch) % (uint64_t)M);
    for (int64_t j = 0; j < batch; ++j) {
      const int64_t m = (start + j) % M;
      const float *xm = x + (size_t)m * d;
      if (!sample_admissible(xm, d)) { bad += 1; continue; }
      const int32_t i = layer_cell(&lg, xm);
      const float *g = grid + (size_t)i * d;
      double d2 = 0.0;
      for (int c = 0; c < d; ++c) {
        const double dx = (double)xm[c] - (double)g[c];
        d2 = d2 + dx * dx;
        sum[(size_t)i * d + c] += fixed_scaled((double)xm[c], 0x1p24);
      }
      cnt[i] += 1;
      used += 1;
      dist += fixed_scaled(d2, 0x1p16);
    }
    free(lg.aux);
    if (distortion) distortion[t] = used > 0 ? ((double)dist * 0x1p-16) / (double)used : 0.0;
    for (int32_t i = 0; i < N; ++i) {
      if (cnt[i] == 0) continue;
      for (int c = 0; c < d; ++c) {
        const double mean = ((double)sum[(size_t)i * d + c] * 0x1p-24) / (double)cnt[i];
        const double g = (double)grid[(size_t)i * d + c];
        grid[(size_t)i * d + c] = gamma == 1.0 ? (float)mean : (float)(g + gamma * (mean - g));
      }
    }
  }
  if (rejected) *rejected = bad;
  free(sum);
  free(cnt);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Stratified time-layer estimate (not in the paper): the samples of     */
/* X_k are drawn cell by cell from the marginal conditioned on the cell. */
/* ------------------------------------------------------------------ */
/* ln x in FP64 for finite x > 0: x = 2^e f with f in [1, 2) read from the
   bits (subnormals scaled by 2^54 first), f folded into [sqrt(1/2),
   sqrt(2)) by an exact halving; ln f = 2 atanh(s), s = (f - 1) / (f + 1),
   as 2 s sum_{k=0..11} s^(2k) / (2k + 1) (Horner in s^2 with fma, the
   coefficients 1 / (2k + 1) rounded to FP64); ln x = e ln2 + ln f. */
double oracle_ln64(double x) {
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  int e = 0;
  if (((bits >> 52) & 0x7FF) == 0) {
    x = x * 0x1p54;
    memcpy(&bits, &x, sizeof bits);
    e = -54;
  }
  e += (int)((bits >> 52) & 0x7FF) - 1023;
  bits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
  double f;
  memcpy(&f, &bits, sizeof f);
  if (f > 1.4142135623730951) {
    f = 0.5 * f;
    e += 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double P = 1.0 / 23.0;
  for (int k = 10; k >= 0; --k) P = fma(P, s2, 1.0 / (double)(2 * k + 1));
  const double lnf = (2.0 * s) * P;
  return fma((double)e, 0.6931471805599453, lnf);
}

/* Standard normal quantile, Wichura's algorithm AS 241 (PPND16, Applied
   Statistics 37, 1988): a rational function of (p - 1/2)^2 in the centre,
   of sqrt(-ln min(p, 1 - p)) in the tails (ln from oracle_ln64); Horner
   with separate multiply and add.  p <= 0 gives -inf, p >= 1 +inf. */
static double horner8(const double *c, double r) {
  double v = c[7];
  for (int k = 6; k >= 0; --k) v = v * r + c[k];
  return v;
}

double oracle_ppnd16(double p) {
  static const double A[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                              1.9715909503065514427e+3, 1.3731693765509461125e+4,
                              4.5921953931549871457e+4, 6.7265770927008700853e+4,
                              3.3430575583588128105e+4, 2.5090809287301226727e+3};
  static const double B[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                              5.3941960214247511077e+3, 2.1213794301586595867e+4,
                              3.9307895800092710610e+4, 2.8729085735721942674e+4,
                              5.2264952788528545610e+3};
  static const double C[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                              5.76949722146069140550e0, 3.64784832476320460504e0,
                              1.27045825245236838258e0, 2.41780725177450611770e-1,
                              2.27238449892691845833e-2, 7.74545014278341407640e-4};
  static const double D[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                              6.89767334985100004550e-1, 1.48103976427480074590e-1,
                              1.51986665636164571966e-2, 5.47593808499534494600e-4,
                              1.05075007164441684324e-9};
  static const double E[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                              1.78482653991729133580e0, 2.96560571828504891230e-1,
                              2.65321895265761230930e-2, 1.24266094738807843860e-3,
                              2.71155556874348757815e-5, 2.01033439929228813265e-7};
  static const double F[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                              1.48753612908506148525e-2, 7.86869131145613259100e-4,
                              1.84631831751005468180e-5, 1.42151175831644588870e-7,
                              2.04426310338993978564e-15};
  if (!(p > 0.0)) return -INFINITY;
  if (!(p < 1.0)) return INFINITY;
  const double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    return q * horner8(A, r) / horner8(B, r);
  }
  double r = q < 0.0 ? p : 1.0 - p;
  r = sqrt(-oracle_ln64(r));
  double x;
  if (r <= 5.0) {
    r = r - 1.6;
    x = horner8(C, r) / horner8(D, r);
  } else {
    r = r - 5.0;
    x = horner8(E, r) / horner8(F, r);
  }
  return q < 0.0 ? -x : x;
}

/* Marginal probabilities below the cell edges of a 1-D layer: e[0] = 0,
   e[N] = 1, e[r + 1] = Phi(((double)m_r - mu) / L) for the FP32 midpoints
   m_r = (x_r + x_{r+1}) / 2, with Phi(a) = erfc(-a / sqrt 2) / 2 (the
   multiplier 1 / sqrt 2 rounded to FP64). */
void oracle_strat_edges(const float *g, int32_t N, float mu, float L, double *e) {
  e[0] = 0.0;
  e[N] = 1.0;
  for (int32_t r = 0; r + 1 < N; ++r) {
    const float m = 0.5f * (g[r] + g[r + 1]);
    const double a = ((double)m - (double)mu) / (double)L;
    e[r + 1] = 0.5 * erfc(-a * 0.70710678118654752440);
  }
}

/* Samples of row (stratum) i: alloc 0: M (equal allocation); alloc 1:
   max(1, rint(M (e_{i+1} - e_i))) in FP64 (proportional allocation). */
int64_t oracle_strat_row(const double *e, int32_t i, uint64_t M, int32_t alloc) {
  if (alloc == 0) return (int64_t)M;
  const int64_t r = (int64_t)rint((double)M * (e[i + 1] - e[i]));
  return r > 1 ? r : 1;
}

/* Sample t of row i of layer k: Philox counter (t, k, contract, 4 + 256 i);
   u = (k52 + 1/2) 2^-52 with k52 = (r0 >> 12) 2^32 + r1;
   p = e_i + u (e_{i+1} - e_i) (separate multiply and add), kept inside
   [2^-1074, 1 - 2^-53]; z = PPND16(p);
   X_k = fma(L_k, (float)z, mu_k); eps = first Box-Muller normal of (r2, r3);
   X_{k+1} = fma(T_k, eps, fma(A_k, X_k, b_k)). */
void oracle_strat_pair(const oracle_model *mdl, int32_t k, const double *e, int32_t i,
                       uint64_t t, uint64_t seed, uint32_t contract, float *x, float *y) {
  uint32_t key[2], r[4],
      ctr[4] = {(uint32_t)t, (uint32_t)k, contract, 4u + 256u * (uint32_t)i};
  seed_key(seed, key);
  oracle_philox4x32_10(ctr, key, r);
  const double k52 = (double)(r[0] >> 12) * 4294967296.0 + (double)r[1];
  const double u = (k52 + 0.5) * 0x1p-52;
  const double tt = u * (e[i + 1] - e[i]);
  double p = e[i] + tt;
  /* p rounds to 0 or 1 only in cells beyond ~8 standard deviations; the
     nearest representable probabilities keep every sample finite */
  if (!(p < 1.0)) p = 0x1.fffffffffffffp-1;
  if (!(p > 0.0)) p = 0x1p-1074;
  const double z = oracle_ppnd16(p);
  float eps, unused;
  oracle_box_muller(r[2], r[3], &eps, &unused);
  const float xk = fmaf(mdl->L[(size_t)k], (float)z, mdl->mu[(size_t)k]);
  *x = xk;
  *y = fmaf(mdl->T[(size_t)k], eps, fmaf(mdl->A[(size_t)k], xk, mdl->b[(size_t)k]));
}

/* counts[k][i][j] = #{samples of row i of layer k in cell j of layer k+1};
   row i has oracle_strat_row(e_k, i, M, alloc) samples.  d = 1 only. */
int oracle_transitions_stratified(const oracle_model *mdl, const float *grid, const int32_t *N,
                                  uint64_t M, int32_t alloc, uint64_t seed, uint32_t contract,
                                  int32_t *counts) {
  if (!mdl || mdl->d != 1 || N[0] != 1) return 1;
  const int32_t n = mdl->n;
  int64_t poff = 0, coff = 0;
  for (int32_t k = 0; k < n; ++k) {
    const float *g0 = grid + poff, *g1 = grid + poff + N[k];
    double *e = (double *)malloc(sizeof(double) * (size_t)(N[k] + 1));
    oracle_strat_edges(g0, N[k], mdl->mu[k], mdl->L[k], e);
    layer_grid lg;
    layer_grid_init(&lg, g1, N[k + 1], 1);
    int32_t *ck = counts + coff;
    memset(ck, 0, sizeof(int32_t) * (size_t)N[k] * N[k + 1]);
    for (int32_t i = 0; i < N[k]; ++i) {
      const int64_t Mi = oracle_strat_row(e, i, M, alloc);
      for (int64_t t = 0; t < Mi; ++t) {
        float x, y;
        oracle_strat_pair(mdl, k, e, i, (uint64_t)t, seed, contract, &x, &y);
        ck[(int64_t)i * N[k + 1] + layer_cell(&lg, &y)] += 1;
      }
    }
    free(lg.aux);
    free(e);
    poff += N[k];
    coff += (int64_t)N[k] * N[k + 1];
  }
  return 0;
}
