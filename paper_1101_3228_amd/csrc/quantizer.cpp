// Quadratic-optimal quantizer of the standard normal law in one dimension
// (Sec. 2, eq. Qerr), FP64 on the host.  A grid x_1 < ... < x_N is
// stationary when every point is the mean of N(0,1) over its Voronoi cell
// (a_i, a_{i+1}), a_i = (x_{i-1} + x_i) / 2:
//   F_i(x) = x_i (Phi(a_{i+1}) - Phi(a_i)) - (phi(a_i) - phi(a_{i+1})) = 0.
// The Jacobian of F is tridiagonal; Newton's method from the quantiles of
// N(0, 3) (the point density phi^{1/3} of asymptotically optimal grids)
// converges in a few tens of steps where Lloyd's fixed-point map needs
// O(N^2) sweeps.  The paper takes such grids from a precomputed table; this
// generates them.
#include <cmath>
#include <vector>

#include "qtree.h"

namespace {

double pdf(double x) { return std::isinf(x) ? 0.0 : std::exp(-0.5 * x * x) * 0.3989422804014327; }

// P(lo < Z < hi) from the nearer tail so that upper cells keep their digits
double mass(double lo, double hi) {
  if (lo > 0) return 0.5 * (std::erfc(lo * M_SQRT1_2) - std::erfc(hi * M_SQRT1_2));
  return 0.5 * (std::erfc(-hi * M_SQRT1_2) - std::erfc(-lo * M_SQRT1_2));
}

double normal_quantile(double u) {
  // bisection on the CDF (host set-up only)
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * std::erfc(-mid * M_SQRT1_2) < u) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

void residual(const std::vector<double>& x, std::vector<double>& F, std::vector<double>& lo,
              std::vector<double>& di, std::vector<double>& up) {
  const int N = (int)x.size();
  std::vector<double> a(N + 1);
  a[0] = -INFINITY;
  a[N] = INFINITY;
  for (int i = 1; i < N; ++i) a[i] = 0.5 * (x[i - 1] + x[i]);
  for (int i = 0; i < N; ++i) {
    const double P = mass(a[i], a[i + 1]);
    const double pa = pdf(a[i]), pb = pdf(a[i + 1]);
    F[i] = x[i] * P - (pa - pb);
    const double tb = std::isinf(a[i + 1]) ? 0.0 : 0.5 * pb * (x[i] - a[i + 1]);
    const double ta = std::isinf(a[i]) ? 0.0 : 0.5 * pa * (x[i] - a[i]);
    di[i] = P + tb - ta;
    up[i] = tb;   // dF_i / dx_{i+1}
    lo[i] = -ta;  // dF_i / dx_{i-1}
  }
}

// Largest |x_i - centroid_i| (the Lloyd step length); x must be increasing.
double lloyd_gap(const std::vector<double>& x, std::vector<double>* centroid) {
  const int N = (int)x.size();
  double gap = 0.0;
  for (int i = 0; i < N; ++i) {
    const double a = i == 0 ? -INFINITY : 0.5 * (x[i - 1] + x[i]);
    const double b = i + 1 == N ? INFINITY : 0.5 * (x[i] + x[i + 1]);
    const double c = (pdf(a) - pdf(b)) / mass(a, b);
    if (centroid) (*centroid)[i] = c;
    gap = std::fmax(gap, std::fabs(x[i] - c));
  }
  return gap;
}

bool increasing(const std::vector<double>& x) {
  for (size_t i = 0; i + 1 < x.size(); ++i)
    if (!(x[i] < x[i + 1])) return false;
  return true;
}

}  // namespace

extern "C" qtree_status qtree_gauss_quantizer(int32_t N, double* out) {
  if (N < 1 || !out) return QTREE_EINVAL;
  if (N == 1) {
    out[0] = 0.0;
    return QTREE_OK;
  }
  std::vector<double> x(N), F(N), lo(N), di(N), up(N), dx(N), c(N), g(N), cen(N), trial(N);
  for (int i = 0; i < N; ++i) x[i] = std::sqrt(3.0) * normal_quantile((i + 0.5) / N);
  double gap = lloyd_gap(x, &cen);
  // Newton converges quadratically down to the rounding floor of the
  // residual (~1e-13); below 1e-9 the loop stops once the gap has not halved
  // for four steps and keeps the best grid seen.
  std::vector<double> best = x;
  double best_gap = gap;
  int stall = 0;
  for (int it = 0; it < 10000 && gap > 1e-14 && stall < 4; ++it) {
    residual(x, F, lo, di, up);
    // Thomas algorithm for J dx = -F
    c[0] = up[0] / di[0];
    g[0] = -F[0] / di[0];
    for (int i = 1; i < N; ++i) {
      const double m = di[i] - lo[i] * c[i - 1];
      c[i] = up[i] / m;
      g[i] = (-F[i] - lo[i] * g[i - 1]) / m;
    }
    dx[N - 1] = g[N - 1];
    for (int i = N - 2; i >= 0; --i) dx[i] = g[i] - c[i] * dx[i + 1];
    // accept the Newton step (halved as needed) only if it keeps the grid
    // increasing and shortens the Lloyd step; otherwise take one Lloyd step
    bool taken = false;
    for (double t = 1.0; t > 1e-3; t *= 0.5) {
      for (int i = 0; i < N; ++i) trial[i] = x[i] + t * dx[i];
      if (!increasing(trial)) continue;
      const double tg = lloyd_gap(trial, nullptr);
      if (tg < gap) {
        x.swap(trial);
        taken = true;
        break;
      }
    }
    if (!taken) x = cen;
    gap = lloyd_gap(x, &cen);
    stall = (gap < 1e-9 && !(gap < 0.5 * best_gap)) ? stall + 1 : 0;
    if (gap < best_gap) {
      best_gap = gap;
      best = x;
    }
  }
  x.swap(best);
  // symmetrise (the law is symmetric; removes the last rounding asymmetry)
  for (int i = 0; i < N / 2; ++i) {
    const double v = 0.5 * (x[N - 1 - i] - x[i]);
    x[i] = -v;
    x[N - 1 - i] = v;
  }
  if (N % 2) x[N / 2] = 0.0;
  for (int i = 0; i < N; ++i) out[i] = x[i];
  return QTREE_OK;
}
