// Cosine-series stand-in for one axis of the Gaussian spatial kernel.
//
// The paper derives its exact O(1) decomposition for the Manhattan kernel
// (Sec. 2.1, Eq. 1-2) and states that the same route serves other spatial
// weights (Sec. 2.1, closing paragraph).  A weight is decomposable into a
// fixed set of image-wide weight terms exactly when its translates span a
// finite space; the Gaussian does not, so it is replaced per axis by
//   g~(t) = a_0 + sum_{k=1..K} a_k cos(w_k t),   0 < w_1 < ... < w_K,
// whose translates do: cos(w (x - xc)) = cos(w x) cos(w xc) + sin(w x) sin(w xc),
// giving 2K + 1 weight terms per axis.
//
// Fit, at the integer offsets of the window t in [-r, r], to
// exp(-t^2 / (2 sigma^2)) with sigma = n / 4:
//   1. harmonic starts: w_k = 2 pi k / P for integer periods P in [n, 6n]
//      (every one, or ~256 evenly spread for large n), coefficients by linear
//      least squares, ranked by the 1-D maximum error;
//   2. the frequencies of the best starts are then refined by Levenberg-
//      Marquardt on the least-squares residual, the coefficients being the
//      linear least-squares solution for the current frequencies (variable
//      projection);
//   3. among the refined and harmonic candidates with well-conditioned
//      coefficients (sum |a_k| <= 2), the one with the smallest worst-case
//      error of the normalised 2-D histogram wins (max over all pixel subsets
//      of the difference in normalised weight: the larger of the positive and
//      negative parts).
// Free frequencies reach ~4e-8 at K = 3 where harmonics of one period reach
// ~6e-6 (and ~9e-7 at K = 4), so three terms per axis (49 weight terms)
// suffice for a 1e-5 histogram bar.  The search runs once per K for a
// reference side (255); other sides refine its frequencies scaled to their
// size, and fall back to the search if that does worse.  A window with r + 1 <= K + 1 distinct
// |offsets| is interpolated exactly by harmonic terms and is not refined.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace swih {

namespace {

struct Fit {
  std::vector<double> a, om;
  double err = 0.0;
  bool ok = false;
};

// Weighted least squares over t = 0..r (t and -t give identical rows, so rows
// t > 0 weigh sqrt 2) through Householder QR of the (r+1) x (K+1) matrix.
// On success fills a (K+1) and, if res is given, the weighted residuals.
bool lsq(int r, double sigma, const std::vector<double>& om, std::vector<double>& a,
         std::vector<double>* res) {
  const int m = r + 1, n = (int)om.size();
  if (m < n) return false;
  std::vector<double> A((size_t)m * n), y(m);
  for (int t = 0; t <= r; ++t) {
    const double wt = t == 0 ? 1.0 : std::sqrt(2.0);
    for (int k = 0; k < n; ++k) A[(size_t)t * n + k] = wt * std::cos(om[k] * (double)t);
    y[t] = wt * std::exp(-(double)t * t / (2.0 * sigma * sigma));
  }
  const std::vector<double> A0 = A, y0 = y;
  for (int c = 0; c < n; ++c) {
    double nrm = 0.0;
    for (int i = c; i < m; ++i) nrm += A[(size_t)i * n + c] * A[(size_t)i * n + c];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = A[(size_t)c * n + c] > 0 ? -nrm : nrm;
    std::vector<double> v(m, 0.0);
    for (int i = c; i < m; ++i) v[i] = A[(size_t)i * n + c];
    v[c] -= alpha;
    double vv = 0.0;
    for (int i = c; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = c; j < n; ++j) {
      double s = 0.0;
      for (int i = c; i < m; ++i) s += v[i] * A[(size_t)i * n + j];
      s = 2.0 * s / vv;
      for (int i = c; i < m; ++i) A[(size_t)i * n + j] -= s * v[i];
    }
    double s = 0.0;
    for (int i = c; i < m; ++i) s += v[i] * y[i];
    s = 2.0 * s / vv;
    for (int i = c; i < m; ++i) y[i] -= s * v[i];
  }
  a.assign(n, 0.0);
  for (int c = n - 1; c >= 0; --c) {
    double s = y[c];
    for (int j = c + 1; j < n; ++j) s -= A[(size_t)c * n + j] * a[j];
    const double d = A[(size_t)c * n + c];
    if (std::fabs(d) < 1e-300) return false;
    a[c] = s / d;
  }
  for (double v : a)
    if (!std::isfinite(v)) return false;
  if (res) {
    res->assign(m, 0.0);
    for (int t = 0; t < m; ++t) {
      double s = -y0[t];
      for (int k = 0; k < n; ++k) s += A0[(size_t)t * n + k] * a[k];
      (*res)[t] = s;
    }
  }
  return true;
}

double series_at(const std::vector<double>& a, const std::vector<double>& om, int t) {
  double s = 0.0;
  for (size_t k = 0; k < a.size(); ++k) s += a[k] * std::cos(om[k] * (double)t);
  return s;
}

// Worst normalised 2-D histogram error of the square window with this series.
double worst_error_2d(int r, double sigma, const std::vector<double>& a, const std::vector<double>& om) {
  const int n = 2 * r + 1;
  std::vector<double> g(n), gt(n);
  double S = 0.0, St = 0.0;
  for (int t = -r; t <= r; ++t) {
    g[t + r] = std::exp(-(double)t * t / (2.0 * sigma * sigma));
    gt[t + r] = series_at(a, om, t);
    S += g[t + r];
    St += gt[t + r];
  }
  S = S * S;
  St = St * St;
  double pos = 0.0, neg = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double d = gt[i] * gt[j] / St - g[i] * g[j] / S;
      if (d > 0) pos += d; else neg -= d;
    }
  return pos > neg ? pos : neg;
}

double worst_error_1d(int r, double sigma, const std::vector<double>& a, const std::vector<double>& om) {
  double e = 0.0;
  for (int t = 0; t <= r; ++t)
    e = std::fmax(e, std::fabs(series_at(a, om, t) - std::exp(-(double)t * t / (2.0 * sigma * sigma))));
  return e;
}

std::vector<double> harmonic(int K, double P) {
  std::vector<double> om(K + 1);
  for (int k = 0; k <= K; ++k) om[k] = 2.0 * M_PI * (double)k / P;
  return om;
}

// Frequencies from their positive gaps: w_0 = 0, w_k = w_{k-1} + |d_k|.
std::vector<double> from_gaps(const std::vector<double>& d) {
  std::vector<double> om(d.size() + 1, 0.0);
  for (size_t k = 0; k < d.size(); ++k) om[k + 1] = om[k] + std::fabs(d[k]);
  return om;
}

double cost_of(int r, double sigma, const std::vector<double>& d, std::vector<double>* res) {
  std::vector<double> a, rr;
  if (!lsq(r, sigma, from_gaps(d), a, &rr)) return INFINITY;
  double c = 0.0;
  for (double v : rr) c += v * v;
  if (res) *res = rr;
  return c;
}

// Solves the small system M x = v (n x n, row-major) by Gaussian elimination
// with partial pivoting; false if singular.
bool solve_small(std::vector<double> M, std::vector<double> v, int n, std::vector<double>& x) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(M[(size_t)i * n + c]) > std::fabs(M[(size_t)p * n + c])) p = i;
    if (std::fabs(M[(size_t)p * n + c]) < 1e-300) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)c * n + j], M[(size_t)p * n + j]);
      std::swap(v[c], v[p]);
    }
    for (int i = c + 1; i < n; ++i) {
      const double f = M[(size_t)i * n + c] / M[(size_t)c * n + c];
      for (int j = c; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)c * n + j];
      v[i] -= f * v[c];
    }
  }
  x.assign(n, 0.0);
  for (int c = n - 1; c >= 0; --c) {
    double s = v[c];
    for (int j = c + 1; j < n; ++j) s -= M[(size_t)c * n + j] * x[j];
    x[c] = s / M[(size_t)c * n + c];
  }
  return true;
}

// Levenberg-Marquardt over the K frequency gaps, forward-difference Jacobian.
std::vector<double> refine(int r, double sigma, const std::vector<double>& om0) {
  const int K = (int)om0.size() - 1;
  std::vector<double> d(K);
  for (int k = 0; k < K; ++k) d[k] = om0[k + 1] - om0[k];
  std::vector<double> res;
  double cost = cost_of(r, sigma, d, &res);
  if (!std::isfinite(cost)) return om0;
  const int m = (int)res.size();
  double lambda = 1e-3;
  for (int it = 0; it < 200 && cost > 0.0; ++it) {
    std::vector<double> J((size_t)m * K), rj;
    for (int j = 0; j < K; ++j) {
      std::vector<double> dj = d;
      const double h = 1e-7 * std::fmax(std::fabs(d[j]), 1e-6);
      dj[j] += h;
      if (!std::isfinite(cost_of(r, sigma, dj, &rj))) return from_gaps(d);
      for (int i = 0; i < m; ++i) J[(size_t)i * K + j] = (rj[i] - res[i]) / h;
    }
    std::vector<double> JtJ((size_t)K * K, 0.0), g(K, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < K; ++j) {
        g[j] -= J[(size_t)i * K + j] * res[i];
        for (int l = 0; l < K; ++l) JtJ[(size_t)j * K + l] += J[(size_t)i * K + j] * J[(size_t)i * K + l];
      }
    bool improved = false;
    double new_cost = cost;
    while (lambda < 1e12) {
      std::vector<double> M = JtJ, step;
      for (int j = 0; j < K; ++j) M[(size_t)j * K + j] += lambda * std::fmax(JtJ[(size_t)j * K + j], 1e-30);
      if (solve_small(M, g, K, step)) {
        std::vector<double> dn = d, rn;
        for (int j = 0; j < K; ++j) dn[j] += step[j];
        const double c = cost_of(r, sigma, dn, &rn);
        if (c < cost) {
          d = dn;
          res = rn;
          new_cost = c;
          improved = true;
          lambda = std::fmax(lambda / 3.0, 1e-12);
          break;
        }
      }
      lambda *= 4.0;
    }
    if (!improved) break;
    const double gain = (cost - new_cost) / cost;
    cost = new_cost;
    if (gain < 1e-12) break;
  }
  return from_gaps(d);
}

Fit candidate(int r, double sigma, const std::vector<double>& om) {
  Fit f;
  if (!lsq(r, sigma, om, f.a, nullptr)) return f;
  double sa = 0.0;
  for (double v : f.a) sa += std::fabs(v);
  for (size_t k = 1; k < om.size(); ++k)
    if (!(om[k] > om[k - 1])) return f;  // coincident frequencies: degenerate
  if (sa > 2.0) return f;                // cancelling coefficients amplify plane rounding
  f.om = om;
  f.err = worst_error_2d(r, sigma, f.a, f.om);
  f.ok = std::isfinite(f.err);
  return f;
}

Fit compute(int n, int K) {
  const int r = (n - 1) / 2;
  const double sigma = n / 4.0;
  if (r <= K) {
    // r + 1 distinct |offsets|: the first r + 1 harmonic terms interpolate them
    // exactly (the rest get zero coefficients); the period with the smallest
    // 2-D error wins.
    Fit best;
    best.err = INFINITY;
    for (int P = n; P <= 6 * n; ++P) {
      const std::vector<double> om = harmonic(K, (double)P);
      std::vector<double> a;
      if (!lsq(r, sigma, std::vector<double>(om.begin(), om.begin() + r + 1), a, nullptr)) continue;
      a.resize(K + 1, 0.0);
      const double e = worst_error_2d(r, sigma, a, om);
      if (e < best.err) {
        best.err = e;
        best.a = a;
        best.om = om;
        best.ok = true;
      }
    }
    return best;
  }
  // 1. harmonic starts ranked by the 1-D error
  struct Start {
    double e1;
    int P;
  };
  std::vector<Start> starts;
  std::vector<double> a;
  // at most ~256 periods, evenly spread, so large windows fit quickly
  const int stepP = std::max(1, 5 * n / 256);
  for (int P = n; P <= 6 * n; P += stepP) {
    if (!lsq(r, sigma, harmonic(K, (double)P), a, nullptr)) continue;
    starts.push_back({worst_error_1d(r, sigma, a, harmonic(K, (double)P)), P});
  }
  std::sort(starts.begin(), starts.end(), [](const Start& x, const Start& y) {
    return x.e1 < y.e1 || (x.e1 == y.e1 && x.P < y.P);
  });
  // 2. refine the best few and a spread of periods
  std::vector<int> Ps;
  for (size_t i = 0; i < starts.size() && i < 4; ++i) Ps.push_back(starts[i].P);
  for (int f = 1; f <= 6; ++f) Ps.push_back(f * n);
  Fit best;
  best.err = INFINITY;
  auto consider = [&](const Fit& f) {
    if (f.ok && f.err < best.err) best = f;
  };
  for (int P : Ps) {
    const std::vector<double> om0 = harmonic(K, (double)P);
    consider(candidate(r, sigma, om0));
    consider(candidate(r, sigma, refine(r, sigma, om0)));
  }
  return best;
}

// The best frequencies scale as 1 / n (the kernel's shape is fixed relative to
// the window), so a window of another side starts from a reference fit scaled
// by n_ref / n and needs only the refinement: ~0.1-1 ms instead of the search.
constexpr int kRefSide = 255;

Fit compute_scaled(int n, int K, const Fit& ref) {
  const int r = (n - 1) / 2;
  const double sigma = n / 4.0;
  std::vector<double> om0(ref.om.size());
  for (size_t k = 0; k < om0.size(); ++k) om0[k] = ref.om[k] * (double)kRefSide / (double)n;
  return candidate(r, sigma, refine(r, sigma, om0));
}

std::mutex g_mu;
std::map<std::pair<int, int>, Fit> g_cache;

bool cached(int n, int K, Fit& f) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find({n, K});
  if (it == g_cache.end()) return false;
  f = it->second;
  return true;
}

// The reference side's fit, searched (and cached) on first use.
bool reference(int K, Fit& ref) {
  if (cached(kRefSide, K, ref)) return true;
  ref = compute(kRefSide, K);
  if (!ref.ok) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[{kRefSide, K}] = ref;
  return true;
}

}  // namespace

// Returns 0 on success, -1 for bad arguments or a failed fit.
int gauss_fit(int n, int K, double* a_out, double* om_out, double* err_out) {
  if (n < 1 || n > 4095 || (n % 2) == 0 || K < 1 || K > 8) return -1;
  Fit f;
  if (!cached(n, K, f)) {
    if (n == 1) {
      // a single offset: g(0) = 1 exactly with a_0 = 1
      f.a.assign(K + 1, 0.0);
      f.a[0] = 1.0;
      f.om = harmonic(K, 1.0);
      f.err = 0.0;
      f.ok = true;
    } else {
      Fit ref;
      if (n != kRefSide && (n - 1) / 2 > K && reference(K, ref)) {
        // refinement from the scaled reference, kept when it is as good as
        // the search finds (a worst 2-D error within 2x of the reference's)
        f = compute_scaled(n, K, ref);
        if (f.ok && f.err > 2.0 * ref.err + 1e-15) f.ok = false;
      }
      if (!f.ok) f = compute(n, K);
      if (!f.ok) return -1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[{n, K}] = f;
  }
  for (int k = 0; k <= K; ++k) {
    if (a_out) a_out[k] = f.a[k];
    if (om_out) om_out[k] = f.om[k];
  }
  if (err_out) *err_out = f.err;
  return 0;
}

// Mass of the series over t in [-r, r]: sum_t g~(t).
double gauss_axis_mass(int n, int K, const double* a, const double* om) {
  const int r = (n - 1) / 2;
  double s = 0.0;
  for (int t = -r; t <= r; ++t)
    for (int k = 0; k <= K; ++k) s += a[k] * std::cos(om[k] * (double)t);
  return s;
}

}  // namespace swih
