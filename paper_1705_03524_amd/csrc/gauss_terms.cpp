// Cosine-series stand-in for one axis of the Gaussian spatial kernel.
//
// The paper derives its exact O(1) decomposition for the Manhattan kernel
// (Sec. 2.1, Eq. 1-2) and states that the same route serves other spatial
// weights (Sec. 2.1, closing paragraph).  A weight is decomposable into a
// fixed set of image-wide weight terms exactly when its translates span a
// finite space; the Gaussian does not, so it is replaced per axis by
//   g~(t) = sum_{k=0..K} a_k cos(2 pi k t / P)
// whose translates do: cos(w (x - xc)) = cos(w x) cos(w xc) + sin(w x) sin(w xc).
// The coefficients are least-squares fitted at the integer offsets of the
// window, t in [-r, r], to exp(-t^2 / (2 sigma^2)) with sigma = n / 4, and the
// integer period P is chosen for the smallest worst-case error of the
// normalised 2-D histogram (max over all pixel subsets of the difference in
// normalised weight, i.e. the larger of the positive and negative parts)
// among the periods with the smallest 1-D maximum error.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace swih {

namespace {

struct Fit {
  std::vector<double> a;
  int P = 0;
  double err = 0.0;
};

// Weighted least squares on t = 0..r (t and -t give identical rows) through
// Householder QR of the (r+1) x (K+1) matrix.
static bool lsq_fit(int r, double sigma, int K, int P, std::vector<double>& a) {
  const int m = r + 1, n = K + 1;
  if (m < n) return false;
  std::vector<double> A((size_t)m * n), y(m);
  for (int t = 0; t <= r; ++t) {
    const double wt = t == 0 ? 1.0 : std::sqrt(2.0);
    for (int k = 0; k <= K; ++k) {
      const long ph = ((long)k * t) % P;
      A[(size_t)t * n + k] = wt * std::cos(2.0 * M_PI * (double)ph / (double)P);
    }
    y[t] = wt * std::exp(-(double)t * t / (2.0 * sigma * sigma));
  }
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
  return true;
}

static void profiles(int r, double sigma, int P, const std::vector<double>& a,
                     std::vector<double>& g, std::vector<double>& gt) {
  const int n = 2 * r + 1;
  g.resize(n);
  gt.resize(n);
  for (int t = -r; t <= r; ++t) {
    g[t + r] = std::exp(-(double)t * t / (2.0 * sigma * sigma));
    double s = 0.0;
    const long at = t < 0 ? -(long)t : (long)t;
    for (size_t k = 0; k < a.size(); ++k) {
      const long ph = ((long)k * at) % P;
      s += a[k] * std::cos(2.0 * M_PI * (double)ph / (double)P);
    }
    gt[t + r] = s;
  }
}

// Worst normalised 2-D histogram error of the square window with this series.
static double worst_error_2d(const std::vector<double>& g, const std::vector<double>& gt) {
  double S = 0.0, St = 0.0;
  for (double v : g) S += v;
  for (double v : gt) St += v;
  S = S * S;
  St = St * St;
  double pos = 0.0, neg = 0.0;
  const size_t n = g.size();
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) {
      const double d = gt[i] * gt[j] / St - g[i] * g[j] / S;
      if (d > 0) pos += d; else neg -= d;
    }
  return pos > neg ? pos : neg;
}

static double worst_error_1d(const std::vector<double>& g, const std::vector<double>& gt) {
  double e = 0.0;
  for (size_t i = 0; i < g.size(); ++i) e = std::fmax(e, std::fabs(g[i] - gt[i]));
  return e;
}

static Fit compute(int n, int K) {
  const int r = (n - 1) / 2;
  const double sigma = n / 4.0;
  // A window with r + 1 <= K distinct |offsets| is interpolated exactly by its
  // first r + 1 terms; the remaining coefficients are zero.
  const int Ke = K < r ? K : r;
  // Every integer period in [n, 6n] is fitted and ranked by the cheap 1-D
  // maximum error; the best few are then ranked by the 2-D criterion, which
  // costs n^2 each.
  constexpr int kFinalists = 8;
  struct Cand {
    double e1;
    int P;
  };
  std::vector<Cand> cands;
  std::vector<double> a, g, gt;
  for (int P = n; P <= 6 * n; ++P) {
    if (!lsq_fit(r, sigma, Ke, P, a)) continue;
    a.resize(K + 1, 0.0);
    profiles(r, sigma, P, a, g, gt);
    cands.push_back({worst_error_1d(g, gt), P});
  }
  std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) {
    return x.e1 < y.e1 || (x.e1 == y.e1 && x.P < y.P);
  });
  if (cands.size() > kFinalists) cands.resize(kFinalists);
  Fit best;
  best.err = INFINITY;
  for (const Cand& c : cands) {
    lsq_fit(r, sigma, Ke, c.P, a);
    a.resize(K + 1, 0.0);
    profiles(r, sigma, c.P, a, g, gt);
    const double e = worst_error_2d(g, gt);
    if (e < best.err || (e == best.err && c.P < best.P)) {
      best.err = e;
      best.P = c.P;
      best.a = a;
    }
  }
  return best;
}

std::mutex g_mu;
std::map<std::pair<int, int>, Fit> g_cache;

}  // namespace

// Returns 0 on success, -1 for bad arguments or a failed fit.
int gauss_fit(int n, int K, double* a_out, int* P_out, double* err_out) {
  if (n < 1 || n > 4095 || (n % 2) == 0 || K < 1 || K > 8) return -1;
  Fit f;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find({n, K});
    if (it != g_cache.end()) f = it->second;
  }
  if (f.P == 0) {
    if (n == 1) {
      // a single offset: g(0) = 1 exactly with a_0 = 1
      f.a.assign(K + 1, 0.0);
      f.a[0] = 1.0;
      f.P = 1;
      f.err = 0.0;
    } else {
      f = compute(n, K);
      if (f.P == 0) return -1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[{n, K}] = f;
  }
  if (a_out)
    for (int k = 0; k <= K; ++k) a_out[k] = f.a[k];
  if (P_out) *P_out = f.P;
  if (err_out) *err_out = f.err;
  return 0;
}

// Mass of the series over t in [-r, r]: sum_t g~(t).
double gauss_axis_mass(int n, int K, const double* a, int P) {
  const int r = (n - 1) / 2;
  double s = 0.0;
  for (int t = -r; t <= r; ++t) {
    const long at = t < 0 ? -(long)t : (long)t;
    for (int k = 0; k <= K; ++k) {
      const long ph = ((long)k * at) % P;
      s += a[k] * std::cos(2.0 * M_PI * (double)ph / (double)P);
    }
  }
  return s;
}

}  // namespace swih
