// Host-side numerics of libbse (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstddef>

namespace bse_host {

uint64_t splitmix64_draw(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void stochastic_signs(uint64_t seed, int n_stoch, int n_occ, int8_t* xi) {
  for (int l = 0; l < n_stoch; ++l)
    for (int s = 0; s < n_occ; ++s)
      xi[(size_t)l * n_occ + s] =
          (splitmix64_draw(seed, (uint64_t)l * n_occ + s) >> 63) == 0 ? (int8_t)1 : (int8_t)-1;
}

void time_weights(int n_steps, double dt, double gamma, double* w) {
  for (int n = 0; n <= n_steps; ++n) {
    const double t = n * dt;
    const double c = (n == 0 || n == n_steps) ? 0.5 : 1.0;
    w[n] = c * std::exp(-0.5 * gamma * gamma * t * t) * dt;
  }
}

// Sturm counts (eigenvalues of T below x) at nx points at once: the points'
// recurrences are independent, so interleaving them keeps the divider busy.
void sturm_counts(const std::vector<double>& a, const std::vector<double>& b2, int m, const double* x, int nx,
                  int* cnt) {
  constexpr int XB = 32;
  for (int x0 = 0; x0 < nx; x0 += XB) {
    const int nb = std::min(XB, nx - x0);
    double q[XB];
    int c[XB];
    for (int j = 0; j < nb; ++j) {
      q[j] = a[0] - x[x0 + j];
      c[j] = q[j] < 0;
    }
    for (int i = 1; i < m; ++i)
      for (int j = 0; j < nb; ++j) {
        const double qq = (std::fabs(q[j]) < 1e-300) ? 1e-300 : q[j];
        q[j] = a[i] - x[x0 + j] - b2[i - 1] / qq;
        c[j] += q[j] < 0;
      }
    for (int j = 0; j < nb; ++j) cnt[x0 + j] = c[j];
  }
}

// The k lowest eigenpairs of the symmetric tridiagonal T (diagonal a,
// off-diagonal b): bisection on Sturm counts until each bracket is below
// tol relative to its magnitude, then inverse iteration.
void tridiag_lowest(const std::vector<double>& a, const std::vector<double>& b, int m, int k,
                    std::vector<double>& theta, std::vector<std::vector<double>>& vecs, double tol) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const double span = std::max(hi - lo, 1e-30);
  // a zero pivot of the shifted elimination is replaced by eps |T| (the
  // matrix scale), so that the solve stays finite (a 1 x 1 T, or a shift
  // that hits an eigenvalue exactly)
  const double tscale = std::max(std::max(std::fabs(lo), std::fabs(hi)), 1e-300);
  const double piv0 = 2.220446049250313e-16 * tscale;
  std::vector<double> b2(std::max(m - 1, 1));
  for (int i = 0; i + 1 < m; ++i) b2[i] = b[i] * b[i];
  // bisection of the k lowest eigenvalues, all brackets advanced together
  std::vector<double> l(k, lo - 1e-12 * span), h(k, hi + 1e-12 * span), mid(k);
  std::vector<int> act(k), cnt(k);
  for (int it = 0; it < 200; ++it) {
    int na = 0;
    for (int j = 0; j < k; ++j)
      if (h[j] - l[j] > tol * std::max(1.0, std::fabs(l[j]) + std::fabs(h[j]))) {
        act[na] = j;
        mid[na++] = 0.5 * (l[j] + h[j]);
      }
    if (!na) break;
    sturm_counts(a, b2, m, mid.data(), na, cnt.data());
    for (int q = 0; q < na; ++q) {
      const int j = act[q];
      if (cnt[q] > j) h[j] = mid[q]; else l[j] = mid[q];
    }
  }
  theta.assign(k, 0.0);
  for (int j = 0; j < k; ++j) theta[j] = 0.5 * (l[j] + h[j]);
  vecs.assign(k, std::vector<double>(m, 0.0));
  uint64_t seed = 977;
  for (int j = 0; j < k; ++j) {
    std::vector<double>& y = vecs[j];
    for (int i = 0; i < m; ++i) {
      seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
      y[i] = ((seed >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    }
    const double sh = theta[j] + 1e-13 * span;
    for (int it = 0; it < 4; ++it) {
      // solve (T - sh I) z = y by Gaussian elimination with partial pivoting
      std::vector<double> dl(m), d(m), du(m), du2(m, 0.0), z = y;
      for (int i = 0; i < m; ++i) { d[i] = a[i] - sh; if (i < m - 1) { du[i] = b[i]; dl[i] = b[i]; } }
      std::vector<int> piv(m, 0);
      for (int i = 0; i < m - 1; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
          if (d[i] == 0.0) d[i] = piv0;
          const double f = dl[i] / d[i];
          dl[i] = f;
          d[i + 1] -= f * du[i];
        } else {
          const double f = d[i] / dl[i];
          d[i] = dl[i];
          dl[i] = f;
          const double t = du[i];
          du[i] = d[i + 1];
          d[i + 1] = t - f * d[i + 1];
          if (i < m - 2) { du2[i] = du[i + 1]; du[i + 1] = -f * du[i + 1]; }
          piv[i] = 1;
        }
      }
      if (d[m - 1] == 0.0) d[m - 1] = piv0;
      for (int i = 0; i < m - 1; ++i) {
        if (piv[i]) { const double t = z[i]; z[i] = z[i + 1]; z[i + 1] = t - dl[i] * z[i + 1]; }
        else z[i + 1] -= dl[i] * z[i];
      }
      z[m - 1] /= d[m - 1];
      if (m > 1) z[m - 2] = (z[m - 2] - du[m - 2] * z[m - 1]) / d[m - 2];
      for (int i = m - 3; i >= 0; --i) z[i] = (z[i] - du[i] * z[i + 1] - du2[i] * z[i + 2]) / d[i];
      // orthogonalise against earlier vectors (degenerate clusters)
      for (int q = 0; q < j; ++q) {
        double c = 0;
        for (int i = 0; i < m; ++i) c += vecs[q][i] * z[i];
        for (int i = 0; i < m; ++i) z[i] -= c * vecs[q][i];
      }
      // normalise after scaling by the largest component (no overflow of
      // the squares when the shift is within rounding of the eigenvalue)
      double mx = 0;
      for (int i = 0; i < m; ++i) mx = std::max(mx, std::fabs(z[i]));
      if (!(mx > 0) || !std::isfinite(mx)) break;   // keep the previous iterate
      double nrm = 0;
      for (int i = 0; i < m; ++i) nrm += (z[i] / mx) * (z[i] / mx);
      nrm = std::sqrt(nrm) * mx;
      for (int i = 0; i < m; ++i) y[i] = z[i] / nrm;
    }
  }
}

// Least squares of omega[b][m] = c_m + e v[b]: with box means removed,
// e = sum_bm (omega_bm - mean_b omega_bm)(v_b - mean v) / (n_exc sum_b (v_b - mean v)^2).
const char* fit_box_correction(int n_box, int n_exc, const double* omega, const double* v, double* eps_inv,
                               double* c, double* w_k0) {
  if (n_box < 2 || n_exc < 1 || !omega || !v || !eps_inv || !w_k0)
    return "bse_fit_box_correction: need n_box >= 2, n_exc >= 1 and non-null buffers";
  for (int i = 0; i < n_box * n_exc; ++i)
    if (!std::isfinite(omega[i])) return "bse_fit_box_correction: non-finite omega";
  double vm = 0, vmax = 0;
  for (int b = 0; b < n_box; ++b) {
    if (!std::isfinite(v[b])) return "bse_fit_box_correction: non-finite v_bndry";
    vm += v[b];
    vmax = std::max(vmax, std::fabs(v[b]));
  }
  vm /= n_box;
  double spread = 0, den = 0;
  for (int b = 0; b < n_box; ++b) {
    spread = std::max(spread, std::fabs(v[b] - vm));
    den += (v[b] - vm) * (v[b] - vm);
  }
  if (!(spread > 1e-12 * std::max(vmax, 1e-300)))
    return "bse_fit_box_correction: the boxes' boundary potentials coincide";
  std::vector<double> om_mean(n_exc, 0.0);
  for (int b = 0; b < n_box; ++b)
    for (int m = 0; m < n_exc; ++m) om_mean[m] += omega[(size_t)b * n_exc + m];
  for (int m = 0; m < n_exc; ++m) om_mean[m] /= n_box;
  double num = 0;
  for (int b = 0; b < n_box; ++b)
    for (int m = 0; m < n_exc; ++m) num += (omega[(size_t)b * n_exc + m] - om_mean[m]) * (v[b] - vm);
  const double e = num / (n_exc * den);
  *eps_inv = e;
  if (c)
    for (int m = 0; m < n_exc; ++m) c[m] = om_mean[m] - e * vm;
  for (int b = 0; b < n_box; ++b) w_k0[b] = e * v[b];
  return nullptr;
}

}  // namespace bse_host
