#include "tridiag.hpp"

#include <cmath>

namespace tdvp {

bool tridiag_eig(std::vector<double>& d, std::vector<double> e, std::vector<double>& z, int n) {
  z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) z[i + (size_t)n * i] = 1.0;
  if (n == 1) return true;
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      // find a negligible off-diagonal element at or after l
      int m = l;
      for (; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) + dd == dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // Wilkinson shift from the leading 2x2 block at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {  // accumulate the rotation into z
          double zk1 = z[k + (size_t)n * (i + 1)], zk = z[k + (size_t)n * i];
          z[k + (size_t)n * (i + 1)] = s * zk + c * zk1;
          z[k + (size_t)n * i] = c * zk - s * zk1;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

bool tridiag_expm_e1(const std::vector<double>& alpha, const std::vector<double>& beta,
                     std::complex<double> tau, double nrm, std::vector<std::complex<double>>& y) {
  int n = (int)alpha.size();
  std::vector<double> d = alpha, e(beta.begin(), beta.begin() + (n > 0 ? n - 1 : 0)), z;
  if (!tridiag_eig(d, e, z, n)) return false;
  y.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    std::complex<double> f = std::exp(tau * d[k]) * z[0 + (size_t)n * k] * nrm;
    for (int i = 0; i < n; ++i) y[i] += z[i + (size_t)n * k] * f;
  }
  return true;
}

}  // namespace tdvp
