#include "spectral.hpp"

#include <algorithm>
#include <cmath>

namespace hps {

std::vector<double> cheb_points(int p) {
  std::vector<double> x(p);
  const int n = p - 1;
  // -cos(pi j / n) written as a sine of a symmetric argument so that the
  // grid is exactly antisymmetric
  for (int j = 0; j <= n; ++j)
    x[j] = std::sin(M_PI * (2.0 * j - n) / (2.0 * n));
  return x;
}

std::vector<double> legendre_roots(int q) {
  std::vector<double> x(q);
  for (int k = 0; k < q; ++k) {
    double t = std::cos(M_PI * (k + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int m = 1; m < q; ++m) {
        double p2 = ((2.0 * m + 1.0) * t * p1 - m * p0) / (m + 1.0);
        p0 = p1;
        p1 = p2;
      }
      // P_q = p1, P_{q-1} = p0;  P_q' = q (t P_q - P_{q-1}) / (t^2 - 1)
      double dp = q * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    x[k] = t;
  }
  std::sort(x.begin(), x.end());
  // enforce the symmetry of the root set
  for (int k = 0; k < q / 2; ++k) {
    double a = 0.5 * (x[q - 1 - k] - x[k]);
    x[k] = -a;
    x[q - 1 - k] = a;
  }
  if (q % 2) x[q / 2] = 0.0;
  return x;
}

std::vector<double> bary_weights(const std::vector<double> &x) {
  const int n = (int)x.size();
  std::vector<double> w(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) w[j] /= (x[j] - x[k]);
  return w;
}

std::vector<double> diff_matrix(const std::vector<double> &x) {
  const int n = (int)x.size();
  std::vector<double> w = bary_weights(x);
  std::vector<double> D(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d = (w[j] / w[i]) / (x[i] - x[j]);
      D[i * n + j] = d;
      s += d;
    }
    D[i * n + i] = -s;
  }
  return D;
}

std::vector<double> interp_matrix(const std::vector<double> &src,
                                  const std::vector<double> &dst) {
  const int n = (int)src.size(), m = (int)dst.size();
  std::vector<double> w = bary_weights(src);
  std::vector<double> P(m * n, 0.0);
  for (int i = 0; i < m; ++i) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (dst[i] == src[j]) hit = j;
    if (hit >= 0) {
      P[i * n + hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += w[j] / (dst[i] - src[j]);
    for (int j = 0; j < n; ++j) P[i * n + j] = (w[j] / (dst[i] - src[j])) / den;
  }
  return P;
}

}  // namespace hps
