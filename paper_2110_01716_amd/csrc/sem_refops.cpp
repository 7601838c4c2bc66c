// Reference-element operators on Gauss-Lobatto-Legendre points (host, FP64).
//
// The SEM basis is the tensor product of Lagrange interpolants h_i on the
// N+1 GLL points (Algorithms, eq. field1); derivatives are applied as the
// small dense matrix Dhat_il = h_l'(xi_i) (footnote to eq. field1); pMG moves
// between orders with the 1D interpolation matrix Jhat (Implementation, pMG
// paragraph).
//
// Constructions used here:
//   * interior GLL points are the roots of P_N'; Newton's method on P_N' with
//     P_N'' from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P, started
//     from the Chebyshev-Gauss-Lobatto points; weights 2/(N(N+1) P_N(x)^2);
//   * Dhat and Jhat from barycentric Lagrange interpolation (Berrut &
//     Trefethen, SIAM Review 2004): weights lam_j = 1/prod_{k!=j}(x_j-x_k),
//     D_ij = (lam_j/lam_i)/(x_i-x_j), D_ii = -sum_{j!=i} D_ij.
#include <cmath>

#include "sem_internal.h"

namespace sem {

namespace {

// P_N(x) and P_N'(x) by the three-term recurrence and P_N' = N (x P_N - P_{N-1})/(x^2-1).
void legendre_and_deriv(int N, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x;
  if (N == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  *dP = N * (x * p1 - p0) / (x * x - 1.0);
}

double legendre(int N, double x) {
  double p0 = 1.0, p1 = x;
  if (N == 0) return 1.0;
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

void barycentric_weights(int n, const double* x, double* lam) {
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (x[j] - x[k]);
    lam[j] = 1.0 / prod;
  }
}

}  // namespace

void gll_points(int N, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -std::cos(pi * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_and_deriv(N, xi, &P, &dP);
      double d2P = (2.0 * xi * dP - N * (N + 1.0) * P) / (1.0 - xi * xi);
      double step = dP / d2P;
      xi -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    x[i] = xi;
  }
  // mirror symmetry: average each pair so that x[N-i] = -x[i] exactly
  for (int i = 1; i < N - i; ++i) {
    double a = 0.5 * (x[N - i] - x[i]);
    x[i] = -a;
    x[N - i] = a;
  }
  if (N % 2 == 0) x[N / 2] = 0.0;
  if (w) {
    for (int i = 0; i <= N; ++i) {
      double P = legendre(N, x[i]);
      w[i] = 2.0 / (N * (N + 1.0) * P * P);
    }
  }
}

void deriv_matrix(int N, double* D) {
  const int n = N + 1;
  double x[kMaxNP], lam[kMaxNP];
  gll_points(N, x, nullptr);
  barycentric_weights(n, x, lam);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      double v = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[i * n + j] = v;
      diag -= v;
    }
    D[i * n + i] = diag;
  }
  // the corner values are known exactly
  D[0] = -N * (N + 1) / 4.0;
  D[N * n + N] = N * (N + 1) / 4.0;
}

void lagrange_matrix(int n_src, const double* src, int n_dst, const double* dst, double* M) {
  double lam[kMaxNP];
  barycentric_weights(n_src, src, lam);
  for (int i = 0; i < n_dst; ++i) {
    int hit = -1;
    for (int j = 0; j < n_src; ++j)
      if (dst[i] == src[j]) hit = j;
    if (hit >= 0) {
      for (int j = 0; j < n_src; ++j) M[i * n_src + j] = (j == hit) ? 1.0 : 0.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n_src; ++j) den += lam[j] / (dst[i] - src[j]);
    for (int j = 0; j < n_src; ++j) M[i * n_src + j] = (lam[j] / (dst[i] - src[j])) / den;
  }
}

}  // namespace sem

extern "C" int sem_reference(int N, double* nodes, double* weights, double* D) {
  return sem::guarded([&] {
    if (N < 1 || N > sem::kMaxN) sem::fail(SEM_EINVAL, "sem_reference: N=%d outside [1,%d]", N, sem::kMaxN);
    double x[sem::kMaxNP], w[sem::kMaxNP];
    sem::gll_points(N, x, w);
    for (int i = 0; i <= N; ++i) {
      if (nodes) nodes[i] = x[i];
      if (weights) weights[i] = w[i];
    }
    if (D) sem::deriv_matrix(N, D);
  });
}

extern "C" int sem_interpolation(int Nc, int Nf, double* J) {
  return sem::guarded([&] {
    if (Nc < 1 || Nc > sem::kMaxN || Nf < 1 || Nf > sem::kMaxN)
      sem::fail(SEM_EINVAL, "sem_interpolation: orders (%d,%d) outside [1,%d]", Nc, Nf, sem::kMaxN);
    if (!J) sem::fail(SEM_EINVAL, "sem_interpolation: J is NULL");
    double xc[sem::kMaxNP], xf[sem::kMaxNP];
    sem::gll_points(Nc, xc, nullptr);
    sem::gll_points(Nf, xf, nullptr);
    sem::lagrange_matrix(Nc + 1, xc, Nf + 1, xf, J);
  });
}
