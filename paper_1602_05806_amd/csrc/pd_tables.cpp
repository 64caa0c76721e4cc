// Host FP64 construction of the 1D tables (arXiv:1602.05806, Section 2.1, eqs. (matrices),
// (pSyst), (l2forward)). Computed once per context and uploaded to the device.
#include "pd_tables.h"

#include <cmath>
#include <cstring>
#include <utility>

namespace pdh {
namespace {

// n-point Gauss-Legendre rule on [-1,1] by Newton iteration on the Legendre three-term
// recurrence, mapped to [0,1].
void gauss_legendre01(int n, double* x01, double* w01) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      double pn = (n == 1) ? x : p1;
      double pnm1 = (n == 1) ? 1.0 : p0;
      dp = n * (x * pn - pnm1) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    double pn = (n == 1) ? x : p1, pnm1 = (n == 1) ? 1.0 : p0;
    dp = n * (x * pn - pnm1) / (x * x - 1.0);
    double w = 2.0 / ((1.0 - x * x) * dp * dp);
    // store ascending on [0,1]
    x01[n - 1 - i] = 0.5 * (x + 1.0);
    w01[n - 1 - i] = 0.5 * w;
  }
}

double lag(const double* xi, int n, int p, double s) {
  double v = 1.0;
  for (int q = 0; q < n; ++q)
    if (q != p) v *= (s - xi[q]) / (xi[p] - xi[q]);
  return v;
}

double dlag(const double* xi, int n, int p, double s) {
  double tot = 0.0;
  for (int r = 0; r < n; ++r) {
    if (r == p) continue;
    double v = 1.0 / (xi[p] - xi[r]);
    for (int q = 0; q < n; ++q)
      if (q != p && q != r) v *= (s - xi[q]) / (xi[p] - xi[q]);
    tot += v;
  }
  return tot;
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major), eigenvectors in
// the columns of V.
void jacobi_eig(int n, double* A, double* V, double* lam) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {          // A <- A J
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {          // A <- J^T A
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {          // V <- V J
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

}  // namespace

bool build_table(int N, Table1D* t, std::string* err) {
  if (N < 0 || N > kMaxN) {
    if (err) *err = "degree N must be in [0, 8]";
    return false;
  }
  *t = Table1D{};
  const int n = N + 1;
  t->N = N;
  t->n = n;
  gauss_legendre01(n, t->xi, t->w);
  // Quadrature for the integrals: N+2 points (exact to degree 2N+3 >= 2N).
  const int nq = N + 2;
  double qx[kMaxn + 2], qw[kMaxn + 2];
  gauss_legendre01(nq, qx, qw);
  const double* xi = t->xi;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double ir = 0, il = 0, ml = 0;
      for (int k = 0; k < nq; ++k) {
        double s = qx[k];
        ir += qw[k] * lag(xi, n, p, 0.5 + 0.5 * s) * dlag(xi, n, q, 0.5 * s);
        il += qw[k] * lag(xi, n, p, 0.5 * s) * dlag(xi, n, q, 0.5 + 0.5 * s);
        ml += qw[k] * lag(xi, n, p, 0.5 * s) * lag(xi, n, q, 0.5 + 0.5 * s);
      }
      // eq. (matrices): jump at the dual-cell midpoint plus the two half-cell integrals
      t->Rt[p * n + q] = lag(xi, n, p, 0.5) * lag(xi, n, q, 0.0) + 0.5 * ir;
      t->Lt[p * n + q] = lag(xi, n, p, 0.5) * lag(xi, n, q, 1.0) - 0.5 * il;
      t->ML[p * n + q] = 0.5 * ml;
    }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) t->MR[p * n + q] = t->ML[q * n + p];
  // Pressure blocks of eq. (pSyst) with R-bar = L~^T, L-bar = R~^T:
  //   C = L~^T M^-1 L~ + R~^T M^-1 R~,  R = -L~^T M^-1 R~,  L = R^T.
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double c = 0, r = 0;
      for (int m = 0; m < n; ++m) {
        double wi = 1.0 / t->w[m];
        c += t->Lt[m * n + p] * wi * t->Lt[m * n + q] + t->Rt[m * n + p] * wi * t->Rt[m * n + q];
        r -= t->Lt[m * n + p] * wi * t->Rt[m * n + q];
      }
      t->Cb[p * n + q] = c;
      t->Rb[p * n + q] = r;
    }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      t->Lb[p * n + q] = t->Rb[q * n + p];
      if (q > p) {   // symmetrise C against rounding
        double s = 0.5 * (t->Cb[p * n + q] + t->Cb[q * n + p]);
        t->Cb[p * n + q] = t->Cb[q * n + p] = s;
      }
    }
  for (int p = 0; p < n; ++p) {
    t->phi0[p] = lag(xi, n, p, 0.0);
    t->phi1[p] = lag(xi, n, p, 1.0);
    for (int m = 0; m < n; ++m) t->Kv[p * n + m] = t->w[m] * dlag(xi, n, p, xi[m]) / t->w[p];
    t->dphi0[p] = dlag(xi, n, p, 0.0);
    t->dphi1[p] = dlag(xi, n, p, 1.0);
  }
  for (int k = 0; k < n; ++k)
    for (int m = 0; m < n; ++m) {
      double a = 0;
      for (int j = 0; j < n; ++j) a += t->Kv[k * n + j] * dlag(xi, n, m, xi[j]);
      t->KD[k * n + m] = a;
    }
  {
    // block-Jacobi tables: S = M^-1/2 C M^-1/2 = U diag(lam) U^T, V = M^-1/2 U
    double Sm[kMaxn * kMaxn], U[kMaxn * kMaxn];
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q)
        Sm[p * n + q] = t->Cb[p * n + q] / std::sqrt(t->w[p] * t->w[q]);
    jacobi_eig(n, Sm, U, t->Plam);
    for (int p = 0; p < n; ++p)
      for (int l = 0; l < n; ++l) t->PV[p * n + l] = U[p * n + l] / std::sqrt(t->w[p]);
  }
  // Null space of (R~ - L~): the cell-periodic solutions of D P = 0. Eigenvectors of
  // S = (R~-L~)^T (R~-L~) whose eigenvalue (a squared singular value of R~-L~) is below
  // (1e-8 ||(R~, L~)||_F)^2. The scale is that of R~ and L~ themselves, not of S: for N = 1,
  // R~ - L~ vanishes up to rounding and every eigenvalue of S is rounding noise. Over degrees
  // 0..8 the null singular values are below 1e-15 and the others above 8e-3 of that norm.
  double S[kMaxn * kMaxn], V[kMaxn * kMaxn], lam[kMaxn];
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double s = 0;
      for (int m = 0; m < n; ++m)
        s += (t->Rt[m * n + p] - t->Lt[m * n + p]) * (t->Rt[m * n + q] - t->Lt[m * n + q]);
      S[p * n + q] = s;
    }
  jacobi_eig(n, S, V, lam);
  double ref2 = 0;
  for (int i = 0; i < n * n; ++i) ref2 += t->Rt[i] * t->Rt[i] + t->Lt[i] * t->Lt[i];
  t->nnull = 0;
  std::memset(t->Pnull, 0, sizeof(t->Pnull));
  for (int i = 0; i < n; ++i) {
    if (std::fabs(lam[i]) <= 1e-16 * ref2) {
      ++t->nnull;
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) t->Pnull[p * n + q] += V[p * n + i] * V[q * n + i];
    }
  }
  // The part of that kernel that is odd about the cell centre: the kernel is invariant under the
  // node reversal J (GL nodes are symmetric), so the projector onto its odd part is
  // Pnull (I - J) / 2. It spans the null space of a direction with Dirichlet pressure walls
  // (odd reflection): the odd mode for odd N, nothing for even N.
  t->nnull_odd = 0;
  double tr = 0.0;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      const double v = 0.5 * (t->Pnull[p * n + q] - t->Pnull[p * n + (n - 1 - q)]);
      t->PnullOdd[p * n + q] = v;
      if (p == q) tr += v;
    }
  t->nnull_odd = (int)std::lround(tr);
  if (t->nnull_odd == 0) std::memset(t->PnullOdd, 0, sizeof(t->PnullOdd));
  return true;
}

bool build_time_table(int M, TimeTable* t, std::string* err) {
  if (M < 0 || M > kMaxM) {
    if (err) *err = "time degree M must be in [0, 4]";
    return false;
  }
  *t = TimeTable{};
  const int m = M + 1;
  t->M = M;
  t->m = m;
  gauss_legendre01(m, t->tau, t->omega);
  double qx[kMaxm + 2], qw[kMaxm + 2];
  gauss_legendre01(m + 2, qx, qw);          // exact for the degree-2M integrands of MV
  for (int p = 0; p < m; ++p) {
    t->psi0[p] = lag(t->tau, m, p, 0.0);
    t->psi1[p] = lag(t->tau, m, p, 1.0);
    for (int q = 0; q < m; ++q) {
      double a = 0.0;
      for (int j = 0; j < m + 2; ++j) a += qw[j] * dlag(t->tau, m, p, qx[j]) * lag(t->tau, m, q, qx[j]);
      t->MV[p * m + q] = a;
    }
  }
  for (int p = 0; p < m; ++p)
    for (int q = 0; q < m; ++q) t->At[p * m + q] = t->psi1[p] * t->psi1[q] - t->MV[p * m + q];
  // Ainv by Gauss-Jordan elimination with partial pivoting
  double A[kMaxm * 2 * kMaxm];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < 2 * m; ++j) A[i * 2 * m + j] = j < m ? t->At[i * m + j] : (j - m == i);
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[r * 2 * m + c]) > std::fabs(A[piv * 2 * m + c])) piv = r;
    if (std::fabs(A[piv * 2 * m + c]) < 1e-14) {
      if (err) *err = "singular time matrix";
      return false;
    }
    if (piv != c)
      for (int j = 0; j < 2 * m; ++j) std::swap(A[c * 2 * m + j], A[piv * 2 * m + j]);
    const double d = A[c * 2 * m + c];
    for (int j = 0; j < 2 * m; ++j) A[c * 2 * m + j] /= d;
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = A[r * 2 * m + c];
      for (int j = 0; j < 2 * m; ++j) A[r * 2 * m + j] -= f * A[c * 2 * m + j];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) t->Ainv[i * m + j] = A[i * 2 * m + m + j];
  return true;
}

}  // namespace pdh
