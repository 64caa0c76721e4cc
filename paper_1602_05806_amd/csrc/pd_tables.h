// Host-side 1D reference-element tables (FP64) of the staggered spectral DG scheme,
// arXiv:1602.05806 Section 2.1: Gauss-Legendre nodal basis on [0,1], the matrices of eq. (matrices),
// the pressure blocks of eq. (pSyst), the L2-projection matrices of eq. (l2forward), and the
// cell-periodic null space of the 1D weak gradient.
#pragma once
#include <string>

namespace pdh {

constexpr int kMaxN = 8;                 // supported degrees 0..kMaxN
constexpr int kMaxn = kMaxN + 1;

struct Table1D {
  int N = 0, n = 1;
  double xi[kMaxn], w[kMaxn];            // GL nodes / weights on [0,1], sum w = 1
  double Rt[kMaxn * kMaxn];              // R~  (row p, column q), eq. (matrices)
  double Lt[kMaxn * kMaxn];              // L~
  double Cb[kMaxn * kMaxn];              // C  = L~^T M^-1 L~ + R~^T M^-1 R~  (diagonal block)
  double Rb[kMaxn * kMaxn];              // R  = -L~^T M^-1 R~  (couples cell i to i+1)
  double Lb[kMaxn * kMaxn];              // L  = R^T            (couples cell i to i-1)
  double ML[kMaxn * kMaxn], MR[kMaxn * kMaxn];   // eq. (l2forward), MR = ML^T
  double phi0[kMaxn], phi1[kMaxn];       // phi_p(0), phi_p(1)
  double Kv[kMaxn * kMaxn];              // Kv[k][m] = w_m phi_k'(xi_m) / w_k (collocated volume term)
  double dphi0[kMaxn], dphi1[kMaxn];     // phi_p'(0), phi_p'(1)
  double KD[kMaxn * kMaxn];              // KD[k][m] = sum_j Kv[k][j] phi_m'(xi_j): volume term of
                                         // the broken gradient (explicit viscous flux)
  // Generalised eigenvectors of the diagonal block: C V = M V diag(lam), V^T M V = I (C is SPD).
  // The cell-diagonal block of alpha M^{xyz} + sum_d c_d (M on the other directions) (x) C is
  // then (V^-T (x) ..) diag(alpha + sum_d c_d lam_{l_d}) (V^-1 (x) ..): the block-Jacobi
  // preconditioner is (V (x) ..) diag(1 / (alpha + sum_d c_d lam_{l_d})) (V^T (x) ..).
  double PV[kMaxn * kMaxn];              // PV[m][l]: component m of eigenvector l
  double Plam[kMaxn];
  int nnull = 0;                         // dimension of null(R~ - L~) (1 for even N, 2 for odd N)
  double Pnull[kMaxn * kMaxn];           // orthogonal projector onto null(R~ - L~)
  int nnull_odd = 0;                     // dimension of its part odd about the cell centre
  double PnullOdd[kMaxn * kMaxn];        // projector onto that part (Dirichlet directions)
};

// Fills t for degree N. Returns false (with a message) for unsupported N.
bool build_table(int N, Table1D* t, std::string* err);

// Time matrices of degree M of the space-time scheme (Section 3, eqs. tmatrix1-tmatrix3) on the
// nodal Gauss-Legendre basis psi_0..psi_M of [0, 1]: M^t = diag(omega), M1 = psi(1) psi(1)^T,
// M0 = psi(0) psi(1)^T, MV[p][q] = int psi_p' psi_q; At = M1 - MV and its inverse.
constexpr int kMaxM = 4;
constexpr int kMaxm = kMaxM + 1;
struct TimeTable {
  int M = 0, m = 1;
  double tau[kMaxm], omega[kMaxm], psi0[kMaxm], psi1[kMaxm];
  double MV[kMaxm * kMaxm], At[kMaxm * kMaxm], Ainv[kMaxm * kMaxm];
};

// Fills t for degree M (0..kMaxM). Returns false (with a message) otherwise.
bool build_time_table(int M, TimeTable* t, std::string* err);

}  // namespace pdh
