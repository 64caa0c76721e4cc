// Once-per-step operators of the fractional step (arXiv:1602.05806 Section 2.1-2.3):
//   * 1D two-cell line operators along one direction: the weak gradient D (eq. weakgradient,
//     velocity update eq. LOvelocityU), its transpose D^T (RHS of eq. LOpressure) and the L2
//     projections between main and dual grids (eqs. l2forward, l2backward);
//   * the explicit DG convection term with the Rusanov flux (eqs. Fu-Fw) combined with one stage
//     of the third-order TVD Runge-Kutta scheme, and the transpose of its linearisation (adjoint
//     of one stage, for gradients through the step).
// These run a few times per time step, not per CG iteration; they read their operands directly
// from global memory (one thread per output DoF, neighbour lines served from L1/L2).
#include "pd_device.h"
#include "pd_launch.h"

namespace pdk {

namespace {

template <int N>
struct LineMats {
  double A0[(N + 1) * (N + 1)], A1[(N + 1) * (N + 1)], w[N + 1];
};

__device__ __forceinline__ long long wrapl(long long i, long long m) {
  i %= m;
  return i < 0 ? i + m : i;
}

// out[cell, l] = accum*out + coef * wperp(l) * sum_m (A0[l_d][m] in[cell+o0 e_d, l(l_d=m)]
//                                                     + A1[l_d][m] in[cell+o1 e_d, l(l_d=m)])
template <int N, int DIM>
__global__ __launch_bounds__(kBlock) void k_line(LineMats<N> M, const double* __restrict__ in,
                                                 double* __restrict__ out, int nx, int ny, int nz,
                                                 int d, int o0, int o1, double coef, int wperp,
                                                 double accum) {
  constexpr int n = N + 1, NC = DIM == 3 ? n * n * n : n * n;
  const long long ncells = (long long)nx * ny * nz;
  const long long tot = ncells * NC;
  const int sd = d == 0 ? 1 : d == 1 ? n : n * n;   // node stride along d
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
       i += (long long)gridDim.x * kBlock) {
    const long long cell = i / NC;
    const int l = (int)(i - cell * NC);
    const int l1 = l % n, l2 = (l / n) % n, l3 = DIM == 3 ? l / (n * n) : 0;
    const int ld = d == 0 ? l1 : d == 1 ? l2 : l3;
    const int lbase = l - ld * sd;
    long long ci = cell % nx, cj = (cell / nx) % ny, ck = cell / ((long long)nx * ny);
    long long c0, c1;
    if (d == 0) {
      c0 = (ck * ny + cj) * nx + wrapl(ci + o0, nx);
      c1 = (ck * ny + cj) * nx + wrapl(ci + o1, nx);
    } else if (d == 1) {
      c0 = (ck * ny + wrapl(cj + o0, ny)) * nx + ci;
      c1 = (ck * ny + wrapl(cj + o1, ny)) * nx + ci;
    } else {
      c0 = (wrapl(ck + o0, nz) * ny + cj) * nx + ci;
      c1 = (wrapl(ck + o1, nz) * ny + cj) * nx + ci;
    }
    const double* p0 = in + c0 * NC + lbase;
    const double* p1 = in + c1 * NC + lbase;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s += M.A0[ld * n + m] * p0[m * sd] + M.A1[ld * n + m] * p1[m * sd];
    double wt = 1.0;
    if (wperp) {
      if (d != 0) wt *= M.w[l1];
      if (d != 1) wt *= M.w[l2];
      if (DIM == 3 && d != 2) wt *= M.w[l3];
    }
    const double v = coef * wt * s;
    out[i] = accum == 0.0 ? v : accum * out[i] + v;
  }
}

template <int N>
struct ConvMats {
  double w[N + 1], phi0[N + 1], phi1[N + 1], Kv[(N + 1) * (N + 1)];
};

// Tables of the explicit viscous flux (explicit-viscosity variant): phi_m'(0), phi_m'(1) and
// KD[k][m] = sum_j Kv[k][j] phi_m'(xi_j) (volume term of the broken gradient).
template <int N>
struct ViscMats {
  double dphi0[N + 1], dphi1[N + 1], KD[(N + 1) * (N + 1)];
};

struct ConvPtrs {
  const double* ucur[3];
  const double* u0[3];
  double* out[3];
};

// One RK stage for component `comp` at every DoF: out = a u0 + b (ucur + dt L(ucur)) with
// L(U)_q = -sum_e h_e^-1 [ (phi_k(1) F_{e,right} - phi_k(0) F_{e,left}) / w_k
//                          - sum_m Kv[k][m] (q v_e)(m) ]   (collocated at the GL nodes)
// and the Rusanov flux F = (q^- v^- + q^+ v^+)/2 - s (q^+ - q^-)/2, s = 2 max(|v_e^-|, |v_e^+|).
// VISC = 1 (explicit-viscosity variant): the flux gains -nu dq/dx_e (broken gradient at the
// nodes; on faces the average of the two sides' normal derivatives) and s the viscous part
// 2 nu (2N+1) / (h_e sqrt(pi/2)); conv = 0 drops the convective flux (unsteady Stokes).
// cr != 0: out = a u0 + cr L(ucur) instead (the rate itself, b and dt unused).
template <int N, int DIM, int VISC>
__global__ __launch_bounds__(kBlock) void k_convect(ConvMats<N> M, ViscMats<N> VM, ConvPtrs P,
                                                    int nx, int ny, int nz, double h0, double h1,
                                                    double h2, double a, double b, double dt,
                                                    double nu, int conv, double cr) {
  constexpr int n = N + 1, NC = DIM == 3 ? n * n * n : n * n;
  const long long ncells = (long long)nx * ny * nz;
  const long long tot = ncells * NC;
  const double hh[3] = {h0, h1, h2};
  for (long long gi = (long long)blockIdx.x * kBlock + threadIdx.x; gi < tot * DIM;
       gi += (long long)gridDim.x * kBlock) {
    const int comp = (int)(gi / tot);
    const long long i = gi - comp * tot;
    const long long cell = i / NC;
    const int l = (int)(i - cell * NC);
    const int lidx[3] = {l % n, (l / n) % n, DIM == 3 ? l / (n * n) : 0};
    const long long ci = cell % nx, cj = (cell / nx) % ny, ck = cell / ((long long)nx * ny);
    const double* q = P.ucur[comp];
    double rate = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
      const int sd = e == 0 ? 1 : e == 1 ? n : n * n;
      const int le = lidx[e];
      const int lbase = l - le * sd;
      long long cl, cr;
      if (e == 0) {
        cl = (ck * ny + cj) * nx + wrapl(ci - 1, nx);
        cr = (ck * ny + cj) * nx + wrapl(ci + 1, nx);
      } else if (e == 1) {
        cl = (ck * ny + wrapl(cj - 1, ny)) * nx + ci;
        cr = (ck * ny + wrapl(cj + 1, ny)) * nx + ci;
      } else {
        cl = (wrapl(ck - 1, nz) * ny + cj) * nx + ci;
        cr = (wrapl(ck + 1, nz) * ny + cj) * nx + ci;
      }
      const double* ve = P.ucur[e];
      const double* qo = q + cell * NC + lbase;
      const double* vo = ve + cell * NC + lbase;
      const double* ql = q + cl * NC + lbase;
      const double* vl = ve + cl * NC + lbase;
      const double* qr = q + cr * NC + lbase;
      const double* vr = ve + cr * NC + lbase;
      double vol = 0.0, q0 = 0.0, q1 = 0.0, v0 = 0.0, v1 = 0.0;
      double qlf = 0.0, vlf = 0.0, qrf = 0.0, vrf = 0.0;
      double kd = 0.0, d0 = 0.0, d1 = 0.0, dlf = 0.0, drf = 0.0;   // VISC: reference derivatives
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double qm = qo[m * sd], vm = vo[m * sd];
        vol += M.Kv[le * n + m] * qm * vm;
        q0 += M.phi0[m] * qm;
        q1 += M.phi1[m] * qm;
        v0 += M.phi0[m] * vm;
        v1 += M.phi1[m] * vm;
        qlf += M.phi1[m] * ql[m * sd];    // left neighbour at its right face
        vlf += M.phi1[m] * vl[m * sd];
        qrf += M.phi0[m] * qr[m * sd];    // right neighbour at its left face
        vrf += M.phi0[m] * vr[m * sd];
        if (VISC) {
          kd += VM.KD[le * n + m] * qm;
          d0 += VM.dphi0[m] * qm;
          d1 += VM.dphi1[m] * qm;
          dlf += VM.dphi1[m] * ql[m * sd];
          drf += VM.dphi0[m] * qr[m * sd];
        }
      }
      double sR = 2.0 * fmax(fabs(v1), fabs(vrf));
      double sL = 2.0 * fmax(fabs(vlf), fabs(v0));
      double FR = 0.5 * (q1 * v1 + qrf * vrf);
      double FL = 0.5 * (qlf * vlf + q0 * v0);
      if (VISC) {
        if (!conv) {
          vol = 0.0;
          sR = sL = 0.0;
          FR = FL = 0.0;
        }
        const double he = hh[e];
        const double sv = 2.0 * nu * (2 * N + 1) / (he * 1.2533141373155002512);   // sqrt(pi/2)
        sR += sv;
        sL += sv;
        vol -= nu * kd / he;
        FR -= 0.5 * nu * (d1 + drf) / he;
        FL -= 0.5 * nu * (dlf + d0) / he;
      }
      FR -= 0.5 * sR * (qrf - q1);
      FL -= 0.5 * sL * (q0 - qlf);
      const double surf = (M.phi1[le] * FR - M.phi0[le] * FL) / M.w[le];
      rate -= (surf - vol) / hh[e];
    }
    const double uc = q[i];
    const double base = a != 0.0 ? a * P.u0[comp][i] : 0.0;
    P.out[comp][i] = cr != 0.0 ? base + cr * rate : base + b * (uc + dt * rate);
  }
}

struct ConvAdjPtrs {
  const double* state[3];   // stage input of the forward RK stage
  const double* obar[3];    // cotangent of the stage output
  const double* acc[3];     // optional term added with acc_coef (may alias out)
  double* out[3];
};

// Transposed linearisation of the convective rate L at one DoF. For the pair (momentum
// component c, direction e) on the line along e through the DoF (cells i-1, i, i+1), with
// g = obar_c / h_e:
//   F_bar(node)   = sum_k Kv[k][node] g_i[k]                                 (volume term)
//   Fhat_bar(R)   = -sum_k g_i[k] phi1_k / w_k + sum_k g_{i+1}[k] phi0_k / w_k  (face i+1/2)
//   Fhat_bar(L)   = -sum_k g_{i-1}[k] phi1_k / w_k + sum_k g_i[k] phi0_k / w_k  (face i-1/2)
// and, through Fhat = (q- v- + q+ v+)/2 - s (q+ - q-)/2 with s = 2 max(|v-|, |v+|) (its
// derivative taken on the branch of the forward state, |v-| >= |v+| selecting v-):
//   qpart: the cotangent of q = U_c at the DoF;  else: that of v = U_e at the DoF.
template <int N>
__device__ __forceinline__ double pair_adjoint(const ConvMats<N>& M, const double* __restrict__ ob,
                                               const double* __restrict__ q,
                                               const double* __restrict__ v, long long cl,
                                               long long co, long long cr, int NC, int lbase,
                                               int sd, int le, double he, bool qpart) {
  constexpr int n = N + 1;
  const double* obl = ob + cl * NC + lbase;
  const double* obo = ob + co * NC + lbase;
  const double* obr = ob + cr * NC + lbase;
  const double* ql = q + cl * NC + lbase;
  const double* qo = q + co * NC + lbase;
  const double* qr = q + cr * NC + lbase;
  const double* vl = v + cl * NC + lbase;
  const double* vo = v + co * NC + lbase;
  const double* vr = v + cr * NC + lbase;
  double Fb = 0.0, FR = 0.0, FL = 0.0;
  double q1o = 0.0, q0o = 0.0, v1o = 0.0, v0o = 0.0, q1l = 0.0, v1l = 0.0, q0r = 0.0, v0r = 0.0;
#pragma unroll
  for (int m = 0; m < n; ++m) {
    const double go = obo[m * sd], gl = obl[m * sd], gr = obr[m * sd];
    const double a1 = M.phi1[m] / M.w[m], a0 = M.phi0[m] / M.w[m];
    Fb += M.Kv[m * n + le] * go;
    FR += gr * a0 - go * a1;
    FL += go * a0 - gl * a1;
    const double qom = qo[m * sd], vom = vo[m * sd];
    q1o += M.phi1[m] * qom;
    q0o += M.phi0[m] * qom;
    v1o += M.phi1[m] * vom;
    v0o += M.phi0[m] * vom;
    q1l += M.phi1[m] * ql[m * sd];
    v1l += M.phi1[m] * vl[m * sd];
    q0r += M.phi0[m] * qr[m * sd];
    v0r += M.phi0[m] * vr[m * sd];
  }
  Fb /= he;
  FR /= he;
  FL /= he;
  // face i+1/2: minus side = this cell, plus side = cell i+1; face i-1/2: minus = i-1, plus = i
  const double sR = 2.0 * fmax(fabs(v1o), fabs(v0r));
  const double sL = 2.0 * fmax(fabs(v1l), fabs(v0o));
  if (qpart)
    return Fb * vo[le * sd] + M.phi1[le] * FR * (0.5 * v1o + 0.5 * sR) +
           M.phi0[le] * FL * (0.5 * v0o - 0.5 * sL);
  double vmb = 0.5 * FR * q1o;
  if (fabs(v1o) >= fabs(v0r)) vmb += 2.0 * ((v1o > 0.0) - (v1o < 0.0)) * (-0.5 * FR * (q0r - q1o));
  double vpb = 0.5 * FL * q0o;
  if (!(fabs(v1l) >= fabs(v0o))) vpb += 2.0 * ((v0o > 0.0) - (v0o < 0.0)) * (-0.5 * FL * (q0o - q1l));
  return Fb * qo[le * sd] + M.phi1[le] * vmb + M.phi0[le] * vpb;
}

// Adjoint of one RK stage: out = acc_coef acc + b (obar + dt J(state)^T obar) for every DoF of
// every component; J is the Jacobian of the convective rate L at the stage input `state`.
template <int N, int DIM>
__global__ __launch_bounds__(kBlock) void k_convect_adj(ConvMats<N> M, ConvAdjPtrs P, int nx,
                                                        int ny, int nz, double h0, double h1,
                                                        double h2, double acc_coef, double b,
                                                        double dt) {
  constexpr int n = N + 1, NC = DIM == 3 ? n * n * n : n * n;
  const long long ncells = (long long)nx * ny * nz;
  const long long tot = ncells * NC;
  const double hh[3] = {h0, h1, h2};
  for (long long gi = (long long)blockIdx.x * kBlock + threadIdx.x; gi < tot * DIM;
       gi += (long long)gridDim.x * kBlock) {
    const int comp = (int)(gi / tot);
    const long long i = gi - comp * tot;
    const long long cell = i / NC;
    const int l = (int)(i - cell * NC);
    const int lidx[3] = {l % n, (l / n) % n, DIM == 3 ? l / (n * n) : 0};
    const long long ci = cell % nx, cj = (cell / nx) % ny, ck = cell / ((long long)nx * ny);
    double jt = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
      const int sd = e == 0 ? 1 : e == 1 ? n : n * n;
      const int le = lidx[e];
      const int lbase = l - le * sd;
      long long cl, cr;
      if (e == 0) {
        cl = (ck * ny + cj) * nx + wrapl(ci - 1, nx);
        cr = (ck * ny + cj) * nx + wrapl(ci + 1, nx);
      } else if (e == 1) {
        cl = (ck * ny + wrapl(cj - 1, ny)) * nx + ci;
        cr = (ck * ny + wrapl(cj + 1, ny)) * nx + ci;
      } else {
        cl = (wrapl(ck - 1, nz) * ny + cj) * nx + ci;
        cr = (wrapl(ck + 1, nz) * ny + cj) * nx + ci;
      }
      // this DoF as momentum (pair comp, e)
      jt += pair_adjoint<N>(M, P.obar[comp], P.state[comp], P.state[e], cl, cell, cr, NC, lbase,
                            sd, le, hh[e], true);
      // this DoF as transport velocity along e = comp (pairs c, comp)
      if (e == comp) {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
          jt += pair_adjoint<N>(M, P.obar[c], P.state[c], P.state[e], cl, cell, cr, NC, lbase,
                                sd, le, hh[e], false);
      }
    }
    // L enters the stage as -(surf - vol) / h, already folded into pair_adjoint through the
    // signs of Fb (+) and of the face terms (-), so jt is J^T obar at this DoF
    const double base = P.acc[comp] ? acc_coef * P.acc[comp][i] : 0.0;
    P.out[comp][i] = base + b * (P.obar[comp][i] + dt * jt);
  }
}

inline unsigned grid_for(long long tot) {
  long long b = (tot + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <int N>
hipError_t launch_line_N(const LineLaunch& L, hipStream_t s) {
  LineMats<N> M;
  constexpr int n = N + 1;
  for (int i = 0; i < n * n; ++i) {
    M.A0[i] = L.A0[i];
    M.A1[i] = L.A1[i];
  }
  for (int i = 0; i < n; ++i) M.w[i] = L.w[i];
  const int nz = L.dim == 3 ? L.nc[2] : 1;
  const long long tot = (long long)L.nc[0] * L.nc[1] * nz * (L.dim == 3 ? n * n * n : n * n);
  if (L.dim == 3)
    hipLaunchKernelGGL((k_line<N, 3>), dim3(grid_for(tot)), dim3(kBlock), 0, s, M, L.in, L.out,
                       L.nc[0], L.nc[1], nz, L.d, L.o0, L.o1, L.coef, L.wperp, L.accum);
  else
    hipLaunchKernelGGL((k_line<N, 2>), dim3(grid_for(tot)), dim3(kBlock), 0, s, M, L.in, L.out,
                       L.nc[0], L.nc[1], nz, L.d, L.o0, L.o1, L.coef, L.wperp, L.accum);
  return hipGetLastError();
}

template <int N>
hipError_t launch_conv_N(const ConvLaunch& L, hipStream_t s) {
  ConvMats<N> M;
  constexpr int n = N + 1;
  for (int i = 0; i < n; ++i) {
    M.w[i] = L.w[i];
    M.phi0[i] = L.phi0[i];
    M.phi1[i] = L.phi1[i];
  }
  for (int i = 0; i < n * n; ++i) M.Kv[i] = L.Kv[i];
  ViscMats<N> VM;
  for (int i = 0; i < n; ++i) {
    VM.dphi0[i] = L.dphi0[i];
    VM.dphi1[i] = L.dphi1[i];
  }
  for (int i = 0; i < n * n; ++i) VM.KD[i] = L.KD[i];
  ConvPtrs P;
  for (int c = 0; c < 3; ++c) {
    P.ucur[c] = L.ucur[c];
    P.u0[c] = L.u0[c];
    P.out[c] = L.out[c];
  }
  const int nz = L.dim == 3 ? L.nc[2] : 1;
  const long long tot =
      (long long)L.nc[0] * L.nc[1] * nz * (L.dim == 3 ? n * n * n : n * n) * L.dim;
  const bool visc = L.nu > 0.0;
  const dim3 G(grid_for(tot)), B(kBlock);
  if (L.dim == 3) {
    if (visc)
      hipLaunchKernelGGL((k_convect<N, 3, 1>), G, B, 0, s, M, VM, P, L.nc[0], L.nc[1], nz, L.h[0],
                         L.h[1], L.h[2], L.a, L.b, L.dt, L.nu, L.conv, L.cr);
    else
      hipLaunchKernelGGL((k_convect<N, 3, 0>), G, B, 0, s, M, VM, P, L.nc[0], L.nc[1], nz, L.h[0],
                         L.h[1], L.h[2], L.a, L.b, L.dt, 0.0, 1, L.cr);
  } else {
    if (visc)
      hipLaunchKernelGGL((k_convect<N, 2, 1>), G, B, 0, s, M, VM, P, L.nc[0], L.nc[1], nz, L.h[0],
                         L.h[1], L.h[2], L.a, L.b, L.dt, L.nu, L.conv, L.cr);
    else
      hipLaunchKernelGGL((k_convect<N, 2, 0>), G, B, 0, s, M, VM, P, L.nc[0], L.nc[1], nz, L.h[0],
                         L.h[1], L.h[2], L.a, L.b, L.dt, 0.0, 1, L.cr);
  }
  return hipGetLastError();
}


template <int N>
hipError_t launch_conv_adj_N(const ConvAdjLaunch& L, hipStream_t s) {
  ConvMats<N> M;
  constexpr int n = N + 1;
  for (int i = 0; i < n; ++i) {
    M.w[i] = L.w[i];
    M.phi0[i] = L.phi0[i];
    M.phi1[i] = L.phi1[i];
  }
  for (int i = 0; i < n * n; ++i) M.Kv[i] = L.Kv[i];
  ConvAdjPtrs P;
  for (int c = 0; c < 3; ++c) {
    P.state[c] = L.state[c];
    P.obar[c] = L.obar[c];
    P.acc[c] = L.acc[c];
    P.out[c] = L.out[c];
  }
  const int nz = L.dim == 3 ? L.nc[2] : 1;
  const long long tot =
      (long long)L.nc[0] * L.nc[1] * nz * (L.dim == 3 ? n * n * n : n * n) * L.dim;
  if (L.dim == 3)
    hipLaunchKernelGGL((k_convect_adj<N, 3>), dim3(grid_for(tot)), dim3(kBlock), 0, s, M, P,
                       L.nc[0], L.nc[1], nz, L.h[0], L.h[1], L.h[2], L.acc_coef, L.b, L.dt);
  else
    hipLaunchKernelGGL((k_convect_adj<N, 2>), dim3(grid_for(tot)), dim3(kBlock), 0, s, M, P,
                       L.nc[0], L.nc[1], nz, L.h[0], L.h[1], L.h[2], L.acc_coef, L.b, L.dt);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_line(const LineLaunch& L, hipStream_t s) {
  switch (L.N) {
    case 0: return launch_line_N<0>(L, s);
    case 1: return launch_line_N<1>(L, s);
    case 2: return launch_line_N<2>(L, s);
    case 3: return launch_line_N<3>(L, s);
    case 4: return launch_line_N<4>(L, s);
    case 5: return launch_line_N<5>(L, s);
    case 6: return launch_line_N<6>(L, s);
    case 7: return launch_line_N<7>(L, s);
    case 8: return launch_line_N<8>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_convect_stage(const ConvLaunch& L, hipStream_t s) {
  switch (L.N) {
    case 0: return launch_conv_N<0>(L, s);
    case 1: return launch_conv_N<1>(L, s);
    case 2: return launch_conv_N<2>(L, s);
    case 3: return launch_conv_N<3>(L, s);
    case 4: return launch_conv_N<4>(L, s);
    case 5: return launch_conv_N<5>(L, s);
    case 6: return launch_conv_N<6>(L, s);
    case 7: return launch_conv_N<7>(L, s);
    case 8: return launch_conv_N<8>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdk

namespace pdk {

hipError_t launch_convect_adj_stage(const ConvAdjLaunch& L, hipStream_t s) {
  switch (L.N) {
    case 0: return launch_conv_adj_N<0>(L, s);
    case 1: return launch_conv_adj_N<1>(L, s);
    case 2: return launch_conv_adj_N<2>(L, s);
    case 3: return launch_conv_adj_N<3>(L, s);
    case 4: return launch_conv_adj_N<4>(L, s);
    case 5: return launch_conv_adj_N<5>(L, s);
    case 6: return launch_conv_adj_N<6>(L, s);
    case 7: return launch_conv_adj_N<7>(L, s);
    case 8: return launch_conv_adj_N<8>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdk
