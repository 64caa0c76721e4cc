// Streaming vector kernels of the conjugate-gradient loop (arXiv:1602.05806 Section 2.1: the
// pressure system is solved by a matrix-free CG method) and of the null-space projection.
// Every reduction accumulates in FP64 and writes one partial per block; the consumer (the next
// kernel, or a single-block finalize) re-sums the partials in block order (deterministic:
// repeated runs give bit-identical scalars).
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "pd_device.h"
#include "pd_launch.h"

namespace pdk {

namespace {

constexpr int kStreamBlocks = kMaxStreamPartials;

inline unsigned stream_blocks(long long n, int per_thread) {
  long long b = (n + (long long)kBlock * per_thread - 1) / ((long long)kBlock * per_thread);
  if (b < 1) b = 1;
  if (b > kStreamBlocks) b = kStreamBlocks;
  return (unsigned)b;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(const T* __restrict__ a, const T* __restrict__ b,
                                                long long n, double* __restrict__ partials) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    s += (double)a[i] * (double)b[i];
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Single-block finalize of a stand-alone reduction.
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partials, int n,
                                                     CgState* st, int fin) {
  const double s = sum_partials<kBlock>(partials, n);
  if (threadIdx.x == 0) {
    if (fin == FIN_BNORM) {
      st->bnorm2 = s;
      st->tol2 = st->aux * st->aux * s;
    } else {
      st->aux = s;
    }
  }
}

// CG iteration k, second half: alpha_k = rho_k / <p_k, A p_k> (sigma re-summed from the apply
// kernel's block partials), r -= alpha q, block partials of <r_{k+1}, r_{k+1}>. XU = 1: also
// x += alpha p here (6 vector words per DoF). XU = 0: the x update is left to the apply kernel of
// iteration k + 1 (which reads p_k anyway) or, when the run stops first, to k_x_flush; block 0
// publishes alpha_k with xk = k (3 words per DoF).
template <typename T, int XU>
__global__ __launch_bounds__(kBlock) void k_cg_update(T* __restrict__ x, const T* __restrict__ p,
                                                      const T* __restrict__ q, T* __restrict__ r,
                                                      long long n, CgState* st, int k,
                                                      const double* __restrict__ sigpart, int nsig,
                                                      double* __restrict__ rho_next) {
  if (st->run_u != k) return;        // the apply kernel of iteration k stopped the run
  // The first J elements of this thread are loaded before sigma is reduced (latency overlap).
  constexpr int J = 4;
  const long long i0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long stride = (long long)gridDim.x * kBlock;
  T xv[XU ? J : 1], pv[XU ? J : 1], qv[J], rv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const long long i = i0 + j * stride;
    if (i < n) {
      if (XU) {
        xv[j] = x[i];
        pv[j] = p[i];
      }
      qv[j] = q[i];
      rv[j] = r[i];
    }
  }
  const double sigma = sum_partials<kBlock>(sigpart, nsig);
  const double alpha = st->rho / sigma;
  if (!(sigma > 0.0) || !isfinite(alpha)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
      st->sigma = sigma;
      st->status = -5;
      st->iter = k;
      st->done = 1;
    }
    return;
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->sigma = sigma;
    st->alpha = alpha;
    if (!XU) st->xk = k;
    st->run_a[(k + 1) & 1] = k + 1;
  }
  const T a = (T)alpha;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const long long i = i0 + j * stride;
    if (i < n) {
      if (XU) x[i] = xv[j] + a * pv[j];
      const T rn = rv[j] - a * qv[j];
      r[i] = rn;
      s += (double)rn * (double)rn;
    }
  }
  for (long long i = i0 + J * stride; i < n; i += stride) {
    if (XU) x[i] = x[i] + a * p[i];
    const T rn = r[i] - a * q[i];
    r[i] = rn;
    s += (double)rn * (double)rn;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) rho_next[blockIdx.x] = s;
}

// The deferred form (XU = 0) with 16-byte accesses (float4 / double2): q and r 16-byte aligned,
// the n % W tail elements handled element-wise. Same arithmetic per element as k_cg_update (only
// the summation order of the <r, r> partials differs); J vectors per thread (64 B of each array in
// flight in FP32 against 16 B with element accesses) are loaded before sigma is reduced.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update_vec(const T* __restrict__ q,
                                                          T* __restrict__ r, long long n,
                                                          CgState* st, int k,
                                                          const double* __restrict__ sigpart,
                                                          int nsig, double* __restrict__ rho_next) {
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int W = 16 / (int)sizeof(T);
  constexpr int J = 4;
  if (st->run_u != k) return;        // the apply kernel of iteration k stopped the run
  const long long nv = n / W;
  const V* __restrict__ qv = reinterpret_cast<const V*>(q);
  V* __restrict__ rv = reinterpret_cast<V*>(r);
  const long long i0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long stride = (long long)gridDim.x * kBlock;
  V qa[J], ra[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const long long i = i0 + j * stride;
    if (i < nv) {
      qa[j] = qv[i];
      ra[j] = rv[i];
    }
  }
  const double sigma = sum_partials<kBlock>(sigpart, nsig);
  const double alpha = st->rho / sigma;
  if (!(sigma > 0.0) || !isfinite(alpha)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
      st->sigma = sigma;
      st->status = -5;
      st->iter = k;
      st->done = 1;
    }
    return;
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->sigma = sigma;
    st->alpha = alpha;
    st->xk = k;
    st->run_a[(k + 1) & 1] = k + 1;
  }
  const T a = (T)alpha;
  double s = 0.0;
  auto upd = [&](const V& qq, V& rr) {
    rr.x = rr.x - a * qq.x;
    rr.y = rr.y - a * qq.y;
    s += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
    if constexpr (W == 4) {
      rr.z = rr.z - a * qq.z;
      rr.w = rr.w - a * qq.w;
      s += (double)rr.z * (double)rr.z + (double)rr.w * (double)rr.w;
    }
  };
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const long long i = i0 + j * stride;
    if (i < nv) {
      upd(qa[j], ra[j]);
      rv[i] = ra[j];
    }
  }
  for (long long i = i0 + J * stride; i < nv; i += stride) {
    const V qq = qv[i];
    V rr = rv[i];
    upd(qq, rr);
    rv[i] = rr;
  }
  for (long long e = nv * W + i0; e < n; e += stride) {
    const T rn = r[e] - a * q[e];
    r[e] = rn;
    s += (double)rn * (double)rn;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) rho_next[blockIdx.x] = s;
}

// After a run has stopped: the pending x += alpha_xk p_xk (p_k is in buf[(k + 1) % 2]) unless an
// apply kernel already made it. Called once per stop; the next state reset clears xk.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_x_flush(T* __restrict__ x, const T* __restrict__ pa,
                                                    const T* __restrict__ pb, long long n,
                                                    const CgState* st) {
  const int xk = st->xk;
  if (xk < 0 || st->xused == xk) return;
  const T a = (T)st->alpha;
  const T* __restrict__ p = ((xk + 1) & 1) ? pb : pa;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    x[i] = x[i] + a * p[i];
}

// r = b - q (q may be null: r = b), with block partials of <r, r>.
__global__ __launch_bounds__(kBlock) void k_residual(const double* __restrict__ b,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ r, long long n,
                                                     double* __restrict__ partials) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const double v = q ? b[i] - q[i] : b[i];
    r[i] = v;
    s += v * v;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_axpby(double a, const double* __restrict__ x, double b,
                                                  double* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];   // b == 0: y is write-only
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero(T* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    x[i] = T(0);
}

__global__ void k_state_init(CgState* st, int maxit, double rtol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->rho = 0.0;
    st->sigma = 0.0;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->bnorm2 = 0.0;
    st->tol2 = 0.0;
    st->aux = rtol;
    st->iter = 0;
    st->maxit = maxit;
    st->done = 0;
    st->status = 0;
    st->restart_k = -1;
    st->even_stop = 0;
    st->fresh = 0;
    st->scale = 1.0;
    st->xk = -1;
    st->xused = -1;
    st->idle = 0;
    st->outer = 0;
    st->run_a[0] = 0;
    st->run_a[1] = -1;
    st->run_u = -1;
  }
}

// Set the stopping data of a CG run: tol2 (squared absolute residual bound), maxit; clears done
// and lets the apply kernel of iteration k0 (the run's next iteration) run.
__global__ void k_state_set(CgState* st, int maxit, double tol2, int k0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->run_a[k0 & 1] = k0;
    st->run_a[(k0 + 1) & 1] = -1;
    st->run_u = -1;
    st->tol2 = tol2;
    st->maxit = maxit;
    st->done = 0;
    st->status = 0;
    st->restart_k = -1;
    st->even_stop = 0;
    st->fresh = 0;
    st->xk = -1;
    st->xused = -1;
  }
}

// r32 = (float)(r64 * inv) with block partials of <r32, r32> (in FP64).
__global__ __launch_bounds__(kBlock) void k_to_f32_dot(const double* __restrict__ r64,
                                                       float* __restrict__ r32, long long n,
                                                       double inv, double* __restrict__ partials) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const float v = (float)(inv * r64[i]);
    r32[i] = v;
    s += (double)v * (double)v;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x64 += scale * (double)d32; d32 = 0
__global__ __launch_bounds__(kBlock) void k_flush_f32(double* __restrict__ x64,
                                                      float* __restrict__ d32, long long n,
                                                      double scale) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    x64[i] += scale * (double)d32[i];
    d32[i] = 0.0f;
  }
}

struct W9 {
  double w[9];
};

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_mass(W9 W, int n, const double* __restrict__ x,
                                                 double* __restrict__ y, long long ncells) {
  const int NC = DIM == 3 ? n * n * n : n * n;
  const long long tot = ncells * NC;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
       i += (long long)gridDim.x * kBlock) {
    const int l = (int)(i % NC);
    const int l1 = l % n, l2 = (l / n) % n, l3 = l / (n * n);
    double wt = W.w[l1] * W.w[l2];
    if (DIM == 3) wt *= W.w[l3];
    y[i] = wt * x[i];
  }
}

// ---- cell-block Jacobi preconditioner (the preconditioning the paper names as future work for
// its matrix-free CG, end of Section 2.1): z = P r with P the inverse of the diagonal cell block
// of alpha M + sum_d c_d (M on the other directions) (x) C, applied per cell in the generalised
// eigenbasis of (C, M): z = (V (x) ..) diag(1 / (alpha + sum_d c_d lam_{l_d})) (V^T (x) ..) r.
template <int N>
struct PrecArgs {
  double V[(N + 1) * (N + 1)];   // V[m][l]: component m of eigenvector l
  double lam[N + 1];
  double alpha, c0, c1, c2;
};

// UPD = 1: second half of a preconditioned CG iteration k (r -= alpha_k q first, alpha_k from
// the sigma partials); UPD = 0: z = P r only. Partials of <r, z> and <r, r> per block. Each
// block takes groups of CPB whole cells (grid-stride over the groups, the next group's r and q
// loaded while the current one is transformed). A group is staged in LDS in FP64; each thread
// takes one line of nodes per direction and applies the 1D transform in registers: forward
// along x and y (and z), the diagonal scaling and the backward transform along the last
// direction in one pass, then backward along y (and x). 2d + 2 LDS passes per group, all in FP64.
template <typename T, int N, int DIM, int UPD>
__global__ __launch_bounds__(kBlock) void k_pcg_update(PrecArgs<N> P, const T* __restrict__ q,
                                                       T* __restrict__ r, T* __restrict__ z,
                                                       long long ncells, CgState* st, int k,
                                                       const double* __restrict__ sigpart,
                                                       int nsig, double* __restrict__ rz_next,
                                                       double* __restrict__ rr_next) {
  constexpr int n = N + 1, NC = DIM == 3 ? n * n * n : n * n;
  constexpr int LPC = NC / n;                          // lines per cell and direction
  constexpr int CPB = pcg_cells_per_group(N, DIM);
  constexpr int E = CPB * NC;
  constexpr int J = (E + kBlock - 1) / kBlock;         // elements per thread in the streaming phases
  __shared__ double sa[E], sb[E], sinv[NC];
  T a = T(0);
  if (UPD) {
    if (st->run_u != k) return;        // the apply kernel of iteration k stopped the run
    const double sigma = sum_partials<kBlock>(sigpart, nsig);
    const double alpha = st->rho / sigma;
    if (!(sigma > 0.0) || !isfinite(alpha)) {
      if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->sigma = sigma;
        st->status = -5;
        st->iter = k;
        st->done = 1;
      }
      return;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
      st->sigma = sigma;
      st->alpha = alpha;
      st->xk = k;
      st->run_a[(k + 1) & 1] = k + 1;
    }
    a = (T)alpha;
  }
  // reciprocals of the diagonal of the transformed cell block
  for (int l = threadIdx.x; l < NC; l += kBlock) {
    double d = P.alpha + P.c0 * P.lam[l % n] + P.c1 * P.lam[(l / n) % n];
    if (DIM == 3) d += P.c2 * P.lam[l / (n * n)];
    sinv[l] = 1.0 / d;
  }
  // 1D transform of the line of `cnt` lines starting at element `b` with stride `sd`
  auto line = [&](const double* in, double* out, int b, int sd, bool fwd, bool scale) {
    double v[n], w[n];
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = in[b + m * sd];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) acc += (fwd ? P.V[m * n + i] : P.V[i * n + m]) * v[m];
      w[i] = acc;
    }
    if (scale) {   // the last direction: diagonal scaling, then its backward transform
      const int l0 = b % NC;
#pragma unroll
      for (int i = 0; i < n; ++i) w[i] *= sinv[l0 + i * sd];
#pragma unroll
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) acc += P.V[i * n + m] * w[m];
        v[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) out[b + i * sd] = v[i];
    } else {
#pragma unroll
      for (int i = 0; i < n; ++i) out[b + i * sd] = w[i];
    }
  };
  // first element of line t (t < lines of the group) along direction d
  auto line_base = [&](int t, int d) -> int {
    const int c = t / LPC, li = t - c * LPC;
    int b;
    if (d == 0) b = li * n;                                          // x-line (l2, l3)
    else if (d == 1) b = (li / n) * n * n + (li % n);                // y-line (l1, l3)
    else b = li;                                                     // z-line (l1, l2)
    return c * NC + b;
  };
  double rr = 0.0, rz = 0.0;
  const long long ngroups = (ncells + CPB - 1) / CPB;
  T rn[J], qn[J];
  auto load = [&](long long grp) {
    const long long c0 = grp * CPB;
    const long long base = c0 * NC;
    const int ecount = (int)((ncells - c0 < CPB ? ncells - c0 : CPB) * NC);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = threadIdx.x + kBlock * j;
      if (e < ecount) {
        rn[j] = r[base + e];
        if (UPD) qn[j] = q[base + e];
      }
    }
  };
  long long grp = blockIdx.x;
  if (grp < ngroups) load(grp);
  for (; grp < ngroups; grp += gridDim.x) {
    const long long c0 = grp * CPB;
    const long long base = c0 * NC;
    const int cells = (int)(ncells - c0 < CPB ? ncells - c0 : CPB);
    const int ecount = cells * NC;
    const int lines = cells * LPC;
    double rv[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = threadIdx.x + kBlock * j;
      if (e < ecount) {
        T x = rn[j];
        if (UPD) {
          x = x - a * qn[j];
          r[base + e] = x;
        }
        rv[j] = (double)x;
        rr += rv[j] * rv[j];
        sa[e] = rv[j];
      }
    }
    if (grp + gridDim.x < ngroups) load(grp + gridDim.x);   // in flight during the transforms
    __syncthreads();
    const int t = threadIdx.x;
    if (DIM == 3) {
      if (t < lines) line(sa, sb, line_base(t, 0), 1, true, false);
      __syncthreads();
      if (t < lines) line(sb, sa, line_base(t, 1), n, true, false);
      __syncthreads();
      if (t < lines) line(sa, sa, line_base(t, 2), n * n, true, true);
      __syncthreads();
      if (t < lines) line(sa, sb, line_base(t, 1), n, false, false);
      __syncthreads();
      if (t < lines) line(sb, sa, line_base(t, 0), 1, false, false);
    } else {
      if (t < lines) line(sa, sb, line_base(t, 0), 1, true, false);
      __syncthreads();
      if (t < lines) line(sb, sb, line_base(t, 1), n, true, true);
      __syncthreads();
      if (t < lines) line(sb, sa, line_base(t, 0), 1, false, false);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = threadIdx.x + kBlock * j;
      if (e < ecount) {
        const T zv = (T)sa[e];
        z[base + e] = zv;
        rz += rv[j] * (double)zv;
      }
    }
    __syncthreads();   // sa is rewritten by the next group
  }
  rr = block_sum_all<kBlock>(rr);
  rz = block_sum_all<kBlock>(rz);
  if (threadIdx.x == 0) {
    rr_next[blockIdx.x] = rr;
    rz_next[blockIdx.x] = rz;
  }
}

// Mean kinetic energy of a dual velocity field: partials of sum_i W_i sum_d u_d,i^2 (W_i = product
// of the GL weights of node i); with g[0] non-null also g_d = gs W u_d for every component.
struct Vel3 {
  const double* u[3];
  double* g[3];
};

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_energy(W9 W, int n, Vel3 v, double gs, long long ncells,
                                                   double* __restrict__ partials) {
  const int NC = DIM == 3 ? n * n * n : n * n;
  const long long tot = ncells * NC;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
       i += (long long)gridDim.x * kBlock) {
    const int l = (int)(i % NC);
    const int l1 = l % n, l2 = (l / n) % n, l3 = l / (n * n);
    double wt = W.w[l1] * W.w[l2];
    if (DIM == 3) wt *= W.w[l3];
    double q = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double ud = v.u[d][i];
      q += ud * ud;
      if (v.g[0]) v.g[d][i] = gs * wt * ud;
    }
    s += wt * q;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[s] = bc base[s] + sum_p T[s][p] in[p] (see TimeMix); all inputs of an element are read
// before any output of it is written.
__global__ __launch_bounds__(kBlock) void k_time_mix(TimeMix X, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    double v[5], b[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      v[p] = p < X.m ? X.in[p][i] : 0.0;
      b[p] = (p < X.mo && X.base[p]) ? X.base[p][i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (q >= X.mo) break;
      double acc = X.bc * b[q];
#pragma unroll
      for (int p = 0; p < 5; ++p)
        if (p < X.m) acc += X.T[q * X.m + p] * v[p];
      X.out[q][i] = acc;
    }
  }
}

// ---- null-space projection: per-node sums over cells, then correction per node
constexpr int kNullBlocks = 256;

// per-direction projectors onto the 1D null space ((N+1)^2 each)
struct P81 {
  double P[3][81];
};

// part[b][l] = sum over the cells of block b of v(cell, l)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_node_sums(const T* __restrict__ v, long long ncells,
                                                      int NC, double* __restrict__ part) {
  __shared__ double acc[kBlock];
  __shared__ double out[kMaxNC];
  const long long per = (ncells + gridDim.x - 1) / gridDim.x;
  const long long c0 = (long long)blockIdx.x * per;
  const long long c1 = c0 + per < ncells ? c0 + per : ncells;
  column_sums<T>(v, NC, c0, c1, NC, acc, out);
  for (int l = threadIdx.x; l < NC; l += kBlock) part[(size_t)blockIdx.x * NC + l] = out[l];
}

// corr = (P (x) ... (x) P) (sum of the node partials) / ncells  (single block)
__global__ __launch_bounds__(kBlock) void k_null_finalize(const double* __restrict__ part,
                                                          int nblk, long long ncells, int NC,
                                                          int dim, int n, P81 P,
                                                          double* __restrict__ corr) {
  __shared__ double S[kMaxNC], U[kMaxNC], acc[kBlock];
  column_sums<double>(part, NC, 0, nblk, NC, acc, S);
  for (int l = threadIdx.x; l < NC; l += kBlock) S[l] = S[l] / (double)ncells;
  __syncthreads();
  for (int d = 0; d < dim; ++d) {
    int stride = 1;
    for (int e = 0; e < d; ++e) stride *= n;
    for (int l = threadIdx.x; l < NC; l += kBlock) {
      const int ld = (l / stride) % n;
      const int base = l - ld * stride;
      double s = 0.0;
      for (int m = 0; m < n; ++m) s += P.P[d][ld * n + m] * S[base + m * stride];
      U[l] = s;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < NC; l += kBlock) S[l] = U[l];
    __syncthreads();
  }
  for (int l = threadIdx.x; l < NC; l += kBlock) corr[l] = S[l];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sub_nodes(T* __restrict__ v, long long tot, int NC,
                                                      const double* __restrict__ corr) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < tot;
       i += (long long)gridDim.x * kBlock)
    v[i] = (T)((double)v[i] - corr[i % NC]);
}

}  // namespace

// Scratch of the allocation-free null-space projection: the node-sum partials of the k_node_sums
// blocks (kNullBlocks rows of at most kMaxNC doubles) followed by the correction (kMaxNC
// doubles): 1,499,904 bytes, one copy per device for the life of the process. Host code never
// uses the name `scratch` as an address (on the host it is a stand-in symbol); the device
// address comes from hipGetSymbolAddress, once per device with that device current.
constexpr size_t kNoAllocParts = (size_t)kNullBlocks * kMaxNC;
constexpr size_t kNoAllocDoubles = kNoAllocParts + kMaxNC;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t noalloc_scratch_bytes() { return kNoAllocDoubles * sizeof(double); }

hipError_t launch_project_null_noalloc(bool fp32, void* v, long long ncells, int dim, int n,
                                       const double* const Pdir[3], hipStream_t s) {
  const int NC = dim == 3 ? n * n * n : n * n;
  if (NC > kMaxNC) return hipErrorInvalidValue;
  double* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return e;
  return launch_project_null(fp32, v, ncells, dim, n, Pdir, base, base + kNoAllocParts, s);
}

unsigned stream_grid(long long n) { return stream_blocks(n, 4); }

hipError_t launch_dot(bool fp32, const void* a, const void* b, long long n, double* partials,
                      hipStream_t s) {
  const unsigned G = stream_blocks(n, 4);
  if (fp32)
    hipLaunchKernelGGL(k_dot<float>, dim3(G), dim3(kBlock), 0, s, (const float*)a,
                       (const float*)b, n, partials);
  else
    hipLaunchKernelGGL(k_dot<double>, dim3(G), dim3(kBlock), 0, s, (const double*)a,
                       (const double*)b, n, partials);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nparts, CgState* st, int fin,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nparts, st, fin);
  return hipGetLastError();
}

hipError_t launch_cg_update(bool fp32, void* x, const void* p, const void* q, void* r,
                            long long n, CgState* st, int k, const double* sigpart, int nsig,
                            double* rho_next, hipStream_t s) {
  const unsigned G = stream_blocks(n, 4);
  const bool vec = !x && ((reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(r)) & 15) == 0;
  if (vec) {
    if (fp32)
      hipLaunchKernelGGL(k_cg_update_vec<float>, dim3(G), dim3(kBlock), 0, s, (const float*)q,
                         (float*)r, n, st, k, sigpart, nsig, rho_next);
    else
      hipLaunchKernelGGL(k_cg_update_vec<double>, dim3(G), dim3(kBlock), 0, s, (const double*)q,
                         (double*)r, n, st, k, sigpart, nsig, rho_next);
    return hipGetLastError();
  }
  if (fp32) {
    if (x)
      hipLaunchKernelGGL((k_cg_update<float, 1>), dim3(G), dim3(kBlock), 0, s, (float*)x,
                         (const float*)p, (const float*)q, (float*)r, n, st, k, sigpart, nsig,
                         rho_next);
    else
      hipLaunchKernelGGL((k_cg_update<float, 0>), dim3(G), dim3(kBlock), 0, s, nullptr, nullptr,
                         (const float*)q, (float*)r, n, st, k, sigpart, nsig, rho_next);
  } else {
    if (x)
      hipLaunchKernelGGL((k_cg_update<double, 1>), dim3(G), dim3(kBlock), 0, s, (double*)x,
                         (const double*)p, (const double*)q, (double*)r, n, st, k, sigpart, nsig,
                         rho_next);
    else
      hipLaunchKernelGGL((k_cg_update<double, 0>), dim3(G), dim3(kBlock), 0, s, nullptr, nullptr,
                         (const double*)q, (double*)r, n, st, k, sigpart, nsig, rho_next);
  }
  return hipGetLastError();
}

hipError_t launch_x_flush(bool fp32, void* x, const void* pa, const void* pb, long long n,
                          const CgState* st, hipStream_t s) {
  const unsigned G = stream_blocks(n, 4);
  if (fp32)
    hipLaunchKernelGGL(k_x_flush<float>, dim3(G), dim3(kBlock), 0, s, (float*)x,
                       (const float*)pa, (const float*)pb, n, st);
  else
    hipLaunchKernelGGL(k_x_flush<double>, dim3(G), dim3(kBlock), 0, s, (double*)x,
                       (const double*)pa, (const double*)pb, n, st);
  return hipGetLastError();
}

hipError_t launch_residual(const double* b, const double* q, double* r, long long n,
                           double* partials, hipStream_t s) {
  const unsigned G = stream_blocks(n, 4);
  hipLaunchKernelGGL(k_residual, dim3(G), dim3(kBlock), 0, s, b, q, r, n, partials);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double* x, double b, double* y, long long n,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t launch_zero(bool fp32, void* x, long long n, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_zero<float>, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, (float*)x, n);
  else
    hipLaunchKernelGGL(k_zero<double>, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, (double*)x,
                       n);
  return hipGetLastError();
}

hipError_t launch_state_init(CgState* st, int maxit, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, maxit, rtol);
  return hipGetLastError();
}

hipError_t launch_state_set(CgState* st, int maxit, double tol2, int k0, hipStream_t s) {
  hipLaunchKernelGGL(k_state_set, dim3(1), dim3(64), 0, s, st, maxit, tol2, k0);
  return hipGetLastError();
}

hipError_t launch_to_f32_dot(const double* r64, float* r32, long long n, double inv,
                             double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32_dot, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, r64, r32, n,
                     inv, partials);
  return hipGetLastError();
}

hipError_t launch_flush_f32(double* x64, float* d32, long long n, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_flush_f32, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, x64, d32, n,
                     scale);
  return hipGetLastError();
}

hipError_t launch_energy(int dim, int N, const double* w, const double* const u[3],
                         double* const g[3], double gs, long long ncells, double* partials,
                         hipStream_t s) {
  W9 W;
  for (int i = 0; i < 9; ++i) W.w[i] = i <= N ? w[i] : 0.0;
  const int n = N + 1;
  const long long tot = ncells * (dim == 3 ? n * n * n : n * n);
  Vel3 v;
  for (int d = 0; d < 3; ++d) {
    v.u[d] = d < dim ? u[d] : nullptr;
    v.g[d] = (g && d < dim) ? g[d] : nullptr;
  }
  const unsigned G = stream_grid(tot);
  if (dim == 3)
    hipLaunchKernelGGL(k_energy<3>, dim3(G), dim3(kBlock), 0, s, W, n, v, gs, ncells, partials);
  else
    hipLaunchKernelGGL(k_energy<2>, dim3(G), dim3(kBlock), 0, s, W, n, v, gs, ncells, partials);
  return hipGetLastError();
}

unsigned pcg_grid(long long ncells, int dim, int N) {
  const int CPB = pcg_cells_per_group(N, dim);
  long long g = (ncells + CPB - 1) / CPB;
  if (g < 1) g = 1;
  if (g > kMaxStreamPartials) g = kMaxStreamPartials;
  return (unsigned)g;
}

template <typename T, int N, int DIM>
static hipError_t pcg_launch_NT(bool upd, const void* q, void* r, void* z, long long ncells,
                                CgState* st, int k, const double* sigpart, int nsig,
                                double* rz_next, double* rr_next, const PrecTables& tb,
                                hipStream_t s) {
  PrecArgs<N> P;
  constexpr int n = N + 1;
  for (int i = 0; i < n * n; ++i) P.V[i] = tb.V[i];
  for (int i = 0; i < n; ++i) P.lam[i] = tb.lam[i];
  P.alpha = tb.alpha;
  P.c0 = tb.coef[0];
  P.c1 = tb.coef[1];
  P.c2 = tb.coef[2];
  const dim3 G(pcg_grid(ncells, DIM, N)), B(kBlock);
  if (upd)
    hipLaunchKernelGGL((k_pcg_update<T, N, DIM, 1>), G, B, 0, s, P, (const T*)q, (T*)r, (T*)z,
                       ncells, st, k, sigpart, nsig, rz_next, rr_next);
  else
    hipLaunchKernelGGL((k_pcg_update<T, N, DIM, 0>), G, B, 0, s, P, (const T*)q, (T*)r, (T*)z,
                       ncells, st, k, sigpart, nsig, rz_next, rr_next);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t pcg_launch_N(int dim, bool upd, const void* q, void* r, void* z,
                               long long ncells, CgState* st, int k, const double* sigpart,
                               int nsig, double* rz_next, double* rr_next, const PrecTables& tb,
                               hipStream_t s) {
  return dim == 3 ? pcg_launch_NT<T, N, 3>(upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next,
                                             rr_next, tb, s)
                  : pcg_launch_NT<T, N, 2>(upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next,
                                             rr_next, tb, s);
}

template <typename T>
static hipError_t pcg_launch_T(int dim, int N, bool upd, const void* q, void* r, void* z,
                               long long ncells, CgState* st, int k, const double* sigpart,
                               int nsig, double* rz_next, double* rr_next, const PrecTables& tb,
                               hipStream_t s) {
  switch (N) {
    case 0: return pcg_launch_N<T, 0>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 1: return pcg_launch_N<T, 1>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 2: return pcg_launch_N<T, 2>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 3: return pcg_launch_N<T, 3>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 4: return pcg_launch_N<T, 4>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 5: return pcg_launch_N<T, 5>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 6: return pcg_launch_N<T, 6>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 7: return pcg_launch_N<T, 7>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    case 8: return pcg_launch_N<T, 8>(dim, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next, rr_next, tb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pcg_update(bool fp32, int dim, int N, bool upd, const void* q, void* r, void* z,
                             long long ncells, CgState* st, int k, const double* sigpart, int nsig,
                             double* rz_next, double* rr_next, const PrecTables& P, hipStream_t s) {
  if (fp32)
    return pcg_launch_T<float>(dim, N, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next,
                               rr_next, P, s);
  return pcg_launch_T<double>(dim, N, upd, q, r, z, ncells, st, k, sigpart, nsig, rz_next,
                              rr_next, P, s);
}

hipError_t launch_time_mix(const TimeMix& X, long long n, hipStream_t s) {
  if (X.m < 1 || X.m > 5 || X.mo < 1 || X.mo > 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_time_mix, dim3(stream_blocks(n, 4)), dim3(kBlock), 0, s, X, n);
  return hipGetLastError();
}

hipError_t launch_mass(int dim, int N, const double* w, const double* x, double* y,
                       long long ncells, hipStream_t s) {
  W9 W;
  for (int i = 0; i < 9; ++i) W.w[i] = i <= N ? w[i] : 0.0;
  const int n = N + 1;
  const long long tot = ncells * (dim == 3 ? n * n * n : n * n);
  if (dim == 3)
    hipLaunchKernelGGL(k_mass<3>, dim3(stream_blocks(tot, 4)), dim3(kBlock), 0, s, W, n, x, y,
                       ncells);
  else
    hipLaunchKernelGGL(k_mass<2>, dim3(stream_blocks(tot, 4)), dim3(kBlock), 0, s, W, n, x, y,
                       ncells);
  return hipGetLastError();
}

hipError_t launch_project_null(bool fp32, void* v, long long ncells, int dim, int n,
                               const double* const Pdir[3], double* part, double* corr,
                               hipStream_t s) {
  P81 P;
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < 81; ++i) P.P[d][i] = (d < dim && i < n * n) ? Pdir[d][i] : 0.0;
  const int NC = dim == 3 ? n * n * n : n * n;
  const unsigned G = ncells < kNullBlocks ? (unsigned)ncells : (unsigned)kNullBlocks;
  if (fp32)
    hipLaunchKernelGGL(k_node_sums<float>, dim3(G), dim3(kBlock), 0, s, (const float*)v, ncells,
                       NC, part);
  else
    hipLaunchKernelGGL(k_node_sums<double>, dim3(G), dim3(kBlock), 0, s, (const double*)v,
                       ncells, NC, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_null_finalize, dim3(1), dim3(kBlock), 0, s, (const double*)part, (int)G,
                     ncells, NC, dim, n, P, corr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long tot = ncells * NC;
  if (fp32)
    hipLaunchKernelGGL(k_sub_nodes<float>, dim3(stream_blocks(tot, 4)), dim3(kBlock), 0, s,
                       (float*)v, tot, NC, (const double*)corr);
  else
    hipLaunchKernelGGL(k_sub_nodes<double>, dim3(stream_blocks(tot, 4)), dim3(kBlock), 0, s,
                       (double*)v, tot, NC, (const double*)corr);
  return hipGetLastError();
}

}  // namespace pdk
