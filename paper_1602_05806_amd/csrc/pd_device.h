// Device-side shared definitions of libpd (gfx950): parameter blocks passed by value to the
// kernels, the device-resident CG scalar state and the deterministic block / grid reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdk {

constexpr int kBlock = 256;          // threads of the streaming kernels
constexpr int kMaxPartials = 1 << 16;        // blocks of one operator-apply launch
constexpr int kMaxStreamPartials = 1024;     // blocks of one streaming-kernel launch
constexpr int kMaxNC = 729;          // (N+1)^3 for N = 8

// 1D blocks of the operator of eq. (pSyst) for degree N in precision T, passed as a kernel
// argument so that every (uniform) table access is a scalar load from the kernarg segment.
template <typename T, int N>
struct Blk {
  // The 1D blocks in one of two forms (line3 reads the form line_eo selects):
  //   rows     K = [L | C | R], n x n each, row-major: L couples cell i to cell i-1, C is the
  //            diagonal block, R couples cell i to cell i+1;
  //   even/odd with J the node reversal, R = J L J and C = J C J: per row pair (p, N - p),
  //            p < (N+1)/2, the rows 1/2 (L_p + L_{N-p}) and 1/2 (L_p - L_{N-p}) (n entries
  //            each) and the halves 1/2 (C_p[m] +- C_p[N-m]), m < (N+1)/2, that act on
  //            vc[m] +- vc[N-m]; for odd N + 1 then the middle rows L_{N/2} and C_{N/2}[m <= N/2].
  static constexpr int n = N + 1, P = n / 2;
  T K[3 * n * n];
  T w[N + 1];               // GL weights (1D mass diagonal)
  template <typename Tab>
  __host__ void fill(const Tab& tb, bool eo) {
    if (!eo) {
      for (int i = 0; i < n * n; ++i) {
        K[i] = (T)tb.L[i];
        K[n * n + i] = (T)tb.C[i];
        K[2 * n * n + i] = (T)tb.R[i];
      }
    } else {
      // per pair p: [AL (n) | ACh (H1) | BL (n) | BCh (H0)], H1 = ceil(n/2), H0 = floor(n/2);
      // then for odd n the middle row [L_mid (n) | C_mid (H1)]
      constexpr int H1 = (n + 1) / 2, H0 = n / 2, PS = 3 * n;
      for (int i = 0; i < 3 * n * n; ++i) K[i] = T(0);
      for (int p = 0; p < P; ++p) {
        const int q = n - 1 - p;
        T* c = K + PS * p;
        for (int m = 0; m < n; ++m) {
          c[m] = (T)(0.5 * (tb.L[p * n + m] + tb.L[q * n + m]));
          c[n + H1 + m] = (T)(0.5 * (tb.L[p * n + m] - tb.L[q * n + m]));
        }
        for (int m = 0; m < H0; ++m) {
          c[n + m] = (T)(0.5 * (tb.C[p * n + m] + tb.C[p * n + n - 1 - m]));
          c[2 * n + H1 + m] = (T)(0.5 * (tb.C[p * n + m] - tb.C[p * n + n - 1 - m]));
        }
        if (n & 1) c[n + H0] = (T)tb.C[p * n + H0];
      }
      if (n & 1) {
        T* c = K + PS * P;
        for (int m = 0; m < n; ++m) c[m] = (T)tb.L[P * n + m];
        for (int m = 0; m < H1; ++m) c[n + m] = (T)tb.C[P * n + m];
      }
    }
    for (int i = 0; i < n; ++i) w[i] = (T)tb.w[i];
  }
};

// Form of the line operator for the kernels of dimension DIM, precision T, degree N: true =
// even/odd (about 1.5 (N+1)^2 FMAs per line instead of 3 (N+1)^2, two output rows per
// iteration). Chosen per case by measurement (fused CG apply, ~33M DoFs in 3D, 2D as listed):
// 3D FP64 N = 4 377 -> 350 us, N = 7 636 -> 608, N = 8 1078 -> 1006; 3D FP32 N = 3 169 -> 163,
// N = 4 198 -> 178, N = 5 249 -> 227, N = 6 447 -> 411, N = 7 292 -> 276, N = 8 643 -> 591;
// 2D 512^2 N = 4 FP64 77.6 -> 68.4, FP32 47.2 -> 39.4; 384^2 N = 8 FP32 107 -> 98. Elsewhere
// the two rows' live values cost vector registers and occupancy (256^2 N = 6: FP64 40.8 ->
// 56.2 us, FP32 28.0 -> 34.5; 384^2 N = 8 FP64 207 -> 232; 3D FP64 N = 5 557 -> 705, N = 6
// 690 -> 871) or nothing changes (N <= 1).
template <typename T, int N, int DIM>
__host__ __device__ constexpr bool line_eo() {
  return DIM == 2 ? (N == 4 || (N == 8 && sizeof(T) == 4))
                  : (sizeof(T) == 8 ? (N == 4 || N == 7 || N == 8) : (N >= 3 && N <= 8));
}

// Device-resident scalars of one CG solve. Kernels never synchronise across blocks inside a
// launch: a kernel writes one partial sum per block (plain stores), and every block of the NEXT
// kernel re-sums those partials in block order (kernel boundaries make them visible; the fixed
// order keeps every block's scalar bit-identical and the whole solve deterministic). Block 0
// mirrors the scalars here for the host (convergence polling) and for later kernels.
struct CgState {
  double rho_hist[2];  // rho_k kept in slot k % 2 by block 0 of apply k (rho_{k-1} for apply k)
  double rho;        // <r_k, r_k> of the current iterate (written by block 0 of the apply)
  double sigma;      // <p_k, A p_k>
  double alpha;      // rho / sigma
  double beta;       // rho_k / rho_{k-1}
  double bnorm2;     // <b, b>
  double tol2;       // (rtol ||b||)^2
  double aux;        // scalar result of a stand-alone reduction (FIN_AUX), rtol input of FIN_BNORM
  double scale;      // batched refinement: the FP32 vectors hold r / scale
  double ref;        // batched refinement: FP64 residual / scale at the last replacement
  double best;       // batched refinement: smallest FP64 residual / scale so far
  double res2;       // <r_k, r_k> of the current iterate (the stopping test); equals rho unless
                     // the run is preconditioned (then rho = <r_k, z_k>, z_k = P r_k)
  int iter;          // iterations completed when done
  int maxit;
  int done;          // 1 once converged, out of iterations or broken down (batched refinement:
                     // the FP32 iterations of this problem pause until the next replacement)
  int status;        // 0 ok, -4 no convergence, -5 breakdown
  int restart_k;     // iteration at which beta is forced to 0 (direction restart), -1 = none
  int restarts;      // direction restarts so far (batched refinement)
  int fin;           // batched: 1 once the problem is finished
  int even_stop;     // 1: the tol2 stop is taken at even iterations only (batched refinement)
  int fresh;         // batched: 1 = the next executed iteration starts a new direction (beta = 0)
  int mode64;        // batched: 0 = FP32 iterations with FP64 replacement, 1 = FP64 iterations
  int switched;      // batched: set when the problem has just switched to FP64 iterations
  int stall;         // batched refinement: replacements in a row without a new best residual
  int fallback_k;    // batched refinement: iterations run before the switch to FP64, -1 = none
  int idle;          // batched: iterations spent stopped inside a chunk before a chunk-end resume
  int outer;         // batched: chunk-end FP64 residual evaluations of this problem
  // Single-problem runs fold x += alpha_k p_k into the apply kernel of iteration k + 1, which
  // reads p_k anyway: xk = iteration whose alpha (above) awaits that update, -1 = none; xused =
  // the last such iteration an apply kernel has applied (block 0 records it; no block of the
  // same launch reads it). After a run stops, x is complete once xk == xused or after one
  // flush kernel.
  int xk;
  int xused;
  // Permission stamps of the iterating kernels. The apply kernel of iteration k runs iff
  // run_a[k % 2] == k, the update kernel of iteration k iff run_u == k. Each stamp is written
  // only by a launch that no reader of it overlaps: the apply kernel of iteration k publishes
  // run_u = k (two-kernel form) or run_a[(k + 1) % 2] = k + 1 (one-kernel form), the update
  // kernel of iteration k publishes run_a[(k + 1) % 2] = k + 1, each only when the run goes on;
  // state resets and chunk-end resumes publish run_a for the iteration that starts next. So an
  // early exit never depends on a word that another block of the same launch writes, and every
  // block of a launch takes the same decision (the done flag above is for the host and the
  // chunk-end logic only).
  int run_a[2];
  int run_u;
};

// The apply kernel of iteration k may run (see CgState::run_a).
__device__ __forceinline__ bool apply_may_run(const CgState* st, int k) {
  return st->run_a[k & 1] == k;
}

// Finalizers of the stand-alone reductions (dot kernel + single-block finalize kernel).
enum Finalize : int {
  FIN_BNORM = 3,     // sum = <b, b>: bnorm2 = sum, tol2 = aux^2 * sum (aux holds rtol)
  FIN_AUX = 4        // sum stored in aux
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block in a fixed order; the result is returned to EVERY thread.
template <int NT>
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double red[(NT + 63) / 64];
  __shared__ double tot;
  __syncthreads();
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < (NT + 63) / 64; ++i) s += red[i];
    tot = s;
  }
  __syncthreads();
  return tot;
}

// Sums over rows [r0, r1) of the row-major array a (row stride ld, NC columns), one per column,
// returned in out[0..NC) of every block (shared; acc: kBlock shared doubles of scratch). Every thread works: thread t takes column t % NC of the rows
// r0 + t / NC, r0 + t / NC + G, ... (G = kBlock / NC row groups, four independent accumulators),
// and the G partial sums of a column are added in group order. NC > kBlock: one thread per column.
template <typename T>
__device__ __forceinline__ void column_sums(const T* __restrict__ a, int ld, long long r0,
                                            long long r1, int NC, double* __restrict__ acc,
                                            double* __restrict__ out) {
  if (NC <= kBlock) {
    const int G = kBlock / NC;
    const int g = threadIdx.x / NC, l = threadIdx.x - g * NC;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (g < G) {
      long long r = r0 + g;
      for (; r + 3LL * G < r1; r += 4LL * G) {
        s0 += (double)a[r * ld + l];
        s1 += (double)a[(r + G) * ld + l];
        s2 += (double)a[(r + 2LL * G) * ld + l];
        s3 += (double)a[(r + 3LL * G) * ld + l];
      }
      for (; r < r1; r += G) s0 += (double)a[r * ld + l];
    }
    acc[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int c = threadIdx.x; c < NC; c += kBlock) {
      double t = 0.0;
      for (int q = 0; q < G; ++q) t += acc[q * NC + c];
      out[c] = t;
    }
  } else {
    for (int c = threadIdx.x; c < NC; c += kBlock) {
      double t = 0.0;
      for (long long r = r0; r < r1; ++r) t += (double)a[r * ld + c];
      out[c] = t;
    }
  }
  __syncthreads();
}

// Fixed-order sum of `n` partials written by a previous kernel; result in every thread.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += part[i];
  return block_sum_all<NT>(s);
}

// Scalars of CG iteration k shared by the apply kernel of that iteration: rho_k from the
// partials of <r_k, r_k>, the stop decision, and beta_k = rho_k / rho_{k-1}.
struct IterScalars {
  double rho, beta;
  bool stop;
};

// `writer`: the one block of the problem that mirrors the scalars into st.
// `one`: one kernel per iteration (the next launch is the apply kernel of iteration k + 1).
// res_cur: partials of <r_k, r_k> when the run is preconditioned (rho_cur then holds those of
// <r_k, z_k>); null otherwise.
template <int NT>
__device__ __forceinline__ IterScalars iteration_scalars(CgState* st, int k,
                                                         const double* rho_cur, int nrho,
                                                         bool writer, bool one = false,
                                                         const double* res_cur = nullptr) {
  IterScalars r;
  r.rho = sum_partials<NT>(rho_cur, nrho);
  const double res2 = res_cur ? sum_partials<NT>(res_cur, nrho) : r.rho;
  const double rho_old = k > 0 ? st->rho_hist[(k + 1) & 1] : 0.0;
  r.beta = (k > 0 && k != st->restart_k && !st->fresh) ? r.rho / rho_old : 0.0;
  int status = 1;                               // 1 = keep iterating
  if (!isfinite(r.rho) || !isfinite(res2)) status = -5;
  else if (res2 <= st->tol2 && !(st->even_stop && (k & 1))) status = 0;
  else if (k - st->idle >= st->maxit) status = -4;   // iterations run (batched: idle excluded)
  r.stop = status != 1;
  if (threadIdx.x == 0 && writer) {
    st->rho_hist[k & 1] = r.rho;
    st->rho = r.rho;
    st->res2 = res2;
    st->beta = r.beta;
    st->iter = k;
    if (r.stop) {
      st->status = status;
      st->done = 1;
    } else if (one) {
      st->run_a[(k + 1) & 1] = k + 1;
    } else {
      st->run_u = k;
    }
  }
  return r;
}

// Four sums over the block in a fixed order, returned to every thread.
template <int NT>
__device__ __forceinline__ void block_sum4_all(double (&v)[4]) {
  __shared__ double red4[(NT + 63) / 64][4];
  __shared__ double tot4[4];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red4[wid][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < (NT + 63) / 64; ++w) s += red4[w][threadIdx.x];
    tot4[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = tot4[i];
}

// Scalars of CG iteration k >= 1 in the one-kernel form, where the apply kernel of iteration k
// also makes the residual update of iteration k - 1. The previous launch wrote per block the
// 4-tuple (<p, A p>, <r, A p>, <A p, A p>, <r, r>) of iteration k - 1, so
//   alpha_{k-1} = rho_{k-1} / sigma_{k-1},
//   rho_k = |r_{k-1} - alpha_{k-1} q_{k-1}|^2 = rho_{k-1} - 2 alpha gamma + alpha^2 nu
// (the expansion with the actual inner products, not the exact-arithmetic identity
// gamma = sigma), beta_k = rho_k / rho_{k-1}, and the stop decision on rho_k.
struct FusedScalars {
  double alpha, beta;
  bool stop;
};

template <int NT>
__device__ __forceinline__ FusedScalars fused_scalars(CgState* st, int k,
                                                      const double* __restrict__ part, int np,
                                                      bool writer) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += NT) {
    const double2 a = *reinterpret_cast<const double2*>(part + 4 * i);
    const double2 b = *reinterpret_cast<const double2*>(part + 4 * i + 2);
    s[0] += a.x;
    s[1] += a.y;
    s[2] += b.x;
    s[3] += b.y;
  }
  block_sum4_all<NT>(s);
  const double sigma = s[0], gamma = s[1], nu = s[2], rho_prev = s[3];
  FusedScalars f;
  f.alpha = rho_prev / sigma;
  f.beta = 0.0;
  if (!(sigma > 0.0) || !isfinite(f.alpha)) {
    if (threadIdx.x == 0 && writer) {
      st->sigma = sigma;
      st->status = -5;
      st->iter = k - 1;
      st->done = 1;
    }
    f.stop = true;
    return f;
  }
  const double rho = rho_prev - 2.0 * f.alpha * gamma + f.alpha * f.alpha * nu;
  f.beta = (k != st->restart_k && !st->fresh) ? rho / rho_prev : 0.0;
  int status = 1;
  if (!isfinite(rho)) status = -5;
  else if (rho <= st->tol2 && !(st->even_stop && (k & 1))) status = 0;
  else if (k - st->idle >= st->maxit) status = -4;
  f.stop = status != 1;
  if (threadIdx.x == 0 && writer) {
    st->sigma = sigma;
    st->alpha = f.alpha;
    st->xk = k - 1;                      // x += alpha_{k-1} p_{k-1}: this launch or a flush
    st->rho_hist[(k + 1) & 1] = rho_prev;
    st->rho_hist[k & 1] = rho;
    st->rho = rho;
    st->res2 = rho;
    st->beta = f.beta;
    st->iter = k;
    if (f.stop) {
      st->status = status;
      st->done = 1;
    } else {
      st->xused = k - 1;
      st->run_a[(k + 1) & 1] = k + 1;
    }
  }
  return f;
}

// Map the hardware block index to a logical tile so that each XCD (blocks are dispatched to
// the 8 XCDs round-robin) processes one contiguous range of tiles, keeping neighbouring tiles
// (whose halos overlap) in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned G) {
  const unsigned q = G / 8u, r = G % 8u;
  const unsigned x = b % 8u, idx = b / 8u;
  const unsigned start = (x < r) ? x * (q + 1u) : r * (q + 1u) + (x - r) * q;
  return start + idx;
}

}  // namespace pdk
