// Batched pressure solves: many independent 2D periodic problems of different sizes and degrees
// advanced together. All problems' vectors are packed into one array (problem j at dof_off[j]).
// Every kernel maps its blocks to problems through a table of cumulative block counts over a
// list of problems, so one launch serves every listed problem (the operator kernel: every problem
// of one degree and tile shape). Each problem keeps its own CG state, partial sums, scale, flags
// and precision mode. With the device-resident iteration base, a chunk of iterations plus the
// chunk-end decisions is captured once into a HIP graph and replayed; the host re-captures with
// shorter lists when problems finish or change precision.
#include "pd_apply2d.h"
#include "pd_device.h"
#include "pd_launch.h"

namespace pdk {

namespace {

// index of the last entry <= b in the ascending offsets off[0..n) (off[0] = 0)
__device__ __forceinline__ int find_prob(const int* __restrict__ off, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// list entry of block b of a streaming kernel: problem index j and block lb within the problem
struct Slot {
  int i, j, lb;
};
__device__ __forceinline__ Slot slot_of(const BatchIter& it, const int* __restrict__ off, int b) {
  Slot s;
  s.i = find_prob(off, it.count, b);
  s.j = it.list[s.i];
  s.lb = b - off[s.i];
  return s;
}

// iterating kernels: the problem runs iteration k in this launch's precision. The stamps are
// written by the other kernel of the iteration, the chunk-end decision or the state reset, never
// by another block of the reading launch (see CgState::run_a).
__device__ __forceinline__ bool iterates(const BatchIter& it, const CgState* st, int k,
                                         bool apply) {
  if (st->fin || !(it.want < 0 || st->mode64 == it.want)) return false;
  return apply ? apply_may_run(st, k) : st->run_u == k;
}

// other kernels: skip finished problems when asked, and problems of the other precision.
// want == -2 selects the problems whose FP64 residual is recomputed at a refinement chunk end:
// unfinished FP32-mode problems, and problems that fell back to FP64 iterations and whose
// recurrence has just met the tolerance (their true residual decides).
__device__ __forceinline__ bool serves(const BatchIter& it, const CgState* st) {
  if (it.skip_fin && st->fin) return false;
  if (it.want == -2) return !st->mode64 || (st->done && st->status == 0);
  return it.want < 0 || st->mode64 == it.want;
}

__device__ __forceinline__ double* rho_slot(const BatchIter& it, int j, int parity) {
  return it.rho + (size_t)j * 2 * kMaxStreamPartials + (size_t)(parity & 1) * kMaxStreamPartials;
}

// preconditioned solves: partials of <r, r> (the stopping test), beside those of <r, z> in rho
__device__ __forceinline__ double* res_slot(const BatchIter& it, int j, int parity) {
  return it.res + (size_t)j * 2 * kMaxStreamPartials + (size_t)(parity & 1) * kMaxStreamPartials;
}

// ---- CG update: r -= alpha_j q; partials of <r, r> (next iteration's slot). The matching
// x += alpha_j p_k is deferred: the apply kernel of iteration k + 1 makes it, or k_xflush_batch at
// the end of the chunk when the problem has stopped iterating; block 0 of the problem publishes
// alpha_j with xk = k. The first J elements of each thread are loaded before sigma is reduced.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_batch(BatchIter it, const T* __restrict__ q,
                                                         T* __restrict__ r) {
  const Slot sl = slot_of(it, it.upd_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  CgState* st = it.st + sl.j;
  const int k = *it.kbase + it.koff;
  if (!iterates(it, st, k, false)) return;
  const long long n = P.ndof;
  const long long stride = (long long)P.nupd * kBlock;
  const long long i0 = (long long)sl.lb * kBlock + threadIdx.x;
  T* rj = r + P.dof_off;
  const T* qj = q + P.dof_off;
  constexpr int J = 8;
  T qv[J], rv[J];
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const long long i = i0 + jj * stride;
    if (i < n) {
      qv[jj] = qj[i];
      rv[jj] = rj[i];
    }
  }
  const double sigma = sum_partials<kBlock>(it.sig + P.sig_off, P.nsig);
  const double alpha = st->rho / sigma;
  if (!(sigma > 0.0) || !isfinite(alpha)) {
    if (threadIdx.x == 0 && sl.lb == 0) {
      st->sigma = sigma;
      st->status = -5;
      st->iter = k;
      st->done = 1;
    }
    return;
  }
  const T a = (T)alpha;
  double s = 0.0;
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const long long i = i0 + jj * stride;
    if (i < n) {
      const T rn = rv[jj] - a * qv[jj];
      rj[i] = rn;
      s += (double)rn * (double)rn;
    }
  }
  for (long long i = i0 + J * stride; i < n; i += stride) {
    const T rn = rj[i] - a * qj[i];
    rj[i] = rn;
    s += (double)rn * (double)rn;
  }
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) {
    rho_slot(it, sl.j, it.koff + 1)[sl.lb] = s;
    if (sl.lb == 0) {
      st->alpha = alpha;
      st->xk = k;
      st->run_a[(k + 1) & 1] = k + 1;
      // the direction of this iteration now exists: later iterations may build on it (no reader
      // of this flag runs during this kernel)
      st->fresh = 0;
    }
  }
}

// ---- chunk end, every listed problem: the deferred x += alpha p_xk still pending (the problem
// stopped iterating before the apply kernel of the next iteration made it). FP64-mode problems
// update x64 with the FP64 direction, FP32-mode problems the FP32 correction d32 with the FP32
// direction; p_k sits in buffer (k + 1) % 2 of its precision. The next finalize clears xk.
__global__ __launch_bounds__(kBlock) void k_xflush_batch(BatchIter it, double* __restrict__ x64,
                                                         float* __restrict__ d32,
                                                         const double* __restrict__ pa64,
                                                         const double* __restrict__ pb64,
                                                         const float* __restrict__ pa32,
                                                         const float* __restrict__ pb32) {
  const Slot sl = slot_of(it, it.upd_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  const CgState* st = it.st + sl.j;
  const int xk = st->xk;
  if (xk < 0 || st->xused == xk) return;
  const long long n = P.ndof;
  const long long stride = (long long)P.nupd * kBlock;
  const long long o = P.dof_off;
  if (st->mode64) {
    const double a = st->alpha;
    const double* __restrict__ p = ((xk + 1) & 1) ? pb64 : pa64;
    for (long long i = (long long)sl.lb * kBlock + threadIdx.x; i < n; i += stride)
      x64[o + i] += a * p[o + i];
  } else {
    const float a = (float)st->alpha;
    const float* __restrict__ p = ((xk + 1) & 1) ? pb32 : pa32;
    for (long long i = (long long)sl.lb * kBlock + threadIdx.x; i < n; i += stride)
      d32[o + i] += a * p[o + i];
  }
}

// ---- the operator for every problem of one (degree, tile variant) group
// FUSE: CG iteration form for problems that iterate in this launch's precision; else y = A x.
template <typename T, int N, int V, int FUSE>
__global__ __launch_bounds__(256) void k_apply2d_batch(BatchIter it, const int* __restrict__ grp,
                                                       const int* __restrict__ toff, int ng,
                                                       const T* __restrict__ x,
                                                       const T* __restrict__ pold,
                                                       T* __restrict__ pnew, T* __restrict__ y,
                                                       T* __restrict__ xsol, Blk<T, N> B) {
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int g = find_prob(toff, ng, b);
  const int j = grp[g];
  const BProb& P = it.probs[j];
  CgState* st = it.st + j;
  if (FUSE) {
    if (!iterates(it, st, *it.kbase + it.koff, true)) return;
  } else if (!serves(it, st)) {
    return;
  }
  ApplyArgs<T> a;
  a.x = x + P.dof_off;
  a.pold = FUSE ? pold + P.dof_off : nullptr;
  a.pnew = FUSE ? pnew + P.dof_off : nullptr;
  a.y = y + P.dof_off;
  a.nx = P.nx;
  a.ny = P.ny;
  a.nz = 1;
  a.ntx = P.ntx;
  a.nty = P.nty;
  a.ntz = 1;
  a.kz = 1;
  a.alpha = (T)P.alpha;
  a.c0 = (T)P.c0;
  a.c1 = (T)P.c1;
  a.c2 = T(0);
  a.st = st;
  a.k = it.koff;
  a.kbase = it.kbase;
  a.rho_cur = rho_slot(it, j, it.koff);
  a.res_cur = it.res ? res_slot(it, j, it.koff) : nullptr;
  a.mir[0] = a.mir[1] = a.mir[2] = 0;
  a.nrho = P.nupd;
  a.sigpart = it.sig + P.sig_off;
  a.xsol = FUSE == 2 ? xsol + P.dof_off : nullptr;
  const int tile = b - toff[g];
  apply2d_body<T, N, V, FUSE, 0>(a, B, tile, tile + 1, 1, tile);
}

// ---- streaming passes over the listed problems (see launch_stream_batch)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stream_batch(BatchIter it, const double* __restrict__ b,
                                                         const double* __restrict__ q64,
                                                         double* __restrict__ r64,
                                                         double* __restrict__ x64,
                                                         float* __restrict__ v32) {
  const Slot sl = slot_of(it, it.upd_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  CgState* st = it.st + sl.j;
  if (MODE == 5) {
    if (!st->switched) return;
  } else if (MODE != 1 && !serves(it, st)) {
    return;
  }
  const long long n = P.ndof;
  const long long stride = (long long)P.nupd * kBlock;
  const long long o = P.dof_off;
  const double scale = st->scale;
  double s = 0.0;
  for (long long i = (long long)sl.lb * kBlock + threadIdx.x; i < n; i += stride) {
    if (MODE == 0) {
      const double v = b[o + i] - q64[o + i];
      r64[o + i] = v;
      s += v * v;
    } else if (MODE == 1) {
      x64[o + i] += scale * (double)v32[o + i];
      v32[o + i] = 0.0f;
    } else if (MODE == 2) {
      const float v = (float)(r64[o + i] / scale);
      v32[o + i] = v;
      s += (double)v * (double)v;
    } else if (MODE == 4) {
      const double v = b[o + i];
      r64[o + i] = v;
      s += v * v;
    } else {
      const double v = r64[o + i];
      s += v * v;
    }
  }
  if (MODE == 1) return;
  s = block_sum_all<kBlock>(s);
  if (threadIdx.x == 0) {
    if (MODE == 2 || MODE == 5) rho_slot(it, sl.j, it.koff)[sl.lb] = s;
    else if (MODE == 4) rho_slot(it, sl.j, 0)[sl.lb] = s;
    else it.tmp[(size_t)sl.j * kMaxStreamPartials + sl.lb] = s;
  }
}

// FP32 refinement: replacements in a row without a new smallest FP64 residual after which the
// problem continues in FP64 (FP32 arithmetic has stopped reducing it)
constexpr int kStallLimit = 16;
// FP64 runs: chunk-end checks of the true residual after the recurrence met the tolerance, and
// the largest true / goal ratio that is iterated away (beyond it: FP64 rounding floor)
constexpr int kTrueChecks = 8;
constexpr double kTrueGap = 16.0;

// ---- per-problem finalize (one block per list entry)
// what 0: aux = sum of the tmp partials (residual norm squared)
// what 1: refinement start (sum = ||b||^2): bnorm2; scale = ||b|| (the FP32 vectors hold
//         r / scale); tol2 = the pause threshold max(ru, rtol)^2 of the FP32 iterations (scaled
//         units); a zero or NaN right-hand side finishes the problem at once
// what 2: FP64 start: bnorm2 = sum; tol2 = (rtol_j)^2 * sum
// what 3: chunk end, every unfinished problem. FP64-mode problems whose iterations stopped on
//   the tolerance are checked against the recomputed FP64 residual: finished when it is <= rtol
//   ||b||; else an FP64 run resumes from it with the same direction (within kTrueGap of the
//   goal, at most kTrueChecks times, each halving it; else finished at the rounding floor) and
//   a problem that fell back from the refinement resumes from it with a new direction. Other
//   stops of FP64-mode problems finish them. FP32-mode
//   problems decide from the FP64 residual of the replacement
//   (sum = ||b - A x||^2): finished when it is <= rtol ||b|| (or not finite, or out of
//   iterations); else, when that residual has grown beyond twice the smallest one so far or has
//   not improved for kStallLimit replacements, the problem switches to FP64 iterations from its
//   current x (new direction); else the FP32 iterations resume with the pause threshold lowered
//   to ru times the new residual. A pause on the threshold happens at an even iteration p
//   (even_stop), so the paused problem's last direction, its rho_{p-1} and the partials of
//   <r_p, r_p> sit in the slots that the next chunk (whose first iteration is even) reads: the
//   direction is kept, as for a problem that ran the whole chunk. It restarts (beta = 0 at the
//   next executed iteration) after a pause on a breakdown or a non-finite rho, after a pause
//   whose FP32 residual had fallen more than 1e4 below the last replaced one (FP32 rounding
//   level: the direction is noise), and when the FP32 recurrence residual of the same iteration,
//   still in its rho slot, has drifted more than 4x below the true one.
template <int WHAT>
__global__ __launch_bounds__(kBlock) void k_finalize_batch(BatchIter it) {
  const int j = it.list[blockIdx.x];
  const BProb& P = it.probs[j];
  CgState* st = it.st + j;
  if (WHAT == 3 && threadIdx.x == 0) st->xk = -1;   // the deferred x update was flushed before
  if (WHAT == 3 && st->fin) return;
  const double s = sum_partials<kBlock>(it.tmp + (size_t)j * kMaxStreamPartials, P.nupd);
  // recurrence residual of the chunk's last iteration (preconditioned solves: <r, r>, kept apart
  // from the <r, z> of the rho slots)
  const double rec =
      WHAT == 3 ? sum_partials<kBlock>(it.res ? res_slot(it, j, it.koff) : rho_slot(it, j, it.koff),
                                       P.nupd)
                : 0.0;
  if (threadIdx.x != 0) return;
  if (WHAT == 0) {
    st->aux = s;
  } else if (WHAT == 1) {
    st->bnorm2 = s;
    st->scale = s > 0.0 ? sqrt(s) : 1.0;
    const double t = fmax(P.ru, P.rtol);
    st->tol2 = t * t;
    st->ref = 1.0;
    st->best = 1.0;
    st->even_stop = 1;
    st->aux = s;
    if (!(s > 0.0)) {                 // zero (or NaN) right-hand side: nothing to iterate
      st->done = 1;
      st->fin = 1;
      st->status = isfinite(s) ? 0 : -5;
      st->iter = 0;
    }
  } else if (WHAT == 2) {
    st->bnorm2 = s;
    st->tol2 = P.rtol * P.rtol * s;
    st->aux = s;
    st->ref = 0.0;
    st->even_stop = 1;
  } else {
    st->switched = 0;
    const int k = *it.kbase + it.koff;
    if (st->mode64) {
      // still iterating: it may have sat out this chunk in a plan that listed it with the FP32
      // problems (it switched at an earlier chunk end and the host has not re-captured yet), so
      // its permission stamp is renewed for the next chunk's first iteration
      if (!st->done) {
        st->run_a[k & 1] = k;
        return;
      }
      if (st->status != 0) {           // out of iterations or broken down
        st->fin = 1;
        return;
      }
      // the FP64 recurrence met the tolerance: the recomputed residual decides
      st->aux = s;
      st->outer += 1;
      const double res = sqrt(s);
      const double goal = P.rtol * sqrt(st->bnorm2);
      if (!isfinite(res)) {
        st->fin = 1;
        st->status = -5;
        return;
      }
      if (res <= goal) {
        st->fin = 1;
        return;
      }
      if (st->fallback_k < 0) {
        // an FP64 run: the iterations resume from the recomputed residual (with the same
        // direction: the stop was at an even iteration, so the direction and rho of the
        // previous iteration sit in the slots the next chunk reads) while it is within
        // kTrueGap of the goal, at most kTrueChecks times, each halving it; a larger gap is the
        // FP64 rounding floor of b - A x: finished, the true residual reported
        if (res > kTrueGap * goal || st->outer > kTrueChecks ||
            (st->ref > 0.0 && res > 0.5 * st->ref)) {
          st->fin = 1;
          return;
        }
        st->ref = res;
        // a recurrence that drifted more than 4x below the true residual would make beta huge
        // and the old direction swamp the new residual: restart the direction then (always in
        // preconditioned solves, as in the single-problem solve)
        if (it.res || !(res <= 4.0 * sqrt(st->rho))) {
          st->fresh = 1;
          st->restarts += 1;
        }
      } else {
        // fallen back from the refinement: resume from it with a new direction
        st->fresh = 1;
        st->restarts += 1;
      }
      if (st->iter - st->idle >= st->maxit) {
        st->fin = 1;
        st->status = -4;
        return;
      }
      st->idle += k - st->iter;
      st->done = 0;
      st->run_a[k & 1] = k;
      st->switched = 1;
      return;
    }
    const bool paused = st->done != 0;
    if (!paused) st->iter = k;         // ran every iteration of the chunk
    st->aux = s;
    st->outer += 1;
    const double res = sqrt(s);
    const double goal = P.rtol * sqrt(st->bnorm2);
    const double r = res / st->scale;
    if (!isfinite(res)) {
      st->done = st->fin = 1;
      st->status = -5;
    } else if (res <= goal) {
      st->done = st->fin = 1;
      st->status = 0;
    } else if ((paused && st->status == -4) || st->iter - st->idle >= st->maxit) {
      st->done = st->fin = 1;
      st->status = -4;
    } else {
      if (r < st->best) {
        st->best = r;
        st->stall = 0;
      } else {
        st->stall += 1;
      }
      st->idle += k - st->iter;        // a paused problem resumes at the chunk boundary
      if (r > 2.0 * st->best || st->stall >= kStallLimit) {
        st->mode64 = 1;
        st->switched = 1;
        st->fallback_k = k - st->idle;
        st->fresh = 1;
        st->even_stop = 0;
        st->tol2 = goal * goal;
      } else {
        const bool deep = paused && st->status == 0 && sqrt(rec) < 1e-4 * st->ref;
        if ((paused && st->status != 0) || deep || r > 4.0 * sqrt(rec)) {
          st->fresh = 1;
          st->restarts += 1;
        }
        st->ref = r;
        const double t = fmax(P.ru * res, goal) / st->scale;
        st->tol2 = t * t;
      }
      st->done = 0;
      st->run_a[k & 1] = k;
      st->status = 0;
    }
  }
}

// ---- cell-block Jacobi preconditioner of the listed problems (preconditioned solves)
// z = P r problem by problem, with P the inverse of each cell's diagonal block in its generalised
// eigenbasis (the single-problem k_pcg_update, whose notes apply): each block takes groups of
// cells of its problem (grid-stride over the problem's nupd blocks), one line of nodes per
// direction and thread, the next group's r and q loaded while the current one is transformed.
// One launch per degree over the listed problems of that degree (the eigenbasis is the degree's;
// the diagonal scaling uses each problem's own cell sizes).
template <int N>
struct PcgTab {
  double V[(N + 1) * (N + 1)];   // V[m][l]: component m of eigenvector l
  double lam[N + 1];
};

template <typename T, int N, int SEL>
__global__ __launch_bounds__(kBlock) void k_pcg_update_batch(BatchIter it, PcgTab<N> tab,
                                                             const T* __restrict__ q,
                                                             T* __restrict__ r,
                                                             T* __restrict__ z) {
  constexpr int n = N + 1, NC = n * n;
  constexpr int CPB = pcg_cells_per_group(N, 2);
  constexpr int E = CPB * NC;
  constexpr int J = (E + kBlock - 1) / kBlock;
  constexpr bool UPD = SEL == 0;
  __shared__ double sa[E], sb[E], sinv[NC];
  const Slot sl = slot_of(it, it.upd_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  CgState* st = it.st + sl.j;
  T a = T(0);
  double alpha = 0.0;
  int k = 0, parity = it.koff;
  if (UPD) {
    k = *it.kbase + it.koff;
    if (!iterates(it, st, k, false)) return;
    const double sigma = sum_partials<kBlock>(it.sig + P.sig_off, P.nsig);
    alpha = st->rho / sigma;
    if (!(sigma > 0.0) || !isfinite(alpha)) {
      if (threadIdx.x == 0 && sl.lb == 0) {
        st->sigma = sigma;
        st->status = -5;
        st->iter = k;
        st->done = 1;
      }
      return;
    }
    a = (T)alpha;
    parity = it.koff + 1;
  } else if (SEL == 2 ? !st->switched : !serves(it, st)) {
    return;
  }
  for (int l = threadIdx.x; l < NC; l += kBlock)
    sinv[l] = 1.0 / (P.alpha + P.c0 * tab.lam[l % n] + P.c1 * tab.lam[l / n]);
  // 1D transform of one line (first element b, stride sd); scale: the diagonal scaling and the
  // backward transform of the last direction in the same pass
  auto line = [&](const double* in, double* out, int b, int sd, bool fwd, bool scale) {
    double v[n], w[n];
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = in[b + m * sd];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) acc += (fwd ? tab.V[m * n + i] : tab.V[i * n + m]) * v[m];
      w[i] = acc;
    }
    if (scale) {
      const int l0 = b % NC;
#pragma unroll
      for (int i = 0; i < n; ++i) w[i] *= sinv[l0 + i * sd];
#pragma unroll
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) acc += tab.V[i * n + m] * w[m];
        v[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < n; ++i) out[b + i * sd] = v[i];
    } else {
#pragma unroll
      for (int i = 0; i < n; ++i) out[b + i * sd] = w[i];
    }
  };
  const long long ncells = P.ncells;
  const long long ngroups = (ncells + CPB - 1) / CPB;
  T* __restrict__ rj = r + P.dof_off;
  const T* __restrict__ qj = UPD ? q + P.dof_off : nullptr;
  T* __restrict__ zj = z + P.dof_off;
  double rr = 0.0, rz = 0.0;
  T rn[J], qn[J];
  auto load = [&](long long grp) {
    const long long c0 = grp * CPB;
    const long long base = c0 * NC;
    const int ecount = (int)((ncells - c0 < CPB ? ncells - c0 : CPB) * NC);
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const int e = threadIdx.x + kBlock * jj;
      if (e < ecount) {
        rn[jj] = rj[base + e];
        if (UPD) qn[jj] = qj[base + e];
      }
    }
  };
  long long grp = sl.lb;
  if (grp < ngroups) load(grp);
  for (; grp < ngroups; grp += P.nupd) {
    const long long c0 = grp * CPB;
    const long long base = c0 * NC;
    const int cells = (int)(ncells - c0 < CPB ? ncells - c0 : CPB);
    const int ecount = cells * NC;
    const int lines = cells * n;
    double rv[J];
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const int e = threadIdx.x + kBlock * jj;
      if (e < ecount) {
        T x = rn[jj];
        if (UPD) {
          x = x - a * qn[jj];
          rj[base + e] = x;
        }
        rv[jj] = (double)x;
        rr += rv[jj] * rv[jj];
        sa[e] = rv[jj];
      }
    }
    if (grp + P.nupd < ngroups) load(grp + P.nupd);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < lines) line(sa, sb, (t / n) * NC + (t % n) * n, 1, true, false);   // x-lines
    __syncthreads();
    if (t < lines) line(sb, sb, (t / n) * NC + (t % n), n, true, true);         // y-lines
    __syncthreads();
    if (t < lines) line(sb, sa, (t / n) * NC + (t % n) * n, 1, false, false);  // x-lines
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const int e = threadIdx.x + kBlock * jj;
      if (e < ecount) {
        const T zv = (T)sa[e];
        zj[base + e] = zv;
        rz += rv[jj] * (double)zv;
      }
    }
    __syncthreads();   // sa is rewritten by the next group
  }
  rr = block_sum_all<kBlock>(rr);
  rz = block_sum_all<kBlock>(rz);
  if (threadIdx.x == 0) {
    rho_slot(it, sl.j, parity)[sl.lb] = rz;
    res_slot(it, sl.j, parity)[sl.lb] = rr;
    if (UPD && sl.lb == 0) {
      st->alpha = alpha;
      st->xk = k;
      st->run_a[(k + 1) & 1] = k + 1;
      st->fresh = 0;
    }
  }
}

template <typename T, int N>
hipError_t pcg_batch_N(const BatchIter& it, int sel, const double* V, const double* lam,
                       const void* q, void* r, void* z, hipStream_t s) {
  PcgTab<N> tab;
  constexpr int n = N + 1;
  for (int i = 0; i < n * n; ++i) tab.V[i] = V[i];
  for (int i = 0; i < n; ++i) tab.lam[i] = lam[i];
  const dim3 G(it.upd_blocks), B(kBlock);
  if (sel == 0)
    hipLaunchKernelGGL((k_pcg_update_batch<T, N, 0>), G, B, 0, s, it, tab, (const T*)q, (T*)r, (T*)z);
  else if (sel == 1)
    hipLaunchKernelGGL((k_pcg_update_batch<T, N, 1>), G, B, 0, s, it, tab, (const T*)q, (T*)r, (T*)z);
  else
    hipLaunchKernelGGL((k_pcg_update_batch<T, N, 2>), G, B, 0, s, it, tab, (const T*)q, (T*)r, (T*)z);
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_batch_T(const BatchIter& it, int N, int sel, const double* V, const double* lam,
                       const void* q, void* r, void* z, hipStream_t s) {
  switch (N) {
    case 0: return pcg_batch_N<T, 0>(it, sel, V, lam, q, r, z, s);
    case 1: return pcg_batch_N<T, 1>(it, sel, V, lam, q, r, z, s);
    case 2: return pcg_batch_N<T, 2>(it, sel, V, lam, q, r, z, s);
    case 3: return pcg_batch_N<T, 3>(it, sel, V, lam, q, r, z, s);
    case 4: return pcg_batch_N<T, 4>(it, sel, V, lam, q, r, z, s);
    case 5: return pcg_batch_N<T, 5>(it, sel, V, lam, q, r, z, s);
    case 6: return pcg_batch_N<T, 6>(it, sel, V, lam, q, r, z, s);
    case 7: return pcg_batch_N<T, 7>(it, sel, V, lam, q, r, z, s);
    case 8: return pcg_batch_N<T, 8>(it, sel, V, lam, q, r, z, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- null-space projection of the listed problems: node sums, correction, subtraction
__global__ __launch_bounds__(kBlock) void k_node_sums_batch(BatchIter it, const double* __restrict__ v) {
  const Slot sl = slot_of(it, it.ns_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  if (!serves(it, it.st + sl.j)) return;
  const int nb = P.nns;
  const long long per = (P.ncells + nb - 1) / nb;
  const long long c0 = (long long)sl.lb * per;
  const long long c1 = c0 + per < P.ncells ? c0 + per : P.ncells;
  const int NC = P.NC;
  __shared__ double acc[kBlock];
  __shared__ double out[kMaxNC2D];
  column_sums<double>(v + P.dof_off, NC, c0, c1, NC, acc, out);
  for (int l = threadIdx.x; l < NC; l += kBlock)
    it.nsp[((size_t)sl.j * kNsBlocksBatch + sl.lb) * kMaxNC2D + l] = out[l];
}

__global__ __launch_bounds__(kBlock) void k_null_finalize_batch(BatchIter it) {
  const int j = it.list[blockIdx.x];
  const BProb& P = it.probs[j];
  if (!serves(it, it.st + j)) return;
  __shared__ double S[kMaxNC2D], U[kMaxNC2D], acc[kBlock];
  const int nb = P.nns;
  const int n = P.N + 1, NC = P.NC;
  const double* Pn = it.pnull + P.N * 81;
  column_sums<double>(it.nsp + (size_t)j * kNsBlocksBatch * kMaxNC2D, kMaxNC2D, 0, nb, NC, acc, S);
  for (int l = threadIdx.x; l < NC; l += kBlock) S[l] = S[l] / (double)P.ncells;
  __syncthreads();
  for (int d = 0; d < 2; ++d) {
    const int stride = d == 0 ? 1 : n;
    for (int l = threadIdx.x; l < NC; l += kBlock) {
      const int ld = (l / stride) % n;
      const int base = l - ld * stride;
      double s = 0.0;
      for (int m = 0; m < n; ++m) s += Pn[ld * n + m] * S[base + m * stride];
      U[l] = s;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < NC; l += kBlock) S[l] = U[l];
    __syncthreads();
  }
  for (int l = threadIdx.x; l < NC; l += kBlock) it.corr[(size_t)j * kMaxNC2D + l] = S[l];
}

__global__ __launch_bounds__(kBlock) void k_sub_nodes_batch(BatchIter it, double* __restrict__ v) {
  const Slot sl = slot_of(it, it.upd_off, blockIdx.x);
  const BProb& P = it.probs[sl.j];
  if (!serves(it, it.st + sl.j)) return;
  const long long stride = (long long)P.nupd * kBlock;
  const double* cj = it.corr + (size_t)sl.j * kMaxNC2D;
  for (long long i = (long long)sl.lb * kBlock + threadIdx.x; i < P.ndof; i += stride)
    v[P.dof_off + i] -= cj[i % P.NC];
}

__global__ void k_tick(int* kbase, int by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *kbase += by;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_all(T* __restrict__ v, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    v[i] = T(0);
}

__global__ void k_state_init_batch(CgState* st, int count, int maxit, double tol2, int mode64) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    CgState& s = st[j];
    s.rho_hist[0] = s.rho_hist[1] = 0.0;
    s.rho = s.sigma = s.alpha = s.beta = 0.0;
    s.bnorm2 = s.aux = 0.0;
    s.tol2 = tol2;
    s.scale = s.ref = s.best = 1.0;
    s.iter = 0;
    s.maxit = maxit;
    s.done = 0;
    s.status = 0;
    s.restart_k = -1;
    s.restarts = 0;
    s.fin = 0;
    s.even_stop = 0;
    s.fresh = 1;
    s.mode64 = mode64;
    s.switched = 0;
    s.stall = 0;
    s.fallback_k = -1;
    s.xk = -1;
    s.xused = -1;
    s.idle = 0;
    s.outer = 0;
    s.run_a[0] = 0;
    s.run_a[1] = -1;
    s.run_u = -1;
  }
}

template <typename T, int N, int V>
hipError_t launch_group_N(const BatchIter& it, const BatchGroup& g, bool fuse, const void* x,
                          const void* pold, void* pnew, void* y, void* xsol, const OpTables& tb,
                          hipStream_t s) {
  Blk<T, N> B;
  B.fill(tb, line_eo<T, N, 2>());   // (the batched kernel runs the 2D tile body)
  if (fuse)
    hipLaunchKernelGGL((k_apply2d_batch<T, N, V, 2>), dim3(g.blocks), dim3(256), 0, s, it,
                       g.grp, g.toff, g.ng, (const T*)x, (const T*)pold, (T*)pnew, (T*)y,
                       (T*)xsol, B);
  else
    hipLaunchKernelGGL((k_apply2d_batch<T, N, V, 0>), dim3(g.blocks), dim3(256), 0, s, it,
                       g.grp, g.toff, g.ng, (const T*)x, (const T*)pold, (T*)pnew, (T*)y,
                       (T*)nullptr, B);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_group_V(const BatchIter& it, const BatchGroup& g, bool fuse, const void* x,
                          const void* pold, void* pnew, void* y, void* xsol, const OpTables& tb,
                          hipStream_t s) {
  switch (g.variant) {
    case 1: return launch_group_N<T, N, 1>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 2: return launch_group_N<T, N, 2>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    default: return launch_group_N<T, N, 0>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
  }
}

template <typename T>
hipError_t launch_group_T(const BatchIter& it, const BatchGroup& g, bool fuse, const void* x,
                          const void* pold, void* pnew, void* y, void* xsol, const OpTables& tb,
                          hipStream_t s) {
  switch (g.N) {
    case 0: return launch_group_V<T, 0>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 1: return launch_group_V<T, 1>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 2: return launch_group_V<T, 2>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 3: return launch_group_V<T, 3>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 4: return launch_group_V<T, 4>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 5: return launch_group_V<T, 5>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 6: return launch_group_V<T, 6>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 7: return launch_group_V<T, 7>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    case 8: return launch_group_V<T, 8>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_apply_batch(const BatchIter& it, const BatchGroup& g, bool fp32, bool fuse,
                              const void* x, const void* pold, void* pnew, void* y, void* xsol,
                              const OpTables& tb, hipStream_t s) {
  if (g.blocks == 0) return hipSuccess;
  return fp32 ? launch_group_T<float>(it, g, fuse, x, pold, pnew, y, xsol, tb, s)
              : launch_group_T<double>(it, g, fuse, x, pold, pnew, y, xsol, tb, s);
}

hipError_t launch_update_batch(const BatchIter& it, bool fp32, const void* q, void* r,
                               hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_update_batch<float>, dim3(it.upd_blocks), dim3(kBlock), 0, s, it,
                       (const float*)q, (float*)r);
  else
    hipLaunchKernelGGL(k_update_batch<double>, dim3(it.upd_blocks), dim3(kBlock), 0, s, it,
                       (const double*)q, (double*)r);
  return hipGetLastError();
}

hipError_t launch_xflush_batch(const BatchIter& it, double* x64, float* d32, const double* pa64,
                               const double* pb64, const float* pa32, const float* pb32,
                               hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xflush_batch, dim3(it.upd_blocks), dim3(kBlock), 0, s, it, x64, d32, pa64,
                     pb64, pa32, pb32);
  return hipGetLastError();
}

hipError_t launch_stream_batch(int mode, const BatchIter& it, const double* b, const double* q64,
                               double* r64, double* x64, float* v32, hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  const dim3 G(it.upd_blocks), T(kBlock);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_stream_batch<0>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    case 1: hipLaunchKernelGGL(k_stream_batch<1>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    case 2: hipLaunchKernelGGL(k_stream_batch<2>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    case 3: hipLaunchKernelGGL(k_stream_batch<3>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    case 4: hipLaunchKernelGGL(k_stream_batch<4>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    case 5: hipLaunchKernelGGL(k_stream_batch<5>, G, T, 0, s, it, b, q64, r64, x64, v32); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize_batch(int what, const BatchIter& it, hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  const dim3 G(it.count), T(kBlock);
  switch (what) {
    case 0: hipLaunchKernelGGL(k_finalize_batch<0>, G, T, 0, s, it); break;
    case 1: hipLaunchKernelGGL(k_finalize_batch<1>, G, T, 0, s, it); break;
    case 2: hipLaunchKernelGGL(k_finalize_batch<2>, G, T, 0, s, it); break;
    case 3: hipLaunchKernelGGL(k_finalize_batch<3>, G, T, 0, s, it); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pcg_update_batch(const BatchIter& it, int N, bool fp32, int sel,
                                   const double* V, const double* lam, const void* q, void* r,
                                   void* z, hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  if (!it.res || sel < 0 || sel > 2) return hipErrorInvalidValue;
  return fp32 ? pcg_batch_T<float>(it, N, sel, V, lam, q, r, z, s)
              : pcg_batch_T<double>(it, N, sel, V, lam, q, r, z, s);
}

hipError_t launch_project_null_batch(const BatchIter& it, double* v, hipStream_t s) {
  if (it.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_sums_batch, dim3(it.ns_blocks), dim3(kBlock), 0, s, it,
                     (const double*)v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_null_finalize_batch, dim3(it.count), dim3(kBlock), 0, s, it);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sub_nodes_batch, dim3(it.upd_blocks), dim3(kBlock), 0, s, it, v);
  return hipGetLastError();
}

hipError_t launch_tick(int* kbase, int by, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, kbase, by);
  return hipGetLastError();
}

hipError_t launch_zero_all(bool fp32, void* v, long long n, hipStream_t s) {
  long long g = (n + kBlock * 4 - 1) / (kBlock * 4);
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  if (fp32)
    hipLaunchKernelGGL(k_zero_all<float>, dim3((unsigned)g), dim3(kBlock), 0, s, (float*)v, n);
  else
    hipLaunchKernelGGL(k_zero_all<double>, dim3((unsigned)g), dim3(kBlock), 0, s, (double*)v, n);
  return hipGetLastError();
}

hipError_t launch_state_init_batch(CgState* st, int count, int maxit, double tol2, int mode64,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_state_init_batch, dim3((count + 63) / 64), dim3(64), 0, s, st, count,
                     maxit, tol2, mode64);
  return hipGetLastError();
}

}  // namespace pdk
