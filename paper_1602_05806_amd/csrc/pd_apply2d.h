// Shared pieces of the operator-apply kernels (single-problem and batched launches): kernel
// argument block, periodic index wrap, the 1D three-cell line operator and the 2D tile body.
// The kernel design notes are at the top of pd_apply_kernels.h.
#pragma once
#include "pd_device.h"

namespace pdk {

template <typename T>
struct ApplyArgs {
  const T* x;       // operand (FUSE = 0) or residual r (FUSE = 1)
  const T* pold;    // FUSE = 1: previous search direction
  T* pnew;          // FUSE = 1: new search direction (must not alias pold)
  T* y;             // result
  int nx, ny, nz;
  int ntx, nty, ntz;
  int kz;           // 3D: planes per column segment
  T alpha;          // mass coefficient
  T c0, c1, c2;     // coefficient of each direction (beta / h_d^2)
  // FUSE = 1: CG iteration k, partials of rho_k and rho_{k-1}, sigma partials (one per block)
  CgState* st;
  int k;              // iteration index, or offset from *kbase when kbase is set
  const int* kbase;   // device-resident iteration base (graph-replayed batched runs) or null
  const double* rho_cur;
  const double* res_cur;   // preconditioned runs: partials of <r_k, r_k> (x is then z = P r)
  int nrho;
  double* sigpart;
  T* xsol;            // FUSE = 2, 3: CG iterate, x += alpha_{k-1} p_old on owned cells
  // FUSE = 3 (one kernel per CG iteration, 2D): the residual update of iteration k - 1 is made
  // here, r_k = r_{k-1} - alpha_{k-1} q_{k-1}, from x = r_{k-1} and qprev = q_{k-1} (halo cells
  // included, so both are double-buffered: rout and y must not alias x and qprev). first = 1:
  // x already holds r_k (iteration 0, or a run resumed after a residual replacement) with the
  // partials of <r_k, r_k> in rho_cur; nothing is updated. Each block writes the 4-tuple
  // (<p, A p>, <r, A p>, <A p, A p>, <r, r>) of its owned cells to fout[4 slot ..], and the
  // next launch reads the npart tuples of this one from fin.
  const T* qprev;
  T* rout;
  const double* fin;
  double* fout;
  int npart;
  int first;
  int remap;          // single-problem 2D launch: 1 = XCD-contiguous tile ranges (xcd_remap)
  // mir[d] = 1: homogeneous Dirichlet pressure walls across direction d (the cells beyond a
  // wall hold the odd reflection -J of the adjacent cell: index mirrored, node order reversed
  // along d, sign flipped); 0: periodic wrap
  int mir[3];
};

// Mirror a cell index beyond a Dirichlet wall onto the domain: -1 -> 0, m -> m - 1, ...
__device__ __forceinline__ int mirror_index(int i, int m) {
  return i < 0 ? -1 - i : 2 * m - 1 - i;
}

__device__ __forceinline__ int wrapi(int i, int m) {
  i %= m;
  return i < 0 ? i + m : i;
}


// One output row l of the 1D three-cell operator (row form of the blocks): sum_m L[l][m] vl[m] +
// C[l][m] vc[m] + R[l][m] vr[m], with three independent accumulators (the FMA latency is not
// serialised over 3(N+1) terms). Called with a run-time row index from a rolled loop, so the
// coefficients of the rows being computed are scalar-loaded per iteration instead of keeping
// all 3(N+1)^2 of them live.
template <typename T, int N>
__device__ __forceinline__ T row3(const Blk<T, N>& B, int l, const T (&vl)[N + 1],
                                  const T (&vc)[N + 1], const T (&vr)[N + 1]) {
  constexpr int n = N + 1;
  const T* L = B.K;
  const T* C = B.K + n * n;
  const T* R = B.K + 2 * n * n;
  T al = T(0), ac = T(0), ar = T(0);
#pragma unroll
  for (int m = 0; m < n; ++m) {
    al += L[l * n + m] * vl[m];
    ac += C[l * n + m] * vc[m];
    ar += R[l * n + m] * vr[m];
  }
  return (al + ac) + ar;
}

// Apply the 1D three-cell operator to one line: out(l) = L vl + C vc + R vr at every row l, in
// the form line_eo<T, N, DIM> selects (the host fills Blk in that form).
//   rows      row3 per row, two rows per iteration where the scalar-register budget allows it;
//   even/odd  with s = vl + J vr and d = vl - J vr (J the node reversal, R = J L J), rows p and
//             N - p are e + o and e - o, e = 1/2 (L_p + L_{N-p}) s + 1/2 (C_p + C_{N-p}) vc,
//             o = 1/2 (L_p - L_{N-p}) d + 1/2 (C_p - C_{N-p}) vc; as C = J C J, the C parts
//             are sums over m < (N+1)/2 of the half rows on vc[m] + vc[N-m] and vc[m] - vc[N-m]:
//             about 1.5 (N+1)^2 FMAs per line.
template <typename T, int N, int DIM, typename F>
__device__ __forceinline__ void line3(const Blk<T, N>& B, const T (&vl)[N + 1],
                                      const T (&vc)[N + 1], const T (&vr)[N + 1], F&& out) {
  constexpr int n = N + 1;
  if constexpr (line_eo<T, N, DIM>()) {
    constexpr int P = n / 2, H1 = (n + 1) / 2, H0 = n / 2, PS = 3 * n;
    T s[n], d[n], ce[H1], co[H0 > 0 ? H0 : 1];
#pragma unroll
    for (int m = 0; m < n; ++m) {
      s[m] = vl[m] + vr[n - 1 - m];
      d[m] = vl[m] - vr[n - 1 - m];
    }
#pragma unroll
    for (int m = 0; m < H0; ++m) {
      ce[m] = vc[m] + vc[n - 1 - m];
      co[m] = vc[m] - vc[n - 1 - m];
    }
    if constexpr (n & 1) ce[H0] = vc[H0];
#pragma unroll 1
    for (int p = 0; p < P; ++p) {
      const T* c = B.K + PS * p;
      T e0 = T(0), e1 = T(0), o0 = T(0), o1 = T(0);
#pragma unroll
      for (int m = 0; m < n; ++m) {
        e0 += c[m] * s[m];
        o0 += c[n + H1 + m] * d[m];
      }
#pragma unroll
      for (int m = 0; m < H1; ++m) e1 += c[n + m] * ce[m];
#pragma unroll
      for (int m = 0; m < H0; ++m) o1 += c[2 * n + H1 + m] * co[m];
      const T e = e0 + e1, o = o0 + o1;
      out(p, e + o);
      out(n - 1 - p, e - o);
    }
    if constexpr (n & 1) {
      const T* c = B.K + PS * P;
      T e0 = T(0), e1 = T(0);
#pragma unroll
      for (int m = 0; m < n; ++m) e0 += c[m] * s[m];
#pragma unroll
      for (int m = 0; m < H1; ++m) e1 += c[n + m] * ce[m];
      out(P, e0 + e1);
    }
  } else {
    constexpr bool pairs = 2 * 3 * n * (int)sizeof(T) / 4 <= 36;   // SGPRs of two rows
    if constexpr (pairs) {
#pragma unroll 1
      for (int l = 0; l + 1 < n; l += 2) {
        const T r0 = row3<T, N>(B, l, vl, vc, vr);
        const T r1 = row3<T, N>(B, l + 1, vl, vc, vr);
        out(l, r0);
        out(l + 1, r1);
      }
      if (n & 1) out(n - 1, row3<T, N>(B, n - 1, vl, vc, vr));
    } else {
#pragma unroll 1
      for (int l = 0; l < n; ++l) out(l, row3<T, N>(B, l, vl, vc, vr));
    }
  }
}

__device__ __forceinline__ int wrap_small(int i, int m) {
  // i in [-m, 2m) for every caller except grids narrower than a tile (loop handles those)
  while (i < 0) i += m;
  while (i >= m) i -= m;
  return i;
}

// ------------------------------------------------------------------ 2D tile kernel

// 2D tile shapes. Variant V = 0 is the largest of 8x8, 8x4, 4x4, 4x2, 2x2 whose LDS footprint
// (box + accumulator) fits 40 KB; V = 1 and V = 2 are the next one and two sizes down (more
// workgroups and occupancy, more halo). The batched solver's autotuner picks V per size bucket.
template <typename T, int N, int V = 0>
struct Tile2D {
  static constexpr int n = N + 1, NC = n * n;
  static constexpr bool fits(int tx, int ty) {
    return ((tx + 2) * (ty + 2) + tx * ty) * NC * (int)sizeof(T) <= 40960;
  }
  static constexpr int first = fits(8, 8) ? 0 : fits(8, 4) ? 1 : fits(4, 4) ? 2 : fits(4, 2) ? 3 : 4;
  static constexpr int idx = first + V < 4 ? first + V : 4;
  static constexpr int TX = idx == 0 ? 8 : idx == 1 ? 8 : idx == 2 ? 4 : idx == 3 ? 4 : 2;
  static constexpr int TY = idx == 0 ? 8 : idx == 1 ? 4 : idx == 2 ? 4 : idx == 3 ? 2 : 2;
};

// 2D: LDS holds the tile and its face halos as a (TX+2) x (TY+2) box of cells (corners unused),
// box cell (bi, bj) = tile cell (bi-1, bj-1). Box row bj is one contiguous run of cells in global
// memory unless it crosses the periodic seam, so staging is a flat copy per row. The workgroup
// processes tiles t_begin, t_begin + t_stride, ... below t_end.
// MIR: the grid has Dirichlet walls (a.mir); the periodic form carries none of their code.
template <typename T, int N, int V, int FUSE, int PF, bool MIR = false>
__device__ __forceinline__ void apply2d_body(const ApplyArgs<T>& a, const Blk<T, N>& B,
                                             int t_begin, int t_end, int t_stride, int slot) {
  constexpr bool RU = FUSE == 3;                // residual update folded in
  using TL = Tile2D<T, N, V>;
  constexpr int n = N + 1, NC = n * n, TX = TL::TX, TY = TL::TY, NT = TX * TY;
  constexpr int BX = TX + 2;                    // box width in cells
  constexpr int RI = BX * NC;                   // elements of an interior box row
  constexpr int RH = TX * NC;                   // elements of a halo box row (no corners)
  constexpr int JI = (RI + 255) / 256, JH = (RH + 255) / 256;
  __shared__ T xs[(TY + 2) * BX * NC];
  __shared__ T ys[NT * NC];
  // launches queued after the run stopped exit before loading anything
  const int kit = FUSE ? (a.kbase ? *a.kbase + a.k : a.k) : 0;
  if (FUSE) {
    if (!apply_may_run(a.st, kit)) return;
  }
  const T* __restrict__ xg = a.x;
  const T* __restrict__ pg = a.pold;
  T* __restrict__ png = a.pnew;
  T* __restrict__ yg = a.y;
  const int tid = threadIdx.x;
  T rvi[TY][JI], pvi[TY][JI], rvh[2][JH], pvh[2][JH];
  T xvi[FUSE >= 2 ? TY : 1][FUSE >= 2 ? JI : 1];   // FUSE >= 2: x of the owned cells
  T qvi[RU ? TY : 1][RU ? JI : 1], qvh[RU ? 2 : 1][RU ? JH : 1];   // q_{k-1}
  T rki[RU ? TY : 1][RU ? JI : 1];              // r_k of the owned cells (for <r_k, A p_k>)
  const bool rupd = RU && !a.first;

  // global element index of box element e of box row bj (bj in 0..TY+1) of the tile at (tx0, ty0);
  // neg: the element is the odd reflection of that source across a Dirichlet wall
  auto gindex = [&](int tx0, int ty0, int bj, int e, bool& neg) -> size_t {
    const int first = (bj == 0 || bj == TY + 1) ? 0 : -1;   // first tile column of the row
    const int cr = e / NC;
    int l = e - cr * NC;
    int ri = tx0 + first + cr, rj = ty0 + bj - 1;
    neg = false;
    if (MIR && a.mir[0] && (ri < 0 || ri >= a.nx)) {
      ri = mirror_index(ri, a.nx);
      l = (l / n) * n + (n - 1 - l % n);
      neg = !neg;
    }
    if (MIR && a.mir[1] && (rj < 0 || rj >= a.ny)) {
      rj = mirror_index(rj, a.ny);
      l = (n - 1 - l / n) * n + l % n;
      neg = !neg;
    }
    const int gi = wrap_small(ri, a.nx);
    const int gj = wrap_small(rj, a.ny);
    return ((size_t)gj * a.nx + gi) * NC + l;
  };
  // box rows [bj_lo, bj_hi) of a tile into registers
  auto stage_load = [&](int tile, int bj_lo, int bj_hi) {
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    const bool flat = tx0 >= 1 && tx0 + TX + 1 <= a.nx;        // no row crosses the x seam / a wall
#pragma unroll
    for (int bj = 0; bj < TY + 2; ++bj) {
      if (bj < bj_lo || bj >= bj_hi) continue;
      const bool halo = bj == 0 || bj == TY + 1;
      const int rj = ty0 + bj - 1;
      const bool rowflat = flat && !(MIR && a.mir[1] && (rj < 0 || rj >= a.ny));
      const int gj = wrap_small(rj, a.ny);
      const size_t row0 = ((size_t)gj * a.nx + (halo ? tx0 : tx0 - 1)) * NC;
      constexpr int J = JI > JH ? JI : JH;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int e = tid + 256 * j;
        if (e < (halo ? RH : RI)) {
          bool neg = false;
          const size_t g = rowflat ? row0 + e : gindex(tx0, ty0, bj, e, neg);
          T rv = xg[g], pv = T(0), qv = T(0);
          if (FUSE) pv = pg[g];
          if (rupd) qv = a.qprev[g];
          if (halo) {
            if (j < JH) {
              rvh[bj ? 1 : 0][j] = rv;
              pvh[bj ? 1 : 0][j] = pv;
              if (RU) qvh[bj ? 1 : 0][j] = qv;
            }
          } else if (j < JI) {
            rvi[bj - 1][j] = rv;
            pvi[bj - 1][j] = pv;
            if (RU) qvi[bj - 1][j] = qv;
            if (FUSE >= 2 && e >= NC && e < (TX + 1) * NC) xvi[bj - 1][j] = a.xsol[g];
          }
        }
      }
    }
  };

  if (t_begin < t_end) stage_load(t_begin, 0, TY + 2);
  T beta = T(0);
  bool xupd = false;   // FUSE = 2: x += xalpha p_old on the owned cells
  T xalpha = T(0);
  if (rupd) {
    const FusedScalars sc = fused_scalars<256>(a.st, a.k, a.fin, a.npart, t_begin == 0);
    if (sc.stop) return;
    beta = (T)sc.beta;
    xupd = true;
    xalpha = (T)sc.alpha;
  } else if (FUSE) {
    const int k = kit;
    const IterScalars sc = iteration_scalars<256>(a.st, k, a.rho_cur, a.nrho, t_begin == 0, RU,
                                                  a.res_cur);
    if (sc.stop) return;
    beta = (T)sc.beta;
    if (FUSE == 2) {
      xupd = k >= 1 && a.st->xk == k - 1;
      xalpha = (T)a.st->alpha;
      if (xupd && t_begin == 0 && threadIdx.x == 0) a.st->xused = k - 1;
    }
  }
  double dot = 0.0, gam = 0.0, nu = 0.0, rr = 0.0;   // RU: <r, A p>, <A p, A p>, <r, r>
  for (int tile = t_begin; tile < t_end; tile += t_stride) {
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    // registers -> LDS (p = r + beta p_old formed here; owned cells also stored to global)
#pragma unroll
    for (int bj = 0; bj < TY + 2; ++bj) {
      const bool halo = bj == 0 || bj == TY + 1;
      constexpr int J = JI > JH ? JI : JH;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int e = tid + 256 * j;
        if (e < (halo ? RH : RI) && (halo ? j < JH : j < JI)) {
          T v = halo ? rvh[bj ? 1 : 0][j] : rvi[bj - 1][j];
          if (rupd) v = v - xalpha * (halo ? qvh[bj ? 1 : 0][j] : qvi[bj - 1][j]);
          if (FUSE) {
            const T rk = v;
            // beta = 0 (first iteration, restart) must not read p_old, which may hold anything
            if (beta != T(0)) v = v + beta * (halo ? pvh[bj ? 1 : 0][j] : pvi[bj - 1][j]);
            if (!halo) {
              const int bi = e / NC;                 // box column: own cells are 1..TX
              const int ui = tx0 + bi - 1, uj = ty0 + bj - 1;
              if (bi >= 1 && bi <= TX && ui < a.nx && uj < a.ny) {
                const size_t g = ((size_t)uj * a.nx + ui) * NC + (e - bi * NC);
                png[g] = v;
                if (FUSE >= 2 && xupd) a.xsol[g] = xvi[bj - 1][j] + xalpha * pvi[bj - 1][j];
                if (RU) {
                  if (rupd) a.rout[g] = rk;
                  rki[bj - 1][j] = rk;
                  rr += (double)rk * (double)rk;
                }
              }
            }
          }
          if constexpr (MIR) {
            // the sign of a reflected element is applied here, not to the loaded value, so
            // that the loads of a prefetched tile are not waited for when they are issued
            // (owned cells are never reflected: the values stored above carry no sign)
            const int ri = tx0 + (halo ? 0 : -1) + e / NC, rj = ty0 + bj - 1;
            const bool nx_ = a.mir[0] && (ri < 0 || ri >= a.nx);
            const bool ny_ = a.mir[1] && (rj < 0 || rj >= a.ny);
            if (nx_ != ny_) v = -v;
          }
          xs[(bj * BX + (halo ? 1 : 0)) * NC + e] = v;
        }
      }
    }
    __syncthreads();
    // the next tile's loads, in flight during the compute below: half of the box rows before the
    // x-lines, half before the y-lines (issuing all at once stalls this wave's x-lines while the
    // memory pipeline drains)
    constexpr int HALF = (TY + 2) / 2;
    if (PF && tile + t_stride < t_end) stage_load(tile + t_stride, 0, HALF);

    // x-lines: (cell c, l2); nodes l1 = 0..N
    for (int L = tid; L < NT * n; L += 256) {
      const int c = L / n, l2 = L - c * n;
      const int ci = c % TX, cj = c / TX;
      const int bc = ((cj + 1) * BX + ci + 1) * NC + l2 * n;
      T vl[n], vc[n], vr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vl[m] = xs[bc - NC + m];
        vc[m] = xs[bc + m];
        vr[m] = xs[bc + NC + m];
      }
      const T wgt = a.c0 * B.w[l2];
      line3<T, N, 2>(B, vl, vc, vr, [&](int l1, T v) { ys[c * NC + l2 * n + l1] = wgt * v; });
    }
    __syncthreads();
    if (PF && tile + t_stride < t_end) stage_load(tile + t_stride, HALF, TY + 2);

    // y-lines: (cell c, l1); nodes l2 = 0..N; final values are stored here
    for (int L = tid; L < NT * n; L += 256) {
      const int c = L / n, l1 = L - c * n;
      const int ci = c % TX, cj = c / TX;
      const int bc = ((cj + 1) * BX + ci + 1) * NC + l1;
      T vl[n], vc[n], vr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vl[m] = xs[bc - BX * NC + m * n];
        vc[m] = xs[bc + m * n];
        vr[m] = xs[bc + BX * NC + m * n];
      }
      const int ui = tx0 + ci, uj = ty0 + cj;
      const bool valid = ui < a.nx && uj < a.ny;
      const size_t base = ((size_t)uj * a.nx + ui) * NC;
      const T wgt = a.c1 * B.w[l1];
      const T wm = a.alpha * B.w[l1];
      line3<T, N, 2>(B, vl, vc, vr, [&](int l2, T v) {
        const T xc = xs[bc + l2 * n];
        const T val = ys[c * NC + l2 * n + l1] + wgt * v + wm * B.w[l2] * xc;
        if (valid) {
          yg[base + l2 * n + l1] = val;
          dot += (double)xc * (double)val;
          if (RU) {
            nu += (double)val * (double)val;
            ys[c * NC + l2 * n + l1] = val;     // read back below for <r_k, A p_k>
          }
        }
      });
    }
    __syncthreads();
    if (RU) {
      // <r_k, A p_k> over the owned cells: r_k from registers (staging layout), A p_k from the
      // accumulator, which the y-lines overwrote with the final values (the next tile's x-lines
      // write it only after the staging barrier)
#pragma unroll
      for (int bj = 1; bj <= TY; ++bj) {
#pragma unroll
        for (int j = 0; j < JI; ++j) {
          const int e = tid + 256 * j;
          if (e < RI) {
            const int bi = e / NC;
            const int ui = tx0 + bi - 1, uj = ty0 + bj - 1;
            if (bi >= 1 && bi <= TX && ui < a.nx && uj < a.ny)
              gam += (double)rki[bj - 1][j] * (double)ys[((bj - 1) * TX + bi - 1) * NC + e - bi * NC];
          }
        }
      }
    }
    if (!PF && tile + t_stride < t_end) stage_load(tile + t_stride, 0, TY + 2);
  }
  if (RU) {
    double s4[4] = {dot, gam, nu, rr};
    block_sum4_all<256>(s4);
    if (threadIdx.x == 0) {
      double* o = a.fout + 4 * (size_t)slot;
      *reinterpret_cast<double2*>(o) = make_double2(s4[0], s4[1]);
      *reinterpret_cast<double2*>(o + 2) = make_double2(s4[2], s4[3]);
    }
  } else if (FUSE) {
    const double s = block_sum_all<256>(dot);
    if (threadIdx.x == 0) a.sigpart[slot] = s;
  }
}

}  // namespace pdk
