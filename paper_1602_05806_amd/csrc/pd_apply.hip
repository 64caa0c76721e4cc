// Matrix-free application of alpha M^{xyz} + sum_d c_d (M on the other directions) (x) H_d, the
// pressure / viscous operator of arXiv:1602.05806 eqs. (pSyst) and (implicitviscosity), applied
// dimension by dimension with the 1D blocks L, C, R (eq. tensorP1): along every line of nodes in
// direction d, (H_d x)_i = L x_{i-1} + C x_i + R x_{i+1} over the three cells of that line.
//
// Two kernel shapes (both memory-bound streaming kernels on gfx950, VALU FMA with the 1D blocks
// in scalar registers loaded from the kernarg segment):
//   2D  one workgroup per TX x TY tile of cells; tile + face halos staged in LDS; the x-lines
//       write partial results to an LDS accumulator, the y-lines finish and store.
//   3D  one workgroup per TX x TY column of cells marching over a range of planes along z. Each
//       thread owns one z-line of one cell and keeps the z-lines of planes k-1, k, k+1 in
//       registers, so the z coupling never touches LDS and every cell is read from HBM once
//       (plus two boundary planes per column segment). The x- and y-lines of plane k go through
//       LDS with the plane's x/y face halos.
// FUSE = 1 is the CG form: the search direction p = r + beta p_old is formed while loading
// (beta read from the device-resident CG state), stored for the owned cells, and the block sums of
// <p, A p> feed the grid reduction that sets alpha = rho / <p, A p>.
#include "pd_device.h"
#include "pd_launch.h"

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
  int k;
  const double* rho_cur;
  int nrho;
  double* sigpart;
};

__device__ __forceinline__ int wrapi(int i, int m) {
  i %= m;
  return i < 0 ? i + m : i;
}


// One output row l of the 1D three-cell operator: sum_m L[l][m] vl[m] + C[l][m] vc[m] + R[l][m] vr[m],
// with three independent accumulators (the FMA latency is not serialised over 3(N+1) terms).
// Called with a run-time row index from a rolled loop, so the coefficients of the rows being
// computed are scalar-loaded per iteration instead of keeping all 3(N+1)^2 of them live.
template <typename T, int N>
__device__ __forceinline__ T row3(const Blk<T, N>& B, int l, const T (&vl)[N + 1],
                                  const T (&vc)[N + 1], const T (&vr)[N + 1]) {
  constexpr int n = N + 1;
  T al = T(0), ac = T(0), ar = T(0);
#pragma unroll
  for (int m = 0; m < n; ++m) {
    al += B.L[l * n + m] * vl[m];
    ac += B.C[l * n + m] * vc[m];
    ar += B.R[l * n + m] * vr[m];
  }
  return (al + ac) + ar;
}

// Apply the 1D three-cell operator to one line: out(l) = op(l) for every row l, two rows per
// iteration where the scalar-register budget allows it.
template <typename T, int N, typename F>
__device__ __forceinline__ void line3(const Blk<T, N>& B, const T (&vl)[N + 1],
                                      const T (&vc)[N + 1], const T (&vr)[N + 1], F&& out) {
  constexpr int n = N + 1;
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

__device__ __forceinline__ int wrap_small(int i, int m) {
  // i in [-m, 2m) for every caller except grids narrower than a tile (loop handles those)
  while (i < 0) i += m;
  while (i >= m) i -= m;
  return i;
}

// ------------------------------------------------------------------ 2D tile kernel

template <typename T, int N>
struct Tile2D {
  static constexpr int n = N + 1, NC = n * n;
  static constexpr bool fits(int tx, int ty) {
    return ((tx + 2) * (ty + 2) + tx * ty) * NC * (int)sizeof(T) <= 40960;
  }
  static constexpr int TX = fits(8, 8) ? 8 : fits(8, 4) ? 8 : fits(4, 4) ? 4 : fits(4, 2) ? 4 : 2;
  static constexpr int TY = fits(8, 8) ? 8 : fits(8, 4) ? 4 : fits(4, 4) ? 4 : fits(4, 2) ? 2 : 2;
};

// 2D: LDS holds the tile and its face halos as a (TX+2) x (TY+2) box of cells (corners unused),
// box cell (bi, bj) = tile cell (bi-1, bj-1). Box row bj is one contiguous run of cells in global
// memory unless it crosses the periodic seam, so staging is a flat copy per row.
template <typename T, int N, int FUSE, int PF>
__global__ __launch_bounds__(256) void k_apply2d(ApplyArgs<T> a, Blk<T, N> B) {
  using TL = Tile2D<T, N>;
  constexpr int n = N + 1, NC = n * n, TX = TL::TX, TY = TL::TY, NT = TX * TY;
  constexpr int BX = TX + 2;                    // box width in cells
  constexpr int RI = BX * NC;                   // elements of an interior box row
  constexpr int RH = TX * NC;                   // elements of a halo box row (no corners)
  constexpr int JI = (RI + 255) / 256, JH = (RH + 255) / 256;
  __shared__ T xs[(TY + 2) * BX * NC];
  __shared__ T ys[NT * NC];
  if (FUSE) {
    if (a.st->done) return;
  }
  const T* __restrict__ xg = a.x;
  const T* __restrict__ pg = a.pold;
  T* __restrict__ png = a.pnew;
  T* __restrict__ yg = a.y;
  // Persistent workgroups: this one owns the contiguous tile range [t_begin, t_end) (each XCD
  // gets a contiguous range of workgroups, so neighbouring tiles share an L2).
  const unsigned lw = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = a.ntx * a.nty;
  const int t_begin = (int)lw * a.kz;           // kz = tiles per workgroup in 2D
  const int t_end = min(t_begin + a.kz, ntiles);
  const int tid = threadIdx.x;
  T rvi[TY][JI], pvi[TY][JI], rvh[2][JH], pvh[2][JH];

  // global element index of box element e of box row bj (bj in 0..TY+1) of the tile at (tx0, ty0)
  auto gindex = [&](int tx0, int ty0, int bj, int e) -> size_t {
    const int first = (bj == 0 || bj == TY + 1) ? 0 : -1;   // first tile column of the row
    const int cr = e / NC, l = e - cr * NC;
    const int gi = wrap_small(tx0 + first + cr, a.nx);
    const int gj = wrap_small(ty0 + bj - 1, a.ny);
    return ((size_t)gj * a.nx + gi) * NC + l;
  };
  auto stage_load = [&](int tile) {
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    const bool flat = tx0 >= 1 && tx0 + TX + 1 <= a.nx;        // no row crosses the x seam
#pragma unroll
    for (int bj = 0; bj < TY + 2; ++bj) {
      const bool halo = bj == 0 || bj == TY + 1;
      const int gj = wrap_small(ty0 + bj - 1, a.ny);
      const size_t row0 = ((size_t)gj * a.nx + (halo ? tx0 : tx0 - 1)) * NC;
      constexpr int J = JI > JH ? JI : JH;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int e = tid + 256 * j;
        if (e < (halo ? RH : RI)) {
          const size_t g = flat ? row0 + e : gindex(tx0, ty0, bj, e);
          T rv = xg[g], pv = T(0);
          if (FUSE) pv = pg[g];
          if (halo) {
            if (j < JH) { rvh[bj ? 1 : 0][j] = rv; pvh[bj ? 1 : 0][j] = pv; }
          } else if (j < JI) {
            rvi[bj - 1][j] = rv;
            pvi[bj - 1][j] = pv;
          }
        }
      }
    }
  };

  if (t_begin < t_end) stage_load(t_begin);
  T beta = T(0);
  if (FUSE) {
    const IterScalars sc = iteration_scalars<256>(a.st, a.k, a.rho_cur, a.nrho);
    if (sc.stop) return;
    beta = (T)sc.beta;
  }
  double dot = 0.0;
  for (int tile = t_begin; tile < t_end; ++tile) {
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
          if (FUSE) {
            v = v + beta * (halo ? pvh[bj ? 1 : 0][j] : pvi[bj - 1][j]);
            if (!halo) {
              const int bi = e / NC;                 // box column: own cells are 1..TX
              const int ui = tx0 + bi - 1, uj = ty0 + bj - 1;
              if (bi >= 1 && bi <= TX && ui < a.nx && uj < a.ny)
                png[((size_t)uj * a.nx + ui) * NC + (e - bi * NC)] = v;
            }
          }
          xs[(bj * BX + (halo ? 1 : 0)) * NC + e] = v;
        }
      }
    }
    __syncthreads();
    if (PF && tile + 1 < t_end) stage_load(tile + 1);   // in flight during the compute below

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
      line3<T, N>(B, vl, vc, vr, [&](int l1, T v) { ys[c * NC + l2 * n + l1] = wgt * v; });
    }
    __syncthreads();

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
      line3<T, N>(B, vl, vc, vr, [&](int l2, T v) {
        const T xc = xs[bc + l2 * n];
        const T val = ys[c * NC + l2 * n + l1] + wgt * v + wm * B.w[l2] * xc;
        if (valid) {
          yg[base + l2 * n + l1] = val;
          dot += (double)xc * (double)val;
        }
      });
    }
    __syncthreads();
    if (!PF && tile + 1 < t_end) stage_load(tile + 1);
  }
  if (FUSE) {
    const double s = block_sum_all<256>(dot);
    if (threadIdx.x == 0) a.sigpart[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ 3D z-marching kernel

template <int N>
struct Tile3D {
  static constexpr int TX = N == 0 ? 16 : N == 1 ? 8 : N == 2 ? 8 : N <= 4 ? 4 : N == 5 ? 4 : 2;
  static constexpr int TY = N == 0 ? 16 : N == 1 ? 8 : N == 2 ? 4 : N <= 4 ? 4 : 2;
  static constexpr int NTH = TX * TY * (N + 1) * (N + 1);
};

template <typename T, int N, int FUSE, int PF>
__global__ __launch_bounds__(Tile3D<N>::NTH) void k_apply3d(ApplyArgs<T> a, Blk<T, N> B) {
  constexpr int n = N + 1, NP = n * n, NC = n * n * n;
  constexpr int TX = Tile3D<N>::TX, TY = Tile3D<N>::TY, NT = TX * TY, NTH = Tile3D<N>::NTH;
  constexpr int S_XL = NT, S_XR = NT + TY, S_YL = NT + 2 * TY, S_YR = NT + 2 * TY + TX;
  constexpr int NS = NT + 2 * TY + 2 * TX;
  constexpr int NH = NS - NT;
  __shared__ T xs[NS * NC];
  __shared__ T ys[NT * NC];
  __shared__ int hbase[NS];     // in-plane cell index (j*nx + i, wrapped) of every halo slot
  if (FUSE) {
    if (a.st->done) return;
  }
  const T* __restrict__ xg = a.x;
  const T* __restrict__ pg = a.pold;
  T* __restrict__ png = a.pnew;
  const unsigned tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tcol = (int)(tile % (unsigned)(a.ntx * a.nty));
  const int zseg = (int)(tile / (unsigned)(a.ntx * a.nty));
  const int tx0 = (tcol % a.ntx) * TX, ty0 = (tcol / a.ntx) * TY;
  const int k0 = zseg * a.kz;
  const int k1 = min(k0 + a.kz, a.nz);
  for (int s = NT + (int)threadIdx.x; s < NS; s += NTH) {
    int hi, hj;
    if (s < S_XR) { hi = -1; hj = s - S_XL; }
    else if (s < S_YL) { hi = TX; hj = s - S_XR; }
    else if (s < S_YR) { hi = s - S_YL; hj = -1; }
    else { hi = s - S_YR; hj = TY; }
    hbase[s] = wrapi(ty0 + hj, a.ny) * a.nx + wrapi(tx0 + hi, a.nx);
  }
  __syncthreads();   // hbase ready

  const int t = threadIdx.x;
  const int c = t / NP, lp = t - c * NP;          // cell in the plane tile, z-line (l1 + n l2)
  const int ci = c % TX, cj = c / TX;
  const int ui = tx0 + ci, uj = ty0 + cj;
  const bool valid = ui < a.nx && uj < a.ny;
  const int gi = wrapi(ui, a.nx), gj = wrapi(uj, a.ny);
  const size_t plane = (size_t)a.nx * a.ny;
  T beta = T(0);

  auto zbase = [&](int k) -> size_t {
    return (((size_t)wrap_small(k, a.nz) * a.ny + gj) * a.nx + gi) * NC + lp;
  };
  T zp[n], zc[n], zn[n];
  {
    // first two planes of this thread's z-line; the CG scalars are reduced while they load
    const size_t bp = zbase(k0 - 1), bc = zbase(k0);
    T pp[n], pc[n];
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zp[l3] = xg[bp + l3 * NP];
      zc[l3] = xg[bc + l3 * NP];
      if (FUSE) {
        pp[l3] = pg[bp + l3 * NP];
        pc[l3] = pg[bc + l3 * NP];
      }
    }
    if (FUSE) {
      const IterScalars sc = iteration_scalars<NTH>(a.st, a.k, a.rho_cur, a.nrho);
      if (sc.stop) return;
      beta = (T)sc.beta;
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zp[l3] = zp[l3] + beta * pp[l3];
        zc[l3] = zc[l3] + beta * pc[l3];
        if (valid) png[bc + l3 * NP] = zc[l3];
      }
    }
  }
  // per-thread x-line and y-line coordinates (one line per thread in each direction)
  const int xl23 = lp;                        // x-line: (l2, l3) = (lp % n, lp / n)
  const int yl1 = lp % n, yl3 = lp / n;       // y-line: (l1, l3)
  const int zl1 = lp % n, zl2 = lp / n;       // z-line: (l1, l2)
  const int sxl = (ci == 0) ? S_XL + cj : c - 1;
  const int sxr = (ci == TX - 1) ? S_XR + cj : c + 1;
  const int syl = (cj == 0) ? S_YL + ci : c - TX;
  const int syr = (cj == TY - 1) ? S_YR + ci : c + TX;
  const T wx = a.c0 * B.w[xl23 % n] * B.w[xl23 / n];
  const T wy = a.c1 * B.w[yl1] * B.w[yl3];
  const T wz = a.c2 * B.w[zl1] * B.w[zl2];
  const T wm = a.alpha * B.w[zl1] * B.w[zl2];
  double dot = 0.0;

  // x/y halo cells of a plane: one wave per cell (wave-uniform addressing). When the register
  // budget allows, plane k+1's halo is prefetched during plane k's compute.
  constexpr int NWV = NTH / 64;                // full waves (a partial last wave stays idle)
  static_assert(NWV >= 1, "3D tile needs at least one full wave");
  constexpr int HPW = (NH + NWV - 1) / NWV;
  constexpr int LR = (NC + 63) / 64;
  constexpr bool PREF = PF && HPW * LR <= 8;
  constexpr int HR = PREF ? HPW : 1;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = t & 63;
  T hv[HR][LR], hp[HR][LR];
  auto halo_load = [&](int k) {
    const size_t pb = (size_t)wrap_small(k, a.nz) * plane;
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
        const size_t g = (pb + (size_t)hbase[s]) * NC;
#pragma unroll
        for (int r = 0; r < LR; ++r) {
          const int l = lane + 64 * r;
          if (l < NC) {
            hv[i][r] = xg[g + l];
            if (FUSE) hp[i][r] = pg[g + l];
          }
        }
      }
    }
  };
  auto halo_store = [&]() {
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
#pragma unroll
        for (int r = 0; r < LR; ++r) {
          const int l = lane + 64 * r;
          if (l < NC) xs[s * NC + l] = FUSE ? (T)(hv[i][r] + beta * hp[i][r]) : hv[i][r];
        }
      }
    }
  };
  auto halo_direct = [&](int k) {
    const size_t pb = (size_t)wrap_small(k, a.nz) * plane;
#pragma unroll 1
    for (int i = 0; i < HPW; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
        const size_t g = (pb + (size_t)hbase[s]) * NC;
        for (int l = lane; l < NC; l += 64)
          xs[s * NC + l] = FUSE ? (T)(xg[g + l] + beta * pg[g + l]) : xg[g + l];
      }
    }
  };
  if constexpr (PREF) halo_load(k0);

  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) xs[c * NC + l3 * NP + lp] = zc[l3];
    if constexpr (PREF) halo_store();
    else halo_direct(k);
    __syncthreads();
    // plane k+1: own z-line and (prefetch) halo, in flight during the x/y phases
    const size_t bn = zbase(k + 1);
    T pn[n];
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zn[l3] = xg[bn + l3 * NP];
      if (FUSE) pn[l3] = pg[bn + l3 * NP];
    }
    if constexpr (PREF) {
      if (k + 1 < k1) halo_load(k + 1);
    }
    {  // x-line (l2, l3) of cell c
      T vl[n], vc[n], vr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vl[m] = xs[sxl * NC + xl23 * n + m];
        vc[m] = xs[c * NC + xl23 * n + m];
        vr[m] = xs[sxr * NC + xl23 * n + m];
      }
      line3<T, N>(B, vl, vc, vr, [&](int l1, T v) { ys[c * NC + xl23 * n + l1] = wx * v; });
    }
    __syncthreads();
    {  // y-line (l1, l3) of cell c
      T vl[n], vc[n], vr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vl[m] = xs[syl * NC + yl3 * NP + m * n + yl1];
        vc[m] = xs[c * NC + yl3 * NP + m * n + yl1];
        vr[m] = xs[syr * NC + yl3 * NP + m * n + yl1];
      }
      line3<T, N>(B, vl, vc, vr,
                  [&](int l2, T v) { ys[c * NC + yl3 * NP + l2 * n + yl1] += wy * v; });
    }
    __syncthreads();
    if (FUSE) {
      const bool own_next = valid && (k + 1 < k1);
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zn[l3] = zn[l3] + beta * pn[l3];
        if (own_next) png[bn + l3 * NP] = zn[l3];
      }
    }
    {  // own z-line (l1, l2) from registers; final values
      const size_t bc = zbase(k);
      T* __restrict__ yg = a.y;
      line3<T, N>(B, zp, zc, zn, [&](int l3, T v) {
        const T xc = xs[c * NC + l3 * NP + lp];
        const T val = ys[c * NC + l3 * NP + lp] + wz * v + wm * B.w[l3] * xc;
        if (valid) {
          yg[bc + l3 * NP] = val;
          dot += (double)xc * (double)val;
        }
      });
    }
    __syncthreads();
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zp[l3] = zc[l3];
      zc[l3] = zn[l3];
    }
  }
  if (FUSE) {
    const double s = block_sum_all<NTH>(dot);
    if (threadIdx.x == 0) a.sigpart[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ launchers

template <typename T, int N>
static Blk<T, N> make_blk(const OpTables& tb) {
  Blk<T, N> B;
  constexpr int n = N + 1;
  for (int i = 0; i < n * n; ++i) {
    B.L[i] = (T)tb.L[i];
    B.C[i] = (T)tb.C[i];
    B.R[i] = (T)tb.R[i];
  }
  for (int i = 0; i < n; ++i) B.w[i] = (T)tb.w[i];
  return B;
}

// Grid geometry of one launch: tiles per direction, planes per 3D column segment, blocks.
struct Geom {
  int ntx, nty, ntz, kz;
  unsigned long long blocks;
};

template <typename T, int N>
static Geom geometry(const ApplyLaunch& L) {
  Geom g;
  const int nx = L.nc[0], ny = L.nc[1], nz = L.dim == 3 ? L.nc[2] : 1;
  if (L.dim == 2) {
    using TL = Tile2D<T, N>;
    g.ntx = (nx + TL::TX - 1) / TL::TX;
    g.nty = (ny + TL::TY - 1) / TL::TY;
    // persistent workgroups: about 4 per CU on 256 CUs, each over kz consecutive tiles
    const long long ntiles = (long long)g.ntx * g.nty;
    long long per = 1;   // one tile per workgroup measured best on 256^2 N=6 (2D grids are small)
    if (L.tiles_per_wg > 0) per = L.tiles_per_wg;
    g.kz = (int)per;
    g.ntz = 1;
    g.blocks = (unsigned long long)((ntiles + per - 1) / per);
    return g;
  } else {
    using TL = Tile3D<N>;
    g.ntx = (nx + TL::TX - 1) / TL::TX;
    g.nty = (ny + TL::TY - 1) / TL::TY;
    const long long cols = (long long)g.ntx * g.nty;
    // planes per segment: about 1024 workgroups, segments of at least 4 planes (64^3 N=4: 16)
    int kz = (int)((cols * nz) / 1024);
    if (kz < 4) kz = 4;
    if (kz > nz) kz = nz;
    if (L.kz_override > 0) kz = L.kz_override < nz ? L.kz_override : nz;
    g.kz = kz;
    g.ntz = (nz + kz - 1) / kz;
  }
  g.blocks = (unsigned long long)g.ntx * g.nty * g.ntz;
  return g;
}

template <typename T, int N>
static hipError_t launch_apply_N(const ApplyLaunch& L, hipStream_t s) {
  ApplyArgs<T> a;
  a.x = (const T*)L.x;
  a.pold = (const T*)L.pold;
  a.pnew = (T*)L.pnew;
  a.y = (T*)L.y;
  a.nx = L.nc[0];
  a.ny = L.nc[1];
  a.nz = L.dim == 3 ? L.nc[2] : 1;
  a.alpha = (T)L.alpha;
  a.c0 = (T)L.coef[0];
  a.c1 = (T)L.coef[1];
  a.c2 = (T)L.coef[2];
  a.st = L.st;
  a.k = L.k;
  a.rho_cur = L.rho_cur;
  a.nrho = L.nrho;
  a.sigpart = L.sigpart;
  const Blk<T, N> B = make_blk<T, N>(*L.tab);
  const Geom g = geometry<T, N>(L);
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.ntz = g.ntz;
  a.kz = g.kz;
  if (g.blocks > (unsigned long long)kMaxPartials) return hipErrorInvalidValue;
  const unsigned G = (unsigned)g.blocks;
  const bool pf = L.prefetch != 0;
  if (L.dim == 2) {
    if (L.fuse) {
      if (pf) hipLaunchKernelGGL((k_apply2d<T, N, 1, 1>), dim3(G), dim3(256), 0, s, a, B);
      else hipLaunchKernelGGL((k_apply2d<T, N, 1, 0>), dim3(G), dim3(256), 0, s, a, B);
    } else {
      hipLaunchKernelGGL((k_apply2d<T, N, 0, 0>), dim3(G), dim3(256), 0, s, a, B);
    }
  } else {
    constexpr int NTH = Tile3D<N>::NTH;
    if (L.fuse) {
      if (pf) hipLaunchKernelGGL((k_apply3d<T, N, 1, 1>), dim3(G), dim3(NTH), 0, s, a, B);
      else hipLaunchKernelGGL((k_apply3d<T, N, 1, 0>), dim3(G), dim3(NTH), 0, s, a, B);
    } else {
      hipLaunchKernelGGL((k_apply3d<T, N, 0, 0>), dim3(G), dim3(NTH), 0, s, a, B);
    }
  }
  return hipGetLastError();
}

template <typename T, int N>
static unsigned blocks_N(const ApplyLaunch& L) {
  return (unsigned)geometry<T, N>(L).blocks;
}

template <typename T>
static hipError_t launch_apply_T(const ApplyLaunch& L, hipStream_t s) {
  switch (L.N) {
    case 0: return launch_apply_N<T, 0>(L, s);
    case 1: return launch_apply_N<T, 1>(L, s);
    case 2: return launch_apply_N<T, 2>(L, s);
    case 3: return launch_apply_N<T, 3>(L, s);
    case 4: return launch_apply_N<T, 4>(L, s);
    case 5: return launch_apply_N<T, 5>(L, s);
    case 6: return launch_apply_N<T, 6>(L, s);
    case 7: return launch_apply_N<T, 7>(L, s);
    case 8: return launch_apply_N<T, 8>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply(const ApplyLaunch& L, hipStream_t s) {
  return L.fp32 ? launch_apply_T<float>(L, s) : launch_apply_T<double>(L, s);
}

template <typename T>
static unsigned apply_blocks_T(const ApplyLaunch& L) {
  switch (L.N) {
    case 0: return blocks_N<T, 0>(L);
    case 1: return blocks_N<T, 1>(L);
    case 2: return blocks_N<T, 2>(L);
    case 3: return blocks_N<T, 3>(L);
    case 4: return blocks_N<T, 4>(L);
    case 5: return blocks_N<T, 5>(L);
    case 6: return blocks_N<T, 6>(L);
    case 7: return blocks_N<T, 7>(L);
    case 8: return blocks_N<T, 8>(L);
    default: return 0;
  }
}

unsigned apply_blocks(const ApplyLaunch& L) {
  return L.fp32 ? apply_blocks_T<float>(L) : apply_blocks_T<double>(L);
}

}  // namespace pdk
