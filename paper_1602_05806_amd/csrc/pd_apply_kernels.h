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
//       LDS with the plane's x/y face halos. A coalesced form (k_apply3d_co) moves each plane's
//       values in memory order and reads the z-lines back from LDS; it is used where it measured
//       faster (Co3D).
// FUSE = 1 is the CG form: the search direction p = r + beta p_old is formed while loading
// (beta read from the device-resident CG state), stored for the owned cells, and the block sums of
// <p, A p> feed the grid reduction that sets alpha = rho / <p, A p>. FUSE = 2 adds the deferred x
// update of the previous iteration, x += alpha_{k-1} p_old, on the owned cells (p_old is loaded
// anyway). FUSE = 3 (2D) also makes the residual update of the previous iteration while loading,
// r_k = r_{k-1} - alpha_{k-1} q_{k-1}, so that one kernel is one CG iteration: 8 vector words
// per DoF (r, q, p, x read; r, q, p, x written) against 6 + 3 for FUSE = 2 and the update
// kernel, and one kernel boundary fewer. The scalars come from the expansion of |r_k|^2 with
// the inner products <r, A p> and <A p, A p> of the previous launch (fused_scalars).
//
// The kernels and their launchers are instantiated per (precision, degree) in pd_apply_inst.hip
// (one object per pair, compiled in parallel); pd_apply.hip dispatches to them.
#pragma once
#include <hip/hip_ext.h>

#include <algorithm>

#include "pd_apply2d.h"
#include "pd_device.h"
#include "pd_launch.h"

namespace pdk {

// Single problem: persistent workgroups; workgroup lw takes tiles lw, lw + G, lw + 2G, ... (G
// workgroups), so that at every step the workgroups of one XCD (lw is the XCD-contiguous index)
// hold a contiguous band of tiles whose halos they share in that XCD's L2, and the band of the
// next step is prefetched during the current one. 256^2 N = 6 FP64, 3 tiles per workgroup:
// 40.9 us per launch against 44.2 us with each workgroup taking 3 consecutive tiles; N = 8:
// 63.3 against 66.1 us. For a launch of one tile per workgroup that the device holds at once
// (a.remap = 0) lw is the dispatch order itself, which deals neighbouring tiles to different
// XCDs: 256^2 N = 6 FP32 28.6 against 30.3 us, 256^2 N = 3 FP64 16.7 against 17.5 us (with
// several tiles per workgroup or several waves the XCD-contiguous index is as fast or faster).
// MIR: Dirichlet walls (a grid with walls runs tile variant 0 with prefetch).
template <typename T, int N, int V, int FUSE, int PF, bool MIR = false>
__global__ __launch_bounds__(256) void k_apply2d(ApplyArgs<T> a, Blk<T, N> B) {
  const unsigned lw = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int ntiles = a.ntx * a.nty;
  apply2d_body<T, N, V, FUSE, PF, MIR>(a, B, (int)lw, ntiles, (int)gridDim.x, blockIdx.x);
}

// ------------------------------------------------------------------ 3D z-marching kernel

template <int N>
struct Tile3D {
  // cells per column tile; N = 5 takes 4 x 4 (557 against 908 us per FP64 apply at 54^3 with
  // 4 x 2), N = 6..8 keep 2 x 2 (4 x 2 at N = 6: 847 against 694 us at 46^3)
  static constexpr int TX = N == 0 ? 16 : N == 1 ? 8 : N == 2 ? 8 : N <= 5 ? 4 : 2;
  static constexpr int TY = N == 0 ? 16 : N == 1 ? 8 : N == 2 ? 4 : N <= 5 ? 4 : 2;
  static constexpr int NTH = TX * TY * (N + 1) * (N + 1);
};

// MIR: the grid has Dirichlet walls (a.mir); the periodic kernel carries none of their code.
template <typename T, int N, int FUSE, int PF, bool MIR>
__global__ __launch_bounds__(Tile3D<N>::NTH) void k_apply3d(ApplyArgs<T> a, Blk<T, N> B) {
  constexpr int n = N + 1, NP = n * n, NC = n * n * n;
  constexpr int TX = Tile3D<N>::TX, TY = Tile3D<N>::TY, NT = TX * TY, NTH = Tile3D<N>::NTH;
  constexpr int S_XL = NT, S_XR = NT + TY, S_YL = NT + 2 * TY, S_YR = NT + 2 * TY + TX;
  constexpr int NS = NT + 2 * TY + 2 * TX;
  constexpr int NH = NS - NT;
  // the staging buffer alternates between planes when two fit in the 160 KB of LDS, which
  // removes the barrier at the end of each plane (1.7 % at 64^3 N = 4, 2.7 % at 96^3 N = 2,
  // 3 % at 54^3 N = 5); not for N >= 6, where the second buffer costs resident workgroups
  // (46^3 N = 6: 931 against 694 us per FP64 apply, 40^3 N = 7: 1024 against 637 us)
  constexpr bool DB = N <= 5 && (2 * NS * NC + NT * NC) * sizeof(T) + 2 * NS * sizeof(int) <= 160 * 1024;
  __shared__ T xsb[DB ? 2 : 1][NS * NC];
  __shared__ T ys[NT * NC];
  __shared__ int hbase[NS];     // in-plane cell index (j*nx + i, wrapped) of every halo slot
  __shared__ int hmir[NS];      // bit 0 / 1: the slot is the odd reflection across an x / y wall
  // launches queued after the run stopped exit before loading anything
  const int kit = FUSE ? (a.kbase ? *a.kbase + a.k : a.k) : 0;
  if (FUSE) {
    if (!apply_may_run(a.st, kit)) return;
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
    int ri = tx0 + hi, rj = ty0 + hj, m = 0;
    if (MIR && a.mir[0] && (ri < 0 || ri >= a.nx)) {
      ri = mirror_index(ri, a.nx);
      m |= 1;
    }
    if (MIR && a.mir[1] && (rj < 0 || rj >= a.ny)) {
      rj = mirror_index(rj, a.ny);
      m |= 2;
    }
    hbase[s] = wrapi(rj, a.ny) * a.nx + wrapi(ri, a.nx);
    if constexpr (MIR) hmir[s] = m;
  }
  __syncthreads();   // hbase ready

  const int t = threadIdx.x;
  const int c = t / NP, lp = t - c * NP;          // cell in the plane tile, z-line (l1 + n l2)
  const int ci = c % TX, cj = c / TX;
  const int ui = tx0 + ci, uj = ty0 + cj;
  const bool valid = ui < a.nx && uj < a.ny;
  // a ragged tile's cells beyond a Dirichlet wall hold the odd reflection of the cells inside
  // (they are the x / y neighbours of the last valid cells); their z-lines read the mirrored
  // source line with the sign flipped
  int si = ui, sj = uj, slp = lp;
  T sgn = T(1);
  if (MIR && a.mir[0] && ui >= a.nx) {
    si = mirror_index(ui, a.nx);
    slp = (slp / n) * n + (n - 1 - slp % n);
    sgn = -sgn;
  }
  if (MIR && a.mir[1] && uj >= a.ny) {
    sj = mirror_index(uj, a.ny);
    slp = (n - 1 - slp / n) * n + slp % n;
    sgn = -sgn;
  }
  const int gi = wrapi(si, a.nx), gj = wrapi(sj, a.ny);
  const size_t plane = (size_t)a.nx * a.ny;
  T beta = T(0);
  bool xupd = false;   // FUSE = 2: x += xalpha p_old on the owned z-line
  T xalpha = T(0);

  auto zbase = [&](int k) -> size_t {
    return (((size_t)wrap_small(k, a.nz) * a.ny + gj) * a.nx + gi) * NC + slp;
  };

  T zp[n], zc[n], zn[n];
  {
    // first two planes of this thread's z-line; the CG scalars are reduced while they load
    const size_t bp = zbase(k0 - 1), bc = zbase(k0);
    T pp[n], pc[n], xc[FUSE == 2 ? n : 1];
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zp[l3] = sgn * xg[bp + l3 * NP];
      zc[l3] = sgn * xg[bc + l3 * NP];
      if (FUSE) {
        pp[l3] = sgn * pg[bp + l3 * NP];
        pc[l3] = sgn * pg[bc + l3 * NP];
      }
      if (FUSE == 2) xc[l3] = a.xsol[bc + l3 * NP];
    }
    if (FUSE) {
      const int k = kit;
      const IterScalars sc = iteration_scalars<NTH>(a.st, k, a.rho_cur, a.nrho, blockIdx.x == 0,
                                                    false, a.res_cur);
      if (sc.stop) return;
      beta = (T)sc.beta;
      if (FUSE == 2) {
        xupd = k >= 1 && a.st->xk == k - 1;
        xalpha = (T)a.st->alpha;
        if (xupd && blockIdx.x == 0 && threadIdx.x == 0) a.st->xused = k - 1;
      }
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zp[l3] = zp[l3] + beta * pp[l3];
        zc[l3] = zc[l3] + beta * pc[l3];
        if (valid) {
          png[bc + l3 * NP] = zc[l3];
          if (FUSE == 2 && xupd) a.xsol[bc + l3 * NP] = xc[l3] + xalpha * pc[l3];
        }
      }
    }
    // the plane below a Dirichlet wall at z = 0: odd reflection of plane 0 (stores are valid
    // cells' own planes only, so valid stores are unaffected)
    if (MIR && a.mir[2] && k0 == 0) {
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) zp[l3] = -zc[n - 1 - l3];
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
  T* xs = xsb[0];   // staging buffer of the current plane (alternates when double-buffered)
  const int lane = t & 63;
  T hv[HR][LR], hp[HR][LR];
  // source element of halo element l of slot s (odd reflection across x / y walls)
  auto hsrc = [&](int s, int l, T& sg) -> int {
    sg = T(1);
    if constexpr (!MIR) return l;
    const int m = hmir[s];
    if (m & 1) {
      l = l - l % n + (n - 1 - l % n);
      sg = -sg;
    }
    if (m & 2) {
      const int l2 = (l / n) % n;
      l = l + (n - 1 - 2 * l2) * n;
      sg = -sg;
    }
    return l;
  };
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
            // (raw values: a wall's sign is applied when they are staged, so that nothing
            // here waits for the loads)
            T sg;
            const int ls = hsrc(s, l, sg);
            hv[i][r] = xg[g + ls];
            if (FUSE) hp[i][r] = pg[g + ls];
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
          if (l < NC) {
            T sg;
            hsrc(s, l, sg);
            xs[s * NC + l] = sg * (FUSE ? (T)(hv[i][r] + beta * hp[i][r]) : hv[i][r]);
          }
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
        for (int l = lane; l < NC; l += 64) {
          T sg;
          const int ls = hsrc(s, l, sg);
          xs[s * NC + l] = sg * (FUSE ? (T)(xg[g + ls] + beta * pg[g + ls]) : xg[g + ls]);
        }
      }
    }
  };
  if constexpr (PREF) halo_load(k0);

  for (int k = k0; k < k1; ++k) {
    xs = xsb[DB ? ((k - k0) & 1) : 0];
    // plane k+1: own z-line loads first (in flight through this plane's staging barrier and
    // the x/y phases: 5 % faster at 64^3 N = 4 than issuing them after the barrier), then the
    // (prefetch) halo
    const size_t bn = zbase(k + 1);
    const bool own_next = valid && (k + 1 < k1);
    T pn[n], xn[FUSE == 2 ? n : 1];
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zn[l3] = xg[bn + l3 * NP];   // (a wall's sign is applied after the y-lines)
      if (FUSE) pn[l3] = pg[bn + l3 * NP];
      if (FUSE == 2 && xupd && own_next) xn[l3] = a.xsol[bn + l3 * NP];
    }
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) xs[c * NC + l3 * NP + lp] = zc[l3];
    if constexpr (PREF) halo_store();
    else halo_direct(k);
    __syncthreads();
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
      line3<T, N, 3>(B, vl, vc, vr, [&](int l1, T v) { ys[c * NC + xl23 * n + l1] = wx * v; });
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
      line3<T, N, 3>(B, vl, vc, vr,
                  [&](int l2, T v) { ys[c * NC + yl3 * NP + l2 * n + yl1] += wy * v; });
    }
    __syncthreads();
    if (FUSE) {
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zn[l3] = sgn * (zn[l3] + beta * pn[l3]);   // (sgn = 1 for the owned cells)
        if (own_next) {
          png[bn + l3 * NP] = zn[l3];
          if (FUSE == 2 && xupd) a.xsol[bn + l3 * NP] = xn[l3] + xalpha * pn[l3];
        }
      }
    }
    if (!FUSE) {
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) zn[l3] = sgn * zn[l3];
    }
    // the plane above a Dirichlet wall at z = L: odd reflection of the last plane
    if (MIR && a.mir[2] && k + 1 == a.nz) {
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) zn[l3] = -zc[n - 1 - l3];
    }
    {  // own z-line (l1, l2) from registers; final values
      const size_t bc = zbase(k);
      T* __restrict__ yg = a.y;
      line3<T, N, 3>(B, zp, zc, zn, [&](int l3, T v) {
        const T xc = xs[c * NC + l3 * NP + lp];
        const T val = ys[c * NC + l3 * NP + lp] + wz * v + wm * B.w[l3] * xc;
        if (valid) {
          yg[bc + l3 * NP] = val;
          dot += (double)xc * (double)val;
        }
      });
    }
    if constexpr (!DB) __syncthreads();
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

// Coalesced form of the 3D kernel (N <= 5). The tile's cells of one plane lie in
// global memory as TY rows of TX * (N+1)^3 consecutive values, in the same order as the staging
// buffer: thread t moves values t, t + NTH, ..., so every wave's load or store covers 64
// consecutive values (the z-line form above touches (N+1)^2-value pieces of several cells per
// instruction). The z-line of each thread is then read back from the staging buffer. Both the
// staging buffer and (when LDS allows) the accumulator alternate between planes: two barriers
// per plane, and the accumulator of plane k is stored to y, coalesced, during plane k + 1.
template <typename T, int N>
struct Co3D {
  static constexpr int n = N + 1, NC = n * n * n;
  static constexpr int NT = Tile3D<N>::TX * Tile3D<N>::TY;
  static constexpr int NS = NT + 2 * Tile3D<N>::TY + 2 * Tile3D<N>::TX;
  static constexpr long XS = 2L * NS * NC * (long)sizeof(T), YS = (long)NT * NC * (long)sizeof(T);
  static constexpr bool OK = N <= 5 && XS + YS + NS * 4L <= 160L * 1024;
  static constexpr bool YDB = XS + 2 * YS + NS * 4L <= 160L * 1024;
  // where it is used (per-launch means of the fused CG apply, ~33M DoFs, against the z-line
  // form, both with the row form of the line operator): FP32 N = 1..4 (128^3 N = 1: 91.5
  // against 108.8 us; 96^3 N = 2: 174 / 216; 80^3 N = 3: 169 / 194; 64^3 N = 4: 196 / 210) and
  // FP64 N = 1 (208.5 / 219). FP64 N = 2..5 and FP32 N = 5 stay on the z-line form (64^3 N = 4
  // FP64: 385 against 378 us, with the even/odd line form 358.8 against 357.3; 54^3 N = 5 FP32:
  // 267 / 249, the coalesced form needs 129 registers there), and so does N = 0 (one value
  // per cell: nothing to coalesce).
  static constexpr bool USE = OK && (sizeof(T) == 4 ? (N >= 1 && N <= 4) : N == 1);
};

// MIR: Dirichlet walls, as in the z-line form (the periodic kernel carries none of their code).
template <typename T, int N, int FUSE, int PF, bool MIR = false>
__global__ __launch_bounds__(Tile3D<N>::NTH) void k_apply3d_co(ApplyArgs<T> a, Blk<T, N> B) {
  constexpr int n = N + 1, NP = n * n, NC = n * n * n;
  constexpr int TX = Tile3D<N>::TX, TY = Tile3D<N>::TY, NT = TX * TY, NTH = Tile3D<N>::NTH;
  constexpr int S_XL = NT, S_XR = NT + TY, S_YL = NT + 2 * TY, S_YR = NT + 2 * TY + TX;
  constexpr int NS = NT + 2 * TY + 2 * TX;
  constexpr int NH = NS - NT;
  constexpr bool YDB = Co3D<T, N>::YDB;
  static_assert(Co3D<T, N>::OK, "coalesced 3D form needs two staging buffers");
  static_assert(NTH * n == NT * NC, "n values per thread cover the tile's plane");
  __shared__ T xsb[2][NS * NC];
  __shared__ T ysb[YDB ? 2 : 1][NT * NC];
  __shared__ int hbase[NS];
  __shared__ int hmir[MIR ? NS : 1];   // bit 0 / 1: the slot is the odd reflection across an x / y wall
  const int kit = FUSE ? (a.kbase ? *a.kbase + a.k : a.k) : 0;
  if (FUSE) {
    if (!apply_may_run(a.st, kit)) return;
  }
  const T* __restrict__ xg = a.x;
  const T* __restrict__ pg = a.pold;
  T* __restrict__ png = a.pnew;
  T* __restrict__ yg = a.y;
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
    int ri = tx0 + hi, rj = ty0 + hj, m = 0;
    if (MIR && a.mir[0] && (ri < 0 || ri >= a.nx)) {
      ri = mirror_index(ri, a.nx);
      m |= 1;
    }
    if (MIR && a.mir[1] && (rj < 0 || rj >= a.ny)) {
      rj = mirror_index(rj, a.ny);
      m |= 2;
    }
    hbase[s] = wrapi(rj, a.ny) * a.nx + wrapi(ri, a.nx);
    if constexpr (MIR) hmir[s] = m;
  }

  const int t = threadIdx.x;
  const int c = t / NP, lp = t - c * NP;          // z-line of this thread: cell c, (l1, l2) = lp
  const int ci = c % TX, cj = c / TX;
  const int ui = tx0 + ci, uj = ty0 + cj;
  const bool valid = ui < a.nx && uj < a.ny;
  // a ragged tile's cells beyond a Dirichlet wall hold the odd reflection of the cells inside:
  // the z-line of such a cell reads the mirrored source line with the sign flipped
  int si = ui, sj = uj, slp = lp;
  T sgn = T(1);
  if (MIR && a.mir[0] && ui >= a.nx) {
    si = mirror_index(ui, a.nx);
    slp = (slp / n) * n + (n - 1 - slp % n);
    sgn = -sgn;
  }
  if (MIR && a.mir[1] && uj >= a.ny) {
    sj = mirror_index(uj, a.ny);
    slp = (n - 1 - slp / n) * n + slp % n;
    sgn = -sgn;
  }
  const int gi = wrapi(si, a.nx), gj = wrapi(sj, a.ny);
  const size_t plane = (size_t)a.nx * a.ny * NC;  // values per plane
  // values t + NTH i of the tile's plane: in-plane offset and whether the cell is in the grid
  // (a ragged tile's cells beyond the edge hold the periodic images, or beyond a wall the odd
  // reflections (bit i of neg), read but never stored)
  int off[n];
  unsigned own = 0, neg = 0;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const int e = t + NTH * i;
    const int rj = e / (TX * NC), o = e - rj * (TX * NC);
    const int rc = o / NC;
    int q = o - rc * NC, ri = tx0 + rc, rjj = ty0 + rj;
    if (ri < a.nx && rjj < a.ny) own |= 1u << i;
    if (MIR && a.mir[0] && ri >= a.nx) {
      ri = mirror_index(ri, a.nx);
      q = q - q % n + (n - 1 - q % n);
      neg ^= 1u << i;
    }
    if (MIR && a.mir[1] && rjj >= a.ny) {
      rjj = mirror_index(rjj, a.ny);
      q = q + (n - 1 - 2 * ((q / n) % n)) * n;
      neg ^= 1u << i;
    }
    off[i] = (wrapi(rjj, a.ny) * a.nx + wrapi(ri, a.nx)) * NC + q;
  }
  __syncthreads();   // hbase ready

  T beta = T(0);
  bool xupd = false;   // FUSE = 2: x += xalpha p_old on the owned values
  T xalpha = T(0);
  T zp[n], zc[n];
  {
    // planes k0 - 1 and k0 of this thread's z-line; the CG scalars are reduced while they load
    const size_t bp = (size_t)wrap_small(k0 - 1, a.nz) * plane + ((size_t)gj * a.nx + gi) * NC + slp;
    const size_t bc = (size_t)k0 * plane + ((size_t)gj * a.nx + gi) * NC + slp;
    T pp[n], pc[n], xc[FUSE == 2 ? n : 1];
#pragma unroll
    for (int l3 = 0; l3 < n; ++l3) {
      zp[l3] = sgn * xg[bp + l3 * NP];
      zc[l3] = sgn * xg[bc + l3 * NP];
      if (FUSE) {
        pp[l3] = sgn * pg[bp + l3 * NP];
        pc[l3] = sgn * pg[bc + l3 * NP];
      }
      if (FUSE == 2) xc[l3] = a.xsol[bc + l3 * NP];
    }
    if (FUSE) {
      const int k = kit;
      const IterScalars sc = iteration_scalars<NTH>(a.st, k, a.rho_cur, a.nrho, blockIdx.x == 0,
                                                    false, a.res_cur);
      if (sc.stop) return;
      beta = (T)sc.beta;
      if (FUSE == 2) {
        xupd = k >= 1 && a.st->xk == k - 1;
        xalpha = (T)a.st->alpha;
        if (xupd && blockIdx.x == 0 && threadIdx.x == 0) a.st->xused = k - 1;
      }
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zp[l3] = zp[l3] + beta * pp[l3];
        zc[l3] = zc[l3] + beta * pc[l3];
        if (valid) {
          png[bc + l3 * NP] = zc[l3];
          if (FUSE == 2 && xupd) a.xsol[bc + l3 * NP] = xc[l3] + xalpha * pc[l3];
        }
      }
    }
    // the plane below a Dirichlet wall at z = 0: odd reflection of plane 0
    if (MIR && a.mir[2] && k0 == 0) {
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) zp[l3] = -zc[n - 1 - l3];
    }
  }
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

  // x/y halo cells of a plane: one wave per cell (wave-uniform addressing)
  constexpr int NWV = NTH / 64;
  static_assert(NWV >= 1, "3D tile needs at least one full wave");
  constexpr int HPW = (NH + NWV - 1) / NWV;
  constexpr int LR = (NC + 63) / 64;
  constexpr bool PREF = PF && HPW * LR <= 8;
  constexpr int HR = PREF ? HPW : 1;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = t & 63;
  T hv[HR][LR], hp[HR][LR];
  // source element of halo element l of slot s (odd reflection across x / y walls)
  auto hsrc = [&](int s, int l, T& sg) -> int {
    sg = T(1);
    if constexpr (!MIR) return l;
    const int m = hmir[s];
    if (m & 1) {
      l = l - l % n + (n - 1 - l % n);
      sg = -sg;
    }
    if (m & 2) {
      l = l + (n - 1 - 2 * ((l / n) % n)) * n;
      sg = -sg;
    }
    return l;
  };
  auto halo_load = [&](int k) {
    const size_t pb = (size_t)wrap_small(k, a.nz) * plane;
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
        const size_t g = pb + (size_t)hbase[s] * NC;
#pragma unroll
        for (int r = 0; r < LR; ++r) {
          const int l = lane + 64 * r;
          if (l < NC) {
            // (raw values: a wall's sign is applied when they are staged)
            T sg;
            const int ls = hsrc(s, l, sg);
            hv[i][r] = xg[g + ls];
            if (FUSE) hp[i][r] = pg[g + ls];
          }
        }
      }
    }
  };
  auto halo_store = [&](T* xs) {
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
#pragma unroll
        for (int r = 0; r < LR; ++r) {
          const int l = lane + 64 * r;
          if (l < NC) {
            T sg;
            hsrc(s, l, sg);
            xs[s * NC + l] = sg * (FUSE ? (T)(hv[i][r] + beta * hp[i][r]) : hv[i][r]);
          }
        }
      }
    }
  };
  auto halo_direct = [&](T* xs, int k) {
    const size_t pb = (size_t)wrap_small(k, a.nz) * plane;
#pragma unroll 1
    for (int i = 0; i < HPW; ++i) {
      const int s = NT + wave + NWV * i;
      if (wave < NWV && s < NS) {
        const size_t g = pb + (size_t)hbase[s] * NC;
        for (int l = lane; l < NC; l += 64) {
          T sg;
          const int ls = hsrc(s, l, sg);
          xs[s * NC + l] = sg * (FUSE ? (T)(xg[g + ls] + beta * pg[g + ls]) : xg[g + ls]);
        }
      }
    }
  };
  // plane k0 into staging buffer 0
#pragma unroll
  for (int l3 = 0; l3 < n; ++l3) xsb[0][c * NC + l3 * NP + lp] = zc[l3];
  halo_direct(xsb[0], k0);
  __syncthreads();

  for (int k = k0; k < k1; ++k) {
    const int cur = (k - k0) & 1;
    T* xs = xsb[cur];
    T* xnx = xsb[cur ^ 1];
    T* ys = ysb[YDB ? cur : 0];
    const bool store_next = k + 1 < k1;
    const size_t pbn = (size_t)wrap_small(k + 1, a.nz) * plane;
    // plane k+1: own values (coalesced) and halo, in flight through the x/y phases
    T xo[n], po[n], xso[FUSE == 2 ? n : 1];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      xo[i] = xg[pbn + off[i]];
      if (FUSE) po[i] = pg[pbn + off[i]];
      if (FUSE == 2 && xupd && store_next && ((own >> i) & 1)) xso[i] = a.xsol[pbn + off[i]];
    }
    if constexpr (PREF) {
      if (store_next) halo_load(k + 1);
    }
    {  // x-line (l2, l3) of cell c
      T vl[n], vc[n], vr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vl[m] = xs[sxl * NC + xl23 * n + m];
        vc[m] = xs[c * NC + xl23 * n + m];
        vr[m] = xs[sxr * NC + xl23 * n + m];
      }
      line3<T, N, 3>(B, vl, vc, vr, [&](int l1, T v) { ys[c * NC + xl23 * n + l1] = wx * v; });
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
      line3<T, N, 3>(B, vl, vc, vr,
                  [&](int l2, T v) { ys[c * NC + yl3 * NP + l2 * n + yl1] += wy * v; });
    }
    // plane k+1 into the other staging buffer; p and x of its owned values to global memory
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const T v = FUSE ? (T)(xo[i] + beta * po[i]) : xo[i];
      // (owned values are never reflected: the values stored below carry no sign)
      xnx[t + NTH * i] = MIR && ((neg >> i) & 1) ? -v : v;
      if (FUSE && store_next && ((own >> i) & 1)) {
        png[pbn + off[i]] = v;
        if (FUSE == 2 && xupd) a.xsol[pbn + off[i]] = xso[i] + xalpha * po[i];
      }
    }
    if (store_next) {   // (the last plane's neighbour above is needed for its z-lines only)
      if constexpr (PREF) halo_store(xnx);
      else halo_direct(xnx, k + 1);
    }
    if constexpr (YDB) {
      // y of plane k - 1 (its accumulator, completed before this plane's first barrier)
      if (k > k0) {
        const T* yp = ysb[cur ^ 1];
        const size_t pbp = (size_t)(k - 1) * plane;
#pragma unroll
        for (int i = 0; i < n; ++i)
          if ((own >> i) & 1) yg[pbp + off[i]] = yp[t + NTH * i];
      }
    }
    __syncthreads();
    {  // own z-line (l1, l2): planes k-1, k from registers, k+1 from staging; final values
      T zn[n];
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) zn[l3] = xnx[c * NC + l3 * NP + lp];
      // the plane above a Dirichlet wall at z = L: odd reflection of the last plane
      if (MIR && a.mir[2] && k + 1 == a.nz) {
#pragma unroll
        for (int l3 = 0; l3 < n; ++l3) zn[l3] = -zc[n - 1 - l3];
      }
      const size_t bc = (size_t)k * plane + ((size_t)gj * a.nx + gi) * NC + lp;
      line3<T, N, 3>(B, zp, zc, zn, [&](int l3, T v) {
        const T xc = xs[c * NC + l3 * NP + lp];
        const T val = ys[c * NC + l3 * NP + lp] + wz * v + wm * B.w[l3] * xc;
        if constexpr (YDB) ys[c * NC + l3 * NP + lp] = val;
        if (valid) {
          if constexpr (!YDB) yg[bc + l3 * NP] = val;
          dot += (double)xc * (double)val;
        }
      });
#pragma unroll
      for (int l3 = 0; l3 < n; ++l3) {
        zp[l3] = zc[l3];
        zc[l3] = zn[l3];
      }
    }
    if constexpr (!YDB) __syncthreads();   // the accumulator is rewritten by the next x-lines
  }
  if constexpr (YDB) {
    __syncthreads();
    const T* yp = ysb[(k1 - 1 - k0) & 1];
    const size_t pbp = (size_t)(k1 - 1) * plane;
#pragma unroll
    for (int i = 0; i < n; ++i)
      if ((own >> i) & 1) yg[pbp + off[i]] = yp[t + NTH * i];
  }
  if (FUSE) {
    const double s = block_sum_all<NTH>(dot);
    if (threadIdx.x == 0) a.sigpart[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ launchers

template <typename T, int N>
static Blk<T, N> make_blk(const OpTables& tb, int dim) {
  Blk<T, N> B;
  B.fill(tb, dim == 3 ? line_eo<T, N, 3>() : line_eo<T, N, 2>());
  return B;
}

// Grid geometry of one launch: tiles per direction, planes per 3D column segment, blocks.
struct Geom {
  int ntx, nty, ntz, kz;
  unsigned long long blocks;
  int remap = 1;   // 2D: XCD-contiguous tile ranges (see k_apply2d)
};

// Workgroups of the fused 2D kernel (tile variant v, prefetch pf) the device holds at once:
// occupancy per CU (registers, LDS) times CUs, queried once per device and shape.
template <typename T, int N, int F>
static const void* kernel_2d(int v, int pf) {
  return pf ? (v == 1 ? (const void*)k_apply2d<T, N, 1, F, 1>
                      : v == 2 ? (const void*)k_apply2d<T, N, 2, F, 1>
                               : (const void*)k_apply2d<T, N, 0, F, 1>)
            : (v == 1 ? (const void*)k_apply2d<T, N, 1, F, 0>
                      : v == 2 ? (const void*)k_apply2d<T, N, 2, F, 0>
                               : (const void*)k_apply2d<T, N, 0, F, 0>);
}

// The 2D kernel of fused form `fuse` for a grid with walls (tile variant 0, prefetch on).
template <typename T, int N>
static const void* kernel_2d_walls(int fuse) {
  switch (fuse) {
    case 3: return (const void*)k_apply2d<T, N, 0, 3, 1, true>;
    case 2: return (const void*)k_apply2d<T, N, 0, 2, 1, true>;
    case 1: return (const void*)k_apply2d<T, N, 0, 1, 1, true>;
    default: return (const void*)k_apply2d<T, N, 0, 0, 0, true>;
  }
}

// (fused forms 1, 2 use the form-2 kernel; form 3 its own)
template <typename T, int N>
static long long resident_2d(int fuse, int v, int pf, bool mir) {
  constexpr int kDev = 16;
  static int cache[kDev][2][3][2][2];
  static bool init[kDev][2][3][2][2];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) return 0;
  const int f3 = fuse == 3 ? 1 : 0;
  const int w = mir ? 1 : 0;
  if (!init[dev][f3][v][pf][w]) {
    const void* f = mir ? kernel_2d_walls<T, N>(fuse)
                  : f3 ? kernel_2d<T, N, 3>(v, pf) : kernel_2d<T, N, 2>(v, pf);
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev][f3][v][pf][w] = per_cu * cus;
    init[dev][f3][v][pf][w] = true;
  }
  return cache[dev][f3][v][pf][w];
}

// The 3D kernel of fused form 0, 1 or 2 and prefetch flag pf: the coalesced form where Co3D
// selects it, else the z-line form; a grid with walls (mir) runs the halo-prefetch variant.
template <typename T, int N>
static const void* kernel_3d(int fuse, int pf, bool mir) {
  if constexpr (Co3D<T, N>::USE) {
    if (mir) {
      return fuse == 2 ? (const void*)k_apply3d_co<T, N, 2, 1, true>
           : fuse == 1 ? (const void*)k_apply3d_co<T, N, 1, 1, true>
                       : (const void*)k_apply3d_co<T, N, 0, 0, true>;
    }
  }
  if (mir) {
    return fuse == 2 ? (const void*)k_apply3d<T, N, 2, 1, true>
         : fuse == 1 ? (const void*)k_apply3d<T, N, 1, 1, true>
                     : (const void*)k_apply3d<T, N, 0, 0, true>;
  }
  if constexpr (Co3D<T, N>::USE) {
    return fuse == 2 ? (pf ? (const void*)k_apply3d_co<T, N, 2, 1> : (const void*)k_apply3d_co<T, N, 2, 0>)
         : fuse == 1 ? (pf ? (const void*)k_apply3d_co<T, N, 1, 1> : (const void*)k_apply3d_co<T, N, 1, 0>)
                     : (const void*)k_apply3d_co<T, N, 0, 0>;
  }
  return fuse == 2 ? (pf ? (const void*)k_apply3d<T, N, 2, 1, false> : (const void*)k_apply3d<T, N, 2, 0, false>)
       : fuse == 1 ? (pf ? (const void*)k_apply3d<T, N, 1, 1, false> : (const void*)k_apply3d<T, N, 1, 0, false>)
                   : (const void*)k_apply3d<T, N, 0, 0, false>;
}

// Workgroups of the 3D kernel (fused form 0, 1 or 2; prefetch pf; walls mir) the device holds at
// once.
template <typename T, int N>
static long long resident_3d(int fuse, int pf, bool mir) {
  constexpr int kDev = 16;
  static int cache[kDev][3][2][2];
  static bool init[kDev][3][2][2];
  int dev = 0;
  if (fuse < 0 || fuse > 2 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) return 0;
  if (fuse == 0) pf = 0;
  const int w = mir ? 1 : 0;
  if (!init[dev][fuse][pf][w]) {
    const void* f = kernel_3d<T, N>(fuse, pf, mir);
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, Tile3D<N>::NTH, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev][fuse][pf][w] = per_cu * cus;
    init[dev][fuse][pf][w] = true;
  }
  return cache[dev][fuse][pf][w];
}

template <typename T, int N>
static Geom geometry(const ApplyLaunch& L) {
  Geom g;
  const int nx = L.nc[0], ny = L.nc[1], nz = L.dim == 3 ? L.nc[2] : 1;
  if (L.dim == 2) {
    int tx = Tile2D<T, N, 0>::TX, ty = Tile2D<T, N, 0>::TY;
    if (L.tile_variant == 1) { tx = Tile2D<T, N, 1>::TX; ty = Tile2D<T, N, 1>::TY; }
    if (L.tile_variant == 2) { tx = Tile2D<T, N, 2>::TX; ty = Tile2D<T, N, 2>::TY; }
    g.ntx = (nx + tx - 1) / tx;
    g.nty = (ny + ty - 1) / ty;
    const long long ntiles = (long long)g.ntx * g.nty;
    // Fused CG form: when the tiles exceed what the device holds at once, each workgroup takes
    // up to 3 consecutive tiles (the next one prefetched during the current one's contraction)
    // so that the launch runs in one wave of workgroups (256^2 N = 6 FP64: 2048 tiles, 768
    // resident, 3 per workgroup measured 4 % faster than 1). One tile per workgroup otherwise.
    long long per = 1;
    long long res = 0;
    if (L.tiles_per_wg > 0) {
      per = L.tiles_per_wg;
    } else if (L.fuse) {
      res = resident_2d<T, N>(L.fuse, L.tile_variant, L.prefetch != 0,
                              L.mir[0] || L.mir[1] || L.mir[2]);
      // (the one-kernel form holds fewer workgroups: 4 tiles each at 256^2 N = 6 FP64)
      const long long cap = L.fuse == 3 ? 4 : 3;
      if (res > 0) per = std::min<long long>(cap, std::max<long long>(1, (ntiles + res - 1) / res));
    }
    // Large grids: at most kTarget2D workgroups (every block of the next launch re-sums one
    // partial per block, and the partial buffers hold kMaxPartials). 1024^2 N = 6 FP64 (32768
    // tiles): 607-614 us per fused launch for 3 to 16 tiles per workgroup alike.
    constexpr long long kTarget2D = 8192;
    per = std::max(per, (ntiles + kTarget2D - 1) / kTarget2D);
    g.kz = (int)per;
    g.ntz = 1;
    g.blocks = (unsigned long long)((ntiles + per - 1) / per);
    g.remap = (per == 1 && res > 0 && (long long)g.blocks <= res) ? 0 : 1;
    return g;
  } else {
    using TL = Tile3D<N>;
    g.ntx = (nx + TL::TX - 1) / TL::TX;
    g.nty = (ny + TL::TY - 1) / TL::TY;
    const long long cols = (long long)g.ntx * g.nty;
    // planes per segment: the workgroups run in waves of `res` (what the device holds at once)
    // and a segment of kz planes costs about kz + 2 plane steps (two boundary planes re-read),
    // so kz minimises waves * (kz + 2), ties to the longer segment; at least 4 planes.
    // 64^3 N = 4: FP64 (one workgroup per CU) 64 planes, FP32 32 (6 % faster than 16 in FP64);
    // 48^3 N = 3 FP64 (144 columns): 85 us per apply against 101 us with one wave of 27-plane
    // segments (the second wave held 32 workgroups).
    const long long res = resident_3d<T, N>(L.fuse, L.prefetch != 0, L.mir[0] || L.mir[1] || L.mir[2]);
    int kz = (int)((cols * nz) / 1024);
    if (res > 0) {
      long long best = -1;
      for (int z = std::min(4, nz); z <= nz; ++z) {
        const long long waves = (cols * ((nz + z - 1) / z) + res - 1) / res;
        const long long cost = waves * (z + 2);
        if (best < 0 || cost <= best) {
          best = cost;
          kz = z;
        }
      }
    }
    if (kz < 4) kz = 4;
    if (kz > nz) kz = nz;
    if (L.kz_override > 0) kz = L.kz_override < nz ? L.kz_override : nz;
    // no more than kMaxPartials workgroups: longer segments when the columns allow it (more
    // columns than that are rejected at setup)
    if (cols > 0 && cols <= kMaxPartials) {
      const long long segs = kMaxPartials / cols;
      const int kmin = (int)((nz + segs - 1) / segs);
      if (kz < kmin) kz = kmin;
    }
    g.kz = kz;
    g.ntz = (nz + kz - 1) / kz;
  }
  g.blocks = (unsigned long long)g.ntx * g.nty * g.ntz;
  return g;
}

template <typename T, int N>
hipError_t launch_apply_N(const ApplyLaunch& L, hipStream_t s) {
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
  a.kbase = nullptr;
  a.rho_cur = L.rho_cur;
  a.res_cur = L.res_cur;
  for (int d = 0; d < 3; ++d) a.mir[d] = L.mir[d];
  a.nrho = L.nrho;
  a.sigpart = L.sigpart;
  a.xsol = (T*)L.xsol;
  a.qprev = (const T*)L.qprev;
  a.rout = (T*)L.rout;
  a.fin = L.fin;
  a.fout = L.fout;
  a.npart = L.npart;
  a.first = L.first;
  if (L.fuse == 3 && L.dim != 2) return hipErrorInvalidValue;
  const Blk<T, N> B = make_blk<T, N>(*L.tab, L.dim);
  const Geom g = geometry<T, N>(L);
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.ntz = g.ntz;
  a.kz = g.kz;
  a.remap = g.remap;
  if (g.blocks > (unsigned long long)kMaxPartials) return hipErrorInvalidValue;
  const unsigned G = (unsigned)g.blocks;
  const bool pf = L.prefetch != 0;
  // extended launch: the optional start/stop events are taken from the dispatch itself (no
  // separate marker packets around the kernel)
  hipEvent_t e0 = L.ev_start, e1 = L.ev_stop;
  const bool walls = L.mir[0] || L.mir[1] || L.mir[2];
  if (L.dim == 2 && walls) {
    // walls: tile variant 0 with prefetch (pd_api sets both for such grids)
    if (L.tile_variant != 0 || (L.fuse && !pf)) return hipErrorInvalidValue;
    const void* f = kernel_2d_walls<T, N>(L.fuse);
    void* args[] = {&a, (void*)&B};
    const hipError_t e = hipExtLaunchKernel(f, dim3(G), dim3(256), args, 0, s, e0, e1, 0);
    if (e != hipSuccess) return e;
  } else if (L.dim == 2) {
#define PD_A2D(VV)                                                                              \
  if (L.fuse == 3) {                                                                            \
    if (pf) hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 3, 1>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B); \
    else hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 3, 0>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B);   \
  } else if (L.fuse == 2) {                                                                     \
    if (pf) hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 2, 1>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B); \
    else hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 2, 0>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B);   \
  } else if (L.fuse) {                                                                          \
    if (pf) hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 1, 1>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B); \
    else hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 1, 0>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B);   \
  } else {                                                                                      \
    hipExtLaunchKernelGGL((k_apply2d<T, N, VV, 0, 0>), dim3(G), dim3(256), 0, s, e0, e1, 0, a, B);       \
  }
    if (L.tile_variant == 1) { PD_A2D(1) }
    else if (L.tile_variant == 2) { PD_A2D(2) }
    else { PD_A2D(0) }
#undef PD_A2D
  } else {
    constexpr int NTH = Tile3D<N>::NTH;
    if (walls || Co3D<T, N>::USE) {
      const void* f = kernel_3d<T, N>(L.fuse, walls ? 1 : (L.fuse && pf ? 1 : 0), walls);
      void* args[] = {&a, (void*)&B};
      const hipError_t e = hipExtLaunchKernel(f, dim3(G), dim3(NTH), args, 0, s, e0, e1, 0);
      if (e != hipSuccess) return e;
    } else if (L.fuse == 2) {
      if (pf) hipExtLaunchKernelGGL((k_apply3d<T, N, 2, 1, false>), dim3(G), dim3(NTH), 0, s, e0, e1, 0, a, B);
      else hipExtLaunchKernelGGL((k_apply3d<T, N, 2, 0, false>), dim3(G), dim3(NTH), 0, s, e0, e1, 0, a, B);
    } else if (L.fuse) {
      if (pf) hipExtLaunchKernelGGL((k_apply3d<T, N, 1, 1, false>), dim3(G), dim3(NTH), 0, s, e0, e1, 0, a, B);
      else hipExtLaunchKernelGGL((k_apply3d<T, N, 1, 0, false>), dim3(G), dim3(NTH), 0, s, e0, e1, 0, a, B);
    } else {
      hipExtLaunchKernelGGL((k_apply3d<T, N, 0, 0, false>), dim3(G), dim3(NTH), 0, s, e0, e1, 0, a, B);
    }
  }
  return hipGetLastError();
}

template <typename T, int N>
unsigned blocks_N(const ApplyLaunch& L) {
  return (unsigned)geometry<T, N>(L).blocks;
}

}  // namespace pdk
