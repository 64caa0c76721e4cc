// Host-side launch descriptors shared by the kernel translation units and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>

#include "pd_device.h"

namespace pdk {

// Cells per group of the block-Jacobi preconditioner kernels: as many as keep one line of N+1
// nodes per direction per thread (n^(d-1) lines per cell and direction, at most kBlock lines).
__host__ __device__ constexpr int pcg_cells_per_group(int N, int dim) {
  return (dim == 3 ? kBlock / ((N + 1) * (N + 1)) : kBlock / (N + 1)) < 1
             ? 1
             : (dim == 3 ? kBlock / ((N + 1) * (N + 1)) : kBlock / (N + 1));
}

// FP64 copies of the 1D tables a launch needs (converted to the kernel precision at launch).
struct OpTables {
  double L[81], C[81], R[81], w[9];
};

struct ApplyLaunch {
  int dim = 2, N = 0;
  int nc[3] = {1, 1, 1};
  bool fp32 = false;
  int fuse = 0;              // 1: CG iteration form (p = r + beta p_old; sigma partials)
                             // 2: the same plus the deferred x += alpha_{k-1} p_old into xsol
                             // 3: 2 plus the residual update r -= alpha_{k-1} q_{k-1}
  const void* x = nullptr;   // operand (fuse = 0) or r (fuse = 1, 2)
  const void* pold = nullptr;
  void* pnew = nullptr;
  void* y = nullptr;
  double alpha = 0.0;
  double coef[3] = {0, 0, 0};
  // fuse = 1 only: CG state, iteration index, partials of rho_k, sigma partials out
  CgState* st = nullptr;
  int k = 0;
  const double* rho_cur = nullptr;
  const double* res_cur = nullptr;   // preconditioned: partials of <r, r> (x = z = P r)
  int nrho = 0;
  double* sigpart = nullptr;
  void* xsol = nullptr;      // fuse = 2, 3: the CG iterate x (updated in place for owned cells)
  // fuse = 3 (2D only): one kernel per CG iteration; the residual update of iteration k - 1 is
  // made here from x = r_{k-1} and qprev = q_{k-1} into rout (see ApplyArgs); fin / fout: the
  // 4-tuple partials of the previous / this launch (npart tuples each); first = 1 when x already
  // holds r_k with the partials of <r_k, r_k> in rho_cur.
  const void* qprev = nullptr;
  void* rout = nullptr;
  const double* fin = nullptr;
  double* fout = nullptr;
  int npart = 0;
  int first = 0;
  int kz_override = 0;       // 3D: planes per column segment (0 = automatic)
  int tiles_per_wg = 0;      // 2D: tiles per persistent workgroup (0 = automatic)
  int prefetch = 1;          // prefetch the next tile (2D) / next plane's halo (3D) into registers
  int tile_variant = 0;      // 2D tile shape (0 = largest fitting, 1 / 2 = one / two sizes smaller)
  int mir[3] = {0, 0, 0};    // 1: homogeneous Dirichlet pressure walls across direction d
  const OpTables* tab = nullptr;
  hipEvent_t ev_start = nullptr;   // optional events stamped at the kernel's start and end
  hipEvent_t ev_stop = nullptr;
};

hipError_t launch_apply(const ApplyLaunch& L, hipStream_t s);
// number of blocks (= partials) the apply kernel launches for this shape
unsigned apply_blocks(const ApplyLaunch& L);

// ---- streaming vector kernels (pd_vec.hip). Reductions write one partial per block; the
// consumer (next kernel or the single-block finalize) re-sums them in block order.
unsigned stream_grid(long long n);   // blocks (= partials) of every streaming kernel of length n
hipError_t launch_dot(bool fp32, const void* a, const void* b, long long n, double* partials,
                      hipStream_t s);
hipError_t launch_finalize(const double* partials, int nparts, CgState* st, int fin,
                           hipStream_t s);
// CG iteration k, second half (see k_cg_update): r -= alpha_k q, partials of rho_{k+1}; with
// x (and p) non-null also x += alpha_k p, else the x update is deferred (fused apply form 2)
hipError_t launch_cg_update(bool fp32, void* x, const void* p, const void* q, void* r,
                            long long n, CgState* st, int k, const double* sigpart, int nsig,
                            double* rho_next, hipStream_t s);
// Cell-block Jacobi preconditioner of alpha M + sum_d coef[d] (M on the other directions) (x) C
// (the diagonal cell blocks of the operator; see pdh::Table1D::PV).
struct PrecTables {
  double V[81], lam[9];
  double alpha = 0.0, coef[3] = {0, 0, 0};
};
// Preconditioned CG, second half of iteration k (upd = true): alpha_k from the sigma partials,
// r -= alpha_k q, z = P r, partials of <r, z> (rz_next) and <r, r> (rr_next); publishes alpha_k
// and xk for the deferred x update and the stamp of the next apply. upd = false: z = P r and
// the partials only (start of a run or after a residual replacement; no stamp check). Partials:
// pcg_grid(...) of each.
hipError_t launch_pcg_update(bool fp32, int dim, int N, bool upd, const void* q, void* r, void* z,
                             long long ncells, CgState* st, int k, const double* sigpart, int nsig,
                             double* rz_next, double* rr_next, const PrecTables& P, hipStream_t s);
unsigned pcg_grid(long long ncells, int dim, int N);
// the x update still pending when a run stopped (see k_x_flush)
hipError_t launch_x_flush(bool fp32, void* x, const void* pa, const void* pb, long long n,
                          const CgState* st, hipStream_t s);
// r = b - q (q == nullptr: r = b) with partials of <r, r>
hipError_t launch_residual(const double* b, const double* q, double* r, long long n,
                           double* partials, hipStream_t s);
// y = a*x + b*y (FP64); with b == 0 the old y is not read (it may hold NaN)
hipError_t launch_axpby(double a, const double* x, double b, double* y, long long n,
                        hipStream_t s);
// fill with zero (a kernel, not a memset, so that captured graphs hold no memset nodes)
hipError_t launch_zero(bool fp32, void* x, long long n, hipStream_t s);
// reset CG state for a new solve: maxit, rtol (kept in aux for FIN_BNORM), done = 0
hipError_t launch_state_init(CgState* st, int maxit, double rtol, hipStream_t s);
// set tol2 / maxit of a CG run, clear its done flag and let iteration k0 run next (starts or
// resumes a run at iteration k0)
hipError_t launch_state_set(CgState* st, int maxit, double tol2, int k0, hipStream_t s);
// r32 = (float)(inv * r64) with partials of <r32, r32> (residual replacement)
hipError_t launch_to_f32_dot(const double* r64, float* r32, long long n, double inv,
                             double* partials, hipStream_t s);
// x64 += scale * (double)d32, then d32 = 0 (flush of the FP32 correction)
hipError_t launch_flush_f32(double* x64, float* d32, long long n, double scale, hipStream_t s);
// y = W^{(x)d} x (nodal mass weights), FP64
hipError_t launch_mass(int dim, int N, const double* w, const double* x, double* y,
                       long long ncells, hipStream_t s);

// Kinetic energy of a dual velocity field: partials (stream_grid(ncells * (N+1)^dim) of them)
// of sum_i W_i sum_d u_d,i^2; with g non-null also g[d] = gs * W * u[d].
hipError_t launch_energy(int dim, int N, const double* w, const double* const u[3],
                         double* const g[3], double gs, long long ncells, double* partials,
                         hipStream_t s);

// ---- null-space projection (pd_vec.hip)
// corr = (P_z (x) P_y (x) P_x) (sum over cells of v) / ncells, then v -= corr per cell; Pdir[d]:
// host (N+1)^2 projector onto the 1D null space of direction d.
// part: 256 * (N+1)^dim doubles; corr: (N+1)^dim doubles.
hipError_t launch_project_null(bool fp32, void* v, long long ncells, int dim, int n,
                               const double* const Pdir[3], double* part, double* corr,
                               hipStream_t s);

// The same projection with its scratch (node-sum partials and correction) in a fixed device
// array of the library instead of caller- or context-owned memory: no allocation. Calls that
// overlap on one device race on that array.
hipError_t launch_project_null_noalloc(bool fp32, void* v, long long ncells, int dim, int n,
                                       const double* const Pdir[3], hipStream_t s);
// device address of the fixed scratch array on the current device (looked up once per device)
hipError_t noalloc_scratch(double** out);
size_t noalloc_scratch_bytes();

// ---- line operators and convection (pd_ops.hip)
struct LineLaunch {
  int dim = 2, N = 0;
  int nc[3] = {1, 1, 1};
  int d = 0;                 // direction of the 1D operator
  int o0 = 0, o1 = 0;        // cell offsets of the two inputs along d
  double A0[81], A1[81];     // out_line = A0 in(i+o0) + A1 in(i+o1)
  double coef = 1.0;         // scale
  int wperp = 0;             // multiply by the GL weights of the other directions
  double w[9];
  double accum = 0.0;        // out = accum*out + coef*(...)
  const double* in = nullptr;
  double* out = nullptr;
};
hipError_t launch_line(const LineLaunch& L, hipStream_t s);

struct ConvLaunch {
  int dim = 2, N = 0;
  int nc[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  double w[9], phi0[9], phi1[9], Kv[81];
  // explicit viscous flux (nu > 0): -nu grad q with the broken gradient, averaged normal
  // derivatives on faces and the viscous Rusanov speed 2 nu (2N+1) / (h_e sqrt(pi/2))
  double nu = 0.0;
  int conv = 1;                                          // 0: viscous flux only
  double dphi0[9], dphi1[9], KD[81];
  const double* ucur[3] = {nullptr, nullptr, nullptr};   // stage input (main grid)
  const double* u0[3] = {nullptr, nullptr, nullptr};     // step start
  double* out[3] = {nullptr, nullptr, nullptr};
  double a = 0.0, b = 1.0, dt = 0.0;                     // out = a u0 + b (ucur + dt L(ucur))
  double cr = 0.0;                                       // != 0: out = a u0 + cr L(ucur)
};
hipError_t launch_convect_stage(const ConvLaunch& L, hipStream_t s);

// Time mixing over the nodes of a space-time slab, elementwise over n values:
// out[s] = bc * base[s] + sum_p T[s][p] in[p] for s < mo (base[s] may be null; outputs may alias
// inputs or bases: every thread reads all its inputs before writing).
struct TimeMix {
  const double* in[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const double* base[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double* out[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double T[25] = {0};
  double bc = 0.0;
  int m = 1, mo = 1;
};
hipError_t launch_time_mix(const TimeMix& X, long long n, hipStream_t s);

// Adjoint of one RK stage out = a u0 + b (ucur + dt L(ucur)): with obar the cotangent of out,
// out_adj = acc_coef acc + b (obar + dt J(state)^T obar) is the cotangent reaching ucur = state
// (plus acc); the a u0 part is a plain scaling done by the caller.
struct ConvAdjLaunch {
  int dim = 2, N = 0;
  int nc[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  double w[9], phi0[9], phi1[9], Kv[81];
  const double* state[3] = {nullptr, nullptr, nullptr};
  const double* obar[3] = {nullptr, nullptr, nullptr};
  const double* acc[3] = {nullptr, nullptr, nullptr};
  double* out[3] = {nullptr, nullptr, nullptr};
  double acc_coef = 0.0, b = 1.0, dt = 0.0;
};
hipError_t launch_convect_adj_stage(const ConvAdjLaunch& L, hipStream_t s);

// ---- batched 2D solves (pd_batch.hip)
constexpr int kMaxNC2D = 81;      // (N+1)^2 for N = 8
constexpr int kNsBlocksBatch = 64;

// One problem of a batch (device-resident array, one per precision: the tile counts and the
// sigma-partial offsets depend on the tile shape of that precision).
struct BProb {
  int nx, ny, N, NC;
  long long dof_off, ndof, ncells;
  int ntx, nty;          // operator tiles of the chosen tile variant
  int sig_off, nsig;     // partials of <p, A p> written by the operator kernel
  int nupd;              // blocks per problem of the streaming kernels (= partials of <r, r>)
  int nns;               // node-sum blocks of the null-space projection
  int variant;
  double c0, c1, alpha;  // operator coefficients: alpha M + c0 (x-part) + c1 (y-part)
  double rtol;
  double ru;             // refinement: FP32 iterations pause once their residual dropped by ru
};

// Arguments shared by the batched kernels (passed by value). The streaming, projection and
// finalize kernels serve the problems of `list` (count entries); block b of a streaming kernel
// belongs to list entry i with upd_off[i] <= b < upd_off[i+1].
struct BatchIter {
  const BProb* probs;
  CgState* st;           // one CG state per problem
  const int* list;       // problem indices
  const int* upd_off;    // cumulative streaming blocks over list, count + 1 entries
  const int* ns_off;     // cumulative node-sum blocks over list, count + 1 entries
  int count, upd_blocks, ns_blocks;
  int want;              // serve problems with mode64 == want (-1: any; -2: residual check)
  int skip_fin;          // non-iterating kernels skip finished problems
  double* rho;           // problems x 2 x kMaxStreamPartials (iteration parity)
  double* sig;           // sigma partials (one buffer per precision)
  double* tmp;           // problems x kMaxStreamPartials
  double* nsp;           // problems x kNsBlocksBatch x kMaxNC2D node-sum partials
  double* corr;          // problems x kMaxNC2D null-space corrections
  const double* pnull;   // 9 x 81 projectors onto null(R~ - L~), by degree
  // preconditioned solves (else nullptr): partials of <r, r> (problems x 2 x kMaxStreamPartials,
  // iteration parity; rho then holds those of <r, z>)
  double* res;
  const int* kbase;      // device iteration base of the replayed chunk
  int koff;              // iteration offset of this launch within the chunk
};

// Problems of one (degree, tile variant) group served by one operator launch.
struct BatchGroup {
  int N, variant;
  const int* grp;        // problem indices (device)
  const int* toff;       // cumulative tiles, ng + 1 entries (device)
  int ng;
  unsigned blocks;
};

// fuse: CG iteration form (skips problems whose done flag is set or whose mode differs from
// it.want), including the deferred x += alpha_{k-1} p_old into xsol (the iterate of this
// precision: FP32 correction or FP64 x); else y = A x for the group's problems that are not
// finished (xsol unused).
hipError_t launch_apply_batch(const BatchIter& it, const BatchGroup& g, bool fp32, bool fuse,
                              const void* x, const void* pold, void* pnew, void* y, void* xsol,
                              const OpTables& tb, hipStream_t s);
// r -= alpha q with partials of <r, r>; publishes alpha and xk for the deferred x update
hipError_t launch_update_batch(const BatchIter& it, bool fp32, const void* q, void* r,
                               hipStream_t s);
// chunk end: the deferred x update of every listed problem that stopped before making it
hipError_t launch_xflush_batch(const BatchIter& it, double* x64, float* d32, const double* pa64,
                               const double* pb64, const float* pa32, const float* pb32,
                               hipStream_t s);
// Streaming passes over the list (problems with fin set are skipped except by mode 1):
// 0: r64 = b - q64 (partials of <r64, r64> into tmp); 1: x64 += scale d32, d32 = 0;
// 2: r32 = r64 / scale (partials into the rho slot koff & 1), problems in FP32 mode;
// 3: partials of <r64, r64> into tmp; 4: r64 = b (partials into rho slot 0);
// 5: partials of <r64, r64> into the rho slot koff & 1 for problems that just (re)started FP64
//    iterations from a recomputed residual.
hipError_t launch_stream_batch(int mode, const BatchIter& it, const double* b, const double* q64,
                               double* r64, double* x64, float* v32, hipStream_t s);
// what 0: aux = sum; 1: refinement start; 2: FP64 start; 3: chunk-end decision (see kernel)
hipError_t launch_finalize_batch(int what, const BatchIter& it, hipStream_t s);
// Cell-block Jacobi preconditioner of the listed problems, which all have degree N (V: the
// (N+1)^2 eigenbasis, lam: its N+1 eigenvalues). sel 0: the second half of a preconditioned
// iteration (alpha from the sigma partials, r -= alpha q, z = P r, partials of <r, z> and
// <r, r> in the slots of the next iteration); sel 1: z = P r of the problems the iterator serves,
// partials in the slots of iteration koff; sel 2: the same for the problems resuming from a
// recomputed residual (switched).
hipError_t launch_pcg_update_batch(const BatchIter& it, int N, bool fp32, int sel,
                                   const double* V, const double* lam, const void* q, void* r,
                                   void* z, hipStream_t s);
hipError_t launch_project_null_batch(const BatchIter& it, double* v, hipStream_t s);
hipError_t launch_tick(int* kbase, int by, hipStream_t s);
hipError_t launch_zero_all(bool fp32, void* v, long long n, hipStream_t s);
// reset every state: maxit, tol2, precision mode (0 FP32 refinement, 1 FP64)
hipError_t launch_state_init_batch(CgState* st, int count, int maxit, double tol2, int mode64,
                                   hipStream_t s);
// tile counts of the 2D operator for a tile variant (host helper)
void tiles2d(int N, bool fp32, int variant, int nx, int ny, int* ntx, int* nty);

}  // namespace pdk
