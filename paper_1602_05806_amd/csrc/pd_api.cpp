// C-ABI of libpd: context set-up, matrix-free operator application, conjugate-gradient solves
// (FP64 and FP32 inner solves with FP64 iterative refinement) and the semi-implicit fractional
// step of arXiv:1602.05806 Section 2.1-2.3 (eqs. LOdiffusionU-LOvelocityW).
#include "pd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pd_launch.h"
#include "pd_tables.h"

using pdk::CgState;

struct pd_ctx {
  int dim = 2, N = 0, n = 1, NC = 1;
  int nc[3] = {1, 1, 1};
  int per[3] = {1, 1, 1};      // 0: homogeneous Dirichlet pressure walls across direction d
  bool periodic = true;        // every direction periodic
  double len[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  double dt = 0, theta = 1, nu = 0;
  long long ncells = 0, ndof = 0;
  pdh::Table1D tab;
  pdk::OpTables optab;
  std::string err;
  // settings
  int step_prec = PD_FP64;
  double p_rtol = 1e-10, v_rtol = 1e-12, ru_factor = 0.1;
  int maxit = 100000, convection = 1, timing = 0, check_every = 32;
  int kz = 0, tiles_per_wg = 0, prefetch = 1;   // operator-kernel launch shape
  int tile_variant = 0;                          // 2D tile shape (0 = largest fitting)
  int defer_x = 1;         // 1: x update made by the next apply kernel, 0: by the update kernel
  int one_kernel = 0;      // 2D: one kernel per CG iteration (residual update folded in)
  int explicit_visc = 0;   // 1: viscous flux in the explicit TVD-RK3 step, no viscous solve
  int precond = 0;         // 1: cell-block Jacobi preconditioned CG (pd_cg_solve, pd_step)
  // device workspace
  CgState* st = nullptr;       // CG state of the (inner) solve
  CgState* st2 = nullptr;      // outer refinement / residual norms
  double* rhopart = nullptr;   // 2 x stream-grid partials of <r, r> (iteration parity)
  double* sigpart = nullptr;   // apply-grid partials of <p, A p>
  double* tmppart = nullptr;   // partials of stand-alone reductions
  double* null_part = nullptr;
  double* null_corr = nullptr;
  double *r64 = nullptr, *pa64 = nullptr, *pb64 = nullptr, *q64 = nullptr, *bw64 = nullptr;
  float *r32 = nullptr, *pa32 = nullptr, *pb32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  // 2D one-kernel CG iterations: second residual and A p buffers, 2 x 4-tuple partials
  double *r64b = nullptr, *q64b = nullptr, *fpart = nullptr;
  float *r32b = nullptr, *q32b = nullptr;
  // preconditioned runs: z = P r in both precisions, 2 x partials of <r, r>
  double* z64 = nullptr;
  float* z32 = nullptr;
  double* rrpart = nullptr;
  double* um[3] = {nullptr, nullptr, nullptr};
  double* s1[3] = {nullptr, nullptr, nullptr};
  double* s2[3] = {nullptr, nullptr, nullptr};
  double* qbuf = nullptr;
  double* at[4][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr},
                      {nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};   // adjoint work
  double* abar = nullptr;                             // adjoint pressure right-hand side
  // space-time step: node iterates U_s, right-hand sides R_s and pressure-gradient work W_s
  // (dual grids, per node and component), pressure increments dP_s, pi_{*->#} U^n and two
  // main-grid work arrays per component, one pressure right-hand side
  double* stU[pdh::kMaxm][3] = {};
  double* stR[pdh::kMaxm][3] = {};
  double* stW[pdh::kMaxm][3] = {};
  double* stdP[pdh::kMaxm] = {};
  double* stum0[3] = {};
  double* sta[3] = {};
  double* stb[3] = {};
  double* strhs = nullptr;
  CgState* hst = nullptr;      // pinned host mirror, 2 slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<hipEvent_t> tev;
  double t_ms[2] = {0, 0};
  long long t_cnt[2] = {0, 0};
  double t_words[2] = {6, 6};  // vector words per DoF of the timed launches (8, 6 or 4)
  hipStream_t last_stream = nullptr;
};

namespace {

thread_local std::string g_setup_err;

int fail(pd_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  else g_setup_err = m;
  return code;
}

#define PD_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, PD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

hipStream_t S(void* s) { return (hipStream_t)s; }

template <typename T>
int dev_alloc(pd_ctx* c, T** p, size_t count) {
  if (*p) return PD_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T) + 256);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, PD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return PD_OK;
}

void op_coefs(const pd_ctx* c, int op, double* alpha, double coef[3]) {
  const double beta = (op == PD_OP_PRESSURE) ? c->dt : c->nu * c->dt;
  *alpha = (op == PD_OP_PRESSURE) ? 0.0 : 1.0;
  for (int d = 0; d < 3; ++d) coef[d] = d < c->dim ? beta / (c->h[d] * c->h[d]) : 0.0;
}

pdk::ApplyLaunch base_launch(const pd_ctx* c, int op, bool fp32) {
  pdk::ApplyLaunch L;
  L.dim = c->dim;
  L.N = c->N;
  for (int d = 0; d < 3; ++d) L.nc[d] = c->nc[d];
  L.fp32 = fp32;
  op_coefs(c, op, &L.alpha, L.coef);
  L.tab = &c->optab;
  L.kz_override = c->kz;
  L.tiles_per_wg = c->tiles_per_wg;
  L.prefetch = c->prefetch;
  L.tile_variant = c->tile_variant;
  for (int d = 0; d < c->dim; ++d) L.mir[d] = c->per[d] ? 0 : 1;
  if (!c->periodic) {   // grids with walls run one kernel shape: tile variant 0, prefetch on
    L.tile_variant = 0;
    L.prefetch = 1;
  }
  return L;
}

int plain_apply(pd_ctx* c, int op, bool fp32, const void* x, void* y, hipStream_t s) {
  pdk::ApplyLaunch L = base_launch(c, op, fp32);
  L.x = x;
  L.y = y;
  PD_HIP(c, pdk::launch_apply(L, s));
  return PD_OK;
}

// Per-direction projectors onto the 1D null space: the cell-periodic kernel of D along periodic
// directions, its odd part along Dirichlet directions. false when a direction has none (then
// the operator has no null space and the projection is the identity).
bool null_projectors(const pd_ctx* c, const double* P[3]) {
  for (int d = 0; d < 3; ++d) {
    P[d] = c->tab.Pnull;
    if (d < c->dim && !c->per[d]) {
      if (c->tab.nnull_odd == 0) return false;
      P[d] = c->tab.PnullOdd;
    }
  }
  return true;
}

int project_null(pd_ctx* c, bool fp32, void* v, hipStream_t s) {
  const double* P[3];
  if (!null_projectors(c, P)) return PD_OK;
  PD_HIP(c, pdk::launch_project_null(fp32, v, c->ncells, c->dim, c->n, P, c->null_part,
                                     c->null_corr, s));
  return PD_OK;
}

int require_periodic(pd_ctx* c, const char* what) {
  if (c->periodic) return PD_OK;
  return fail(c, PD_EINVAL, std::string(what) + ": fully periodic grids only (the Dirichlet "
                            "walls cover the pressure and viscous operators and their solves)");
}

// <a, b> -> st->aux (FIN_AUX) or bnorm2/tol2 (FIN_BNORM), on the stream.
int dot_into(pd_ctx* c, bool fp32, const void* a, const void* b, CgState* st, int fin,
             hipStream_t s) {
  PD_HIP(c, pdk::launch_dot(fp32, a, b, c->ndof, c->tmppart, s));
  PD_HIP(c, pdk::launch_finalize(c->tmppart, (int)pdk::stream_grid(c->ndof), st, fin, s));
  return PD_OK;
}

int read_state(pd_ctx* c, const CgState* dev, CgState* host, hipStream_t s) {
  PD_HIP(c, hipMemcpyAsync(host, dev, sizeof(CgState), hipMemcpyDeviceToHost, s));
  PD_HIP(c, hipStreamSynchronize(s));
  return PD_OK;
}

// Device buffers of one CG run: residual r, the two search-direction buffers (iteration k reads
// buf[k % 2] and writes buf[(k + 1) % 2]) and q = A p. The one-kernel form also double-buffers
// r and q: iteration k reads r_{k-1} and q_{k-1} from {r, rb}[(k + 1) % 2], {q, qb}[(k + 1) % 2]
// and writes r_k, q_k to {r, rb}[k % 2], {q, qb}[k % 2]; a run (re)started at iteration k takes
// r_k from {r, rb}[k % 2].
struct CgBuffers {
  void *r, *pa, *pb, *q;
  void *rb = nullptr, *qb = nullptr;
};

// A chunked conjugate-gradient run on the device, FP64 or FP32 vectors (FP64 scalars).
// One-kernel form (2D, opt-in): the apply kernel of iteration k also makes the residual update
// of iteration k - 1 (r_k = r_{k-1} - alpha_{k-1} q_{k-1} while loading r and q for its tile and
// halo) and the x update, so one iteration is one kernel and 8 vector words per DoF. Measured
// at 256^2 N = 6 it is not faster: the tile kernel streams at the same rate as with 6 words
// (about 3.6 TB/s), so the 3 words moved out of the update kernel (5.3 TB/s) cost about what
// the saved kernel boundary gains (FP64 57 us per iteration kernel against 44 + 15 us; FP32
// slower).
// Iteration k = apply kernel (p_k = r_k + beta_k p_{k-1}, q = A p_k, partials of <p_k, q>) +
// update kernel (x += alpha_k p_k, r -= alpha_k q, partials of <r_{k+1}, r_{k+1}>). Deferred
// form (default): the x update rides on the apply kernel of iteration k + 1, which reads p_k
// anyway (9 vector words per DoF and iteration instead of 10; the update still pending when the
// run stops is flushed at the end). Measured at 256^2 N = 6 and 64^3 N = 4: 0-8 % (2D) and 13 %
// (3D) less time per FP64 iteration, 9 % less (2D) and 1 % more (3D) per FP32 iteration.
// The run can be stopped by a host predicate on the polled state and resumed at the exact
// iteration.
struct CgRun {
  int op = 0;
  bool fp32 = false;
  void* x = nullptr;
  CgBuffers B{};
  CgState* st = nullptr;
  hipStream_t s = nullptr;
  bool timed = false;
  bool defer = true;         // x update made by the next apply kernel (else by the update kernel)
  bool one = false;          // one kernel per iteration (2D)
  int kfirst = 0;            // iteration at which the run was (re)started: r_k given, no update
  int k = 0;                 // next iteration to launch / iterations completed after a stop
  int nrho = 0, nsig = 0;
  double* rho[2] = {nullptr, nullptr};
  pdk::ApplyLaunch L;
  // preconditioned run: z = P r (cell-block Jacobi); rho[] then holds the partials of <r, z>
  // and rr[] those of <r, r> (the stopping test)
  bool pc = false;
  void* z = nullptr;
  double* rr[2] = {nullptr, nullptr};
  pdk::PrecTables P;
};

pdk::PrecTables prec_tables(const pd_ctx* c, int op) {
  pdk::PrecTables P;
  const int n = c->n;
  for (int i = 0; i < 81; ++i) P.V[i] = i < n * n ? c->tab.PV[i] : 0.0;
  for (int i = 0; i < 9; ++i) P.lam[i] = i < n ? c->tab.Plam[i] : 0.0;
  op_coefs(c, op, &P.alpha, P.coef);
  return P;
}

// z = P r with the partials of <r, z> and <r, r> in the slots of iteration slot (start of a
// preconditioned run, or its restart from a replaced residual)
int pcg_init(pd_ctx* c, const struct CgRun* R, int slot, hipStream_t s);

// Prepare a run whose residual r_0 and the partials of <r_0, r_0> (in rho[0]) are in place and
// whose CG state holds tol2 / maxit.
int cg_prepare(pd_ctx* c, CgRun* R) {
  R->pc = c->precond != 0;
  R->nrho = R->pc ? (int)pdk::pcg_grid(c->ncells, c->dim, c->N) : (int)pdk::stream_grid(c->ndof);
  R->rho[0] = c->rhopart;
  R->rho[1] = c->rhopart + pdk::kMaxStreamPartials;
  if (R->pc) {
    R->z = R->fp32 ? (void*)c->z32 : (void*)c->z64;
    R->rr[0] = c->rrpart;
    R->rr[1] = c->rrpart + pdk::kMaxStreamPartials;
    R->P = prec_tables(c, R->op);
  }
  R->L = base_launch(c, R->op, R->fp32);
  R->defer = c->defer_x != 0;
  R->one = c->one_kernel != 0 && c->dim == 2 && R->B.rb && R->B.qb && !R->pc;
  R->L.fuse = R->one ? 3 : R->defer ? 2 : 1;
  R->L.xsol = (R->one || R->defer) ? R->x : nullptr;
  R->L.st = R->st;
  R->L.nrho = R->nrho;
  R->L.sigpart = c->sigpart;
  R->nsig = (int)pdk::apply_blocks(R->L);
  R->L.npart = R->nsig;
  R->k = 0;
  R->kfirst = 0;
  PD_HIP(c, pdk::launch_zero(R->fp32, R->B.pa, c->ndof, R->s));
  if (R->pc) return pcg_init(c, R, 0, R->s);
  return PD_OK;
}

int pcg_init(pd_ctx* c, const CgRun* R, int slot, hipStream_t s) {
  PD_HIP(c, pdk::launch_pcg_update(R->fp32, c->dim, c->N, false, nullptr, R->B.r, R->z, c->ncells,
                                   R->st, 0, nullptr, 0, R->rho[slot & 1], R->rr[slot & 1], R->P,
                                   s));
  return PD_OK;
}

int cg_launch(pd_ctx* c, CgRun* R) {
  const int k = R->k;
  void* buf[2] = {R->B.pa, R->B.pb};
  pdk::ApplyLaunch& L = R->L;
  L.k = k;
  L.rho_cur = R->rho[k & 1];
  L.res_cur = R->pc ? R->rr[k & 1] : nullptr;
  L.x = R->pc ? R->z : R->B.r;
  L.pold = buf[k & 1];
  L.pnew = buf[(k + 1) & 1];
  L.y = R->B.q;
  if (R->one) {
    void* rb[2] = {R->B.r, R->B.rb};
    void* qb[2] = {R->B.q, R->B.qb};
    L.first = k == R->kfirst;
    L.x = L.first ? rb[k & 1] : rb[(k + 1) & 1];
    L.rout = rb[k & 1];
    L.qprev = qb[(k + 1) & 1];
    L.y = qb[k & 1];
    L.fin = c->fpart + 4 * (size_t)pdk::kMaxPartials * ((k + 1) & 1);
    L.fout = c->fpart + 4 * (size_t)pdk::kMaxPartials * (k & 1);
  }
  L.ev_start = L.ev_stop = nullptr;
  if (R->timed && k % c->timing == 0) {       // every timing-th launch carries events
    const size_t j = (size_t)(k / c->timing);
    while (c->tev.size() < 2 * (j + 1)) {
      hipEvent_t e;
      PD_HIP(c, hipEventCreate(&e));
      c->tev.push_back(e);
    }
    L.ev_start = c->tev[2 * j];
    L.ev_stop = c->tev[2 * j + 1];
  }
  PD_HIP(c, pdk::launch_apply(L, R->s));
  if (R->pc)
    PD_HIP(c, pdk::launch_pcg_update(R->fp32, c->dim, c->N, true, R->B.q, R->B.r, R->z,
                                     c->ncells, R->st, k, c->sigpart, R->nsig, R->rho[(k + 1) & 1],
                                     R->rr[(k + 1) & 1], R->P, R->s));
  else if (!R->one)
    PD_HIP(c, pdk::launch_cg_update(R->fp32, R->defer ? nullptr : R->x,
                                    R->defer ? nullptr : buf[(k + 1) & 1], R->B.q, R->B.r,
                                    c->ndof, R->st, k, c->sigpart, R->nsig,
                                    R->rho[(k + 1) & 1], R->s));
  ++R->k;
  return PD_OK;
}

// Launch iterations in chunks until the device reports done or stop(polled state) is true; the
// next chunk is already queued while a chunk's state is inspected. On return the stream is
// synchronised, x holds the iterate of the last completed iteration, *fin the final state and
// R->k the number of completed iterations.
template <typename Pred>
int cg_run_until(pd_ctx* c, CgRun* R, int maxit, Pred stop, CgState* fin) {
  const int chunk = c->check_every > 0 ? c->check_every : 32;
  int slot = 0;
  bool pending[2] = {false, false};
  bool finished = false;
  while (!finished) {
    for (int i = 0; i < chunk; ++i) {
      int rc = cg_launch(c, R);
      if (rc) return rc;
    }
    PD_HIP(c, hipMemcpyAsync(&c->hst[slot], R->st, sizeof(CgState), hipMemcpyDeviceToHost, R->s));
    PD_HIP(c, hipEventRecord(c->ev[slot], R->s));
    pending[slot] = true;
    const int prev = slot ^ 1;
    if (pending[prev]) {
      PD_HIP(c, hipEventSynchronize(c->ev[prev]));
      pending[prev] = false;
      if (c->hst[prev].done || stop(c->hst[prev])) finished = true;
    }
    slot ^= 1;
    if (R->k > maxit + 2 * chunk) finished = true;
  }
  PD_HIP(c, pdk::launch_x_flush(R->fp32, R->x, R->B.pa, R->B.pb, c->ndof, R->st, R->s));
  int rc = read_state(c, R->st, fin, R->s);
  if (rc) return rc;
  if (fin->done) R->k = fin->iter;
  return PD_OK;
}

void cg_collect_timing(pd_ctx* c, const CgRun& R) {
  if (!R.timed) return;
  const int tslot = R.fp32 ? 1 : 0;
  c->t_words[tslot] = R.one ? 8.0 : R.defer ? 6.0 : 4.0;
  // sampled launches of the completed iterations (launches queued after the stop exit at once)
  for (int k = 0; k < R.k; k += c->timing) {
    const size_t j = (size_t)(k / c->timing);
    if (2 * j + 1 >= c->tev.size()) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->tev[2 * j], c->tev[2 * j + 1]) == hipSuccess) {
      c->t_ms[tslot] += ms;
      c->t_cnt[tslot] += 1;
    }
  }
}

// r64 = b - A x in FP64 (projected for the pressure operator); *norm = ||r64||.
int fp64_residual(pd_ctx* c, int op, const double* b, const double* x, hipStream_t s,
                  double* norm) {
  int rc = plain_apply(c, op, false, x, c->q64, s);
  if (rc) return rc;
  PD_HIP(c, pdk::launch_residual(b, c->q64, c->r64, c->ndof, c->tmppart, s));
  if (op == PD_OP_PRESSURE) {
    rc = project_null(c, false, c->r64, s);
    if (rc) return rc;
  }
  rc = dot_into(c, false, c->r64, c->r64, c->st2, pdk::FIN_AUX, s);
  if (rc) return rc;
  CgState h;
  rc = read_state(c, c->st2, &h, s);
  if (rc) return rc;
  *norm = std::sqrt(h.aux);
  return PD_OK;
}

// Verifications of the true residual after the FP64 recurrence met the tolerance, and the
// largest true / goal ratio that is iterated away (beyond it: FP64 rounding floor).
constexpr int kMaxTrueChecks = 8;
constexpr double kTrueGap = 16.0;

// FP64 conjugate gradients from the initial guess in x; stops on the true residual (see below).
int solve_fp64(pd_ctx* c, int op, const double* b, double* x, double rtol, double bnorm, int maxit,
               bool timed, pd_solve_info* inf, hipStream_t s) {
  CgRun R;
  R.op = op;
  R.fp32 = false;
  R.x = x;
  R.B = CgBuffers{c->r64, c->pa64, c->pb64, c->q64, c->r64b, c->q64b};
  R.st = c->st;
  R.s = s;
  R.timed = timed;
  int rc = plain_apply(c, op, false, x, c->q64, s);
  if (rc) return rc;
  PD_HIP(c, pdk::launch_residual(b, c->q64, c->r64, c->ndof, c->rhopart, s));
  PD_HIP(c, pdk::launch_state_set(c->st, maxit, rtol * rtol * bnorm * bnorm, 0, s));
  if ((rc = cg_prepare(c, &R))) return rc;
  CgState fin;
  inf->outer_iters = 0;
  double prev_res = 0.0;
  for (;;) {
    rc = cg_run_until(c, &R, maxit, [](const CgState&) { return false; }, &fin);
    if (rc) return rc;
    ++inf->outer_iters;
    // The recurrence residual met the tolerance; after thousands of iterations it can sit below
    // the true one, so b - A x decides. If it is above but within kTrueGap of the goal, it
    // replaces r (partials of <r, r> for iteration R.k) and the run continues with the same
    // direction (a reliable update) unless the recurrence had drifted more than 4x below it (then
    // beta would be huge and the old direction would swamp the new residual: the direction
    // restarts). A larger gap, or a replacement that did not halve the true residual, is the
    // FP64 rounding floor of b - A x (about eps cond(A) |b|): the solve ends there (status PD_OK
    // from the recurrence, the true residual reported).
    if (!(fin.done && fin.status == PD_OK) || R.k >= maxit || inf->outer_iters > kMaxTrueChecks)
      break;
    double res = 0.0;
    if ((rc = fp64_residual(c, op, b, x, s, &res))) return rc;   // overwrites r and A p
    if (!std::isfinite(res)) {
      fin.status = PD_EBREAKDOWN;
      break;
    }
    const double goal = rtol * bnorm;
    if (res <= goal || res > kTrueGap * goal || (prev_res > 0.0 && res > 0.5 * prev_res)) break;
    prev_res = res;
    // preconditioned runs always restart the direction: beta would combine <r, P r> of the
    // replaced residual with that of the recurrence, and on the ill-conditioned odd-degree
    // systems (where a replacement happens at all) the kept direction loses conjugacy
    // (10 x 12 cells of 0.2 x 0.083, N = 7, rtol 1e-12: 48k iterations ending at a true
    // residual of 0.24 with the direction kept)
    if (R.pc || !(res <= 4.0 * std::sqrt(fin.res2))) {
      void* buf[2] = {R.B.pa, R.B.pb};
      PD_HIP(c, pdk::launch_zero(false, buf[R.k & 1], c->ndof, s));
      ++inf->restarts;
    }
    if (R.pc) {
      if ((rc = pcg_init(c, &R, R.k, s))) return rc;
    } else {
      PD_HIP(c, pdk::launch_dot(false, c->r64, c->r64, c->ndof, R.rho[R.k & 1], s));
    }
    if (R.one && (R.k & 1))
      PD_HIP(c, hipMemcpyAsync(c->r64b, c->r64, c->ndof * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    R.kfirst = R.k;
    PD_HIP(c, pdk::launch_state_set(c->st, maxit, rtol * rtol * bnorm * bnorm, R.k, s));
  }
  cg_collect_timing(c, R);
  inf->iters = R.k;
  inf->rel_res_recur = std::sqrt(fin.res2) / bnorm;
  inf->status = fin.done ? fin.status : PD_ENOCONV;
  return PD_OK;
}

// FP32 conjugate gradients with FP64 residual replacement: one CG run on FP32 vectors (r, p,
// A p and the correction d; FP64 dot products). Whenever the recurrence residual has dropped by
// ru_factor since the last replacement, or meets the tolerance, the correction is flushed into
// the FP64 solution (x += s d), the true residual b - A x is recomputed in FP64 and replaces the
// FP32 residual. The search direction is kept, so the run keeps its Krylov information (unlike
// restarted refinement). Stops on the FP64 residual.
int solve_refine(pd_ctx* c, int op, const double* b, double* x, double rtol, double bnorm,
                 int maxit, bool timed, pd_solve_info* inf, hipStream_t s) {
  const long long n = c->ndof;
  double res = 0.0;
  int rc = fp64_residual(c, op, b, x, s, &res);
  if (rc) return rc;
  inf->outer_iters = 0;
  inf->iters = 0;
  inf->rel_res_recur = res / bnorm;
  if (!std::isfinite(res)) {
    inf->status = PD_EBREAKDOWN;
    return PD_OK;
  }
  if (res <= rtol * bnorm) {
    inf->status = PD_OK;
    return PD_OK;
  }
  const double scale = res;                     // the FP32 vectors hold r / scale
  const double tol_rel = rtol * bnorm / scale;  // recurrence tolerance in scaled units
  const double f = c->ru_factor;
  // The FP32 iterations stop on the device once their residual has dropped by f below the last
  // replaced one (or reached the final tolerance); each stop is followed by a replacement.
  auto inner_tol2 = [&](double ref) {
    const double t = std::fmax(f * ref, tol_rel);
    return t * t;
  };
  CgRun R;
  R.op = op;
  R.fp32 = true;
  R.x = c->d32;
  R.B = CgBuffers{c->r32, c->pa32, c->pb32, c->q32, c->r32b, c->q32b};
  R.st = c->st;
  R.s = s;
  R.timed = timed;
  PD_HIP(c, pdk::launch_zero(true, c->d32, n, s));
  PD_HIP(c, pdk::launch_to_f32_dot(c->r64, c->r32, n, 1.0 / scale, c->rhopart, s));
  PD_HIP(c, pdk::launch_state_set(c->st, maxit, inner_tol2(1.0), 0, s));
  if ((rc = cg_prepare(c, &R))) return rc;
  double ref = 1.0;                             // scaled residual norm at the last replacement
  double best = 1.0;                            // smallest scaled FP64 residual so far
  int stall = 0;                                // replacements in a row that did not halve best
  int stalled = 0;                              // FP32 breakdowns in a row without progress
  inf->status = PD_ENOCONV;
  for (;;) {
    CgState fin;
    rc = cg_run_until(c, &R, maxit, [](const CgState&) { return false; }, &fin);
    if (rc) return rc;
    // flush the FP32 correction and recompute the true residual in FP64
    PD_HIP(c, pdk::launch_flush_f32(x, c->d32, n, scale, s));
    rc = fp64_residual(c, op, b, x, s, &res);
    if (rc) return rc;
    ++inf->outer_iters;
    inf->rel_res_recur = res / bnorm;
    if (!std::isfinite(res)) {
      inf->status = PD_EBREAKDOWN;
      break;
    }
    if (res <= rtol * bnorm) {
      inf->status = PD_OK;
      break;
    }
    if (R.k >= maxit) {
      inf->status = PD_ENOCONV;
      break;
    }
    // FP32 arithmetic has stopped reducing the FP64 residual: it grew beyond twice the best
    // one, or kStallRefine replacements in a row did not halve the best one (each replacement
    // normally gains the factor ru_factor). Causes: eps_32 cond(A) near 1 makes FP32 A p
    // meaningless for the smallest eigenvalues, or the goal lies below the FP64 rounding floor
    // of b - A x. The solve continues with FP64 iterations from the current x, whose true-
    // residual checks handle both (measured: 256^2 N = 6 at rtol 1e-12, below the floor of its
    // smooth right-hand side, took 103k FP32 iterations when only 16 non-improving replacements
    // triggered the switch).
    constexpr int kStallRefine = 3;
    const double r = res / scale;
    if (r < 0.5 * best) {
      stall = 0;
    } else {
      ++stall;
    }
    if (r < best) best = r;
    if (r > 2.0 * best || stall >= kStallRefine) {
      cg_collect_timing(c, R);
      inf->fallback_iter = R.k;
      pd_solve_info i64{};
      rc = solve_fp64(c, op, b, x, rtol, bnorm, std::max(0, maxit - R.k), timed, &i64, s);
      if (rc) return rc;
      inf->iters = R.k + i64.iters;
      inf->status = i64.status;
      inf->rel_res_recur = i64.rel_res_recur;
      return PD_OK;
    }
    // An FP32 breakdown (<p, A p> <= 0 once the FP32 residual is rounding noise, which on a
    // singular operator includes null-space components) ends the inner run; the FP64 residual
    // replaces it and the direction restarts. Two in a row without progress end the solve.
    const bool broke = fin.done && fin.status == PD_EBREAKDOWN;
    stalled = broke && !(res / scale < 0.5 * ref) ? stalled + 1 : 0;
    if (stalled >= 2) {
      inf->status = PD_EBREAKDOWN;
      break;
    }
    // residual replacement: r32 = r64 / scale with the partials of <r32, r32> for iteration R.k.
    // If the FP32 recurrence residual had drifted well below the true one, beta would be huge
    // and the old direction would swamp the new residual: restart the direction (p_old = 0).
    const double rec = std::sqrt(fin.res2);
    if (broke || !(res / scale <= 4.0 * rec)) {
      void* buf[2] = {R.B.pa, R.B.pb};
      PD_HIP(c, pdk::launch_zero(true, buf[R.k & 1], n, s));
      ++inf->restarts;
    }
    float* r32k = (R.one && (R.k & 1)) ? c->r32b : c->r32;
    PD_HIP(c, pdk::launch_to_f32_dot(c->r64, r32k, n, 1.0 / scale, R.rho[R.k & 1], s));
    if (R.pc)
      if ((rc = pcg_init(c, &R, R.k, s))) return rc;
    R.kfirst = R.k;
    ref = res / scale;
    PD_HIP(c, pdk::launch_state_set(c->st, maxit, inner_tol2(ref), R.k, s));
  }
  cg_collect_timing(c, R);
  inf->iters = R.k;
  return PD_OK;
}

int solve(pd_ctx* c, int op, int prec, const double* b_in, double* x, double rtol, int maxit,
          pd_solve_info* info, hipStream_t s) {
  if (op != PD_OP_PRESSURE && op != PD_OP_VISCOUS) return fail(c, PD_EINVAL, "unknown operator");
  if (prec != PD_FP64 && prec != PD_FP32_REFINE64)
    return fail(c, PD_EINVAL, "pd_cg_solve precision must be PD_FP64 or PD_FP32_REFINE64");
  if (!b_in || !x) return fail(c, PD_EINVAL, "null array");
  if ((const void*)b_in == (const void*)x) return fail(c, PD_EINVAL, "b and x must not alias");
  if (!(rtol > 0.0)) return fail(c, PD_EINVAL, "rtol must be > 0");
  if (maxit < 0) return fail(c, PD_EINVAL, "maxit must be >= 0");
  c->last_stream = s;
  const long long n = c->ndof;
  PD_HIP(c, hipEventRecord(c->t0, s));
  const double* b = b_in;
  int rc;
  if (op == PD_OP_PRESSURE) {
    PD_HIP(c, pdk::launch_axpby(1.0, b_in, 0.0, c->bw64, n, s));
    if ((rc = project_null(c, false, c->bw64, s))) return rc;
    if ((rc = project_null(c, false, x, s))) return rc;
    b = c->bw64;
  }
  const bool timed = c->timing && op == PD_OP_PRESSURE;
  if ((rc = dot_into(c, false, b, b, c->st2, pdk::FIN_AUX, s))) return rc;
  CgState h;
  if ((rc = read_state(c, c->st2, &h, s))) return rc;
  const double bnorm = std::sqrt(h.aux);
  pd_solve_info inf{};
  inf.status = PD_OK;
  inf.fallback_iter = -1;
  if (bnorm == 0.0) {
    PD_HIP(c, pdk::launch_zero(false, x, n, s));
  } else if (!std::isfinite(bnorm)) {
    inf.status = PD_EBREAKDOWN;
  } else if (prec == PD_FP64) {
    if ((rc = solve_fp64(c, op, b, x, rtol, bnorm, maxit, timed, &inf, s))) return rc;
  } else {
    if ((rc = solve_refine(c, op, b, x, rtol, bnorm, maxit, timed, &inf, s))) return rc;
  }
  if (op == PD_OP_PRESSURE) {
    if ((rc = project_null(c, false, x, s))) return rc;
  }
  if (bnorm > 0.0 && std::isfinite(bnorm)) {
    double res = 0.0;
    if ((rc = fp64_residual(c, op, b, x, s, &res))) return rc;
    inf.rel_res_true = res / bnorm;
  }
  PD_HIP(c, hipEventRecord(c->t1, s));
  PD_HIP(c, hipEventSynchronize(c->t1));
  float ms = 0.f;
  PD_HIP(c, hipEventElapsedTime(&ms, c->t0, c->t1));
  inf.ms = ms;
  if (info) *info = inf;
  return inf.status;
}

void fill_line_common(const pd_ctx* c, pdk::LineLaunch* L) {
  L->dim = c->dim;
  L->N = c->N;
  for (int d = 0; d < 3; ++d) L->nc[d] = c->nc[d];
  for (int i = 0; i < 9; ++i) L->w[i] = i < c->n ? c->tab.w[i] : 0.0;
}

// pi_{*->#} (dir 0) or pi_{#->*} (dir 1) along d.
int l2_project(pd_ctx* c, int d, int dir, const double* in, double* out, hipStream_t s) {
  pdk::LineLaunch L;
  fill_line_common(c, &L);
  const int n = c->n;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      L.A0[p * n + q] = c->tab.ML[p * n + q] / c->tab.w[p];
      L.A1[p * n + q] = c->tab.MR[p * n + q] / c->tab.w[p];
    }
  L.d = d;
  if (dir == 0) {      // eq. (l2forward): U#_i = M^-1 (M^L U*_{i-1} + M^R U*_i)
    L.o0 = -1;
    L.o1 = 0;
  } else {             // eq. (l2backward): U*_i = M^-1 (M^L U#_i + M^R U#_{i+1})
    L.o0 = 0;
    L.o1 = 1;
  }
  L.coef = 1.0;
  L.in = in;
  L.out = out;
  PD_HIP(c, pdk::launch_line(L, s));
  return PD_OK;
}

// b = sum_d h_d^-1 W_perp (R~^T u_d[i-1] - L~^T u_d[i])
int rhs_div(pd_ctx* c, void* const u[3], double* b, hipStream_t s) {
  const int n = c->n;
  for (int d = 0; d < c->dim; ++d) {
    if (!u[d]) return fail(c, PD_EINVAL, "null velocity component");
    pdk::LineLaunch L;
    fill_line_common(c, &L);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        L.A0[p * n + q] = c->tab.Rt[q * n + p];
        L.A1[p * n + q] = -c->tab.Lt[q * n + p];
      }
    L.d = d;
    L.o0 = -1;
    L.o1 = 0;
    L.coef = 1.0 / c->h[d];
    L.wperp = 1;
    L.accum = d == 0 ? 0.0 : 1.0;
    L.in = (const double*)u[d];
    L.out = b;
    PD_HIP(c, pdk::launch_line(L, s));
  }
  return PD_OK;
}

// u_d -= scale dt/h_d M^-1 (R~ q[i+1] - L~ q[i])
int project_velocity(pd_ctx* c, const double* q, void* const u[3], hipStream_t s,
                     double scale = 1.0) {
  const int n = c->n;
  for (int d = 0; d < c->dim; ++d) {
    if (!u[d]) return fail(c, PD_EINVAL, "null velocity component");
    pdk::LineLaunch L;
    fill_line_common(c, &L);
    for (int p = 0; p < n; ++p)
      for (int r = 0; r < n; ++r) {
        L.A0[p * n + r] = c->tab.Rt[p * n + r] / c->tab.w[p];
        L.A1[p * n + r] = -c->tab.Lt[p * n + r] / c->tab.w[p];
      }
    L.d = d;
    L.o0 = 1;
    L.o1 = 0;
    L.coef = -scale * c->dt / c->h[d];
    L.accum = 1.0;
    L.in = q;
    L.out = (double*)u[d];
    PD_HIP(c, pdk::launch_line(L, s));
  }
  return PD_OK;
}

// Transpose of a two-cell line operator out_i = A0 in_{i+o0} + A1 in_{i+o1} (times coef and the
// transverse weights, both diagonal): out_j = A0^T in_{j-o0} + A1^T in_{j-o1}.
void transpose_line(pdk::LineLaunch* L) {
  const int n = L->N + 1;
  double t0[81], t1[81];
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      t0[q * n + p] = L->A0[p * n + q];
      t1[q * n + p] = L->A1[p * n + q];
    }
  for (int i = 0; i < n * n; ++i) {
    L->A0[i] = t0[i];
    L->A1[i] = t1[i];
  }
  L->o0 = -L->o0;
  L->o1 = -L->o1;
}

// Transpose of pi_{*->#} (dir 0) or pi_{#->*} (dir 1) along d.
int l2_project_T(pd_ctx* c, int d, int dir, const double* in, double* out, hipStream_t s) {
  pdk::LineLaunch L;
  fill_line_common(c, &L);
  const int n = c->n;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      L.A0[p * n + q] = c->tab.ML[p * n + q] / c->tab.w[p];
      L.A1[p * n + q] = c->tab.MR[p * n + q] / c->tab.w[p];
    }
  L.d = d;
  L.o0 = dir == 0 ? -1 : 0;
  L.o1 = dir == 0 ? 0 : 1;
  L.coef = 1.0;
  transpose_line(&L);
  L.in = in;
  L.out = out;
  PD_HIP(c, pdk::launch_line(L, s));
  return PD_OK;
}

// ubar_d = accum ubar_d + B_d^T bbar (B_d^T = h_d^-1 W_perp D_d: main -> dual of direction d)
int rhs_div_T(pd_ctx* c, const double* bbar, void* const ubar[3], double accum, hipStream_t s) {
  const int n = c->n;
  for (int d = 0; d < c->dim; ++d) {
    if (!ubar[d]) return fail(c, PD_EINVAL, "null velocity component");
    pdk::LineLaunch L;
    fill_line_common(c, &L);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        L.A0[p * n + q] = c->tab.Rt[q * n + p];
        L.A1[p * n + q] = -c->tab.Lt[q * n + p];
      }
    L.d = d;
    L.o0 = -1;
    L.o1 = 0;
    L.coef = 1.0 / c->h[d];
    L.wperp = 1;
    transpose_line(&L);
    L.accum = accum;
    L.in = bbar;
    L.out = (double*)ubar[d];
    PD_HIP(c, pdk::launch_line(L, s));
  }
  return PD_OK;
}

// qbar = -sum_d G_d^T ubar_d (G_d = dt h_d^-1 M_d^-1 D_d: the velocity update's gradient)
int project_velocity_T(pd_ctx* c, void* const ubar[3], double* qbar, hipStream_t s) {
  const int n = c->n;
  for (int d = 0; d < c->dim; ++d) {
    if (!ubar[d]) return fail(c, PD_EINVAL, "null velocity component");
    pdk::LineLaunch L;
    fill_line_common(c, &L);
    for (int p = 0; p < n; ++p)
      for (int r = 0; r < n; ++r) {
        L.A0[p * n + r] = c->tab.Rt[p * n + r] / c->tab.w[p];
        L.A1[p * n + r] = -c->tab.Lt[p * n + r] / c->tab.w[p];
      }
    L.d = d;
    L.o0 = 1;
    L.o1 = 0;
    L.coef = -c->dt / c->h[d];
    transpose_line(&L);
    L.accum = d == 0 ? 0.0 : 1.0;
    L.in = (const double*)ubar[d];
    L.out = qbar;
    PD_HIP(c, pdk::launch_line(L, s));
  }
  return PD_OK;
}

int ensure_step_buffers(pd_ctx* c) {
  const size_t n = (size_t)c->ndof;
  for (int d = 0; d < c->dim; ++d) {
    int rc;
    if ((rc = dev_alloc(c, &c->um[d], n))) return rc;
    if ((rc = dev_alloc(c, &c->s1[d], n))) return rc;
    if ((rc = dev_alloc(c, &c->s2[d], n))) return rc;
  }
  return dev_alloc(c, &c->qbuf, n);
}

int ensure_st_buffers(pd_ctx* c, int m) {
  const size_t n = (size_t)c->ndof;
  int rc;
  for (int q = 0; q < m; ++q) {
    for (int d = 0; d < c->dim; ++d)
      if ((rc = dev_alloc(c, &c->stU[q][d], n)) || (rc = dev_alloc(c, &c->stR[q][d], n)) ||
          (rc = dev_alloc(c, &c->stW[q][d], n)))
        return rc;
    if ((rc = dev_alloc(c, &c->stdP[q], n))) return rc;
  }
  for (int d = 0; d < c->dim; ++d)
    if ((rc = dev_alloc(c, &c->stum0[d], n)) || (rc = dev_alloc(c, &c->sta[d], n)) ||
        (rc = dev_alloc(c, &c->stb[d], n)))
      return rc;
  return dev_alloc(c, &c->strhs, n);
}

int ensure_adjoint_buffers(pd_ctx* c) {
  int rc = ensure_step_buffers(c);
  if (rc) return rc;
  const size_t n = (size_t)c->ndof;
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < c->dim; ++d)
      if ((rc = dev_alloc(c, &c->at[k][d], n))) return rc;
  return dev_alloc(c, &c->abar, n);
}

void fill_conv_common(const pd_ctx* c, pdk::ConvLaunch* L) {
  L->dim = c->dim;
  L->N = c->N;
  for (int d = 0; d < 3; ++d) {
    L->nc[d] = c->nc[d];
    L->h[d] = c->h[d];
  }
  const int n = c->n;
  for (int i = 0; i < 9; ++i) {
    L->w[i] = i < n ? c->tab.w[i] : 0;
    L->phi0[i] = i < n ? c->tab.phi0[i] : 0;
    L->phi1[i] = i < n ? c->tab.phi1[i] : 0;
  }
  for (int i = 0; i < 81; ++i) L->Kv[i] = i < n * n ? c->tab.Kv[i] : 0;
  L->dt = c->dt;
  L->nu = c->explicit_visc ? c->nu : 0.0;
  L->conv = c->convection;
  for (int i = 0; i < 9; ++i) {
    L->dphi0[i] = i < n ? c->tab.dphi0[i] : 0;
    L->dphi1[i] = i < n ? c->tab.dphi1[i] : 0;
  }
  for (int i = 0; i < 81; ++i) L->KD[i] = i < n * n ? c->tab.KD[i] : 0;
}

// Viscous part of the CFL condition of the explicit scheme (eq. CFL with CFL = 1):
// dt (2N+1)^2 sum_d 2 nu / h_d^2 <= 1.
bool explicit_visc_stable(const pd_ctx* c) {
  double s = 0.0;
  for (int d = 0; d < c->dim; ++d) s += 2.0 * c->nu / (c->h[d] * c->h[d]);
  return c->dt * (2.0 * c->N + 1.0) * (2.0 * c->N + 1.0) * s <= 1.0;
}

// The first two Shu-Osher stages: s1 = U + dt L(U); s2 = 3/4 U + 1/4 (s1 + dt L(s1)).
int rk_stages12(pd_ctx* c, double* const um[3], double* const s1[3], double* const s2[3],
                hipStream_t s) {
  pdk::ConvLaunch L;
  fill_conv_common(c, &L);
  for (int d = 0; d < c->dim; ++d) {
    L.ucur[d] = um[d];
    L.u0[d] = um[d];
    L.out[d] = s1[d];
  }
  L.a = 0.0;
  L.b = 1.0;
  PD_HIP(c, pdk::launch_convect_stage(L, s));
  for (int d = 0; d < c->dim; ++d) {
    L.ucur[d] = s1[d];
    L.out[d] = s2[d];
  }
  L.a = 0.75;
  L.b = 0.25;
  PD_HIP(c, pdk::launch_convect_stage(L, s));
  return PD_OK;
}

int convect(pd_ctx* c, double* const um[3], hipStream_t s) {
  // Shu-Osher TVD RK3: U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
  //                    U  = 1/3 U + 2/3 (U2 + dt L(U2))
  int rc = rk_stages12(c, um, c->s1, c->s2, s);
  if (rc) return rc;
  pdk::ConvLaunch L;
  fill_conv_common(c, &L);
  for (int d = 0; d < c->dim; ++d) {
    L.ucur[d] = c->s2[d];
    L.u0[d] = um[d];
    L.out[d] = um[d];
  }
  L.a = 1.0 / 3.0;
  L.b = 2.0 / 3.0;
  PD_HIP(c, pdk::launch_convect_stage(L, s));
  return PD_OK;
}

// Adjoint of the three RK stages at the forward states U (um), U1 (s1), U2 (s2): given the
// cotangent fbar of the RK3 result, write the cotangent of U into out. Work vectors: wa, wb
// (fbar, wa, wb and out distinct). In reverse stage order:
//   U2bar = 2/3 (fbar + dt J(U2)^T fbar),        Ubar  = 1/3 fbar
//   U1bar = 1/4 (U2bar + dt J(U1)^T U2bar),      Ubar += 3/4 U2bar
//   Ubar += U1bar + dt J(U)^T U1bar
int convect_adjoint(pd_ctx* c, double* const um[3], double* const s1[3], double* const s2[3],
                    double* const fbar[3], double* const wa[3], double* const wb[3],
                    double* const out[3], hipStream_t s) {
  const long long n = c->ndof;
  pdk::ConvAdjLaunch L;
  L.dim = c->dim;
  L.N = c->N;
  for (int d = 0; d < 3; ++d) {
    L.nc[d] = c->nc[d];
    L.h[d] = c->h[d];
  }
  const int nn = c->n;
  for (int i = 0; i < 9; ++i) {
    L.w[i] = i < nn ? c->tab.w[i] : 0;
    L.phi0[i] = i < nn ? c->tab.phi0[i] : 0;
    L.phi1[i] = i < nn ? c->tab.phi1[i] : 0;
  }
  for (int i = 0; i < 81; ++i) L.Kv[i] = i < nn * nn ? c->tab.Kv[i] : 0;
  L.dt = c->dt;
  for (int d = 0; d < c->dim; ++d) {
    L.state[d] = s2[d];
    L.obar[d] = fbar[d];
    L.acc[d] = nullptr;
    L.out[d] = wa[d];
  }
  L.acc_coef = 0.0;
  L.b = 2.0 / 3.0;
  PD_HIP(c, pdk::launch_convect_adj_stage(L, s));
  for (int d = 0; d < c->dim; ++d)
    PD_HIP(c, pdk::launch_axpby(1.0 / 3.0, fbar[d], 0.0, out[d], n, s));
  for (int d = 0; d < c->dim; ++d) {
    L.state[d] = s1[d];
    L.obar[d] = wa[d];
    L.out[d] = wb[d];
  }
  L.b = 0.25;
  PD_HIP(c, pdk::launch_convect_adj_stage(L, s));
  for (int d = 0; d < c->dim; ++d)
    PD_HIP(c, pdk::launch_axpby(0.75, wa[d], 1.0, out[d], n, s));
  for (int d = 0; d < c->dim; ++d) {
    L.state[d] = um[d];
    L.obar[d] = wb[d];
    L.acc[d] = out[d];
    L.out[d] = out[d];
  }
  L.acc_coef = 1.0;
  L.b = 1.0;
  PD_HIP(c, pdk::launch_convect_adj_stage(L, s));
  return PD_OK;
}

}  // namespace

extern "C" {

int pd_setup(pd_ctx** out, int dim, const int ncell[3], const double len[3], int N, double dt,
             double theta, double nu, unsigned periodic_mask, void* hip_stream) {
  if (!out) return fail(nullptr, PD_EINVAL, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(nullptr, PD_EINVAL, "dim must be 2 or 3");
  if (!ncell || !len) return fail(nullptr, PD_EINVAL, "ncell/len is NULL");
  for (int d = 0; d < dim; ++d) {
    if (ncell[d] < 1) return fail(nullptr, PD_EINVAL, "ncell[d] must be >= 1");
    if (!(len[d] > 0.0)) return fail(nullptr, PD_EINVAL, "len[d] must be > 0");
  }
  if (!(dt > 0.0)) return fail(nullptr, PD_EINVAL, "dt must be > 0");
  if (!(theta >= 0.5 && theta <= 1.0)) return fail(nullptr, PD_EINVAL, "theta must be in [0.5, 1]");
  if (!(nu >= 0.0)) return fail(nullptr, PD_EINVAL, "nu must be >= 0");
  const unsigned need = (1u << dim) - 1u;
  if (periodic_mask & ~need)
    return fail(nullptr, PD_EINVAL, "periodic_mask has bits beyond dim");
  pd_ctx* c = new pd_ctx();
  std::string e;
  if (!pdh::build_table(N, &c->tab, &e)) {
    delete c;
    return fail(nullptr, PD_EINVAL, e);
  }
  c->dim = dim;
  c->N = N;
  c->n = N + 1;
  for (int d = 0; d < 3; ++d) c->per[d] = d < dim ? (int)((periodic_mask >> d) & 1u) : 1;
  c->periodic = (periodic_mask & need) == need;
  c->NC = dim == 3 ? c->n * c->n * c->n : c->n * c->n;
  c->ncells = 1;
  for (int d = 0; d < dim; ++d) {
    c->nc[d] = ncell[d];
    c->len[d] = len[d];
    c->h[d] = len[d] / ncell[d];
    c->ncells *= ncell[d];
  }
  c->ndof = c->ncells * c->NC;
  if (c->ncells > (1LL << 31) / 2) {
    delete c;
    return fail(nullptr, PD_EINVAL, "grid too large");
  }
  // one operator launch holds at most kMaxPartials workgroups (2D grids always fit: workgroups
  // take more tiles; a 3D workgroup owns one column of cells, so the columns must fit)
  for (int f = 0; f < 2; ++f) {
    pdk::ApplyLaunch L;
    L.dim = dim;
    L.N = N;
    for (int d = 0; d < 3; ++d) L.nc[d] = d < dim ? ncell[d] : 1;
    L.fp32 = f == 1;
    if (pdk::apply_blocks(L) > (unsigned)pdk::kMaxPartials) {
      delete c;
      return fail(nullptr, PD_EINVAL,
                  "grid too large: more cell columns than one operator launch holds");
    }
  }
  c->dt = dt;
  c->theta = theta;
  c->nu = nu;
  for (int i = 0; i < c->n * c->n; ++i) {
    c->optab.L[i] = c->tab.Lb[i];
    c->optab.C[i] = c->tab.Cb[i];
    c->optab.R[i] = c->tab.Rb[i];
  }
  for (int i = 0; i < c->n; ++i) c->optab.w[i] = c->tab.w[i];
  const size_t n = (size_t)c->ndof;
  int rc = PD_OK;
  if ((rc = dev_alloc(c, &c->st, 1)) || (rc = dev_alloc(c, &c->st2, 1)) ||
      (rc = dev_alloc(c, &c->rhopart, 2 * (size_t)pdk::kMaxStreamPartials)) ||
      (rc = dev_alloc(c, &c->sigpart, pdk::kMaxPartials)) ||
      (rc = dev_alloc(c, &c->tmppart, pdk::kMaxStreamPartials)) ||
      (rc = dev_alloc(c, &c->null_part, (size_t)256 * c->NC)) ||
      (rc = dev_alloc(c, &c->null_corr, (size_t)c->NC)) || (rc = dev_alloc(c, &c->r64, n)) ||
      (rc = dev_alloc(c, &c->pa64, n)) || (rc = dev_alloc(c, &c->pb64, n)) ||
      (rc = dev_alloc(c, &c->q64, n)) || (rc = dev_alloc(c, &c->bw64, n)) ||
      (rc = dev_alloc(c, &c->r32, n)) || (rc = dev_alloc(c, &c->pa32, n)) ||
      (rc = dev_alloc(c, &c->pb32, n)) || (rc = dev_alloc(c, &c->q32, n)) ||
      (rc = dev_alloc(c, &c->d32, n))) {
    g_setup_err = c->err;
    pd_destroy(c);
    return rc;
  }
  hipStream_t s = S(hip_stream);
  hipError_t he = hipHostMalloc((void**)&c->hst, 2 * sizeof(CgState), hipHostMallocDefault);
  if (he == hipSuccess) he = hipEventCreate(&c->ev[0]);
  if (he == hipSuccess) he = hipEventCreate(&c->ev[1]);
  if (he == hipSuccess) he = hipEventCreate(&c->t0);
  if (he == hipSuccess) he = hipEventCreate(&c->t1);
  if (he == hipSuccess) he = hipMemsetAsync(c->st, 0, sizeof(CgState), s);
  if (he == hipSuccess) he = hipMemsetAsync(c->st2, 0, sizeof(CgState), s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  double* scratch_dev = nullptr;   // fixed scratch of pd_project_null_noalloc on this device
  if (he == hipSuccess) he = pdk::noalloc_scratch(&scratch_dev);
  if (he != hipSuccess) {
    g_setup_err = std::string("setup: ") + hipGetErrorString(he);
    pd_destroy(c);
    return PD_EDEVICE;
  }
  c->last_stream = s;
  *out = c;
  return PD_OK;
}

void pd_destroy(pd_ctx* c) {
  if (!c) return;
  if (c->last_stream) (void)hipStreamSynchronize(c->last_stream);
  (void)hipDeviceSynchronize();
  void* bufs[] = {c->st, c->st2, c->rhopart, c->sigpart, c->tmppart, c->null_part, c->null_corr,
                  c->r64, c->pa64, c->pb64, c->q64, c->bw64, c->r32, c->pa32, c->pb32, c->q32,
                  c->d32, c->qbuf, c->r64b, c->q64b, c->fpart, c->r32b, c->q32b, c->z64,
                  c->z32, c->rrpart};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (int d = 0; d < 3; ++d) {
    if (c->um[d]) (void)hipFree(c->um[d]);
    if (c->s1[d]) (void)hipFree(c->s1[d]);
    if (c->s2[d]) (void)hipFree(c->s2[d]);
    for (int k = 0; k < 4; ++k)
      if (c->at[k][d]) (void)hipFree(c->at[k][d]);
  }
  if (c->abar) (void)hipFree(c->abar);
  for (int q = 0; q < pdh::kMaxm; ++q) {
    for (int d = 0; d < 3; ++d) {
      if (c->stU[q][d]) (void)hipFree(c->stU[q][d]);
      if (c->stR[q][d]) (void)hipFree(c->stR[q][d]);
      if (c->stW[q][d]) (void)hipFree(c->stW[q][d]);
    }
    if (c->stdP[q]) (void)hipFree(c->stdP[q]);
  }
  for (int d = 0; d < 3; ++d) {
    if (c->stum0[d]) (void)hipFree(c->stum0[d]);
    if (c->sta[d]) (void)hipFree(c->sta[d]);
    if (c->stb[d]) (void)hipFree(c->stb[d]);
  }
  if (c->strhs) (void)hipFree(c->strhs);
  if (c->hst) (void)hipHostFree(c->hst);
  for (int i = 0; i < 2; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  delete c;
}

const char* pd_last_error(const pd_ctx* c) { return c ? c->err.c_str() : g_setup_err.c_str(); }

int pd_sizes(const pd_ctx* c, long long* ncells, long long* ndof, int* dim) {
  if (!c) return PD_EINVAL;
  if (ncells) *ncells = c->ncells;
  if (ndof) *ndof = c->ndof;
  if (dim) *dim = c->dim;
  return PD_OK;
}

int pd_nodes(const pd_ctx* c, double* xi, double* w) {
  if (!c) return PD_EINVAL;
  for (int i = 0; i < c->n; ++i) {
    if (xi) xi[i] = c->tab.xi[i];
    if (w) w[i] = c->tab.w[i];
  }
  return PD_OK;
}

int pd_table_1d(int N, int which, double* out) {
  if (!out || which < PD_TAB_NODES || which > PD_TAB_PLAM) return PD_EINVAL;
  pdh::Table1D t;
  std::string e;
  if (!pdh::build_table(N, &t, &e)) return PD_EINVAL;
  const int n = t.n;
  const double* src = nullptr;
  int cnt = n * n;
  switch (which) {
    case PD_TAB_NODES: src = t.xi; cnt = n; break;
    case PD_TAB_WEIGHTS: src = t.w; cnt = n; break;
    case PD_TAB_L: src = t.Lb; break;
    case PD_TAB_C: src = t.Cb; break;
    case PD_TAB_R: src = t.Rb; break;
    case PD_TAB_PNULL_ODD: src = t.PnullOdd; break;
    case PD_TAB_PV: src = t.PV; break;
    case PD_TAB_PLAM: src = t.Plam; cnt = n; break;
    default: src = t.Pnull; break;
  }
  for (int i = 0; i < cnt; ++i) out[i] = src[i];
  return cnt;
}

int pd_apply(pd_ctx* c, int op, int prec, const void* x, void* y, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (op != PD_OP_PRESSURE && op != PD_OP_VISCOUS) return fail(c, PD_EINVAL, "unknown operator");
  if (prec != PD_FP64 && prec != PD_FP32) return fail(c, PD_EINVAL, "pd_apply: prec must be PD_FP64 or PD_FP32");
  if (!x || !y) return fail(c, PD_EINVAL, "null array");
  if (x == y) return fail(c, PD_EINVAL, "x and y must not alias");
  c->last_stream = S(hip_stream);
  return plain_apply(c, op, prec == PD_FP32, x, y, S(hip_stream));
}

int pd_cg_solve(pd_ctx* c, int op, int prec, const void* b, void* x, double rtol, int maxit,
                pd_solve_info* info, void* hip_stream) {
  if (!c) return PD_EINVAL;
  return solve(c, op, prec, (const double*)b, (double*)x, rtol, maxit, info, S(hip_stream));
}

int pd_rhs_div(pd_ctx* c, void* const u[3], void* b, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_rhs_div")) return rc0;
  if (!u || !b) return fail(c, PD_EINVAL, "null array");
  c->last_stream = S(hip_stream);
  return rhs_div(c, u, (double*)b, S(hip_stream));
}

int pd_project_velocity(pd_ctx* c, const void* q, void* const u[3], void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_project_velocity")) return rc0;
  if (!q || !u) return fail(c, PD_EINVAL, "null array");
  c->last_stream = S(hip_stream);
  return project_velocity(c, (const double*)q, u, S(hip_stream));
}

int pd_project_null(pd_ctx* c, int prec, void* v, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (!v) return fail(c, PD_EINVAL, "null array");
  if (prec != PD_FP64 && prec != PD_FP32) return fail(c, PD_EINVAL, "prec must be PD_FP64 or PD_FP32");
  c->last_stream = S(hip_stream);
  return project_null(c, prec == PD_FP32, v, S(hip_stream));
}

int pd_project_null_noalloc(pd_ctx* c, int prec, void* v, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (!v) return fail(c, PD_EINVAL, "null array");
  if (prec != PD_FP64 && prec != PD_FP32) return fail(c, PD_EINVAL, "prec must be PD_FP64 or PD_FP32");
  if ((size_t)(256 + 1) * c->NC * sizeof(double) > pdk::noalloc_scratch_bytes())
    return fail(c, PD_EINVAL, "pd_project_null_noalloc: (N+1)^dim exceeds the fixed scratch");
  c->last_stream = S(hip_stream);
  const double* P[3];
  if (!null_projectors(c, P)) return PD_OK;
  PD_HIP(c, pdk::launch_project_null_noalloc(prec == PD_FP32, v, c->ncells, c->dim, c->n, P,
                                             S(hip_stream)));
  return PD_OK;
}

int pd_l2_project(pd_ctx* c, int d, int dir, const void* in, void* out, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_l2_project")) return rc0;
  if (d < 0 || d >= c->dim || (dir != 0 && dir != 1)) return fail(c, PD_EINVAL, "bad direction");
  if (!in || !out || in == out) return fail(c, PD_EINVAL, "null or aliased array");
  c->last_stream = S(hip_stream);
  return l2_project(c, d, dir, (const double*)in, (double*)out, S(hip_stream));
}

int pd_convect(pd_ctx* c, void* const um[3], void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_convect")) return rc0;
  if (!um) return fail(c, PD_EINVAL, "null array");
  for (int d = 0; d < c->dim; ++d)
    if (!um[d]) return fail(c, PD_EINVAL, "null velocity component");
  int rc = ensure_step_buffers(c);
  if (rc) return rc;
  c->last_stream = S(hip_stream);
  double* m[3] = {(double*)um[0], (double*)um[1], c->dim == 3 ? (double*)um[2] : nullptr};
  return convect(c, m, S(hip_stream));
}

int pd_step(pd_ctx* c, void* const u[3], void* p, pd_solve_info info[4], void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_step")) return rc0;
  if (!u || !p) return fail(c, PD_EINVAL, "null array");
  for (int d = 0; d < c->dim; ++d)
    if (!u[d]) return fail(c, PD_EINVAL, "null velocity component");
  int rc = ensure_step_buffers(c);
  if (rc) return rc;
  hipStream_t s = S(hip_stream);
  c->last_stream = s;
  const long long n = c->ndof;
  pd_solve_info loc[4];
  std::memset(loc, 0, sizeof(loc));
  // 1. pi_{*->#}
  for (int d = 0; d < c->dim; ++d)
    if ((rc = l2_project(c, d, 0, (const double*)u[d], c->um[d], s))) return rc;
  const bool evisc = c->explicit_visc && c->nu > 0.0;
  if (evisc && !explicit_visc_stable(c))
    return fail(c, PD_EINVAL, "explicit viscosity: dt exceeds the viscous CFL limit "
                              "1 / ((2N+1)^2 sum_d 2 nu / h_d^2)");
  // 2. explicit convection (TVD RK3), with the viscous flux in the explicit-viscosity variant
  if (c->convection || evisc)
    if ((rc = convect(c, c->um, s))) return rc;
  // 3. implicit viscosity on the main grid: (M + nu dt K) U = M F, initial guess F
  if (c->nu > 0.0 && !c->explicit_visc) {
    for (int d = 0; d < c->dim; ++d) {
      PD_HIP(c, pdk::launch_mass(c->dim, c->N, c->tab.w, c->um[d], c->s1[d], c->ncells, s));
      rc = solve(c, PD_OP_VISCOUS, c->step_prec, c->s1[d], c->um[d], c->v_rtol, c->maxit, &loc[d], s);
      if (rc != PD_OK) {
        if (info) std::memcpy(info, loc, sizeof(loc));
        return rc;
      }
    }
  }
  // 4. pi_{#->*}
  for (int d = 0; d < c->dim; ++d)
    if ((rc = l2_project(c, d, 1, c->um[d], (double*)u[d], s))) return rc;
  // 5. b = sum_d B_d U*_d, pressure solve for q = P^{n+theta} from q = 0
  if ((rc = rhs_div(c, u, c->s2[0], s))) return rc;
  PD_HIP(c, pdk::launch_zero(false, c->qbuf, n, s));
  rc = solve(c, PD_OP_PRESSURE, c->step_prec, c->s2[0], c->qbuf, c->p_rtol, c->maxit, &loc[3], s);
  if (info) std::memcpy(info, loc, sizeof(loc));
  if (rc != PD_OK) return rc;
  // 6. velocity update, 7. P^{n+1} = (q - (1-theta) P^n) / theta
  if ((rc = project_velocity(c, c->qbuf, u, s))) return rc;
  PD_HIP(c, pdk::launch_axpby(1.0 / c->theta, c->qbuf, -(1.0 - c->theta) / c->theta, (double*)p, n, s));
  PD_HIP(c, hipStreamSynchronize(s));
  return PD_OK;
}

int pd_step_st(pd_ctx* c, int M, void* const u[3], void* p_nodes, pd_solve_info* info,
               void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_step_st")) return rc0;
  if (!u || !p_nodes) return fail(c, PD_EINVAL, "null array");
  for (int d = 0; d < c->dim; ++d) {
    if (!u[d] || u[d] == p_nodes) return fail(c, PD_EINVAL, "null or aliased velocity component");
    for (int e = 0; e < d; ++e)
      if (u[e] == u[d]) return fail(c, PD_EINVAL, "aliased velocity components");
  }
  pdh::TimeTable tt;
  std::string terr;
  if (!pdh::build_time_table(M, &tt, &terr)) return fail(c, PD_EINVAL, terr);
  const bool evisc = c->explicit_visc && c->nu > 0.0;
  if (M >= 1 && c->nu > 0.0 && !c->explicit_visc)
    return fail(c, PD_EINVAL, "pd_step_st: M >= 1 needs nu = 0 or PD_CFG_EXPLICIT_VISC (the "
                              "space-time implicit viscous solve is not provided)");
  if (evisc && !explicit_visc_stable(c))
    return fail(c, PD_EINVAL, "explicit viscosity: dt exceeds the viscous CFL limit "
                              "1 / ((2N+1)^2 sum_d 2 nu / h_d^2)");
  const int m = tt.m;
  int rc = ensure_step_buffers(c);
  if (rc || (rc = ensure_st_buffers(c, m))) return rc;
  hipStream_t s = S(hip_stream);
  c->last_stream = s;
  const long long n = c->ndof;
  const int dim = c->dim;
  pd_solve_info loc[3 + pdh::kMaxm * pdh::kMaxm];
  std::memset(loc, 0, sizeof(loc));
  double* P[pdh::kMaxm];
  for (int q = 0; q < m; ++q) P[q] = (double*)p_nodes + (size_t)q * n;
  auto report = [&](int count) {
    if (info) std::memcpy(info, loc, sizeof(pd_solve_info) * count);
  };
  // F^n of the first iteration: the semi-implicit predictor (pi_{*->#}, TVD-RK3 advection with
  // the explicit viscous flux in that variant, implicit viscous solve for M = 0), and
  // pi_{*->#} U^n for the advective term of the later iterations
  for (int d = 0; d < dim; ++d) {
    if ((rc = l2_project(c, d, 0, (const double*)u[d], c->um[d], s))) return rc;
    PD_HIP(c, pdk::launch_axpby(1.0, c->um[d], 0.0, c->stum0[d], n, s));
  }
  if (c->convection || evisc)
    if ((rc = convect(c, c->um, s))) return rc;
  if (c->nu > 0.0 && !c->explicit_visc) {
    for (int d = 0; d < dim; ++d) {
      PD_HIP(c, pdk::launch_mass(dim, c->N, c->tab.w, c->um[d], c->s1[d], c->ncells, s));
      rc = solve(c, PD_OP_VISCOUS, c->step_prec, c->s1[d], c->um[d], c->v_rtol, c->maxit, &loc[d], s);
      if (rc != PD_OK) {
        report(3);
        return rc;
      }
    }
  }
  for (int q = 0; q < m; ++q) PD_HIP(c, pdk::launch_zero(false, P[q], n, s));
  const int total = 3 + m * m;
  for (int k = 0; k < m; ++k) {
    // right-hand sides R_p of the momentum equations on the dual grids
    for (int p = 0; p < m; ++p) {
      if (k == 0) {
        for (int d = 0; d < dim; ++d)
          PD_HIP(c, pdk::launch_axpby(tt.psi0[p], c->um[d], 0.0, c->stb[d], n, s));
      } else {
        // psi_p(0) pi_{*->#} U^n + dt omega_p L(pi_{*->#} U_p)  (eq. Fu_ST at node p)
        for (int d = 0; d < dim; ++d)
          if ((rc = l2_project(c, d, 0, c->stU[p][d], c->sta[d], s))) return rc;
        pdk::ConvLaunch L;
        fill_conv_common(c, &L);
        for (int d = 0; d < dim; ++d) {
          L.ucur[d] = c->sta[d];
          L.u0[d] = c->stum0[d];
          L.out[d] = c->stb[d];
        }
        L.a = tt.psi0[p];
        L.cr = c->dt * tt.omega[p];
        if (c->convection || evisc) {
          PD_HIP(c, pdk::launch_convect_stage(L, s));
        } else {
          for (int d = 0; d < dim; ++d)
            PD_HIP(c, pdk::launch_axpby(tt.psi0[p], c->stum0[d], 0.0, c->stb[d], n, s));
        }
      }
      for (int d = 0; d < dim; ++d)
        if ((rc = l2_project(c, d, 1, c->stb[d], c->stR[p][d], s))) return rc;
      // pressure term of the current iterate on the dual grids: - omega_p G P_p
      if (k > 0)
        if ((rc = project_velocity(c, P[p], (void* const*)c->stR[p], s, tt.omega[p]))) return rc;
    }
    // decoupled pressure corrections: omega_s A_p dP_s = sum_d B_d R_{s,d}
    for (int q = 0; q < m; ++q) {
      if ((rc = rhs_div(c, (void* const*)c->stR[q], c->strhs, s))) return rc;
      PD_HIP(c, pdk::launch_axpby(1.0 / tt.omega[q], c->strhs, 0.0, c->strhs, n, s));
      PD_HIP(c, pdk::launch_zero(false, c->stdP[q], n, s));
      pd_solve_info* si = &loc[3 + k * m + q];
      rc = solve(c, PD_OP_PRESSURE, c->step_prec, c->strhs, c->stdP[q], c->p_rtol, c->maxit, si, s);
      if (rc != PD_OK) {
        report(total);
        return rc;
      }
      for (int d = 0; d < dim; ++d) PD_HIP(c, pdk::launch_zero(false, c->stW[q][d], n, s));
      if ((rc = project_velocity(c, c->stdP[q], (void* const*)c->stW[q], s))) return rc;   // -G dP
      PD_HIP(c, pdk::launch_axpby(1.0, c->stdP[q], 1.0, P[q], n, s));
    }
    // U_s = sum_p Ainv[s][p] (R_p + omega_p W_p), W_p = -G dP_p
    for (int d = 0; d < dim; ++d) {
      pdk::TimeMix X;
      X.m = X.mo = m;
      for (int q = 0; q < m; ++q) {
        X.in[q] = c->stR[q][d];
        X.out[q] = c->stU[q][d];
      }
      for (int i = 0; i < m * m; ++i) X.T[i] = tt.Ainv[i];
      PD_HIP(c, pdk::launch_time_mix(X, n, s));
      pdk::TimeMix Y;
      Y.m = Y.mo = m;
      Y.bc = 1.0;
      for (int q = 0; q < m; ++q) {
        Y.in[q] = c->stW[q][d];
        Y.base[q] = c->stU[q][d];
        Y.out[q] = c->stU[q][d];
      }
      for (int q = 0; q < m; ++q)
        for (int p = 0; p < m; ++p) Y.T[q * m + p] = tt.Ainv[q * m + p] * tt.omega[p];
      PD_HIP(c, pdk::launch_time_mix(Y, n, s));
    }
  }
  // slab end value u(t^{n+1}) = sum_s psi_s(1) U_s
  for (int d = 0; d < dim; ++d) {
    pdk::TimeMix X;
    X.m = m;
    X.mo = 1;
    for (int q = 0; q < m; ++q) {
      X.in[q] = c->stU[q][d];
      X.T[q] = tt.psi1[q];
    }
    X.out[0] = (double*)u[d];
    PD_HIP(c, pdk::launch_time_mix(X, n, s));
  }
  report(total);
  PD_HIP(c, hipStreamSynchronize(s));
  return PD_OK;
}

int pd_time_table(int M, int which, double* out) {
  pdh::TimeTable t;
  if (!out || !pdh::build_time_table(M, &t, nullptr)) return PD_EINVAL;
  const int m = t.m;
  const double* src = nullptr;
  int cnt = m;
  switch (which) {
    case PD_TTAB_NODES: src = t.tau; break;
    case PD_TTAB_WEIGHTS: src = t.omega; break;
    case PD_TTAB_PSI0: src = t.psi0; break;
    case PD_TTAB_PSI1: src = t.psi1; break;
    case PD_TTAB_MV: src = t.MV; cnt = m * m; break;
    case PD_TTAB_AINV: src = t.Ainv; cnt = m * m; break;
    default: return PD_EINVAL;
  }
  for (int i = 0; i < cnt; ++i) out[i] = src[i];
  return cnt;
}

int pd_l2_project_adjoint(pd_ctx* c, int d, int dir, const void* in, void* out,
                          void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_l2_project_adjoint")) return rc0;
  if (d < 0 || d >= c->dim || (dir != 0 && dir != 1)) return fail(c, PD_EINVAL, "bad direction");
  if (!in || !out || in == out) return fail(c, PD_EINVAL, "null or aliased array");
  c->last_stream = S(hip_stream);
  return l2_project_T(c, d, dir, (const double*)in, (double*)out, S(hip_stream));
}

int pd_rhs_div_adjoint(pd_ctx* c, const void* bbar, void* const ubar[3], void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_rhs_div_adjoint")) return rc0;
  if (!bbar || !ubar) return fail(c, PD_EINVAL, "null array");
  c->last_stream = S(hip_stream);
  return rhs_div_T(c, (const double*)bbar, ubar, 0.0, S(hip_stream));
}

int pd_project_velocity_adjoint(pd_ctx* c, void* const ubar[3], void* qbar, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_project_velocity_adjoint")) return rc0;
  if (!ubar || !qbar) return fail(c, PD_EINVAL, "null array");
  c->last_stream = S(hip_stream);
  return project_velocity_T(c, ubar, (double*)qbar, S(hip_stream));
}

int pd_convect_adjoint(pd_ctx* c, void* const um[3], void* const ubar[3], void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_convect_adjoint")) return rc0;
  if (c->explicit_visc)
    return fail(c, PD_EINVAL, "the adjoint covers the convective flux only (PD_CFG_EXPLICIT_VISC set)");
  if (!um || !ubar) return fail(c, PD_EINVAL, "null array");
  for (int d = 0; d < c->dim; ++d)
    if (!um[d] || !ubar[d] || um[d] == ubar[d]) return fail(c, PD_EINVAL, "null or aliased component");
  int rc = ensure_adjoint_buffers(c);
  if (rc) return rc;
  hipStream_t s = S(hip_stream);
  c->last_stream = s;
  const long long n = c->ndof;
  double* u0[3] = {(double*)um[0], (double*)um[1], c->dim == 3 ? (double*)um[2] : nullptr};
  if ((rc = rk_stages12(c, u0, c->s1, c->s2, s))) return rc;
  // the cotangent is read from ubar into a work vector, the result written back into ubar
  for (int d = 0; d < c->dim; ++d)
    PD_HIP(c, pdk::launch_axpby(1.0, (const double*)ubar[d], 0.0, c->at[0][d], n, s));
  double* out[3] = {(double*)ubar[0], (double*)ubar[1], c->dim == 3 ? (double*)ubar[2] : nullptr};
  return convect_adjoint(c, u0, c->s1, c->s2, c->at[0], c->at[1], c->at[2], out, s);
}

int pd_step_adjoint(pd_ctx* c, void* const u[3], void* const ubar[3], pd_solve_info info[4],
                    void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_step_adjoint")) return rc0;
  if (!u || !ubar) return fail(c, PD_EINVAL, "null array");
  for (int d = 0; d < c->dim; ++d)
    if (!u[d] || !ubar[d] || u[d] == ubar[d]) return fail(c, PD_EINVAL, "null or aliased component");
  if (c->explicit_visc)
    return fail(c, PD_EINVAL, "the adjoint covers the implicit-viscosity step only");
  int rc = ensure_adjoint_buffers(c);
  if (rc) return rc;
  hipStream_t s = S(hip_stream);
  c->last_stream = s;
  const long long n = c->ndof;
  pd_solve_info loc[4];
  std::memset(loc, 0, sizeof(loc));
  for (int d = 0; d < 4; ++d) loc[d].fallback_iter = -1;
  double* T1[3] = {c->at[0][0], c->at[0][1], c->at[0][2]};
  double* T2[3] = {c->at[1][0], c->at[1][1], c->at[1][2]};
  double* T3[3] = {c->at[2][0], c->at[2][1], c->at[2][2]};
  double* T4[3] = {c->at[3][0], c->at[3][1], c->at[3][2]};
  // forward states of the step's convection: U = pi_{*->#} U^n, and the RK stage inputs
  for (int d = 0; d < c->dim; ++d)
    if ((rc = l2_project(c, d, 0, (const double*)u[d], c->um[d], s))) return rc;
  if (c->convection)
    if ((rc = rk_stages12(c, c->um, c->s1, c->s2, s))) return rc;
  // 6: U^{n+1}_d = U*_d - G_d q  ->  qbar = -sum_d G_d^T ubar_d
  if ((rc = project_velocity_T(c, ubar, c->qbuf, s))) return rc;
  // 5: q = A_p^+ b (symmetric)  ->  bbar = A_p^+ qbar
  PD_HIP(c, pdk::launch_zero(false, c->abar, n, s));
  rc = solve(c, PD_OP_PRESSURE, c->step_prec, c->qbuf, c->abar, c->p_rtol, c->maxit, &loc[3], s);
  if (rc != PD_OK) {
    if (info) std::memcpy(info, loc, sizeof(loc));
    return rc;
  }
  // b = sum_d B_d U*_d  ->  U*bar_d = ubar_d + B_d^T bbar
  for (int d = 0; d < c->dim; ++d)
    PD_HIP(c, pdk::launch_axpby(1.0, (const double*)ubar[d], 0.0, T1[d], n, s));
  void* t1v[3] = {T1[0], T1[1], T1[2]};
  if ((rc = rhs_div_T(c, c->abar, t1v, 1.0, s))) return rc;
  // 4: U*_d = pi_{#->*} U#_d
  for (int d = 0; d < c->dim; ++d)
    if ((rc = l2_project_T(c, d, 1, T1[d], T2[d], s))) return rc;
  // 3: U#_d = A_v^-1 M F_d  ->  Fbar_d = M A_v^-1 U#bar_d (A_v symmetric, M diagonal)
  double** fbar = T2;
  if (c->nu > 0.0) {
    for (int d = 0; d < c->dim; ++d) {
      PD_HIP(c, pdk::launch_zero(false, T3[d], n, s));
      rc = solve(c, PD_OP_VISCOUS, c->step_prec, T2[d], T3[d], c->v_rtol, c->maxit, &loc[d], s);
      if (rc != PD_OK) {
        if (info) std::memcpy(info, loc, sizeof(loc));
        return rc;
      }
      PD_HIP(c, pdk::launch_mass(c->dim, c->N, c->tab.w, T3[d], T1[d], c->ncells, s));
    }
    fbar = T1;
  }
  // 2: F = RK3(U)  ->  Ubar = RK3 adjoint at the forward stages (um, s1, s2)
  double** ubm = fbar;
  if (c->convection) {
    double** wa = fbar == T1 ? T2 : T1;
    if ((rc = convect_adjoint(c, c->um, c->s1, c->s2, fbar, wa, T3, T4, s))) return rc;
    ubm = T4;
  }
  // 1: U_d = pi_{*->#} U^n_d  ->  ubar_d = pi_{*->#}^T Ubar_d
  for (int d = 0; d < c->dim; ++d)
    if ((rc = l2_project_T(c, d, 0, ubm[d], (double*)ubar[d], s))) return rc;
  if (info) std::memcpy(info, loc, sizeof(loc));
  PD_HIP(c, hipStreamSynchronize(s));
  return PD_OK;
}

int pd_kinetic_energy(pd_ctx* c, void* const u[3], double gscale, void* const grad[3],
                      double* energy, void* hip_stream) {
  if (!c) return PD_EINVAL;
  if (int rc0 = require_periodic(c, "pd_kinetic_energy")) return rc0;
  if (!u || !energy) return fail(c, PD_EINVAL, "null argument");
  if (!std::isfinite(gscale)) return fail(c, PD_EINVAL, "gscale must be finite");
  for (int d = 0; d < c->dim; ++d) {
    if (!u[d]) return fail(c, PD_EINVAL, "null velocity component");
    if (grad && !grad[d]) return fail(c, PD_EINVAL, "null gradient component");
    if (grad)
      for (int e = 0; e < c->dim; ++e)
        if (grad[d] == u[e]) return fail(c, PD_EINVAL, "grad must not alias u");
  }
  hipStream_t s = S(hip_stream);
  c->last_stream = s;
  const double* uu[3] = {nullptr, nullptr, nullptr};
  double* gg[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < c->dim; ++d) {
    uu[d] = (const double*)u[d];
    if (grad) gg[d] = (double*)grad[d];
  }
  // (1/|Omega|) int |v|^2/2 with |cell|/|Omega| = 1/ncells on the uniform grid
  const double inv_cells = 1.0 / (double)c->ncells;
  PD_HIP(c, pdk::launch_energy(c->dim, c->N, c->tab.w, uu, grad ? gg : nullptr,
                               gscale * inv_cells, c->ncells, c->tmppart, s));
  PD_HIP(c, pdk::launch_finalize(c->tmppart, (int)pdk::stream_grid(c->ndof), c->st2,
                                 pdk::FIN_AUX, s));
  CgState h;
  int rc = read_state(c, c->st2, &h, s);
  if (rc) return rc;
  *energy = 0.5 * inv_cells * h.aux;
  return PD_OK;
}

int pd_configure(pd_ctx* c, int key, double v) {
  if (!c) return PD_EINVAL;
  constexpr double kMaxIntSetting = 1 << 30;   // integer settings are converted with (int)
  switch (key) {
    case PD_CFG_STEP_PREC:
      if (v != PD_FP64 && v != PD_FP32_REFINE64) return fail(c, PD_EINVAL, "bad step precision");
      c->step_prec = (int)v;
      break;
    case PD_CFG_P_RTOL:
      if (!(v > 0)) return fail(c, PD_EINVAL, "rtol must be > 0");
      c->p_rtol = v;
      break;
    case PD_CFG_V_RTOL:
      if (!(v > 0)) return fail(c, PD_EINVAL, "rtol must be > 0");
      c->v_rtol = v;
      break;
    case PD_CFG_MAXIT:
      if (!(v >= 0 && v <= kMaxIntSetting)) return fail(c, PD_EINVAL, "maxit must be in [0, 2^30]");
      c->maxit = (int)v;
      break;
    case PD_CFG_CONVECTION:
      c->convection = v != 0.0;
      break;
    case PD_CFG_RU_FACTOR:
      if (!(v > 0 && v < 1)) return fail(c, PD_EINVAL, "replacement factor must be in (0, 1)");
      c->ru_factor = v;
      break;
    case PD_CFG_TIMING:
      if (!(v >= 0.0 && v <= 1e6)) return fail(c, PD_EINVAL, "PD_CFG_TIMING must be in [0, 1e6]");
      c->timing = (int)v;
      break;
    case PD_CFG_CHECK_EVERY:
      if (!(v >= 1 && v <= 1 << 20)) return fail(c, PD_EINVAL, "check interval must be in [1, 2^20]");
      c->check_every = (int)v;
      break;
    case PD_CFG_KZ:
      if (!(v >= 0 && v <= kMaxIntSetting)) return fail(c, PD_EINVAL, "planes per segment must be in [0, 2^30]");
      c->kz = (int)v;
      break;
    case PD_CFG_TILES_PER_WG:
      if (!(v >= 0 && v <= kMaxIntSetting)) return fail(c, PD_EINVAL, "tiles per workgroup must be in [0, 2^30]");
      c->tiles_per_wg = (int)v;
      break;
    case PD_CFG_PREFETCH:
      c->prefetch = v != 0.0;
      break;
    case PD_CFG_TILE_VARIANT:
      if (!(v == 0 || v == 1 || v == 2)) return fail(c, PD_EINVAL, "tile variant must be 0, 1 or 2");
      c->tile_variant = (int)v;
      break;
    case PD_CFG_DEFER_X:
      if (!(v == 0 || v == 1)) return fail(c, PD_EINVAL, "PD_CFG_DEFER_X must be 0 or 1");
      c->defer_x = (int)v;
      break;
    case PD_CFG_PRECOND:
      if (!(v == 0 || v == 1)) return fail(c, PD_EINVAL, "PD_CFG_PRECOND must be 0 or 1");
      if (v == 1) {
        const size_t n = (size_t)c->ndof;
        int rc = PD_OK;
        if ((rc = dev_alloc(c, &c->z64, n)) || (rc = dev_alloc(c, &c->z32, n)) ||
            (rc = dev_alloc(c, &c->rrpart, 2 * (size_t)pdk::kMaxStreamPartials)))
          return rc;
      }
      c->precond = (int)v;
      break;
    case PD_CFG_EXPLICIT_VISC:
      if (!(v == 0 || v == 1)) return fail(c, PD_EINVAL, "PD_CFG_EXPLICIT_VISC must be 0 or 1");
      c->explicit_visc = (int)v;
      break;
    case PD_CFG_ONE_KERNEL:
      if (!(v == 0 || v == 1)) return fail(c, PD_EINVAL, "PD_CFG_ONE_KERNEL must be 0 or 1");
      if (v == 1 && c->dim == 2 && !c->fpart) {
        // the form's second residual and A p buffers and its partials, on first use
        const size_t n = (size_t)c->ndof;
        int rc = PD_OK;
        if ((rc = dev_alloc(c, &c->r64b, n)) || (rc = dev_alloc(c, &c->q64b, n)) ||
            (rc = dev_alloc(c, &c->r32b, n)) || (rc = dev_alloc(c, &c->q32b, n)) ||
            (rc = dev_alloc(c, &c->fpart, 8 * (size_t)pdk::kMaxPartials)))
          return rc;
      }
      c->one_kernel = (int)v;
      break;
    default:
      return fail(c, PD_EINVAL, "unknown configuration key");
  }
  return PD_OK;
}

int pd_timing(pd_ctx* c, int prec, double* total_ms, long long* launches,
              double* bytes_per_launch, int reset) {
  if (!c) return PD_EINVAL;
  if (prec != PD_FP64 && prec != PD_FP32) return fail(c, PD_EINVAL, "prec must be PD_FP64 or PD_FP32");
  if (c->last_stream) PD_HIP(c, hipStreamSynchronize(c->last_stream));
  const int k = prec == PD_FP32 ? 1 : 0;
  if (total_ms) *total_ms = c->t_ms[k];
  if (launches) *launches = c->t_cnt[k];
  // fused CG apply: reads r and p_old, writes p and A p; with the deferred x update it also reads
  // and writes x (6 words per DoF, else 4)
  if (bytes_per_launch) *bytes_per_launch = c->t_words[k] * (double)c->ndof * (k ? 4.0 : 8.0);
  if (reset) {
    c->t_ms[k] = 0;
    c->t_cnt[k] = 0;
  }
  return PD_OK;
}

}  // extern "C"
