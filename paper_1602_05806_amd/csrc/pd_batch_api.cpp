// C-ABI of the batched 2D pressure solver: many independent periodic problems of uneven sizes and
// degrees solved together. The kernels are in pd_batch.hip; this file builds the per-problem
// descriptors and operator groups, picks tile shapes (an autotuner with a text cache), captures
// one chunk of iterations over the active problems into a HIP graph, replays it, and captures
// again over shorter lists as problems finish or change precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <string>
#include <vector>

#include "pd.h"
#include "pd_launch.h"
#include "pd_tables.h"

using pdk::BatchGroup;
using pdk::BatchIter;
using pdk::BProb;
using pdk::CgState;

namespace {

// Problem descriptors of one precision (tile shapes and sigma offsets differ by precision) and
// the operator groups over all problems.
struct PrecSet {
  std::vector<BProb> probs;
  std::vector<int> variants;
  BProb* d_probs = nullptr;
  double* sig = nullptr;         // sigma partials of this precision
  int sig_cap = 0;
};

// Device tables of one problem list: indices, cumulative streaming and node-sum blocks.
struct ListDev {
  const int* list = nullptr;
  const int* upd_off = nullptr;
  const int* ns_off = nullptr;
  int count = 0, upd_blocks = 0, ns_blocks = 0;
};

// Everything one captured chunk refers to: the lists of problems iterating in FP32 (act32) and
// in FP64 (act64), their union, and the operator groups over them. One device allocation.
struct Plan {
  int* dev = nullptr;
  ListDev l32, l64, lall;
  std::vector<BatchGroup> g32;     // FP32 fused iterations over act32
  std::vector<BatchGroup> gallr;   // FP64 residual apply over act32 + act64 (FP64 tile shapes)
  std::vector<BatchGroup> g64;     // FP64 fused iterations over act64
  std::vector<char> in64;          // membership of act64, by problem
  // the same lists split by degree (preconditioner launches, one per degree)
  std::vector<std::pair<int, ListDev>> n32, n64, nall;
  long long dofs = 0;              // active DoFs when captured
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool refine = false;
  int chunk = 0;
};

}  // namespace

struct pd_batch {
  int count = 0;
  double dt = 0.0;
  std::string err = "no error";
  std::vector<pdk::OpTables> tabs;          // by degree
  std::vector<int> N;
  std::vector<long long> off;               // packed offsets, count + 1
  long long total = 0;
  int chunk = 64;
  int use_graph = 1;
  double ru = 1e-2;                         // pause factor of the FP32 iterations
  PrecSet ps[2];                            // [0] FP64, [1] FP32
  Plan all[2];                              // start-of-solve plans (every problem): [FP64, refine]
  int* d_kbase = nullptr;
  CgState* st = nullptr;
  double *rho = nullptr, *tmp = nullptr, *nsp = nullptr, *corr = nullptr, *pnull = nullptr;
  double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr, *q64 = nullptr, *pa64 = nullptr,
         *pb64 = nullptr;
  float *r32 = nullptr, *pa32 = nullptr, *pb32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  // cell-block Jacobi preconditioned solves (PD_BCFG_PRECOND): z = P r per precision, partials
  // of <r, r> beside those of <r, z>, eigenbasis tables by degree (9 x 90)
  int precond = 0;
  double *z64 = nullptr, *res = nullptr;
  float* z32 = nullptr;
  std::vector<double> pv;                   // eigenbasis tables by degree: V[81], lambda[9]
  std::vector<std::pair<int, ListDev>> everyone_n;   // every problem, one list per degree
  int* d_everyone_n = nullptr;
  ListDev everyone;                         // every problem, in order
  int* d_everyone = nullptr;
  std::vector<BatchGroup> g64_all;          // FP64 groups over every problem (final residual)
  int* d_g64_all = nullptr;
  CgState* hst = nullptr;                   // pinned mirror of the states, 2 x count
  hipEvent_t ev[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
  hipStream_t cap = nullptr;                // private stream used only for graph capture
};

namespace {

std::string g_batch_err = "no error";

int bfail(pd_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  else g_batch_err = m;
  return code;
}

#define BHIP(b, call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail(b, PD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

template <typename T>
int balloc(pd_batch* b, T** p, size_t n) {
  hipError_t e = hipMalloc((void**)p, n * sizeof(T) + 256);
  if (e != hipSuccess) {
    *p = nullptr;
    return bfail(b, PD_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return PD_OK;
}

// streaming blocks of one problem (= its partials of <r, r>)
int stream_blocks_for(long long n) {
  long long g = (n + 256LL * 8 - 1) / (256LL * 8);
  if (g < 1) g = 1;
  if (g > pdk::kMaxStreamPartials) g = pdk::kMaxStreamPartials;
  return (int)g;
}

int size_bucket(int side) {
  int b = 1;
  while (b * 2 <= side) b *= 2;
  return b;
}

std::string tune_key(int N, int bucket, bool fp32) {
  return "gfx950:pressure2d:N" + std::to_string(N) + ":s" + std::to_string(bucket) +
         (fp32 ? ":fp32" : ":fp64");
}

std::map<std::string, int> load_cache() {
  std::map<std::string, int> m;
  const char* p = std::getenv("PD_AUTOTUNE_CACHE");
  if (!p || !*p) return m;
  std::ifstream f(p);
  std::string key;
  int v;
  while (f >> key >> v)
    if (v >= 0 && v <= 2) m[key] = v;
  return m;
}

void store_cache(const std::map<std::string, int>& m) {
  const char* p = std::getenv("PD_AUTOTUNE_CACHE");
  if (!p || !*p) return;
  const std::string tmp = std::string(p) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    for (const auto& kv : m) f << kv.first << " " << kv.second << "\n";
    if (!f) return;
  }
  std::rename(tmp.c_str(), p);
}

BatchIter make_iter(const pd_batch* b, int pi, const ListDev& L, int koff, int want,
                    int skip_fin) {
  BatchIter it;
  it.probs = b->ps[pi].d_probs;
  it.st = b->st;
  it.list = L.list;
  it.upd_off = L.upd_off;
  it.ns_off = L.ns_off;
  it.count = L.count;
  it.upd_blocks = L.upd_blocks;
  it.ns_blocks = L.ns_blocks;
  it.want = want;
  it.skip_fin = skip_fin;
  it.rho = b->rho;
  it.sig = b->ps[pi].sig;
  it.tmp = b->tmp;
  it.nsp = b->nsp;
  it.corr = b->corr;
  it.pnull = b->pnull;
  it.res = b->precond ? b->res : nullptr;
  it.kbase = b->d_kbase;
  it.koff = koff;
  return it;
}

// Host image of a list's tables appended to `h`; positions recorded for the device pointers.
struct ListHost {
  size_t list = 0, upd = 0, ns = 0;
  int count = 0, upd_blocks = 0, ns_blocks = 0;
};

ListHost add_list(const std::vector<BProb>& probs, const std::vector<int>& js,
                  std::vector<int>* h) {
  ListHost L;
  L.count = (int)js.size();
  L.list = h->size();
  h->insert(h->end(), js.begin(), js.end());
  h->push_back(0);                              // keeps an empty list addressable
  L.upd = h->size();
  int u = 0;
  for (int j : js) {
    h->push_back(u);
    u += probs[j].nupd;
  }
  h->push_back(u);
  L.ns = h->size();
  int v = 0;
  for (int j : js) {
    h->push_back(v);
    v += probs[j].nns;
  }
  h->push_back(v);
  L.upd_blocks = u;
  L.ns_blocks = v;
  return L;
}

// Operator groups (one per degree and tile variant) over the problems js, with the variants and
// tile counts of precision set P; table positions appended to h.
struct GroupHost {
  BatchGroup g;
  size_t grp = 0, toff = 0;
};

std::vector<GroupHost> add_groups(const PrecSet& P, const std::vector<int>& js,
                                  std::vector<int>* h) {
  std::map<std::pair<int, int>, std::vector<int>> by;
  for (int j : js) by[{P.probs[j].N, P.variants[j]}].push_back(j);
  std::vector<GroupHost> out;
  for (auto& kv : by) {
    GroupHost G;
    G.g.N = kv.first.first;
    G.g.variant = kv.first.second;
    G.g.ng = (int)kv.second.size();
    G.grp = h->size();
    h->insert(h->end(), kv.second.begin(), kv.second.end());
    G.toff = h->size();
    int tiles = 0;
    for (int j : kv.second) {
      h->push_back(tiles);
      tiles += P.probs[j].ntx * P.probs[j].nty;
    }
    h->push_back(tiles);
    G.g.blocks = (unsigned)tiles;
    out.push_back(G);
  }
  return out;
}

ListDev to_dev(const ListHost& L, const int* d) {
  ListDev D;
  D.list = d + L.list;
  D.upd_off = d + L.upd;
  D.ns_off = d + L.ns;
  D.count = L.count;
  D.upd_blocks = L.upd_blocks;
  D.ns_blocks = L.ns_blocks;
  return D;
}

std::vector<BatchGroup> groups_dev(const std::vector<GroupHost>& G, const int* d) {
  std::vector<BatchGroup> out;
  for (const GroupHost& g : G) {
    BatchGroup x = g.g;
    x.grp = d + g.grp;
    x.toff = d + g.toff;
    out.push_back(x);
  }
  return out;
}

void drop_plan(Plan* P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->dev) (void)hipFree(P->dev);
  *P = Plan();
}

// Lists of the problems js split by degree (ascending), table positions appended to h.
std::vector<std::pair<int, ListHost>> add_lists_by_degree(const pd_batch* b,
                                                         const std::vector<int>& js,
                                                         std::vector<int>* h) {
  std::map<int, std::vector<int>> by;
  for (int j : js) by[b->N[j]].push_back(j);
  std::vector<std::pair<int, ListHost>> out;
  for (const auto& kv : by) out.push_back({kv.first, add_list(b->ps[0].probs, kv.second, h)});
  return out;
}

// The preconditioner pass sel (see launch_pcg_update_batch) over per-degree lists, with the
// descriptors of precision set pi (the sigma partials of that precision for sel 0).
int pcg_pass(pd_batch* b, const std::vector<std::pair<int, ListDev>>& lists, int pi, int koff,
             int want, int skip_fin, bool fp32, int sel, const void* q, void* r, void* z,
             hipStream_t s) {
  for (const auto& nl : lists) {
    const int N = nl.first;
    const BatchIter it = make_iter(b, pi, nl.second, koff, want, skip_fin);
    BHIP(b, pdk::launch_pcg_update_batch(it, N, fp32, sel, &b->pv[(size_t)N * 90],
                                         &b->pv[(size_t)N * 90 + 81], q, r, z, s));
  }
  return PD_OK;
}

// Build the device tables of a plan for the given active sets (no graph yet).
int build_plan(pd_batch* b, const std::vector<int>& act32, const std::vector<int>& act64,
               bool refine, Plan* out) {
  drop_plan(out);
  std::vector<int> h;
  const ListHost l32 = add_list(b->ps[1].probs, act32, &h);
  const ListHost l64 = add_list(b->ps[0].probs, act64, &h);
  std::vector<int> un(act32);
  un.insert(un.end(), act64.begin(), act64.end());
  std::sort(un.begin(), un.end());
  const ListHost la = add_list(b->ps[0].probs, un, &h);
  const std::vector<GroupHost> g32 = add_groups(b->ps[1], act32, &h);
  const std::vector<GroupHost> gallr = add_groups(b->ps[0], un, &h);
  const std::vector<GroupHost> g64 = add_groups(b->ps[0], act64, &h);
  const auto h32 = add_lists_by_degree(b, act32, &h);
  const auto h64 = add_lists_by_degree(b, act64, &h);
  const auto hall = add_lists_by_degree(b, un, &h);
  int rc = balloc(b, &out->dev, h.size());
  if (rc) return rc;
  BHIP(b, hipMemcpy(out->dev, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
  out->l32 = to_dev(l32, out->dev);
  out->l64 = to_dev(l64, out->dev);
  out->lall = to_dev(la, out->dev);
  out->g32 = groups_dev(g32, out->dev);
  out->gallr = groups_dev(gallr, out->dev);
  out->g64 = groups_dev(g64, out->dev);
  for (const auto& e : h32) out->n32.push_back({e.first, to_dev(e.second, out->dev)});
  for (const auto& e : h64) out->n64.push_back({e.first, to_dev(e.second, out->dev)});
  for (const auto& e : hall) out->nall.push_back({e.first, to_dev(e.second, out->dev)});
  out->in64.assign(b->count, 0);
  for (int j : act64) out->in64[j] = 1;
  out->dofs = 0;
  for (int j : un) out->dofs += b->ps[0].probs[j].ndof;
  out->refine = refine;
  return PD_OK;
}

// Give every problem of precision set pi its tile variant: tile counts and sigma offsets.
int set_variants(pd_batch* b, int pi, const std::vector<int>& variants) {
  PrecSet& P = b->ps[pi];
  const bool fp32 = pi == 1;
  P.variants = variants;
  int sig = 0;
  for (int j = 0; j < b->count; ++j) {
    BProb& q = P.probs[j];
    pdk::tiles2d(q.N, fp32, variants[j], q.nx, q.ny, &q.ntx, &q.nty);
    q.variant = variants[j];
    q.sig_off = sig;
    q.nsig = q.ntx * q.nty;
    sig += q.nsig;
  }
  if (sig > P.sig_cap) return bfail(b, PD_EINVAL, "sigma partials exceed the workspace");
  for (Plan& p : b->all) drop_plan(&p);
  if (!P.d_probs) {
    const int rc = balloc(b, &P.d_probs, P.probs.size());
    if (rc) return rc;
  }
  BHIP(b, hipMemcpy(P.d_probs, P.probs.data(), P.probs.size() * sizeof(BProb),
                    hipMemcpyHostToDevice));
  if (pi == 0) {
    // FP64 groups over every problem (final residual check)
    std::vector<int> all(b->count), h;
    for (int j = 0; j < b->count; ++j) all[j] = j;
    const std::vector<GroupHost> G = add_groups(P, all, &h);
    if (b->d_g64_all) (void)hipFree(b->d_g64_all);
    b->d_g64_all = nullptr;
    const int rc = balloc(b, &b->d_g64_all, h.size());
    if (rc) return rc;
    BHIP(b, hipMemcpy(b->d_g64_all, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    b->g64_all = groups_dev(G, b->d_g64_all);
  }
  return PD_OK;
}

// Time the fused CG operator of every (degree, size bucket) key with each tile variant on the
// batch's own problems and keep the fastest (a smaller tile must win by 3% to replace variant 0).
int autotune(pd_batch* b, int pi, unsigned flags, std::map<std::string, int>* cache,
             bool* dirty, hipStream_t s) {
  const bool fp32 = pi == 1;
  const int count = b->count;
  PrecSet& P = b->ps[pi];
  std::vector<std::string> key(count);
  std::map<std::string, std::vector<int>> members;
  for (int j = 0; j < count; ++j) {
    const BProb& q = P.probs[j];
    key[j] = tune_key(q.N, size_bucket(std::max(q.nx, q.ny)), fp32);
    members[key[j]].push_back(j);
  }
  std::vector<std::string> todo;
  for (auto& kv : members)
    if ((flags & PD_BATCH_RETUNE) || !cache->count(kv.first)) todo.push_back(kv.first);
  if (!todo.empty()) {
    // zero operands and partials, and states with tol2 = -1, so that no launch stops early
    void* r = fp32 ? (void*)b->r32 : (void*)b->r64;
    void* pa = fp32 ? (void*)b->pa32 : (void*)b->pa64;
    void* pb = fp32 ? (void*)b->pb32 : (void*)b->pb64;
    void* q = fp32 ? (void*)b->q32 : (void*)b->q64;
    void* xs = fp32 ? (void*)b->d32 : (void*)b->x64;   // untouched: xk = -1 in every state
    BHIP(b, pdk::launch_zero_all(fp32, r, b->total, s));
    BHIP(b, pdk::launch_zero_all(fp32, pa, b->total, s));
    BHIP(b, pdk::launch_zero_all(false, b->rho, (long long)count * 2 * pdk::kMaxStreamPartials, s));
    BHIP(b, pdk::launch_state_init_batch(b->st, count, 1 << 30, -1.0, 0, s));
    BHIP(b, hipMemsetAsync(b->d_kbase, 0, sizeof(int), s));
    std::map<std::string, std::vector<double>> us;
    for (int v = 0; v < 3; ++v) {
      int rc = set_variants(b, pi, std::vector<int>(count, v));
      if (rc) return rc;
      std::vector<int> h;
      std::vector<std::vector<GroupHost>> G;
      for (const std::string& k : todo) G.push_back(add_groups(P, members[k], &h));
      int* dh = nullptr;
      if ((rc = balloc(b, &dh, h.size()))) return rc;
      hipError_t e = hipMemcpy(dh, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice);
      const BatchIter it = make_iter(b, pi, b->everyone, 0, -1, 0);
      for (size_t gi = 0; gi < todo.size() && e == hipSuccess; ++gi) {
        const std::vector<BatchGroup> gs = groups_dev(G[gi], dh);   // one group: key fixes N
        const int reps = 20;
        for (int w = 0; w < 3 && e == hipSuccess; ++w)
          for (const BatchGroup& g : gs)
            if (e == hipSuccess)
              e = pdk::launch_apply_batch(it, g, fp32, true, r, pa, pb, q, xs, b->tabs[g.N], s);
        if (e == hipSuccess) e = hipEventRecord(b->t0, s);
        for (int w = 0; w < reps && e == hipSuccess; ++w)
          for (const BatchGroup& g : gs)
            if (e == hipSuccess)
              e = pdk::launch_apply_batch(it, g, fp32, true, r, pa, pb, q, xs, b->tabs[g.N], s);
        if (e == hipSuccess) e = hipEventRecord(b->t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(b->t1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->t0, b->t1);
        us[todo[gi]].push_back(1e3 * ms / reps);
      }
      (void)hipFree(dh);
      if (e != hipSuccess) return bfail(b, PD_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    }
    for (const std::string& k : todo) {
      const std::vector<double>& t = us[k];
      int best = 0;
      for (int v = 1; v < 3; ++v)
        if (t[v] < 0.97 * t[best]) best = v;
      (*cache)[k] = best;
      *dirty = true;
    }
  }
  std::vector<int> vv(count, 0);
  for (int j = 0; j < count; ++j) vv[j] = cache->at(key[j]);
  return set_variants(b, pi, vv);
}

// One chunk over a plan: `chunk` CG iterations of the FP32-mode problems (act32) and of the
// FP64-mode problems (act64); for the refinement, the FP64 residual replacement of act32; the
// chunk-end decisions of every active problem; then the iteration base advances.
int enqueue_chunk(pd_batch* b, const Plan& pl, hipStream_t s) {
  void* p32[2] = {b->pa32, b->pb32};
  void* p64[2] = {b->pa64, b->pb64};
  for (int i = 0; i < b->chunk; ++i) {
    const BatchIter i32 = make_iter(b, 1, pl.l32, i, 0, 0);
    const BatchIter i64 = make_iter(b, 0, pl.l64, i, 1, 0);
    // the operand of the fused direction update: z = P r when preconditioned, else r
    const void* o32 = b->precond ? (const void*)b->z32 : (const void*)b->r32;
    const void* o64 = b->precond ? (const void*)b->z64 : (const void*)b->r64;
    for (const BatchGroup& g : pl.g32)
      BHIP(b, pdk::launch_apply_batch(i32, g, true, true, o32, p32[i & 1], p32[(i + 1) & 1],
                                      b->q32, b->d32, b->tabs[g.N], s));
    for (const BatchGroup& g : pl.g64)
      BHIP(b, pdk::launch_apply_batch(i64, g, false, true, o64, p64[i & 1], p64[(i + 1) & 1],
                                      b->q64, b->x64, b->tabs[g.N], s));
    if (b->precond) {
      int rc = pcg_pass(b, pl.n32, 1, i, 0, 0, true, 0, b->q32, b->r32, b->z32, s);
      if (!rc) rc = pcg_pass(b, pl.n64, 0, i, 1, 0, false, 0, b->q64, b->r64, b->z64, s);
      if (rc) return rc;
    } else {
      BHIP(b, pdk::launch_update_batch(i32, true, b->q32, b->r32, s));
      BHIP(b, pdk::launch_update_batch(i64, false, b->q64, b->r64, s));
    }
  }
  const int K = b->chunk;
  // the deferred x updates of the problems that stopped inside the chunk (and of those still
  // running, whose next apply would have made it): x is complete before anything below reads
  // it; the chunk-end finalize clears xk
  BHIP(b, pdk::launch_xflush_batch(make_iter(b, 0, pl.lall, K, -1, 0), b->x64, b->d32,
                                   (const double*)p64[0], (const double*)p64[1],
                                   (const float*)p32[0], (const float*)p32[1], s));
  // FP64 residual of the unfinished FP32-mode problems and of the FP64-mode problems whose
  // recurrence has met the tolerance
  const BatchIter chk = make_iter(b, 0, pl.lall, K, -2, 1);
  if (pl.refine) {
    // x64 += scale d32 for every FP32-listed problem (also those that stopped inside the chunk)
    BHIP(b, pdk::launch_stream_batch(1, make_iter(b, 0, pl.l32, K, -1, 0), nullptr, nullptr,
                                     nullptr, b->x64, b->d32, s));
  }
  for (const BatchGroup& g : pl.gallr)
    BHIP(b, pdk::launch_apply_batch(chk, g, false, false, b->x64, nullptr, nullptr, b->q64,
                                    nullptr, b->tabs[g.N], s));
  BHIP(b, pdk::launch_stream_batch(0, chk, b->b64, b->q64, b->r64, nullptr, nullptr, s));
  BHIP(b, pdk::launch_project_null_batch(chk, b->r64, s));
  BHIP(b, pdk::launch_stream_batch(3, chk, nullptr, nullptr, b->r64, nullptr, nullptr, s));
  BHIP(b, pdk::launch_finalize_batch(3, make_iter(b, 0, pl.lall, K, -1, 1), s));
  if (pl.refine) {
    const BatchIter i32 = make_iter(b, 0, pl.l32, K, 0, 1);
    BHIP(b, pdk::launch_stream_batch(2, i32, nullptr, nullptr, b->r64, nullptr, b->r32, s));
    // preconditioned: z32 = P r32, partials of <r, z> and <r, r>
    if (b->precond) {
      const int rc = pcg_pass(b, pl.n32, 0, K, 0, 1, true, 1, nullptr, b->r32, b->z32, s);
      if (rc) return rc;
    }
  }
  // partials of <r, r> (preconditioned: z = P r, <r, z> and <r, r>) of the problems resuming
  // from a recomputed residual
  if (b->precond) {
    const int rc = pcg_pass(b, pl.nall, 0, K, -1, 1, false, 2, nullptr, b->r64, b->z64, s);
    if (rc) return rc;
  } else
    BHIP(b, pdk::launch_stream_batch(5, make_iter(b, 0, pl.lall, K, -1, 1), nullptr, nullptr,
                                     b->r64, nullptr, nullptr, s));
  BHIP(b, pdk::launch_tick(b->d_kbase, b->chunk, s));
  return PD_OK;
}

int capture(pd_batch* b, Plan* pl) {
  if (pl->exec && pl->chunk == b->chunk) return PD_OK;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->exec = nullptr;
  pl->graph = nullptr;
  BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_chunk(b, *pl, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, PD_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  pl->graph = g;
  BHIP(b, hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0));
  pl->chunk = b->chunk;
  return PD_OK;
}

int run_plan(pd_batch* b, Plan* pl, hipStream_t s) {
  if (!b->use_graph) return enqueue_chunk(b, *pl, s);
  int rc = capture(b, pl);
  if (rc) return rc;
  BHIP(b, hipGraphLaunch(pl->exec, s));
  return PD_OK;
}

}  // namespace

extern "C" {

const char* pd_batch_last_error(const pd_batch* b) {
  return b ? b->err.c_str() : g_batch_err.c_str();
}

void pd_batch_destroy(pd_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  for (Plan& p : b->all) drop_plan(&p);
  for (PrecSet& P : b->ps) {
    (void)hipFree(P.d_probs);
    (void)hipFree(P.sig);
  }
  void* bufs[] = {b->d_kbase, b->st, b->rho, b->tmp, b->nsp, b->corr, b->pnull, b->b64,
                  b->x64, b->r64, b->q64, b->pa64, b->pb64, b->r32, b->pa32, b->pb32,
                  b->q32, b->d32, b->d_everyone, b->d_g64_all, b->z64, b->z32, b->res,
                  b->d_everyone_n};
  for (void* p : bufs) (void)hipFree(p);
  if (b->hst) (void)hipHostFree(b->hst);
  for (hipEvent_t e : {b->ev[0], b->ev[1], b->t0, b->t1})
    if (e) (void)hipEventDestroy(e);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

int pd_batch_setup(pd_batch** out, int count, const int* ncell, const double* len, const int* N,
                   double dt, unsigned flags, void* hip_stream) {
  if (!out) return bfail(nullptr, PD_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > (1 << 20) || !ncell || !len || !N)
    return bfail(nullptr, PD_EINVAL, "bad problem list");
  if (!(dt > 0.0)) return bfail(nullptr, PD_EINVAL, "dt must be > 0");
  if (flags & ~(unsigned)(PD_BATCH_AUTOTUNE | PD_BATCH_RETUNE))
    return bfail(nullptr, PD_EINVAL, "unknown flags");
  hipStream_t s = (hipStream_t)hip_stream;
  pd_batch* b = new pd_batch();
  auto fin = [&](int code) {
    g_batch_err = b->err;
    pd_batch_destroy(b);
    return code;
  };
  b->count = count;
  b->dt = dt;
  b->tabs.resize(pdh::kMaxN + 1);
  std::vector<double> pn((pdh::kMaxN + 1) * 81, 0.0);
  b->pv.assign((pdh::kMaxN + 1) * 90, 0.0);   // preconditioner V[81], lambda[9]
  for (int d = 0; d <= pdh::kMaxN; ++d) {
    pdh::Table1D t;
    std::string e;
    if (!pdh::build_table(d, &t, &e)) {
      b->err = e;
      return fin(PD_EINVAL);
    }
    for (int i = 0; i < t.n * t.n; ++i) {
      b->tabs[d].L[i] = t.Lb[i];
      b->tabs[d].C[i] = t.Cb[i];
      b->tabs[d].R[i] = t.Rb[i];
      pn[d * 81 + i] = t.Pnull[i];
      b->pv[d * 90 + i] = t.PV[i];
    }
    for (int i = 0; i < t.n; ++i) b->pv[d * 90 + 81 + i] = t.Plam[i];
    for (int i = 0; i < t.n; ++i) b->tabs[d].w[i] = t.w[i];
  }
  std::vector<BProb> probs(count);
  b->N.resize(count);
  b->off.push_back(0);
  long long upd_total = 0;
  for (int j = 0; j < count; ++j) {
    BProb& P = probs[j];
    P.nx = ncell[2 * j];
    P.ny = ncell[2 * j + 1];
    P.N = N[j];
    if (P.nx < 1 || P.ny < 1 || P.N < 0 || P.N > pdh::kMaxN || !(len[2 * j] > 0.0) ||
        !(len[2 * j + 1] > 0.0) || (long long)P.nx * P.ny > (1LL << 26)) {
      b->err = "bad problem " + std::to_string(j);
      return fin(PD_EINVAL);
    }
    b->N[j] = P.N;
    const int n = P.N + 1;
    P.NC = n * n;
    P.ncells = (long long)P.nx * P.ny;
    P.ndof = P.ncells * P.NC;
    P.dof_off = b->total;
    b->total += P.ndof;
    b->off.push_back(b->total);
    P.nupd = stream_blocks_for(P.ndof);
    upd_total += P.nupd;
    P.nns = (int)std::min<long long>(pdk::kNsBlocksBatch, P.ncells);
    const double hx = len[2 * j] / P.nx, hy = len[2 * j + 1] / P.ny;
    P.c0 = dt / (hx * hx);
    P.c1 = dt / (hy * hy);
    P.alpha = 0.0;
    P.rtol = 1e-10;
    P.ru = b->ru;
    P.variant = 0;
    P.ntx = P.nty = P.sig_off = P.nsig = 0;
    if (upd_total > (1 << 30) || b->total > (1LL << 40)) {
      b->err = "batch too large";
      return fin(PD_EINVAL);
    }
  }
  // sigma partials per precision: the largest tile count over the variants
  for (int pi = 0; pi < 2; ++pi) {
    b->ps[pi].probs = probs;
    for (int v = 0; v < 3; ++v) {
      long long tot = 0;
      for (const BProb& P : probs) {
        int tx, ty;
        pdk::tiles2d(P.N, pi == 1, v, P.nx, P.ny, &tx, &ty);
        tot += (long long)tx * ty;
      }
      if (tot > (1LL << 30)) {
        b->err = "batch too large";
        return fin(PD_EINVAL);
      }
      b->ps[pi].sig_cap = std::max(b->ps[pi].sig_cap, (int)tot);
    }
  }
  const size_t n = (size_t)b->total;
  const size_t cnt = (size_t)count;
  int rc = PD_OK;
  if ((rc = balloc(b, &b->d_kbase, 1)) || (rc = balloc(b, &b->st, cnt)) ||
      (rc = balloc(b, &b->rho, cnt * 2 * pdk::kMaxStreamPartials)) ||
      (rc = balloc(b, &b->ps[0].sig, (size_t)b->ps[0].sig_cap)) ||
      (rc = balloc(b, &b->ps[1].sig, (size_t)b->ps[1].sig_cap)) ||
      (rc = balloc(b, &b->tmp, cnt * pdk::kMaxStreamPartials)) ||
      (rc = balloc(b, &b->nsp, cnt * pdk::kNsBlocksBatch * pdk::kMaxNC2D)) ||
      (rc = balloc(b, &b->corr, cnt * pdk::kMaxNC2D)) || (rc = balloc(b, &b->pnull, pn.size())) ||
      (rc = balloc(b, &b->b64, n)) || (rc = balloc(b, &b->x64, n)) ||
      (rc = balloc(b, &b->r64, n)) || (rc = balloc(b, &b->q64, n)) ||
      (rc = balloc(b, &b->pa64, n)) || (rc = balloc(b, &b->pb64, n)) ||
      (rc = balloc(b, &b->r32, n)) || (rc = balloc(b, &b->pa32, n)) ||
      (rc = balloc(b, &b->pb32, n)) || (rc = balloc(b, &b->q32, n)) ||
      (rc = balloc(b, &b->d32, n)) || (rc = balloc(b, &b->z64, n)) ||
      (rc = balloc(b, &b->z32, n)) ||
      (rc = balloc(b, &b->res, cnt * 2 * pdk::kMaxStreamPartials)))
    return fin(rc);
  {
    std::vector<int> all(count), h;
    for (int j = 0; j < count; ++j) all[j] = j;
    const ListHost L = add_list(probs, all, &h);
    if ((rc = balloc(b, &b->d_everyone, h.size()))) return fin(rc);
    if (hipMemcpy(b->d_everyone, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice) !=
        hipSuccess) {
      b->err = "setup: list upload failed";
      return fin(PD_EDEVICE);
    }
    b->everyone = to_dev(L, b->d_everyone);
    std::vector<int> hn;
    const auto ln = add_lists_by_degree(b, all, &hn);
    if ((rc = balloc(b, &b->d_everyone_n, hn.size()))) return fin(rc);
    if (hipMemcpy(b->d_everyone_n, hn.data(), hn.size() * sizeof(int), hipMemcpyHostToDevice) !=
        hipSuccess) {
      b->err = "setup: list upload failed";
      return fin(PD_EDEVICE);
    }
    for (const auto& e : ln) b->everyone_n.push_back({e.first, to_dev(e.second, b->d_everyone_n)});
  }
  hipError_t he = hipHostMalloc((void**)&b->hst, 2 * cnt * sizeof(CgState), hipHostMallocDefault);
  if (he == hipSuccess) he = hipEventCreate(&b->ev[0]);
  if (he == hipSuccess) he = hipEventCreate(&b->ev[1]);
  if (he == hipSuccess) he = hipEventCreate(&b->t0);
  if (he == hipSuccess) he = hipEventCreate(&b->t1);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (he == hipSuccess)
    he = hipMemcpy(b->pnull, pn.data(), pn.size() * sizeof(double), hipMemcpyHostToDevice);

  if (he != hipSuccess) {
    b->err = std::string("setup: ") + hipGetErrorString(he);
    return fin(PD_EDEVICE);
  }
  std::map<std::string, int> cache = load_cache();
  bool dirty = false;
  for (int pi = 0; pi < 2; ++pi) {
    if (flags & (PD_BATCH_AUTOTUNE | PD_BATCH_RETUNE)) {
      rc = autotune(b, pi, flags, &cache, &dirty, s);
    } else {
      std::vector<int> vv(count, 0);
      for (int j = 0; j < count; ++j) {
        const BProb& P = probs[j];
        auto it = cache.find(tune_key(P.N, size_bucket(std::max(P.nx, P.ny)), pi == 1));
        if (it != cache.end()) vv[j] = it->second;
      }
      rc = set_variants(b, pi, vv);
    }
    if (rc) return fin(rc);
  }
  if (dirty) store_cache(cache);
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    b->err = std::string("setup: ") + hipGetErrorString(he);
    return fin(PD_EDEVICE);
  }
  *out = b;
  return PD_OK;
}

int pd_batch_layout(const pd_batch* b, long long* offsets) {
  if (!b || !offsets) return PD_EINVAL;
  for (int j = 0; j <= b->count; ++j) offsets[j] = b->off[j];
  return PD_OK;
}

int pd_batch_variants(const pd_batch* b, int prec, int* variants) {
  if (!b || !variants) return PD_EINVAL;
  if (prec != PD_FP64 && prec != PD_FP32) return PD_EINVAL;
  const PrecSet& P = b->ps[prec == PD_FP32 ? 1 : 0];
  for (int j = 0; j < b->count; ++j) variants[j] = P.variants[j];
  return PD_OK;
}

int pd_batch_configure(pd_batch* b, int key, double v) {
  if (!b) return PD_EINVAL;
  switch (key) {
    case PD_BCFG_CHUNK: {
      if (!(v >= 2 && v <= 4096)) return bfail(b, PD_EINVAL, "chunk must be an even integer in [2, 4096]");
      const int c = (int)v;
      if (v != c || c % 2 != 0) return bfail(b, PD_EINVAL, "chunk must be an even integer in [2, 4096]");
      b->chunk = c;
      break;
    }
    case PD_BCFG_GRAPH:
      b->use_graph = v != 0.0;
      break;
    case PD_BCFG_RU_FACTOR:
      if (!(v > 0.0 && v < 1.0)) return bfail(b, PD_EINVAL, "pause factor must be in (0, 1)");
      b->ru = v;
      break;
    case PD_BCFG_PRECOND: {
      if (!(v == 0.0 || v == 1.0)) return bfail(b, PD_EINVAL, "precond must be 0 or 1");
      const int p = (int)v;
      if (p != b->precond) {
        // the captured chunks embed the kernels and operands of the other form
        (void)hipDeviceSynchronize();
        for (Plan& pl : b->all) drop_plan(&pl);
        b->precond = p;
      }
      break;
    }
    default:
      return bfail(b, PD_EINVAL, "unknown configuration key");
  }
  return PD_OK;
}

int pd_batch_cg_solve(pd_batch* b, int prec, const void* bvec, void* xvec, double rtol, int maxit,
                      pd_solve_info* info, void* hip_stream) {
  if (!b) return PD_EINVAL;
  if (prec != PD_FP64 && prec != PD_FP32_REFINE64)
    return bfail(b, PD_EINVAL, "prec must be PD_FP64 or PD_FP32_REFINE64");
  if (!bvec || !xvec) return bfail(b, PD_EINVAL, "NULL vector");
  if (!(rtol > 0.0)) return bfail(b, PD_EINVAL, "rtol must be > 0");
  if (maxit < 0) return bfail(b, PD_EINVAL, "maxit must be >= 0");
  const bool refine = prec == PD_FP32_REFINE64;
  hipStream_t s = (hipStream_t)hip_stream;
  const int count = b->count;
  const long long n = b->total;
  // the tolerance and pause factor live in the descriptors of both precision sets
  for (PrecSet& P : b->ps) {
    bool changed = false;
    for (BProb& q : P.probs)
      if (q.rtol != rtol || q.ru != b->ru) {
        q.rtol = rtol;
        q.ru = b->ru;
        changed = true;
      }
    if (changed)
      BHIP(b, hipMemcpy(P.d_probs, P.probs.data(), P.probs.size() * sizeof(BProb),
                        hipMemcpyHostToDevice));
  }
  // plan of the first chunks: every problem, in the precision the solve starts with
  Plan& start = b->all[refine ? 1 : 0];
  if (!start.dev) {
    std::vector<int> every(count), none;
    for (int j = 0; j < count; ++j) every[j] = j;
    const int rc = refine ? build_plan(b, every, none, true, &start)
                          : build_plan(b, none, every, false, &start);
    if (rc) return rc;
  }
  const BatchIter all = make_iter(b, 0, b->everyone, 0, -1, 0);
  BHIP(b, hipEventRecord(b->t0, s));
  // start: b64 = b projected onto range(A) per problem, x = 0, directions 0
  BHIP(b, hipMemcpyAsync(b->b64, bvec, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  BHIP(b, pdk::launch_state_init_batch(b->st, count, maxit, 0.0, refine ? 0 : 1, s));
  BHIP(b, hipMemsetAsync(b->d_kbase, 0, sizeof(int), s));
  BHIP(b, pdk::launch_project_null_batch(all, b->b64, s));
  BHIP(b, pdk::launch_zero_all(false, b->x64, n, s));
  BHIP(b, pdk::launch_zero_all(false, b->pa64, n, s));
  BHIP(b, pdk::launch_zero_all(false, b->pb64, n, s));
  if (refine) {
    BHIP(b, pdk::launch_zero_all(true, b->d32, n, s));
    BHIP(b, pdk::launch_zero_all(true, b->pa32, n, s));
    BHIP(b, pdk::launch_zero_all(true, b->pb32, n, s));
    // ||b|| per problem; scale = ||b||; pause threshold of the FP32 iterations
    BHIP(b, pdk::launch_stream_batch(3, all, nullptr, nullptr, b->b64, nullptr, nullptr, s));
    BHIP(b, pdk::launch_finalize_batch(1, all, s));
    // r32 = b / scale with partials of <r32, r32> in the rho slot of iteration 0
    const BatchIter i32 = make_iter(b, 0, b->everyone, 0, 0, 1);
    BHIP(b, pdk::launch_stream_batch(2, i32, nullptr, nullptr, b->b64, nullptr, b->r32, s));
    // preconditioned: z32 = P r32 with the partials of <r, z> and <r, r> of iteration 0
    if (b->precond) {
      const int rcp = pcg_pass(b, b->everyone_n, 0, 0, 0, 1, true, 1, nullptr, b->r32, b->z32, s);
      if (rcp) return rcp;
    }
  } else {
    // r = b with partials in the rho slot of iteration 0; tol2 = rtol^2 ||b||^2
    BHIP(b, pdk::launch_stream_batch(4, all, b->b64, nullptr, b->r64, nullptr, nullptr, s));
    if (b->precond) {
      const int rcp = pcg_pass(b, b->everyone_n, 0, 0, -1, 0, false, 1, nullptr, b->r64, b->z64, s);
      if (rcp) return rcp;
    }
    BHIP(b, pdk::launch_stream_batch(3, all, nullptr, nullptr, b->r64, nullptr, nullptr, s));
    BHIP(b, pdk::launch_finalize_batch(2, all, s));
  }
  // Replay chunks with up to two in flight. The host reads each chunk's states; when a problem
  // has switched to FP64 iterations (it must join the FP64 list) or the active DoFs have fallen
  // below 70% of those of the current plan, it waits for the stream and captures a new plan.
  Plan cur;                                   // re-captured plan (start plan when empty)
  Plan* pl = &start;
  const long long max_chunks = (long long)maxit / b->chunk + 2;
  const size_t sb = (size_t)count * sizeof(CgState);
  long long launched = 0, checked = 0;
  auto launch = [&]() -> int {
    const int slot = (int)(launched & 1);
    const int rc = run_plan(b, pl, s);
    if (rc) return rc;
    BHIP(b, hipMemcpyAsync(b->hst + (size_t)slot * count, b->st, sb, hipMemcpyDeviceToHost, s));
    BHIP(b, hipEventRecord(b->ev[slot], s));
    ++launched;
    return PD_OK;
  };
  auto finished = [&](const CgState* h) {
    for (int j = 0; j < count; ++j)
      if (!h[j].fin) return false;
    return true;
  };
  int rc = PD_OK;
  for (;;) {
    while (launched < max_chunks && launched - checked < 2)
      if ((rc = launch())) {
        drop_plan(&cur);
        return rc;
      }
    const int slot = (int)(checked & 1);
    BHIP(b, hipEventSynchronize(b->ev[slot]));
    const CgState* h = b->hst + (size_t)slot * count;
    ++checked;
    if (finished(h) || (launched >= max_chunks && checked == launched)) break;
    bool need = false;
    long long dofs = 0;
    for (int j = 0; j < count; ++j) {
      if (h[j].fin) continue;
      dofs += b->ps[0].probs[j].ndof;
      if (h[j].mode64 && !pl->in64[j]) need = true;
    }
    if (!need && !(dofs < 0.7 * (double)pl->dofs)) continue;
    // new plan from the states after every queued chunk
    BHIP(b, hipStreamSynchronize(s));
    BHIP(b, hipMemcpy(b->hst, b->st, sb, hipMemcpyDeviceToHost));
    checked = launched;
    if (finished(b->hst) || launched >= max_chunks) break;
    std::vector<int> a32, a64;
    for (int j = 0; j < count; ++j) {
      if (b->hst[j].fin) continue;
      (b->hst[j].mode64 ? a64 : a32).push_back(j);
    }
    Plan next;
    if ((rc = build_plan(b, a32, a64, refine, &next))) {
      drop_plan(&next);
      drop_plan(&cur);
      return rc;
    }
    drop_plan(&cur);
    cur = next;
    pl = &cur;
  }
  // every problem stopped: minimum-norm solution, FP64 true residual, copy out
  BHIP(b, hipStreamSynchronize(s));
  drop_plan(&cur);
  BHIP(b, pdk::launch_project_null_batch(all, b->x64, s));
  for (const BatchGroup& g : b->g64_all)
    BHIP(b, pdk::launch_apply_batch(all, g, false, false, b->x64, nullptr, nullptr, b->q64,
                                    nullptr, b->tabs[g.N], s));
  BHIP(b, pdk::launch_stream_batch(0, all, b->b64, b->q64, b->r64, nullptr, nullptr, s));
  BHIP(b, pdk::launch_finalize_batch(0, all, s));
  BHIP(b, hipMemcpyAsync(xvec, b->x64, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  BHIP(b, hipEventRecord(b->t1, s));
  BHIP(b, hipMemcpyAsync(b->hst, b->st, sb, hipMemcpyDeviceToHost, s));
  BHIP(b, hipStreamSynchronize(s));
  float ms = 0.f;
  BHIP(b, hipEventElapsedTime(&ms, b->t0, b->t1));
  bool any_break = false, any_noconv = false;
  for (int j = 0; j < count; ++j) {
    const CgState& h = b->hst[j];
    const int status = h.fin ? h.status : PD_ENOCONV;
    if (status == PD_EBREAKDOWN) any_break = true;
    else if (status != PD_OK) any_noconv = true;
    if (info) {
      pd_solve_info& o = info[j];
      o.iters = h.iter - h.idle;        // iterations run (not the idle ones of a stopped problem)
      o.outer_iters = h.outer > 1 ? h.outer : 1;
      o.status = status;
      o.restarts = h.restarts;
      o.fallback_iter = refine ? h.fallback_k : -1;
      o.reserved = 0;
      const double bn = std::sqrt(h.bnorm2);
      const double r2 = b->precond ? h.res2 : h.rho;   // preconditioned: rho is <r, z>
      const double rec = (refine && !h.mode64) ? std::sqrt(r2) * h.scale : std::sqrt(r2);
      o.rel_res_recur = bn > 0 ? rec / bn : 0.0;
      o.rel_res_true = bn > 0 ? std::sqrt(h.aux) / bn : 0.0;
      o.ms = ms;
    }
  }
  return any_break ? PD_EBREAKDOWN : any_noconv ? PD_ENOCONV : PD_OK;
}

}  // extern "C"
