// Build (Algorithm 1) and solve (Algorithm 2) drivers of the MI355X solver.
//
// Memory plan of one operator (all FP64 in HBM, row-major):
//   leafT   [nleaf][4q][4q]      leaf DtNs (section 3), kept for refinement;
//   arena0/1                    DtNs of the boxes at even/odd depth: the
//                               children of a merge live in the other arena,
//                               so only two levels of T are ever alive
//                               (Algorithm 1 deletes children's T);
//   S       per merge m3 x me    solution operators (eq:U_parent), kept;
//   W, Q, piv                    per merge augmented system [M | B] (its
//                               left block ends up holding LU(M)), Q = [T13a;
//                               T23b] and pivots: kept per merge when the
//                               upward pass is wanted, else one level of
//                               scratch reused by every level.
#include "solver.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <tuple>

#include "dense.h"
#include "leaf.h"
#include "ops.h"
#include "prof.h"
#include "surrogate.h"

namespace hps {

DeviceMem::~DeviceMem() {
  for (void* p : ptrs) pool_release(p);
}

void* DeviceMem::raw(size_t b) {
  void* p = pool_alloc(b);
  ptrs.push_back(p);
  bytes += b;
  return p;
}

}  // namespace hps

hps_op::~hps_op() {
  for (auto& kv : solve_graphs) (void)hipGraphExecDestroy(kv.second);
  if (h_io) (void)hipHostFree(h_io);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

namespace hps {

// Stream-ordered scratch (hipMallocAsync) comes from the device's default
// pool; by default that pool hands freed memory back at every
// synchronization, so each solve would map its buffers afresh.  Keep it
// cached instead (hps_mem_trim releases it).
static void keep_async_pool() {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return;
  hipMemPool_t pool = nullptr;
  HPS_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = UINT64_MAX;
  HPS_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done.insert(dev);
}

void trim_async_pool() {
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  hipMemPool_t pool = nullptr;
  HPS_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  HPS_HIP(hipMemPoolTrimTo(pool, 0));
}

// Parked operators: destroyed operators whose buffers and descriptors are
// kept for the next build of the same key (most recent first).  Never freed
// at process exit (the HIP runtime may be gone by then).
namespace {
struct ParkList {
  std::mutex mu;
  std::list<hps_op*> ops;
  size_t limit = 2;
};
ParkList& parked() {
  static ParkList* l = new ParkList;
  return *l;
}
}  // namespace

void park_operator(hps_op* op) {
  if (!op) return;
  ParkList& L = parked();
  std::vector<hps_op*> drop;
  {
    std::lock_guard<std::mutex> lk(L.mu);
    if (L.limit == 0 || op->park_key.empty()) {
      drop.push_back(op);
    } else {
      // Graphs and per-build state go; buffers and descriptors stay.
      for (auto& kv : op->solve_graphs) (void)hipGraphExecDestroy(kv.second);
      op->solve_graphs.clear();
      op->solve_counts.clear();
      op->surrogate = nullptr;
      if (op->coeffs != op->coeffs_own) op->coeffs = nullptr;
      L.ops.push_front(op);
      while (L.ops.size() > L.limit) {
        drop.push_back(L.ops.back());
        L.ops.pop_back();
      }
    }
  }
  for (hps_op* d : drop) delete d;
}

std::unique_ptr<hps_op> unpark_operator(const std::vector<long long>& key) {
  ParkList& L = parked();
  std::lock_guard<std::mutex> lk(L.mu);
  for (auto it = L.ops.begin(); it != L.ops.end(); ++it)
    if ((*it)->park_key == key) {
      hps_op* op = *it;
      L.ops.erase(it);
      return std::unique_ptr<hps_op>(op);
    }
  return nullptr;
}

size_t parked_clear() {
  ParkList& L = parked();
  std::list<hps_op*> all;
  {
    std::lock_guard<std::mutex> lk(L.mu);
    all.swap(L.ops);
  }
  size_t n = all.size();
  for (hps_op* op : all) delete op;
  return n;
}

void set_parked_limit(int n) {
  ParkList& L = parked();
  std::vector<hps_op*> drop;
  {
    std::lock_guard<std::mutex> lk(L.mu);
    L.limit = (size_t)std::max(n, 0);
    while (L.ops.size() > L.limit) {
      drop.push_back(L.ops.back());
      L.ops.pop_back();
    }
  }
  for (hps_op* d : drop) delete d;
}

static void init_runtime() {
  dense_init();
  ops_init();
  keep_async_pool();
}

static inline int bdry_size(const BoxRec& b, int q) { return 2 * q * ((b.i1 - b.i0) + (b.j1 - b.j0)); }

// ---------------------------------------------------------------------------
// Plans: everything a build needs that depends only on the shape of the
// problem (section 2 tree, section 4 index maps, section 3.2 leaf tables).
// They are computed once per shape and device and shared by every operator
// of that shape, so repeated builds (coefficient sweeps) skip the host work.
// ---------------------------------------------------------------------------
namespace {

template <class P>
struct PlanCache {
  std::mutex mu;
  std::map<std::vector<long long>, std::pair<unsigned long long, std::shared_ptr<const P>>> items;
  unsigned long long tick = 0;
  static constexpr size_t kMax = 64;  // a heterogeneous batch holds one plan per shape
  std::shared_ptr<const P> get(const std::vector<long long>& key,
                               const std::function<std::shared_ptr<P>()>& make) {
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = items.find(key);
      if (it != items.end()) {
        it->second.first = ++tick;
        return it->second.second;
      }
    }
    std::shared_ptr<const P> p = make();
    std::lock_guard<std::mutex> lk(mu);
    if (items.size() >= kMax) {  // evict the least recently used plan
      auto old = items.begin();
      for (auto it = items.begin(); it != items.end(); ++it)
        if (it->second.first < old->second.first) old = it;
      items.erase(old);
    }
    items[key] = {++tick, p};
    return p;
  }
};

long long bits(double x) {
  long long b;
  std::memcpy(&b, &x, sizeof(b));
  return b;
}

int current_device() {
  int d = 0;
  HPS_HIP(hipGetDevice(&d));
  return d;
}

}  // namespace

std::shared_ptr<const LeafPlan> leaf_plan(int p, int q, double hx, double hy, hipStream_t s) {
  static PlanCache<LeafPlan> cache;
  const std::vector<long long> key{current_device(), p, q, bits(hx), bits(hy)};
  return cache.get(key, [&] {
    auto lp = std::make_shared<LeafPlan>();
    lp->lt = make_leaf_tables(p, q, hx, hy);
    const LeafTables& lt = lp->lt;
    lp->dDx = lp->mem.upload(lt.Dx, s);
    lp->dDy = lp->mem.upload(lt.Dy, s);
    lp->dDxx = lp->mem.upload(lt.Dxx, s);
    lp->dDyy = lp->mem.upload(lt.Dyy, s);
    lp->dG = lp->mem.upload(lt.G, s);
    lp->dP0 = lp->mem.upload(lt.P0, s);
    lp->dP1 = lp->mem.upload(lt.P1, s);
    const int ne = (int)lt.Je.size(), m = 4 * q;
    std::vector<double> L1t((size_t)m * ne);
    for (int r = 0; r < ne; ++r)
      for (int c = 0; c < m; ++c) L1t[(size_t)c * ne + r] = lt.L1[(size_t)r * m + c];
    lp->dL1t = lp->mem.upload(L1t, s);
    std::vector<int> post_node(lt.Ji);
    post_node.insert(post_node.end(), lt.Je.begin(), lt.Je.end());
    lp->dPostNode = lp->mem.upload(post_node, s);
    HPS_HIP(hipStreamSynchronize(s));  // the tables are read from other streams later
    return lp;
  });
}

static std::shared_ptr<const TreePlan> tree_plan(int nx, int ny, int p, int q, double hx, double hy,
                                                 bool keep, hipStream_t s) {
  static PlanCache<TreePlan> cache;
  const std::vector<long long> key{current_device(), nx, ny, p, q, bits(hx), bits(hy), keep};
  return cache.get(key, [&] {
    auto tp = std::make_shared<TreePlan>();
    tp->leaf = leaf_plan(p, q, hx, hy, s);
    tp->tree = build_tree(nx, ny, q);
    const Tree& t = tp->tree;
    std::vector<int> ids;
    box_boundary(t, 0, nx, 0, ny, ids);
    tp->n_bdry = (int)ids.size();
    const int nbox = (int)t.boxes.size();
    std::vector<int> pool;
    tp->levels.assign(t.depth + 1, {});
    std::vector<long long> lvlT(t.depth + 1, 0);
    for (int d = 0; d <= t.depth; ++d)
      for (int b : t.parents_at_level[d]) {
        const MergeMaps g = merge_maps(t, b);
        HPS_REQUIRE(g.m3 <= max_solve_rows(), "merge interface too long for the dense solver");
        MergeRec r{};
        r.box = b;
        r.pool_off = pool.size();
        r.na = g.na;
        r.nb = g.nb;
        r.me = g.me;
        r.m3 = g.m3;
        r.Toff = lvlT[d];
        lvlT[d] += (long long)g.me * g.me;
        for (const auto* v : {&g.pmap, &g.a3, &g.b3, &g.Ie, &g.Ii}) pool.insert(pool.end(), v->begin(), v->end());
        tp->levels[d].push_back(r);
      }
    tp->ar[0] = tp->ar[1] = 0;
    for (int d = 0; d <= t.depth; ++d) tp->ar[d % 2] = std::max(tp->ar[d % 2], lvlT[d]);
    // Upward-pass storage h: only merged boxes have any (a leaf's h is zero,
    // marked by offset -1), so the pass needs no clearing.
    tp->box_hoff.assign(nbox, -1);
    long long hu = 0;
    for (int b = 0; b < nbox; ++b) {
      if (t.boxes[b].ca < 0) continue;
      tp->box_hoff[b] = hu;
      hu += bdry_size(t.boxes[b], q);
    }
    tp->h_units = std::max(hu, 1LL);
    // Pool of index maps followed by the boundary ids of the root.
    tp->pool_host = std::move(pool);
    tp->gamma_off = tp->pool_host.size();
    tp->pool_host.insert(tp->pool_host.end(), ids.begin(), ids.end());
    tp->dpool = tp->mem.upload(tp->pool_host, s);
    tp->gamma = tp->dpool + tp->gamma_off;
    HPS_HIP(hipStreamSynchronize(s));
    return tp;
  });
}

std::unique_ptr<hps_op> plan_operator(const double* coeffs, const double box[4], const int nleaf[2],
                                      int p, int q, const BuildOptions& o) {
  HPS_REQUIRE(coeffs != nullptr && box != nullptr && nleaf != nullptr, "null argument");
  HPS_REQUIRE(p >= 4 && p <= 24, "p must be in [4, 24]");
  HPS_REQUIRE(q >= 1 && q < p,
              "q must satisfy 1 <= q <= p - 1 (with q >= p the corner averaging of L1 leaves a "
              "null mode at every interior cross point, so the merges are singular)");
  HPS_REQUIRE(nleaf[0] >= 1 && nleaf[1] >= 1, "nleaf must be >= 1");
  HPS_REQUIRE(std::isfinite(box[0]) && std::isfinite(box[1]) && std::isfinite(box[2]) &&
                  std::isfinite(box[3]) && box[1] > box[0] && box[3] > box[2],
              "degenerate box");
  init_runtime();
  hipStream_t s = o.stream;
  HPS_REQUIRE(!o.keep_leaf_solution || o.mode != HPS_SURROGATE,
              "keep_leaf_solution needs the FP64 leaf build (not surrogate mode)");
  // Options as the operator keeps them: body loads and the mixed forms need
  // the factors (upward pass, refinement) and the leaf operators.
  BuildOptions eo = o;
  if (o.keep_body) eo.keep_factors = true;
  if (o.mode == HPS_MIXED_SPLIT32 || o.mode == HPS_MIXED_BF16X6) {
    eo.keep_factors = true;
    eo.keep_leaf = true;
  }
  const int nx = nleaf[0], ny = nleaf[1], m = 4 * q;
  const size_t nl = (size_t)nx * ny;
  const size_t ncoef = nl * 6 * p * p;
  const bool keep = eo.keep_factors;
  // Coefficients: the caller's device buffer when only the build reads them;
  // otherwise an owned copy (body-load solves assemble the leaf systems again
  // after the build, when the caller's buffer may be gone).
  auto set_coeffs = [&](hps_op* op) {
    if (o.device_ptrs && !keep) {
      op->coeffs = coeffs;
      return;
    }
    if (!o.device_ptrs)
      for (size_t i = 0; i < ncoef; ++i)
        HPS_REQUIRE(std::isfinite(coeffs[i]), "non-finite coefficient");
    if (!op->coeffs_own) op->coeffs_own = op->mem.alloc<double>(ncoef);
    HPS_HIP(hipMemcpyAsync(op->coeffs_own, coeffs, ncoef * sizeof(double),
                           o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    op->coeffs = op->coeffs_own;
  };
  // An operator of the same shape and kept buffers, destroyed earlier, comes
  // back with its device buffers and descriptors: only the per-build state
  // is set again (coefficient sweeps skip the planning host work).
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  std::vector<long long> key{dev, nx, ny, p, q, bits(box[0]), bits(box[1]), bits(box[2]),
                             bits(box[3]), o.mode, o.device_ptrs, keep, eo.keep_leaf,
                             o.keep_leaf_solution, o.keep_body, o.root_dtn};
  if (std::unique_ptr<hps_op> op = unpark_operator(key)) {
    op->opt = eo;
    op->surrogate = o.surrogate;
    op->judge_samples = o.judge_samples;
    op->judge_tol = o.judge_tol;
    op->judge_worst = 0.0;
    op->n_judged = 0;
    op->n_fallback = 0;
    op->level_cond.clear();
    set_coeffs(op.get());
    return op;
  }
  auto op = std::make_unique<hps_op>();
  op->park_key = key;
  op->nx = nx;
  op->ny = ny;
  op->p = p;
  op->q = q;
  op->mode = o.mode;
  std::memcpy(op->box, box, sizeof(op->box));
  op->opt = eo;
  op->surrogate = o.surrogate;
  op->judge_samples = o.judge_samples;
  op->judge_tol = o.judge_tol;
  const double hx = (box[1] - box[0]) / nx, hy = (box[3] - box[2]) / ny;
  op->plan = tree_plan(nx, ny, p, q, hx, hy, keep, s);
  const TreePlan& P = *op->plan;
  const Tree& t = P.tree;
  op->n_bdry = P.n_bdry;
  op->gamma = P.gamma;
  op->h_units = P.h_units;
  set_coeffs(op.get());
  op->leafT = op->mem.alloc<double>(nl * m * m);
  if (o.keep_leaf_solution) op->leafZ = op->mem.alloc<double>(nl * (size_t)(p - 2) * (p - 2) * m);
  if (o.keep_body) op->leafK = op->mem.alloc<double>(nl * (size_t)(p - 2) * (p - 2) * m);

  // Per merge: the system W = [M | I] (whose elimination leaves M^-1), the
  // gathered right-hand sides B = [-T31a | T32b] and Q = [T13a; T23b].  S =
  // M^-1 B and the pivots are kept for every merge.  W and Q are kept too when
  // the upward pass is wanted (keep_factors); otherwise they, like B always,
  // live in one level of scratch that every level reuses.
  long long totW = 0, totQ = 0, totP = 0, totS = 0, maxW = 0, maxQ = 0, maxB = 0;
  size_t nmerges = 0;
  for (const auto& lv : P.levels) {
    long long lw = 0, lq = 0, lb = 0;
    for (const MergeRec& r : lv) {
      totS += (long long)r.m3 * r.me;
      lw += 2LL * r.m3 * r.m3;
      lq += (long long)r.me * r.m3;
      lb += (long long)r.m3 * r.me;
      totP += r.m3;
      ++nmerges;
    }
    totW += lw;
    totQ += lq;
    maxW = std::max(maxW, lw);
    maxQ = std::max(maxQ, lq);
    maxB = std::max(maxB, lb);
  }
  op->bytes_S = totS * (long long)sizeof(double);
  op->Sk = op->mem.alloc<double>(totS);
  op->Wk = op->mem.alloc<double>(keep ? totW : maxW);
  op->Q = op->mem.alloc<double>(keep ? totQ : maxQ);
  op->Bk = op->mem.alloc<double>(maxB);
  op->piv = op->mem.alloc<int>(totP);
  op->n_merges = nmerges;
  op->pstat = op->mem.alloc<unsigned long long>(2 * std::max<size_t>(nmerges, 1));
  op->arena[0] = op->mem.alloc<double>(P.ar[0]);
  op->arena[1] = op->mem.alloc<double>(P.ar[1]);

  // ---- descriptors ---------------------------------------------------------
  op->levels.assign(t.depth + 1, LevelPlan());
  op->merge_level.assign(t.boxes.size(), -1);
  op->merge_index.assign(t.boxes.size(), -1);
  long long oW = 0, oQ = 0, oP = 0, oz = 0, oS = 0, oB = 0;
  size_t mi = 0;
  const int n_int = (p - 2) * (p - 2);
  long long flops = (long long)nl * ((2LL * n_int * n_int * n_int) / 3 + 2LL * n_int * n_int * m +
                                     2LL * m * m * n_int);
  for (int d = 0; d <= t.depth; ++d) {
    LevelPlan& L = op->levels[d];
    if (!keep) oW = oQ = 0;
    oB = 0;
    for (const MergeRec& r : P.levels[d]) {
      const int b = r.box;
      const BoxRec& B = t.boxes[b];
      MergeDesc md{};
      // Ta, Tb are set below, once every parent DtN has its place.
      md.Tp = op->arena[d % 2] + r.Toff;
      md.W = op->Wk + oW;
      md.ldw = 2 * r.m3;
      md.B = op->Bk + oB;
      md.S = op->Sk + oS;
      md.lds = r.me;
      md.Q = op->Q + oQ;
      md.piv = op->piv + oP;
      md.pstat = op->pstat + 2 * mi;
      const int* base = P.dpool + r.pool_off;
      md.pmap = base;
      md.a3 = base + r.me;
      md.b3 = base + r.me + r.m3;
      md.Ie = base + r.me + 2 * r.m3;
      md.Ii = base + 2 * r.me + 2 * r.m3;
      md.na = r.na;
      md.nb = r.nb;
      md.me = r.me;
      md.m3 = r.m3;
      md.box = b;
      op->merge_level[b] = d;
      op->merge_index[b] = (int)L.h.size();
      L.h.push_back(md);
      SolveDesc sd{md.W, md.piv, md.W + r.m3, r.m3, r.m3, md.ldw, md.ldw, b, 0, md.pstat};
      L.hs.push_back(sd);
      // S = M^-1 B (FP64 in every mode).
      GemmDesc sg{md.W + r.m3, md.B, md.S, nullptr, r.m3, r.me, r.m3, md.ldw, r.me, r.me, 0, 1.0};
      sg.overwrite = 1;
      L.hsg.push_back(sg);
      if (b != 0 || op->opt.root_dtn) {
        GemmDesc gd{md.Q, md.S, md.Tp, nullptr, r.me, r.me, r.m3, r.m3, r.me, r.me, 0, 1.0,
                    md.pmap, md.Ta, md.Tb, md.na, md.nb};
        L.hg.push_back(gd);
      }
      L.ha.push_back(P.box_hoff[B.ca]);
      L.hb.push_back(P.box_hoff[B.cb]);
      auto body_off = [&](int c) {
        const BoxRec& C = t.boxes[c];
        return C.ca < 0 ? P.h_units + (long long)(C.i0 + nx * C.j0) * m : P.box_hoff[c];
      };
      L.hab.push_back(body_off(B.ca));
      L.hbb.push_back(body_off(B.cb));
      L.hp.push_back(P.box_hoff[b]);
      L.zo.push_back(oz);
      L.m3_max = std::max(L.m3_max, r.m3);
      L.me_max = std::max(L.me_max, r.me);
      L.gather_max =
          std::max(L.gather_max, (size_t)r.m3 * md.ldw + 2 * (size_t)r.me * r.m3);
      oW += 2LL * r.m3 * r.m3;
      oQ += (long long)r.me * r.m3;
      oB += (long long)r.m3 * r.me;
      oS += (long long)r.m3 * r.me;
      oP += r.m3;
      oz += r.m3;
      ++mi;
      flops += (2LL * r.m3 * r.m3 * r.m3) / 3 + 2LL * r.m3 * r.m3 * r.me;
      if (b != 0 || op->opt.root_dtn) flops += 2LL * r.me * r.me * r.m3;
    }
  }
  // Children's DtNs: leaves in leafT, inner boxes in the arena of their depth.
  // The Schur products read them too (the parent's pass-through blocks): their
  // descriptors follow the merges in order, one per merge that forms its T.
  for (int d = 0; d <= t.depth; ++d) {
    LevelPlan& L = op->levels[d];
    size_t gi = 0;
    for (MergeDesc& md : L.h) {
      const BoxRec& B = t.boxes[md.box];
      auto child_T = [&](int c) -> const double* {
        const BoxRec& C = t.boxes[c];
        if (C.ca < 0) return op->leafT + (size_t)(C.i0 + nx * C.j0) * m * m;
        return op->levels[C.level].h[op->merge_index[c]].Tp;
      };
      md.Ta = child_T(B.ca);
      md.Tb = child_T(B.cb);
      if (md.box != 0 || op->opt.root_dtn) {
        HPS_REQUIRE(gi < L.hg.size() && L.hg[gi].C == md.Tp, "Schur descriptor out of step");
        L.hg[gi].Ta = md.Ta;
        L.hg[gi].Tb = md.Tb;
        ++gi;
      }
    }
    HPS_REQUIRE(gi == L.hg.size(), "Schur descriptor count mismatch");
  }
  op->z_units = oz;
  op->flops = flops;
  op->rootT = (t.boxes[0].ca >= 0) ? op->arena[0] : op->leafT;

  // One upload of every level's descriptors from a staging buffer the
  // operator keeps (so no wait is needed here).
  size_t total = 0;
  auto reserve = [&](size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~size_t(255);
    return o;
  };
  struct Off { size_t h, hs, hg, hsg, ha, hb, hp, zo, hab, hbb; };
  std::vector<Off> offs(op->levels.size());
  for (size_t d = 0; d < op->levels.size(); ++d) {
    const LevelPlan& L = op->levels[d];
    if (L.h.empty()) continue;
    offs[d] = Off{reserve(L.h.size() * sizeof(MergeDesc)), reserve(L.hs.size() * sizeof(SolveDesc)),
                  reserve(L.hg.size() * sizeof(GemmDesc)), reserve(L.hsg.size() * sizeof(GemmDesc)),
                  reserve(L.ha.size() * 8),
                  reserve(L.hb.size() * 8), reserve(L.hp.size() * 8), reserve(L.zo.size() * 8),
                  reserve(L.hab.size() * 8), reserve(L.hbb.size() * 8)};
  }
  op->staging.assign(total, 0);
  char* dbase = (char*)op->mem.raw(std::max<size_t>(total, 1));
  for (size_t d = 0; d < op->levels.size(); ++d) {
    LevelPlan& L = op->levels[d];
    if (L.h.empty()) continue;
    const Off& f = offs[d];
    auto put = [&](size_t off, const void* src, size_t n) {
      if (n) std::memcpy(op->staging.data() + off, src, n);
      return dbase + off;
    };
    L.d = (MergeDesc*)put(f.h, L.h.data(), L.h.size() * sizeof(MergeDesc));
    L.ds = (SolveDesc*)put(f.hs, L.hs.data(), L.hs.size() * sizeof(SolveDesc));
    L.dg = (GemmDesc*)put(f.hg, L.hg.data(), L.hg.size() * sizeof(GemmDesc));
    L.dsg = (GemmDesc*)put(f.hsg, L.hsg.data(), L.hsg.size() * sizeof(GemmDesc));
    L.dha = (long long*)put(f.ha, L.ha.data(), L.ha.size() * 8);
    L.dhb = (long long*)put(f.hb, L.hb.data(), L.hb.size() * 8);
    L.dhp = (long long*)put(f.hp, L.hp.data(), L.hp.size() * 8);
    L.dzo = (long long*)put(f.zo, L.zo.data(), L.zo.size() * 8);
    L.dhab = (long long*)put(f.hab, L.hab.data(), L.hab.size() * 8);
    L.dhbb = (long long*)put(f.hbb, L.hbb.data(), L.hbb.size() * 8);
  }
  if (total) HPS_HIP(hipMemcpyAsync(dbase, op->staging.data(), total, hipMemcpyHostToDevice, s));
  return op;
}

// ---------------------------------------------------------------------------
// Leaf stage (section 3): all leaves of equal (p, q, h) share launches.
// ---------------------------------------------------------------------------
struct LeafJob {
  const LeafPlan* lp;   // leaf tables of the job's shape
  int leaf;             // leaf index (error reporting)
  const double* coef;   // [6][p*p]
  double* dst;          // [4q][4q]
  double* zdst = nullptr;  // [4q][(p-2)^2]: keeps Z^T, Z = A_ii^-1 A_ie L1, when not null
};

// On by default: 64 x 64 leaves at p = 16 built in 13.7 ms against 14.2 ms
// with the fused register kernel, 128 x 128 at p = 16 in 50.8 against 52.6,
// 32 x 32 at p = 20 in 9.7 against 11.4 (same GPU, same inputs).
static bool g_leaf_bgj = true;
static std::atomic<long long> g_leaf_bgj_fallbacks{0};
void set_leaf_bgj(bool on) { g_leaf_bgj = on; }
bool leaf_bgj_on() { return g_leaf_bgj; }
long long leaf_bgj_fallbacks() { return g_leaf_bgj_fallbacks.load(); }

static void run_leaf_group(const std::vector<LeafJob>& jobs, DeviceMem& tmp, hipStream_t s,
                           int* dstatus, int panel, double tol = 0.0) {
  const LeafPlan& L0 = *jobs[0].lp;
  const int p = L0.lt.p, q = L0.lt.q, n = (p - 2) * (p - 2), m = 4 * q, ld = n + m;
  LeafDev tab{L0.dDx, L0.dDy, L0.dDxx, L0.dDyy, L0.dG, p, n, m, 0};
  bool keepZ = false;
  for (const LeafJob& j : jobs) keepZ = keepZ || j.zdst;
  if (!keepZ && leaf_mfma_fits(n, m)) {
    // MFMA leaf kernel: T straight from the coefficients, Z never stored.
    const int total = (int)jobs.size();
    std::vector<const double*> cp(total);
    std::vector<double*> td(total);
    for (int i = 0; i < total; ++i) {
      cp[i] = jobs[i].coef;
      td[i] = jobs[i].dst;
    }
    const double** dcp = tmp.alloc<const double*>(total);
    double** dtd = tmp.alloc<double*>(total);
    HPS_HIP(hipMemcpyAsync(dcp, cp.data(), total * sizeof(void*), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(dtd, td.data(), total * sizeof(void*), hipMemcpyHostToDevice, s));
    leaf_dtn_mfma(dcp, tab, L0.dP0, L0.dP1, dtd, total, dstatus, -(jobs[0].leaf + 1), s, tol);
    HPS_HIP(hipStreamSynchronize(s));  // the host pointer arrays are freed on return
    return;
  }
  // Blocked Gauss-Jordan on the assembled systems (pivoting inside 64 x 64
  // diagonal blocks, the chunk redone with partial pivoting should a block
  // pivot be small) instead of the fused register kernel or the panel solver.
  const bool use_bgj = leaf_bgj_on() && n >= 64;
  const bool fused = !use_bgj && leaf_lu_fits(n, m);
  // Fused path: only Z (n x m) per leaf; generic path: the augmented system.
  const size_t per = fused ? (size_t)n * m * sizeof(double)
                           : (size_t)n * ld * sizeof(double) + (size_t)n * sizeof(int);
  const size_t budget = (size_t)2 << 30;
  const int total = (int)jobs.size();
  const int CH = (int)std::max<size_t>(1, std::min<size_t>(total, budget / per));
  double* Wslab = tmp.alloc<double>(fused ? (size_t)CH * n * m : (size_t)CH * n * ld);
  int* pslab = fused ? nullptr : tmp.alloc<int>((size_t)CH * n);
  const double** dcp = tmp.alloc<const double*>(CH);
  SolveDesc* dsd = fused ? nullptr : tmp.alloc<SolveDesc>(CH);
  GemmDesc* dgd = tmp.alloc<GemmDesc>(CH);
  const double** dzs = keepZ ? tmp.alloc<const double*>(CH) : nullptr;
  double** dzd = keepZ ? tmp.alloc<double*>(CH) : nullptr;
  // Pivot statistics of the generic path's systems (relative pivot test, and
  // max|A_ii| for the blocked path's fall-back test).
  unsigned long long* dps = (!fused && (tol > 0.0 || use_bgj))
                                ? tmp.alloc<unsigned long long>(2 * (size_t)CH)
                                : nullptr;
  double* binv = use_bgj ? tmp.alloc<double>((size_t)CH * 64 * 64) : nullptr;
  for (int c0 = 0; c0 < total; c0 += CH) {
    const int cnt = std::min(CH, total - c0);
    std::vector<const double*> cp(cnt);
    std::vector<SolveDesc> sd(fused ? 0 : cnt);
    std::vector<GemmDesc> gd(cnt);
    for (int i = 0; i < cnt; ++i) {
      const LeafJob& j = jobs[c0 + i];
      cp[i] = j.coef;
      if (fused) {
        double* Zl = Wslab + (size_t)i * n * m;
        gd[i] = GemmDesc{j.lp->dP1, Zl, j.dst, j.lp->dP0, m, m, n, n, m, m, m, -1.0};
      } else {
        double* W = Wslab + (size_t)i * n * ld;
        sd[i] = SolveDesc{W, pslab + (size_t)i * n, W + n, n, m, ld, ld, -(j.leaf + 1), 0,
                          dps ? dps + 2 * (size_t)i : nullptr};
        gd[i] = GemmDesc{j.lp->dP1, W + n, j.dst, j.lp->dP0, m, m, n, n, ld, m, m, -1.0};
      }
    }
    HPS_HIP(hipMemcpyAsync(dcp, cp.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(dgd, gd.data(), cnt * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
    if (fused) {
      leaf_lu(dcp, tab, cnt, Wslab, dstatus, -(jobs[c0].leaf + 1), s, tol);
    } else {
      HPS_HIP(hipMemcpyAsync(dsd, sd.data(), cnt * sizeof(SolveDesc), hipMemcpyHostToDevice, s));
      leaf_assemble(dcp, tab, cnt, Wslab, s);
      if (dps) {
        pstat_init(dps, cnt, s);
        system_absmax(dsd, cnt, n, s);
      }
      bool solved = false;
      if (use_bgj) {
        set_int(dstatus + 3, 0, s);
        batched_solve_bgj(dsd, sd, dstatus, binv, s, false);
        int fb = 0;
        HPS_HIP(hipMemcpyAsync(&fb, dstatus + 3, sizeof(int), hipMemcpyDeviceToHost, s));
        HPS_HIP(hipStreamSynchronize(s));
        solved = fb == 0;
        if (!solved) {
          g_leaf_bgj_fallbacks.fetch_add(1);
          leaf_assemble(dcp, tab, cnt, Wslab, s);
          pstat_init(dps, cnt, s);
          system_absmax(dsd, cnt, n, s);
        }
      }
      if (!solved) batched_solve(dsd, sd, dstatus, s, panel);
      if (dps && tol > 0.0) pivot_check(dsd, cnt, tol, dstatus, s);
    }
    grouped_gemm(dgd, gd, s, GEMM_F64, PROF_LEAF_GEMM);
    // Kept Z goes out transposed ([4q][(p-2)^2]) for the post-processing loads.
    std::vector<const double*> zs;  // live until the chunk's synchronization below
    std::vector<double*> zd;
    if (keepZ) {
      for (int i = 0; i < cnt; ++i)
        if (jobs[c0 + i].zdst) {
          zs.push_back(fused ? Wslab + (size_t)i * n * m : Wslab + (size_t)i * n * ld + n);
          zd.push_back(jobs[c0 + i].zdst);
        }
      if (!zs.empty()) {
        HPS_HIP(hipMemcpyAsync(dzs, zs.data(), zs.size() * sizeof(void*), hipMemcpyHostToDevice, s));
        HPS_HIP(hipMemcpyAsync(dzd, zd.data(), zd.size() * sizeof(void*), hipMemcpyHostToDevice, s));
        transpose_rows_batch(dzs, dzd, (int)zs.size(), n, m, fused ? m : ld, s);
      }
    }
    HPS_HIP(hipStreamSynchronize(s));  // host descriptor vectors are reused next chunk
  }
}

// Kept body operator (keep_body_operator): K^T = A_ii^-T P1^T for every leaf
// by the batched dense solver on [A_ii^T | P1^T], copied to op->leafK as
// [n][m].  A body-load solve then needs h = K g per leaf only.
static void body_operator_stage(hps_op* op, DeviceMem& tmp, hipStream_t s, int* dstatus) {
  const LeafPlan& LP = op->leaf();
  const int p = op->p, n = (p - 2) * (p - 2), m = 4 * op->q, nl = op->nx * op->ny, ld = n + m;
  HPS_REQUIRE(n <= max_solve_rows(), "leaf too large for the dense solver");
  LeafDev tab{LP.dDx, LP.dDy, LP.dDxx, LP.dDyy, LP.dG, p, n, m, 0};
  const size_t per = (size_t)n * ld * sizeof(double) + (size_t)n * sizeof(int);
  const int CH = (int)std::max<size_t>(1, std::min<size_t>(nl, ((size_t)2 << 30) / per));
  double* Wslab = tmp.alloc<double>((size_t)CH * n * ld);
  int* pslab = tmp.alloc<int>((size_t)CH * n);
  const double** dcp = tmp.alloc<const double*>(CH);
  SolveDesc* dsd = tmp.alloc<SolveDesc>(CH);
  const double** dsrc = tmp.alloc<const double*>(CH);
  double** ddst = tmp.alloc<double*>(CH);
  for (int c0 = 0; c0 < nl; c0 += CH) {
    const int cnt = std::min(CH, nl - c0);
    std::vector<const double*> cp(cnt), src(cnt);
    std::vector<double*> dst(cnt);
    std::vector<SolveDesc> sd(cnt);
    for (int i = 0; i < cnt; ++i) {
      double* Wl = Wslab + (size_t)i * n * ld;
      cp[i] = op->coeffs + (size_t)(c0 + i) * 6 * p * p;
      sd[i] = SolveDesc{Wl, pslab + (size_t)i * n, Wl + n, n, m, ld, ld, -(c0 + i + 1), 0};
      src[i] = Wl + n;
      dst[i] = op->leafK + (size_t)(c0 + i) * n * m;
    }
    HPS_HIP(hipMemcpyAsync(dcp, cp.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(dsd, sd.data(), cnt * sizeof(SolveDesc), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(dsrc, src.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(ddst, dst.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, s));
    leaf_assemble_body_operator(dcp, tab, cnt, Wslab, LP.dP1, s);
    batched_solve(dsd, sd, dstatus, s, 32);
    copy_rows_batch(dsrc, ddst, cnt, n, m, ld, s);
    HPS_HIP(hipStreamSynchronize(s));  // host descriptor vectors are reused next chunk
  }
}

// Leaf stage of a surrogate operator: inference for every leaf, then the judge
// re-solves a seeded sample of leaves plus every leaf whose coefficients leave
// the training ranges with the FP64 leaf solver; judged leaves above the
// tolerance are replaced, and if more than a quarter of the random sample
// fails, every leaf is rebuilt by the FP64 solver.
static void surrogate_leaf_stage(hps_op* op, DeviceMem& tmp, hipStream_t s, int* dstatus) {
  hps_surrogate* sg = op->surrogate;
  HPS_REQUIRE(sg && sg->fitted, "surrogate mode needs a trained surrogate");
  HPS_REQUIRE(sg->p == op->p && sg->q == op->q, "surrogate was trained for another p, q");
  HPS_REQUIRE(std::fabs(sg->hx - op->leaf().lt.hx) <= 1e-12 * sg->hx &&
                  std::fabs(sg->hy - op->leaf().lt.hy) <= 1e-12 * sg->hy,
              "surrogate was trained for another leaf size");
  const int nl = op->nx * op->ny, p = op->p, m = 4 * op->q, mm = m * m, pp = p * p;
  std::vector<const double*> cp(nl);
  std::vector<double*> tp(nl);
  for (int l = 0; l < nl; ++l) {
    cp[l] = op->coeffs + (size_t)l * 6 * pp;
    tp[l] = op->leafT + (size_t)l * mm;
  }
  const double** dcp = tmp.upload(cp, s);
  double** dtp = tmp.upload(tp, s);
  surrogate_predict(sg, dcp, nl, dtp, s);
  // Out-of-distribution flags (10% margin on each field's training range).
  std::vector<double> lohi = {sg->lo[0], sg->lo[1], sg->lo[2], sg->hi[0], sg->hi[1], sg->hi[2]};
  double* dlohi = tmp.upload(lohi, s);
  int* dflag = tmp.alloc<int>(nl);
  leaf_range_flags(dcp, nl, pp, dlohi, 0.1, dflag, s);
  std::vector<int> flag(nl);
  HPS_HIP(hipMemcpyAsync(flag.data(), dflag, nl * sizeof(int), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  std::vector<int> judged;
  std::vector<char> is_sample(nl, 0);
  const int J = std::min(nl, std::max(1, op->judge_samples));
  std::mt19937_64 rng(0x5eedULL + (unsigned long long)nl);
  for (int i = 0; i < J; ++i) {
    int l = (int)(rng() % (unsigned long long)nl);
    if (!is_sample[l]) {
      is_sample[l] = 1;
      judged.push_back(l);
    }
  }
  for (int l = 0; l < nl; ++l)
    if (flag[l] && !is_sample[l]) judged.push_back(l);
  const int nj = (int)judged.size();
  op->n_judged = nj;
  double* ref = tmp.alloc<double>((size_t)nj * mm);
  std::vector<LeafJob> jobs(nj);
  std::vector<double*> jp(nj);
  for (int i = 0; i < nj; ++i) {
    jobs[i] = LeafJob{&op->leaf(), judged[i], cp[judged[i]], ref + (size_t)i * mm};
    jp[i] = tp[judged[i]];
  }
  run_leaf_group(jobs, tmp, s, dstatus, op->opt.panel, op->opt.pivot_tol);
  double** djp = tmp.upload(jp, s);
  double* derr = tmp.alloc<double>(nj);
  block_errors(djp, ref, nj, mm, derr, s);
  std::vector<double> err(nj);
  HPS_HIP(hipMemcpyAsync(err.data(), derr, nj * sizeof(double), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  int bad_sample = 0, replaced = 0;
  double worst = 0.0;
  for (int i = 0; i < nj; ++i) {
    const bool bad = !(err[i] <= op->judge_tol);
    if (bad) ++replaced;
    if (bad && is_sample[judged[i]]) ++bad_sample;
    if (is_sample[judged[i]]) worst = std::max(worst, err[i]);
  }
  op->judge_worst = worst;
  if (4 * bad_sample > J) {
    // The surrogate is not good enough for this field: plain leaf build everywhere.
    std::vector<LeafJob> all(nl);
    for (int l = 0; l < nl; ++l) all[l] = LeafJob{&op->leaf(), l, cp[l], tp[l]};
    run_leaf_group(all, tmp, s, dstatus, op->opt.panel, op->opt.pivot_tol);
    op->n_fallback = nl;
  } else {
    block_replace(djp, ref, nj, mm, derr, op->judge_tol, s);
    op->n_fallback = replaced;
  }
  HPS_HIP(hipStreamSynchronize(s));
}

// Levels whose blocked Gauss-Jordan fell back to partial pivoting (all builds).
static std::atomic<long long> g_bgj_fallbacks{0};

long long bgj_fallbacks() { return g_bgj_fallbacks.load() + g_leaf_bgj_fallbacks.load(); }

void run_build(const std::vector<hps_op*>& ops, hipStream_t s) {
  DeviceMem tmp;
  int* dstatus = tmp.alloc<int>(4);
  HPS_HIP(hipMemsetAsync(dstatus, 0, 4 * sizeof(int), s));
  for (hps_op* op : ops)
    if (op->opt.device_ptrs)
      nonfinite(op->coeffs, (size_t)op->nx * op->ny * 6 * op->p * op->p, dstatus + 2, s);

  // Leaf groups keyed by (p, q, hx, hy); surrogate operators infer their leaves instead.
  std::map<std::tuple<int, int, double, double>, std::vector<LeafJob>> groups;
  const int panel = ops.empty() ? 32 : ops[0]->opt.panel;
  const double tol = ops.empty() ? 0.0 : ops[0]->opt.pivot_tol;  // one value per batch
  for (hps_op* op : ops) pstat_init(op->pstat, op->n_merges, s);
  for (hps_op* op : ops) {
    if (op->mode == HPS_SURROGATE) {
      surrogate_leaf_stage(op, tmp, s, dstatus);
      continue;
    }
    auto key = std::make_tuple(op->p, op->q, op->leaf().lt.hx, op->leaf().lt.hy);
    auto& v = groups[key];
    const int m = 4 * op->q;
    for (int l = 0; l < op->nx * op->ny; ++l)
      v.push_back(LeafJob{&op->leaf(), l, op->coeffs + (size_t)l * 6 * op->p * op->p,
                          op->leafT + (size_t)l * m * m,
                          op->leafZ ? op->leafZ + (size_t)l * op->leaf().lt.n * m : nullptr});
  }
  for (auto& kv : groups) run_leaf_group(kv.second, tmp, s, dstatus, panel, tol);
  for (hps_op* op : ops)
    if (op->leafK) body_operator_stage(op, tmp, s, dstatus);

  // Merges, deepest level first; all operators' merges at one depth together.
  int maxd = 0;
  for (hps_op* op : ops) maxd = std::max(maxd, (int)op->levels.size() - 1);
  // Arithmetic of the Schur products (one mode per batch).
  const int prec = ops.empty() ? GEMM_F64
                   : ops[0]->mode == HPS_MIXED_SPLIT32 ? GEMM_SPLIT32
                   : ops[0]->mode == HPS_MIXED_BF16X6 ? GEMM_BF16X6 : GEMM_F64;
  for (int d = maxd; d >= 0; --d) {
    std::vector<const LevelPlan*> parts;
    for (hps_op* op : ops) {
      if (d >= (int)op->levels.size() || op->levels[d].h.empty()) continue;
      parts.push_back(&op->levels[d]);
    }
    if (parts.empty()) continue;
    // One operator at this depth: its own host and device descriptors.  Several:
    // the concatenation, uploaded for this level.
    std::vector<MergeDesc> cm;
    std::vector<SolveDesc> cs;
    std::vector<GemmDesc> cg, csg;
    const MergeDesc* dm;
    const SolveDesc* dsd;
    const GemmDesc *dgd, *dsg;
    if (parts.size() == 1) {
      dm = parts[0]->d;
      dsd = parts[0]->ds;
      dgd = parts[0]->dg;
      dsg = parts[0]->dsg;
    } else {
      for (const LevelPlan* L : parts) {
        cm.insert(cm.end(), L->h.begin(), L->h.end());
        cs.insert(cs.end(), L->hs.begin(), L->hs.end());
        cg.insert(cg.end(), L->hg.begin(), L->hg.end());
        csg.insert(csg.end(), L->hsg.begin(), L->hsg.end());
      }
      MergeDesc* a = tmp.upload(cm, s);
      SolveDesc* b = tmp.upload(cs, s);
      GemmDesc* c = tmp.upload(cg, s);
      GemmDesc* e = tmp.upload(csg, s);
      HPS_HIP(hipStreamSynchronize(s));
      dm = a;
      dsd = b;
      dgd = c;
      dsg = e;
    }
    const std::vector<MergeDesc>& hm = parts.size() == 1 ? parts[0]->h : cm;
    const std::vector<SolveDesc>& hs = parts.size() == 1 ? parts[0]->hs : cs;
    const std::vector<GemmDesc>& hg = parts.size() == 1 ? parts[0]->hg : cg;
    const std::vector<GemmDesc>& hsg = parts.size() == 1 ? parts[0]->hsg : csg;
    int kmax = 0, m3max = 0, memax = 0;
    for (const MergeDesc& md : hm) {
      m3max = std::max(m3max, md.m3);
      memax = std::max(memax, md.me);
    }
    for (const GemmDesc& g : hg) kmax = std::max(kmax, g.K);
    const int schur_prec = prec == GEMM_BF16X6 && kmax < bf16x6_min_k() ? GEMM_F64 : prec;
    if (merge_small_on() && schur_prec == GEMM_F64 && m3max <= MERGE_SMALL_MAX_M3 &&
        merge_small_lds(m3max, memax) <= MERGE_SMALL_MAX_LDS) {
      // Small merges: the whole level in one launch.
      bool keep = false, root_T = false;
      for (hps_op* op : ops) {
        keep = keep || op->opt.keep_factors;
        root_T = root_T || op->opt.root_dtn;
      }
      merge_small(dm, hm, keep, root_T, dstatus, s);
      continue;
    }
    merge_gather(dm, hm, s);
    int nmax_level = 0;
    for (const SolveDesc& sd : hs) nmax_level = std::max(nmax_level, sd.n);
    bool solved = false;
    if (bgj_min_rows() > 0 && nmax_level >= bgj_min_rows()) {
      // Large systems: blocked Gauss-Jordan with pivoting inside 64 x 64
      // diagonal blocks; should a block pivot be too small, the level is
      // gathered again and solved with partial pivoting.
      double* binv = tmp.alloc<double>(hs.size() * 64 * 64);
      set_int(dstatus + 3, 0, s);
      batched_solve_bgj(dsd, hs, dstatus, binv, s);
      int fb = 0;
      HPS_HIP(hipMemcpyAsync(&fb, dstatus + 3, sizeof(int), hipMemcpyDeviceToHost, s));
      HPS_HIP(hipStreamSynchronize(s));
      solved = fb == 0;
      if (!solved) {
        g_bgj_fallbacks.fetch_add(1);
        merge_gather(dm, hm, s);
        pstat_reset_min(dsd, (int)hs.size(), s);
      }
    }
    if (!solved) batched_solve(dsd, hs, dstatus, s, panel);
    if (parts.size() > 1 && gemm_queue_on()) {
      // Merges of several problems: one persistent launch per product over
      // a largest-first tile queue.
      int* counter = tmp.alloc<int>(1);
      std::vector<TileRef> qs = gemm_tile_queue(hsg);
      TileRef* dqs = tmp.upload(qs, s);
      grouped_gemm_queue(dsg, hsg, dqs, (int)qs.size(), counter, s, PROF_MERGE_S);
      if (schur_prec == GEMM_F64) {
        std::vector<TileRef> qg = gemm_tile_queue(hg);
        TileRef* dqg = tmp.upload(qg, s);
        grouped_gemm_queue(dgd, hg, dqg, (int)qg.size(), counter, s, PROF_GEMM);
        HPS_HIP(hipStreamSynchronize(s));  // the host tile lists die here
      } else {
        HPS_HIP(hipStreamSynchronize(s));
        grouped_gemm(dgd, hg, s, schur_prec);
      }
      continue;
    }
    grouped_gemm(dsg, hsg, s, GEMM_F64, PROF_MERGE_S);
    grouped_gemm(dgd, hg, s, schur_prec);
  }
  int st[4];
  HPS_HIP(hipMemcpyAsync(st, dstatus, sizeof(st), hipMemcpyDeviceToHost, s));
  // Pivot statistics of every merge: the per-depth condition estimates and
  // the relative pivot test.
  std::vector<std::vector<unsigned long long>> ps(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    ps[i].resize(2 * ops[i]->n_merges);
    if (!ps[i].empty())
      HPS_HIP(hipMemcpyAsync(ps[i].data(), ops[i]->pstat, ps[i].size() * 8, hipMemcpyDeviceToHost, s));
  }
  HPS_HIP(hipStreamSynchronize(s));
  if (st[2]) throw Error(HPS_EINVAL, "non-finite coefficient");
  if (st[0]) {
    std::string where = st[1] < 0 ? "leaf " + std::to_string(-st[1] - 1)
                                  : "merge of box " + std::to_string(st[1]);
    throw Error(HPS_ESINGULAR, tol > 0.0 && st[1] < 0
                                   ? "pivot below pivot_tol * max|A_ii| in " + where
                                   : "zero or non-finite pivot in " + where);
  }
  for (size_t i = 0; i < ops.size(); ++i) {
    hps_op* op = ops[i];
    op->level_cond.assign(op->levels.size(), 0.0);
    size_t k = 0;
    for (size_t d = 0; d < op->levels.size(); ++d)
      for (const MergeDesc& md : op->levels[d].h) {
        double amax, pmin;
        std::memcpy(&amax, &ps[i][2 * k], 8);
        const unsigned long long pb = ps[i][2 * k + 1];
        if (pb >= 0x7FF0000000000000ull) pmin = INFINITY;
        else std::memcpy(&pmin, &pb, 8);
        ++k;
        const double est = pmin > 0.0 ? amax / pmin : INFINITY;
        op->level_cond[d] = std::max(op->level_cond[d], est);
        if (tol > 0.0 && !(pmin > tol * amax)) {
          char buf[200];
          std::snprintf(buf, sizeof(buf),
                        "merge of box %d (depth %d): min |pivot| %.3e <= pivot_tol * max|M| = %.3e",
                        md.box, (int)d, pmin, tol * amax);
          throw Error(HPS_ESINGULAR, buf);
        }
      }
  }
}

void leaf_dtn_batch(const double* coeffs, int nleaf, double hx, double hy, int p, int q, double* T,
                    hipStream_t s) {
  HPS_REQUIRE(p >= 4 && p <= 24 && q >= 1 && q < p && nleaf >= 1,
              "bad leaf batch arguments (need 4 <= p <= 24, 1 <= q <= p - 1, nleaf >= 1)");
  init_runtime();
  std::shared_ptr<const LeafPlan> lp = leaf_plan(p, q, hx, hy, s);
  std::vector<LeafJob> jobs(nleaf);
  const int m = 4 * q;
  for (int i = 0; i < nleaf; ++i)
    jobs[i] = LeafJob{lp.get(), i, coeffs + (size_t)i * 6 * p * p, T + (size_t)i * m * m};
  DeviceMem tmp;
  int* dstatus = tmp.alloc<int>(4);
  HPS_HIP(hipMemsetAsync(dstatus, 0, 4 * sizeof(int), s));
  run_leaf_group(jobs, tmp, s, dstatus, 32);
  int st[4];
  HPS_HIP(hipMemcpyAsync(st, dstatus, sizeof(st), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  if (st[0]) throw Error(HPS_ESINGULAR, "zero pivot in leaf " + std::to_string(-st[1] - 1));
}

// ---------------------------------------------------------------------------
// Solve (Algorithm 2) and the refinement pieces.
// ---------------------------------------------------------------------------
// Algorithm 2 over a batch: for every depth, the merges of all problems in
// one launch (each merge carries its problem's solution array).
static void downward_batch(const std::vector<hps_op*>& ops, const std::vector<double*>& u,
                           const std::vector<int>& nrhs, const double* z, hipStream_t s) {
  if (ops.size() == 1) {
    hps_op* op = ops[0];
    const SolveIO io0{u[0], op->tree().N, nrhs[0]};
    for (size_t d = 0; d < op->levels.size(); ++d) {
      const LevelPlan& L = op->levels[d];
      if (L.h.empty()) continue;
      double sb = 0;
      for (const MergeDesc& m : L.h) sb += 8.0 * m.m3 * m.me;
      downward(L.d, nullptr, io0, (int)L.h.size(), L.m3_max, L.me_max, nrhs[0], z,
               z ? L.dzo : nullptr, s, sb);
    }
    return;
  }
  int maxd = 0;
  for (hps_op* op : ops) maxd = std::max(maxd, (int)op->levels.size() - 1);
  std::vector<MergeDesc> hm;
  std::vector<SolveIO> hio;
  std::vector<size_t> off(maxd + 2, 0);
  std::vector<int> m3m(maxd + 1, 0), mem(maxd + 1, 0), nrm(maxd + 1, 0);
  std::vector<double> sb(maxd + 1, 0.0);
  for (int d = 0; d <= maxd; ++d) {
    off[d] = hm.size();
    for (size_t i = 0; i < ops.size(); ++i) {
      hps_op* op = ops[i];
      if (d >= (int)op->levels.size()) continue;
      for (const MergeDesc& m : op->levels[d].h) {
        hm.push_back(m);
        hio.push_back(SolveIO{u[i], op->tree().N, nrhs[i]});
        m3m[d] = std::max(m3m[d], m.m3);
        mem[d] = std::max(mem[d], m.me);
        nrm[d] = std::max(nrm[d], nrhs[i]);
        sb[d] += 8.0 * m.m3 * m.me;
      }
    }
  }
  off[maxd + 1] = hm.size();
  if (hm.empty()) return;
  MergeDesc* dm = nullptr;
  SolveIO* dio = nullptr;
  HPS_HIP(hipMallocAsync((void**)&dm, hm.size() * sizeof(MergeDesc), s));
  HPS_HIP(hipMallocAsync((void**)&dio, hio.size() * sizeof(SolveIO), s));
  HPS_HIP(hipMemcpyAsync(dm, hm.data(), hm.size() * sizeof(MergeDesc), hipMemcpyHostToDevice, s));
  HPS_HIP(hipMemcpyAsync(dio, hio.data(), hio.size() * sizeof(SolveIO), hipMemcpyHostToDevice, s));
  for (int d = 0; d <= maxd; ++d) {
    const int nm = (int)(off[d + 1] - off[d]);
    if (nm == 0) continue;
    const long long* zo = z ? ops[0]->levels[d].dzo : nullptr;
    downward(dm + off[d], dio + off[d], SolveIO{nullptr, 0, 0}, nm, m3m[d], mem[d], nrm[d], z, zo,
             s, sb[d]);
  }
  HPS_HIP(hipFreeAsync(dm, s));
  HPS_HIP(hipFreeAsync(dio, s));
  HPS_HIP(hipStreamSynchronize(s));  // host vectors above must outlive the copies
}

static void downward_all(hps_op* op, double* u, int nrhs, const double* z, hipStream_t s) {
  downward_batch({op}, {u}, {nrhs}, z, s);
}

// Right-hand-side count from which solves run on node-major arrays
// ([nodes][nrhs]) with FP64 MFMA GEMMs: the factors are then read once per
// 64 right-hand sides instead of once per four.  0: never.
static int g_mm_min_rhs = 16;

void set_solve_mm_min_rhs(int v) { g_mm_min_rhs = v; }

static bool use_mm(int nrhs) { return g_mm_min_rhs > 0 && nrhs >= g_mm_min_rhs; }

static double level_s_bytes(const LevelPlan& L) {
  double sb = 0;
  for (const MergeDesc& m : L.h) sb += 8.0 * m.m3 * m.me;
  return sb;
}

// Algorithm 2 on node-major arrays U[i] ([N_i][nrhs_i]); for every depth the
// merges of all operators in one launch.  z: upward-pass terms (one
// operator only), node-major per merge.
static void downward_batch_nm(const std::vector<hps_op*>& ops, const std::vector<double*>& U,
                              const std::vector<int>& nrhs, const double* z, hipStream_t s) {
  if (ops.size() == 1) {
    hps_op* op = ops[0];
    for (const LevelPlan& L : op->levels)
      if (!L.h.empty())
        downward_mm(L.d, (int)L.h.size(), L.m3_max, L.me_max, U[0], nrhs[0], z,
                    z ? L.dzo : nullptr, s, level_s_bytes(L));
    return;
  }
  HPS_REQUIRE(z == nullptr, "batched downward pass takes no source terms");
  int maxd = 0;
  for (hps_op* op : ops) maxd = std::max(maxd, (int)op->levels.size() - 1);
  std::vector<MergeDesc> hm;
  std::vector<SolveIO> hio;
  std::vector<size_t> off(maxd + 2, 0);
  std::vector<int> m3m(maxd + 1, 0), mem(maxd + 1, 0), nrm(maxd + 1, 0);
  std::vector<double> sb(maxd + 1, 0.0);
  for (int d = 0; d <= maxd; ++d) {
    off[d] = hm.size();
    for (size_t i = 0; i < ops.size(); ++i) {
      if (d >= (int)ops[i]->levels.size()) continue;
      for (const MergeDesc& m : ops[i]->levels[d].h) {
        hm.push_back(m);
        hio.push_back(SolveIO{U[i], ops[i]->tree().N, nrhs[i]});
        m3m[d] = std::max(m3m[d], m.m3);
        mem[d] = std::max(mem[d], m.me);
        nrm[d] = std::max(nrm[d], nrhs[i]);
        sb[d] += 8.0 * m.m3 * m.me;
      }
    }
  }
  off[maxd + 1] = hm.size();
  if (hm.empty()) return;
  MergeDesc* dm = nullptr;
  SolveIO* dio = nullptr;
  HPS_HIP(hipMallocAsync((void**)&dm, hm.size() * sizeof(MergeDesc), s));
  HPS_HIP(hipMallocAsync((void**)&dio, hio.size() * sizeof(SolveIO), s));
  HPS_HIP(hipMemcpyAsync(dm, hm.data(), hm.size() * sizeof(MergeDesc), hipMemcpyHostToDevice, s));
  HPS_HIP(hipMemcpyAsync(dio, hio.data(), hio.size() * sizeof(SolveIO), hipMemcpyHostToDevice, s));
  for (int d = 0; d <= maxd; ++d) {
    const int nm = (int)(off[d + 1] - off[d]);
    if (nm > 0)
      downward_mm(dm + off[d], nm, m3m[d], mem[d], nullptr, nrm[d], nullptr, nullptr, s, sb[d],
                  dio + off[d]);
  }
  HPS_HIP(hipFreeAsync(dm, s));
  HPS_HIP(hipFreeAsync(dio, s));
  HPS_HIP(hipStreamSynchronize(s));  // host vectors above must outlive the copies
}

// Upward pass for node-major sources src ([N][nrhs]): fills z ([m3][nrhs]
// per merge); h and rb are scratch (h_units and z_units per right-hand side).
static void upward_all_nm(hps_op* op, const double* src, int nrhs, double* h, double* z,
                          double* rb, hipStream_t s) {
  HPS_REQUIRE(op->opt.keep_factors, "operator was built without keep_factors");
  for (int d = (int)op->levels.size() - 1; d >= 0; --d) {
    const LevelPlan& L = op->levels[d];
    if (L.h.empty()) continue;
    double fl = 0;
    for (const MergeDesc& m : L.h) fl += 2.0 * nrhs * ((double)m.m3 * m.m3 + (double)m.me * m.m3);
    upward_level_nm(L.d, (int)L.h.size(), L.m3_max, L.me_max, src, h, L.dha, L.dhb, L.dhp, rb, z,
                    L.dzo, nrhs, fl, s);
  }
}

// Device buffer freed on the stream at scope exit.
struct AsyncBuf {
  double* p = nullptr;
  hipStream_t s;
  AsyncBuf(size_t n, hipStream_t st) : s(st) {
    HPS_HIP(hipMallocAsync((void**)&p, std::max<size_t>(n, 1) * sizeof(double), s));
  }
  ~AsyncBuf() { (void)hipFreeAsync(p, s); }
  AsyncBuf(const AsyncBuf&) = delete;
  AsyncBuf& operator=(const AsyncBuf&) = delete;
};

static void solve_mm(hps_op* op, const double* f, int nrhs, double* u, hipStream_t s) {
  keep_async_pool();
  const int N = op->tree().N;
  AsyncBuf U((size_t)N * nrhs, s);
  set_boundary_nm(f, op->gamma, op->n_bdry, nrhs, U.p, s);
  downward_batch_nm({op}, {U.p}, {nrhs}, nullptr, s);
  transpose(U.p, N, nrhs, u, s);
}

static bool g_solve_graph = true;

void set_solve_graph(bool on) { g_solve_graph = on; }

// Algorithm 2 as one graph per right-hand-side count: the boundary data go
// into u, then one downward launch per level.  Captured once on a private
// stream (kernels read f and u from op->d_io, so the graph's arguments never
// change) and replayed on the caller's stream after d_io is refreshed.
// Off by default: on config 2 (64 x 64 leaves, 13 levels, one right-hand
// side) the cooperative pass took 313 us against 162 us for the captured
// level-by-level graph; its grid barriers (512 workgroups counting in across
// eight XCDs, then polling) cost more than the graph's launch gaps.
static bool g_solve_persist = false;
void set_solve_persist(bool on) { g_solve_persist = on; }

// Plans the persistent downward pass of op once: one PersistLevel per depth,
// root first; operators with merges of different shapes at one depth keep
// the level-by-level passes.
static bool persist_ready(hps_op* op, hipStream_t s) {
  if (op->persist_state != 0) return op->persist_state > 0;
  std::vector<PersistLevel> lv;
  for (const LevelPlan& L : op->levels) {
    if (L.h.empty()) continue;
    const int m3 = L.h[0].m3, me = L.h[0].me;
    for (const MergeDesc& m : L.h)
      if (m.m3 != m3 || m.me != me) {
        op->persist_state = -1;
        return false;
      }
    lv.push_back(PersistLevel{L.d, (int)L.h.size(), m3, me, 0});
  }
  op->persist_levels = op->mem.alloc<PersistLevel>(std::max<size_t>(lv.size(), 1));
  op->persist_bar = op->mem.alloc<unsigned>(9 * 32);  // top and eight group counters
  op->persist_err = op->mem.alloc<int>(1);
  if (!lv.empty())
    HPS_HIP(hipMemcpyAsync(op->persist_levels, lv.data(), lv.size() * sizeof(PersistLevel),
                           hipMemcpyHostToDevice, s));
  HPS_HIP(hipStreamSynchronize(s));
  op->persist_nlev = (int)lv.size();
  op->persist_state = 1;
  return true;
}

void solve_device(hps_op* op, const double* f, int nrhs, double* u, hipStream_t s) {
  if (use_mm(nrhs)) {
    solve_mm(op, f, nrhs, u, s);
    return;
  }
  if (g_solve_persist && persist_ready(op, s)) {
    // Every level in one cooperative launch (no per-level launch or graph).
    double sb = 0;
    for (const LevelPlan& L : op->levels)
      for (const MergeDesc& m : L.h) sb += 8.0 * m.m3 * m.me;
    int err = 0;
    {
      ProfScope ps(PROF_DOWNWARD, s, 2.0 * nrhs * sb / 8.0, sb);
      downward_persist(op->persist_levels, op->persist_nlev, f, op->gamma, op->n_bdry, u,
                       op->tree().N, nrhs, op->persist_bar, op->persist_err, s);
    }
    HPS_HIP(hipMemcpyAsync(&err, op->persist_err, sizeof(int), hipMemcpyDeviceToHost, s));
    HPS_HIP(hipStreamSynchronize(s));
    if (err) throw Error(HPS_EDEVICE, "persistent downward pass: a level barrier timed out");
    return;
  }
  // The first solve with a right-hand-side count runs launch by launch; the
  // graph is captured on the second (an operator solved once does not pay
  // for the capture).
  const bool first = op->solve_counts[nrhs]++ == 0;
  if (!g_solve_graph || first) {
    set_boundary(f, op->gamma, op->n_bdry, u, op->tree().N, nrhs, s);
    downward_all(op, u, nrhs, nullptr, s);
    return;
  }
  if (!op->d_io) {
    op->d_io = op->mem.alloc<SolveIO>(1);
    HPS_HIP(hipHostMalloc((void**)&op->h_io, sizeof(SolveIO), hipHostMallocDefault));
  }
  auto it = op->solve_graphs.find(nrhs);
  if (it == op->solve_graphs.end()) {
    if (!op->capture_stream)
      HPS_HIP(hipStreamCreateWithFlags(&op->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = op->capture_stream;
    hipGraph_t g = nullptr;
    {
      ProfPause pause;  // no profiling events inside the capture
      HPS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      set_boundary_io(op->d_io, op->gamma, op->n_bdry, nrhs, cs);
      for (const LevelPlan& L : op->levels) {
        if (L.h.empty()) continue;
        double sb = 0;
        for (const MergeDesc& m : L.h) sb += 8.0 * m.m3 * m.me;
        downward(L.d, op->d_io, SolveIO{}, (int)L.h.size(), L.m3_max, L.me_max, nrhs, nullptr,
                 nullptr, cs, sb, true);
      }
      HPS_HIP(hipStreamEndCapture(cs, &g));
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HPS_HIP(e);
    it = op->solve_graphs.emplace(nrhs, ex).first;
  }
  // Every call waits for its stream before returning, so the staging buffer
  // is free again here.
  *op->h_io = SolveIO{u, op->tree().N, nrhs, f};
  HPS_HIP(hipMemcpyAsync(op->d_io, op->h_io, sizeof(SolveIO), hipMemcpyHostToDevice, s));
  double sb = 0;
  for (const LevelPlan& L : op->levels)
    for (const MergeDesc& m : L.h) sb += 8.0 * m.m3 * m.me;
  ProfScope ps(PROF_DOWNWARD, s, 2.0 * nrhs * sb / 8.0, sb);
  HPS_HIP(hipGraphLaunch(it->second, s));
}

void solve_batch_device(const std::vector<hps_op*>& ops, const std::vector<const double*>& f,
                        const std::vector<int>& nrhs, const std::vector<double*>& u,
                        hipStream_t s) {
  if (!ops.empty() && use_mm(*std::min_element(nrhs.begin(), nrhs.end()))) {
    std::vector<std::unique_ptr<AsyncBuf>> bufs;
    std::vector<double*> U;
    for (size_t i = 0; i < ops.size(); ++i) {
      bufs.emplace_back(new AsyncBuf((size_t)ops[i]->tree().N * nrhs[i], s));
      U.push_back(bufs.back()->p);
      set_boundary_nm(f[i], ops[i]->gamma, ops[i]->n_bdry, nrhs[i], U[i], s);
    }
    downward_batch_nm(ops, U, nrhs, nullptr, s);
    for (size_t i = 0; i < ops.size(); ++i) transpose(U[i], ops[i]->tree().N, nrhs[i], u[i], s);
    return;
  }
  for (size_t i = 0; i < ops.size(); ++i)
    set_boundary(f[i], ops[i]->gamma, ops[i]->n_bdry, u[i], ops[i]->tree().N, nrhs[i], s);
  downward_batch(ops, u, nrhs, nullptr, s);
}

double absmax_device(const double* x, size_t n, hipStream_t s) {
  const int blocks = 2048;
  double* part = nullptr;
  HPS_HIP(hipMallocAsync((void**)&part, blocks * sizeof(double), s));
  absmax_partial(x, n, part, blocks, s);
  double h[blocks];
  HPS_HIP(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipFreeAsync(part, s));
  HPS_HIP(hipStreamSynchronize(s));
  double m = 0.0;
  for (int i = 0; i < blocks; ++i) m = std::max(m, h[i]);
  return m;
}

void residual_device(const hps_op* op, const double* u, int nrhs, double* r, hipStream_t s) {
  HPS_REQUIRE(op->opt.keep_leaf, "operator was built without keep_leaf_ops");
  const int nl = op->nx * op->ny, m = 4 * op->q;
  if (use_mm(nrhs)) {
    const int N = op->tree().N;
    AsyncBuf U((size_t)N * nrhs, s), R((size_t)N * nrhs, s), v((size_t)nl * m * nrhs, s);
    transpose(u, nrhs, N, U.p, s);
    interface_residual_nm(op->leafT, U.p, N, nrhs, op->nx, op->ny, op->q, v.p, R.p, s);
    transpose(R.p, N, nrhs, r, s);
    return;
  }
  double* v = nullptr;
  HPS_HIP(hipMallocAsync((void**)&v, (size_t)nrhs * nl * m * sizeof(double), s));
  interface_residual(op->leafT, u, op->tree().N, nrhs, op->nx, op->ny, op->q, v, r, s);
  HPS_HIP(hipFreeAsync(v, s));
}

// Upward pass for sources src ([nrhs][N]): fills z ([nrhs] per merge).
static void upward_all(hps_op* op, const double* src, int nrhs, double* h, double* z,
                       hipStream_t s) {
  HPS_REQUIRE(op->opt.keep_factors, "operator was built without keep_factors");
  for (int d = (int)op->levels.size() - 1; d >= 0; --d) {
    const LevelPlan& L = op->levels[d];
    if (L.h.empty()) continue;
    double fl = 0;
    for (const MergeDesc& m : L.h) fl += 2.0 * nrhs * ((double)m.m3 * m.m3 + (double)m.me * m.m3);
    upward_level(L.d, (int)L.h.size(), L.m3_max, L.me_max, src, op->tree().N, h, L.dha, L.dhb,
                 L.dhp, z, L.dzo, nrhs, fl, s);
  }
}

void solve_with_sources_device(hps_op* op, const double* f, const double* src, int nrhs, double* u,
                               hipStream_t s) {
  if (use_mm(nrhs)) {
    const int N = op->tree().N;
    AsyncBuf S((size_t)N * nrhs, s), U((size_t)N * nrhs, s);
    AsyncBuf h((size_t)op->h_units * nrhs, s), z((size_t)op->z_units * nrhs, s),
        rb((size_t)op->z_units * nrhs, s);
    transpose(src, nrhs, N, S.p, s);
    upward_all_nm(op, S.p, nrhs, h.p, z.p, rb.p, s);
    set_boundary_nm(f, op->gamma, op->n_bdry, nrhs, U.p, s);
    downward_batch_nm({op}, {U.p}, {nrhs}, z.p, s);
    transpose(U.p, N, nrhs, u, s);
    return;
  }
  double *h = nullptr, *z = nullptr;
  HPS_HIP(hipMallocAsync((void**)&h, (size_t)op->h_units * nrhs * sizeof(double), s));
  HPS_HIP(hipMallocAsync((void**)&z, (size_t)std::max<long long>(1, op->z_units) * nrhs *
                                         sizeof(double), s));
  upward_all(op, src, nrhs, h, z, s);
  set_boundary(f, op->gamma, op->n_bdry, u, op->tree().N, nrhs, s);
  downward_all(op, u, nrhs, z, s);
  HPS_HIP(hipFreeAsync(h, s));
  HPS_HIP(hipFreeAsync(z, s));
}

// Body loads (A u = g).  The leaves' particular fluxes h = P1 A_ii^-1 g_i
// either come from the kept body operator K = P1 A_ii^-1 (one batched
// product) or from leaf particular solutions by the batched dense solver on
// [A_ii | G] (G: the load of every right-hand side at the leaf's interior
// nodes), which also give w_i for the grid values.  h enters the
// per-right-hand-side upward pass as the leaves' h (no interface sources);
// Algorithm 2 then adds the resulting z.  uc adds w_i to the post-processed
// grids.

// Particular solutions of every leaf: fluxes into h (unit offset h_units +
// leaf m), and w_i into wpart [nrhs][nl][n] when wpart is not null.
static void body_particular(hps_op* op, const double* g, int nrhs, double* h, double* wpart,
                            hipStream_t s) {
  const LeafPlan& LP = op->leaf();
  const int p = op->p, n = (p - 2) * (p - 2), m = 4 * op->q, nl = op->nx * op->ny;
  const int ld = n + nrhs;
  LeafDev tab{LP.dDx, LP.dDy, LP.dDxx, LP.dDyy, LP.dG, p, n, m, 0};
  const size_t per = (size_t)n * ld * sizeof(double) + (size_t)n * sizeof(int);
  const int CH = (int)std::max<size_t>(1, std::min<size_t>(nl, ((size_t)2 << 30) / per));
  AsyncBuf W((size_t)CH * n * ld, s), piv(((size_t)CH * n + 1) / 2 + 1, s);
  AsyncBuf desc(((size_t)CH * (sizeof(SolveDesc) + sizeof(void*)) + 7) / 8 + 4, s);
  const double** dcp = (const double**)desc.p;
  SolveDesc* dsd = (SolveDesc*)(dcp + CH);
  int* dstatus = (int*)(dsd + CH);
  HPS_HIP(hipMemsetAsync(dstatus, 0, 4 * sizeof(int), s));
  for (int c0 = 0; c0 < nl; c0 += CH) {
    const int cnt = std::min(CH, nl - c0);
    std::vector<const double*> cp(cnt);
    std::vector<SolveDesc> sd(cnt);
    for (int i = 0; i < cnt; ++i) {
      cp[i] = op->coeffs + (size_t)(c0 + i) * 6 * p * p;
      double* Wl = W.p + (size_t)i * n * ld;
      sd[i] = SolveDesc{Wl, (int*)piv.p + (size_t)i * n, Wl + n, n, nrhs, ld, ld, -(c0 + i + 1), 0};
    }
    HPS_HIP(hipMemcpyAsync(dcp, cp.data(), cnt * sizeof(void*), hipMemcpyHostToDevice, s));
    HPS_HIP(hipMemcpyAsync(dsd, sd.data(), cnt * sizeof(SolveDesc), hipMemcpyHostToDevice, s));
    leaf_assemble_body(dcp, tab, cnt, W.p, g, nrhs, nl, c0, s);
    batched_solve(dsd, sd, dstatus, s, 32);
    body_flux(W.p, cnt, n, m, ld, nrhs, LP.dP1, h, op->h_units, wpart, nl, c0, s);
    HPS_HIP(hipStreamSynchronize(s));  // host descriptor vectors are reused next chunk
  }
  int st[4];
  HPS_HIP(hipMemcpyAsync(st, dstatus, sizeof(st), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  if (st[0]) throw Error(HPS_ESINGULAR, "zero or non-finite pivot in the particular solve of leaf " +
                                            std::to_string(-st[1] - 1));
}

void body_solve_device(hps_op* op, const double* f, const double* g, int nrhs, double* u,
                       double* uc, hipStream_t s) {
  HPS_REQUIRE(op->opt.keep_factors, "body loads need an operator built with keep_factors");
  HPS_REQUIRE(!uc || op->leafZ, "grid values need an operator built with keep_leaf_solution");
  HPS_REQUIRE(nrhs >= 1, "bad right-hand-side count");
  const LeafPlan& LP = op->leaf();
  const int p = op->p, n = (p - 2) * (p - 2), m = 4 * op->q, nl = op->nx * op->ny;
  const int N = op->tree().N;
  HPS_REQUIRE(n <= max_solve_rows(), "leaf too large for the dense solver");
  AsyncBuf h((size_t)(op->h_units + (long long)nl * m) * nrhs, s);
  AsyncBuf z((size_t)std::max<long long>(1, op->z_units) * nrhs, s);
  AsyncBuf wpart(uc ? (size_t)nrhs * nl * n : 1, s);
  if (op->leafK && !uc)
    body_flux_kept(op->leafK, g, nrhs, n, m, p, nl, h.p, op->h_units, s);
  else
    body_particular(op, g, nrhs, h.p, uc ? wpart.p : nullptr, s);
  for (int d = (int)op->levels.size() - 1; d >= 0; --d) {
    const LevelPlan& L = op->levels[d];
    if (L.h.empty()) continue;
    double fl = 0;
    for (const MergeDesc& md : L.h) fl += 2.0 * nrhs * ((double)md.m3 * md.m3 + (double)md.me * md.m3);
    upward_level(L.d, (int)L.h.size(), L.m3_max, L.me_max, nullptr, N, h.p, L.dhab, L.dhbb, L.dhp,
                 z.p, L.dzo, nrhs, fl, s);
  }
  set_boundary(f, op->gamma, op->n_bdry, u, N, nrhs, s);
  downward_all(op, u, nrhs, z.p, s);
  if (uc) {
    postprocess_device(op, u, nrhs, uc, s);
    add_particular(uc, wpart.p, LP.dPostNode, n, p * p, nl, nrhs, s);
  }
}

static void refine_report(hps_solve_info* info, int it, double first, double last, bool conv,
                          int max_iter) {
  if (info) {
    info->iters = it;
    info->last_update_rel = last;
    info->first_update_rel = first < 0 ? 0.0 : first;
  }
  if (!conv) {
    char buf[160];
    snprintf(buf, sizeof(buf),
             "refinement did not reach tolerance in %d sweeps (first relative update %.3e, "
             "last %.3e)", max_iter, first, last);
    throw Error(HPS_ENOTCONV, buf);
  }
}

// Refinement on node-major arrays (same sweep as below): residual, upward
// pass, correction by the downward pass, all as grouped MFMA GEMMs.
static void refine_mm(hps_op* op, int nrhs, double* u, double tol, int max_iter, hipStream_t s,
                      hps_solve_info* info) {
  keep_async_pool();
  const int N = op->tree().N, nl = op->nx * op->ny, m = 4 * op->q;
  const size_t nu = (size_t)N * nrhs;
  AsyncBuf U(nu, s), r(nu, s), du(nu, s), v((size_t)nl * m * nrhs, s);
  AsyncBuf h((size_t)op->h_units * nrhs, s), z((size_t)op->z_units * nrhs, s),
      rb((size_t)op->z_units * nrhs, s), zero((size_t)op->n_bdry * nrhs, s);
  HPS_HIP(hipMemsetAsync(zero.p, 0, (size_t)op->n_bdry * nrhs * sizeof(double), s));
  transpose(u, nrhs, N, U.p, s);
  int it = 0;
  double last = 0.0, first = -1.0;
  bool conv = false;
  const double umax = std::max(absmax_device(U.p, nu, s), 1e-300);
  while (it < max_iter) {
    interface_residual_nm(op->leafT, U.p, N, nrhs, op->nx, op->ny, op->q, v.p, r.p, s);
    // Correction with jump(delta) = -r: by linearity delta = -(solution for sources r).
    upward_all_nm(op, r.p, nrhs, h.p, z.p, rb.p, s);
    set_boundary_nm(zero.p, op->gamma, op->n_bdry, nrhs, du.p, s);
    downward_batch_nm({op}, {du.p}, {nrhs}, z.p, s);
    axpy(U.p, du.p, -1.0, nu, s);
    ++it;
    last = absmax_device(du.p, nu, s) / umax;
    if (first < 0) first = last;
    if (last <= tol) {
      conv = true;
      break;
    }
  }
  transpose(U.p, N, nrhs, u, s);
  HPS_HIP(hipStreamSynchronize(s));
  refine_report(info, it, first, last, conv, max_iter);
}

void refine_device(hps_op* op, const double* f, int nrhs, double* u, double tol, int max_iter,
                   hipStream_t s, hps_solve_info* info) {
  HPS_REQUIRE(op->opt.keep_factors && op->opt.keep_leaf,
              "refinement needs keep_leaf_ops and keep_factors");
  const int N = op->tree().N;
  const size_t nu = (size_t)N * nrhs;
  if (use_mm(nrhs)) {
    refine_mm(op, nrhs, u, tol, max_iter, s, info);
    return;
  }
  double *r = nullptr, *du = nullptr, *h = nullptr, *z = nullptr, *zero = nullptr;
  HPS_HIP(hipMallocAsync((void**)&r, nu * sizeof(double), s));
  HPS_HIP(hipMallocAsync((void**)&du, nu * sizeof(double), s));
  HPS_HIP(hipMallocAsync((void**)&h, (size_t)op->h_units * nrhs * sizeof(double), s));
  HPS_HIP(hipMallocAsync((void**)&z, (size_t)std::max<long long>(1, op->z_units) * nrhs *
                                         sizeof(double), s));
  HPS_HIP(hipMallocAsync((void**)&zero, (size_t)op->n_bdry * nrhs * sizeof(double), s));
  HPS_HIP(hipMemsetAsync(zero, 0, (size_t)op->n_bdry * nrhs * sizeof(double), s));
  (void)f;
  int it = 0;
  double last = 0.0, first = -1.0;
  bool conv = false;
  const double umax = std::max(absmax_device(u, nu, s), 1e-300);
  while (it < max_iter) {
    residual_device(op, u, nrhs, r, s);
    // Correction with jump(delta) = -r: by linearity delta = -(solution for sources r).
    upward_all(op, r, nrhs, h, z, s);
    set_boundary(zero, op->gamma, op->n_bdry, du, N, nrhs, s);
    downward_all(op, du, nrhs, z, s);
    axpy(u, du, -1.0, nu, s);
    ++it;
    last = absmax_device(du, nu, s) / umax;
    if (first < 0) first = last;
    if (last <= tol) {
      conv = true;
      break;
    }
  }
  HPS_HIP(hipFreeAsync(r, s));
  HPS_HIP(hipFreeAsync(du, s));
  HPS_HIP(hipFreeAsync(h, s));
  HPS_HIP(hipFreeAsync(z, s));
  HPS_HIP(hipFreeAsync(zero, s));
  HPS_HIP(hipStreamSynchronize(s));
  refine_report(info, it, first, last, conv, max_iter);
}

void root_apply_device(const hps_op* op, const double* f, int nrhs, double* v, hipStream_t s) {
  HPS_REQUIRE(op->opt.root_dtn, "operator was built without the root DtN");
  matvec(op->rootT, op->n_bdry, op->n_bdry, f, nrhs, v, s);
}

// Section 5.3 with the leaf solution operators kept by the build (Remark 3.2).
void postprocess_device(const hps_op* op, const double* u, int nrhs, double* uc, hipStream_t s) {
  HPS_REQUIRE(op->leafZ, "operator was built without keep_leaf_solution");
  const LeafPlan& L = op->leaf();
  leaf_postprocess(op->leafZ, L.dL1t, L.dPostNode, u, op->tree().N, nrhs, op->nx, op->ny, op->p,
                   op->q, uc, s);
}

}  // namespace hps
