// Operator object and the build/solve drivers behind the C ABI.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "common.h"
#include "plan.h"
#include "pool.h"

namespace hps {

// Owner of device allocations (from the device memory cache); returns them on
// destruction.
struct DeviceMem {
  std::vector<void*> ptrs;
  DeviceMem() = default;
  DeviceMem(const DeviceMem&) = delete;
  DeviceMem& operator=(const DeviceMem&) = delete;
  ~DeviceMem();
  void* raw(size_t bytes);
  template <class T>
  T* alloc(size_t n) {
    return (T*)raw(std::max<size_t>(n, 1) * sizeof(T));
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* d = alloc<T>(v.size());
    if (!v.empty()) HPS_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
  }
  size_t bytes = 0;
};

// Merges of one tree depth of one operator (or of a batch when concatenated).
struct LevelPlan {
  std::vector<MergeDesc> h;
  std::vector<SolveDesc> hs;
  std::vector<GemmDesc> hg;                 // Schur products T^tau = diag + Q S
  std::vector<GemmDesc> hsg;                // solution operators S = M^-1 B
  std::vector<long long> ha, hb, hp, zo;    // unit offsets for the upward pass
  // The same child offsets for body-load solves: a leaf child's particular
  // flux sits at unit offset h_units + leaf * 4q (after the merged boxes).
  std::vector<long long> hab, hbb;
  MergeDesc* d = nullptr;
  SolveDesc* ds = nullptr;
  GemmDesc* dg = nullptr;
  GemmDesc* dsg = nullptr;
  long long *dha = nullptr, *dhb = nullptr, *dhp = nullptr, *dzo = nullptr;
  long long *dhab = nullptr, *dhbb = nullptr;
  int m3_max = 0, me_max = 0;
  size_t gather_max = 0;
};

// Shape-only data of the leaf stage for one (p, q, hx, hy): host tables and
// their device copies.
struct LeafPlan {
  LeafTables lt;
  DeviceMem mem;
  double *dDx = nullptr, *dDy = nullptr, *dDxx = nullptr, *dDyy = nullptr, *dG = nullptr,
         *dP0 = nullptr, *dP1 = nullptr;
  // Post-processing (section 5.3): L1 transposed (4q x 4(p-1)) and the
  // Chebyshev node of each post-processing row (interior nodes J_i, then
  // boundary nodes J_e).
  double* dL1t = nullptr;
  int* dPostNode = nullptr;
};
std::shared_ptr<const LeafPlan> leaf_plan(int p, int q, double hx, double hy, hipStream_t s);

// One merge of a tree plan: its box, where its index maps start in the map
// pool, its sizes and where its parent DtN goes in its depth's arena.
struct MergeRec {
  int box;
  size_t pool_off;
  int na, nb, me, m3;
  long long Toff;
};

// Shape-only data of a whole operator: tree, merge maps (host and device),
// root boundary ids and arena sizes.
struct TreePlan {
  std::shared_ptr<const LeafPlan> leaf;
  Tree tree;
  int n_bdry = 0;
  std::vector<std::vector<MergeRec>> levels;   // by depth
  std::vector<int> pool_host;                  // pmap, a3, b3, Ie, Ii per merge, then gamma
  size_t gamma_off = 0;
  DeviceMem mem;
  int* dpool = nullptr;
  int* gamma = nullptr;
  long long ar[2] = {0, 0};
  std::vector<long long> box_hoff;
  long long h_units = 0;
};

struct BuildOptions {
  int mode = HPS_FP64;
  hps_surrogate* surrogate = nullptr;
  int judge_samples = 64;
  double judge_tol = 1e-6;
  hipStream_t stream = nullptr;
  bool device_ptrs = false;
  bool keep_leaf = true;
  bool keep_factors = false;
  bool keep_leaf_solution = false;
  bool keep_body = false;
  bool root_dtn = true;
  int panel = 32;
  double pivot_tol = 0.0;   // relative pivot test (0: exactly zero pivots only)
};

}  // namespace hps

struct hps_op {
  int nx = 0, ny = 0, p = 0, q = 0, mode = HPS_FP64;
  double box[4] = {0, 0, 0, 0};
  std::shared_ptr<const hps::TreePlan> plan;   // shared by every operator of this shape
  hps::DeviceMem mem;
  std::vector<char> staging;        // host image of the device descriptors
  hps::BuildOptions opt;
  const double* coeffs = nullptr;   // device coefficients: an owned copy (host input or
                                    // keep_factors), else the caller's, read by the build only
  double* coeffs_own = nullptr;     // the owned copy's buffer, once allocated
  std::vector<long long> park_key;  // shape and kept buffers (parked-operator reuse)
  double* leafT = nullptr;          // [nleaf][4q][4q]
  double* leafZ = nullptr;          // [nleaf][4q][(p-2)^2]: Z^T, Z = A_ii^-1 A_ie L1, or null
  double* leafK = nullptr;          // [nleaf][(p-2)^2][4q]: K^T, K = P1 A_ii^-1, or null
  double* Wk = nullptr;             // merge systems [M | I] (M^-1 after the elimination)
  double* Bk = nullptr;             // gathered right-hand sides of one level (scratch)
  double* Sk = nullptr;             // solution operators S = M^-1 B of every merge
  double* Q = nullptr;
  int* piv = nullptr;
  size_t n_merges = 0;
  unsigned long long* pstat = nullptr;  // per merge: max|M| and min |pivot| (bit patterns)
  std::vector<double> level_cond;   // per depth: max over its merges of max|M| / min |pivot|
  int* gamma = nullptr;             // boundary ids in S,E,N,W order
  double* arena[2] = {nullptr, nullptr};
  double* rootT = nullptr;
  int n_bdry = 0;
  std::vector<hps::LevelPlan> levels;       // indexed by depth
  std::vector<int> merge_level, merge_index;  // per box: level and index of its merge, or -1
  std::vector<long long> box_hoff;          // unit offset of each box's particular flux
  long long h_units = 0, z_units = 0;       // totals (per right-hand side)
  long long bytes_S = 0, flops = 0;
  int n_fallback = 0;
  hps_surrogate* surrogate = nullptr;   // HPS_SURROGATE mode (not owned)
  int judge_samples = 64;
  double judge_tol = 1e-6;
  double judge_worst = 0.0;             // worst judged error in the random sample
  int n_judged = 0;                     // leaves re-solved in FP64 by the judge
  // Graph-captured plain solves (Algorithm 2), one executable graph per
  // right-hand-side count; f and u reach the kernels through d_io.
  std::map<int, hipGraphExec_t> solve_graphs;
  std::map<int, int> solve_counts;    // plain solves so far, per right-hand-side count
  hps::SolveIO* d_io = nullptr;       // device copy of the current solve's f, u
  // Persistent downward pass: its level table (root first), barrier word and
  // error flag (persist_state 0: not planned yet, 1: planned, -1: levels of
  // mixed merge shapes, not eligible).
  int persist_state = 0, persist_nlev = 0;
  hps::PersistLevel* persist_levels = nullptr;
  unsigned* persist_bar = nullptr;
  int* persist_err = nullptr;
  hps::SolveIO* h_io = nullptr;       // pinned host staging of it
  hipStream_t capture_stream = nullptr;

  const hps::Tree& tree() const { return plan->tree; }
  const hps::LeafPlan& leaf() const { return *plan->leaf; }
  hps_op() = default;
  hps_op(const hps_op&) = delete;
  hps_op& operator=(const hps_op&) = delete;
  ~hps_op();
};

namespace hps {

// Destroyed operators are parked: their device buffers and descriptors wait
// for the next build of the same shape, options and device (at most
// set_parked_limit of them, most recent first; parked_clear frees them all
// and returns how many there were).
void park_operator(hps_op* op);
std::unique_ptr<hps_op> unpark_operator(const std::vector<long long>& key);
size_t parked_clear();
void set_parked_limit(int n);

// Validates, plans and allocates one operator (no kernel launches except
// uploads), or takes back a parked one of the same key.
std::unique_ptr<hps_op> plan_operator(const double* coeffs, const double box[4], const int nleaf[2],
                                      int p, int q, const BuildOptions& o);
// Runs the build of a batch of planned operators: leaf stage grouped by leaf
// shape, merges grouped by depth.
void run_build(const std::vector<hps_op*>& ops, hipStream_t s);
// Leaf DtNs of nleaf equal leaves (device in, device out).
void leaf_dtn_batch(const double* coeffs, int nleaf, double hx, double hy, int p, int q, double* T,
                    hipStream_t s);
// Algorithm 2 (+ optional interface terms).  u, f device pointers.
void solve_device(hps_op* op, const double* f, int nrhs, double* u, hipStream_t s);
// Plain solves below 16 right-hand sides as one cooperative launch (knob
// "solve_persist", default off: measured slower than the level-by-level
// passes of the captured graph).
void set_solve_persist(bool on);
void solve_batch_device(const std::vector<hps_op*>& ops, const std::vector<const double*>& f,
                        const std::vector<int>& nrhs, const std::vector<double*>& u,
                        hipStream_t s);
// Refinement sweeps; returns the number of sweeps and the update sizes.
void refine_device(hps_op* op, const double* f, int nrhs, double* u, double tol, int max_iter,
                   hipStream_t s, hps_solve_info* info);
void residual_device(const hps_op* op, const double* u, int nrhs, double* r, hipStream_t s);
// The same with the flux scratch in a fixed device array (no allocation);
// throws HPS_EINVAL when nrhs * nleaf * 4q doubles exceed it.
void residual_noalloc(const hps_op* op, const double* u, int nrhs, double* r, hipStream_t s);
void solve_with_sources_device(hps_op* op, const double* f, const double* src, int nrhs, double* u,
                               hipStream_t s);
void root_apply_device(const hps_op* op, const double* f, int nrhs, double* v, hipStream_t s);
// Section 5.3: u at every leaf's Chebyshev nodes, uc [nrhs][nleaf][p*p].
void postprocess_device(const hps_op* op, const double* u, int nrhs, double* uc, hipStream_t s);
// Body loads (A u = g): g [nrhs][nleaf][p*p] at the Chebyshev nodes; u [nrhs][N];
// uc (or null) [nrhs][nleaf][p*p], the full solution on every leaf grid.
void body_solve_device(hps_op* op, const double* f, const double* g, int nrhs, double* u,
                       double* uc, hipStream_t s);
double absmax_device(const double* x, size_t n, hipStream_t s);
// Plain solves through captured graphs (default on); off = launch by launch.
void set_solve_graph(bool on);
// Solves, source solves and refinement with at least v right-hand sides run
// on node-major arrays with MFMA GEMMs (default 16; 0: never).
void set_solve_mm_min_rhs(int v);
// Merge levels (over all builds so far) whose blocked Gauss-Jordan fell back
// to partial pivoting.
// Leaf systems by blocked Gauss-Jordan (knob "leaf_bgj", default on): the
// leaves the MFMA leaf kernel does not take (p > 12, or with the leaf
// solution kept) are assembled and eliminated like the large merges.
void set_leaf_bgj(bool on);
bool leaf_bgj_on();
long long bgj_fallbacks();
// Releases the stream-ordered scratch cached in the current device's pool.
void trim_async_pool();

}  // namespace hps
