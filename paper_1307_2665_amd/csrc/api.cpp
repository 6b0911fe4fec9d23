// C ABI of the solver (declared in include/hps.h).  Every entry point catches
// library errors and turns them into a status plus a thread-local message.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dense.h"
#include "hbs.h"
#include "leaf.h"
#include "ops.h"
#include "solver.h"
#include "surrogate.h"
#include "tune.h"

#include <fstream>
#include <sstream>

namespace {

thread_local std::string g_err;

template <class F>
hps_status guard(F&& f) {
  try {
    f();
    return HPS_OK;
  } catch (const hps::Error& e) {
    g_err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return HPS_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return HPS_EINVAL;
  }
}

hps::BuildOptions to_build_options(const hps_build_opts* o) {
  hps::BuildOptions b;
  if (!o) return b;
  b.mode = o->mode;
  b.stream = (hipStream_t)o->stream;
  b.device_ptrs = o->device_ptrs != 0;
  b.keep_leaf = true;
  b.keep_factors = o->keep_factors != 0;
  b.keep_leaf_solution = o->keep_leaf_solution != 0;
  b.keep_body = o->keep_body_operator != 0;
  b.root_dtn = o->compute_root_dtn != 0;
  b.surrogate = const_cast<hps_surrogate*>(o->surrogate);
  b.judge_samples = o->judge_samples > 0 ? o->judge_samples : 64;
  b.judge_tol = o->judge_tol > 0 ? o->judge_tol : 1e-6;
  HPS_REQUIRE(o->pivot_tol >= 0.0 && o->pivot_tol < 1.0, "pivot_tol must be in [0, 1)");
  b.pivot_tol = o->pivot_tol;
  return b;
}

// Device staging of a caller array that may live on the host.
struct Staged {
  double* d = nullptr;
  bool owned = false;
  ~Staged() {
    if (owned && d) hps::pool_release(d);
  }
};

void stage_in(Staged& st, const double* p, size_t n, bool device, hipStream_t s) {
  if (device) {
    st.d = const_cast<double*>(p);
    return;
  }
  st.d = (double*)hps::pool_alloc(std::max<size_t>(n, 1) * sizeof(double));
  st.owned = true;
  if (n) HPS_HIP(hipMemcpyAsync(st.d, p, n * sizeof(double), hipMemcpyHostToDevice, s));
}

void stage_out(const Staged& st, double* p, size_t n, bool device, hipStream_t s) {
  if (!device && n)
    HPS_HIP(hipMemcpyAsync(p, st.d, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

hps_status hps_mem_trim(size_t* freed) {
  return guard([&] {
    (void)hipDeviceSynchronize();
    hps::parked_clear();
    hps::hbs_passes_clear();
    const size_t f = hps::pool_trim();
    hps::trim_async_pool();
    if (freed) *freed = f;
  });
}

hps_status hps_mem_stats(size_t* cached, size_t* in_use) {
  return guard([&] { hps::pool_stats(cached, in_use); });
}

const char* hps_last_error(void) { return g_err.c_str(); }
const char* hps_version(void) { return "hps-mi355x 0.1 (gfx950)"; }

hps_status hps_cheb_nodes(const double box[4], const int nleaf[2], int p, double* xy) {
  return guard([&] {
    HPS_REQUIRE(box && nleaf && xy && p >= 2 && nleaf[0] >= 1 && nleaf[1] >= 1, "bad arguments");
    std::vector<double> v;
    hps::cheb_node_xy(nleaf[0], nleaf[1], p, box, v);
    std::memcpy(xy, v.data(), v.size() * sizeof(double));
  });
}

hps_status hps_gauss_nodes_grid(const double box[4], const int nleaf[2], int q, double* xy, int* N) {
  return guard([&] {
    HPS_REQUIRE(box && nleaf && q >= 1 && nleaf[0] >= 1 && nleaf[1] >= 1, "bad arguments");
    hps::Tree t;
    t.nx = nleaf[0];
    t.ny = nleaf[1];
    t.q = q;
    t.nh = t.nx * (t.ny + 1);
    t.N = q * (t.nx * (t.ny + 1) + (t.nx + 1) * t.ny);
    if (N) *N = t.N;
    if (xy) {
      std::vector<double> v;
      hps::gauss_node_xy(t, box, v);
      std::memcpy(xy, v.data(), v.size() * sizeof(double));
    }
  });
}

hps_status hps_boundary_ids(const int nleaf[2], int q, int* ids, int* n_bdry) {
  return guard([&] {
    HPS_REQUIRE(nleaf && q >= 1 && nleaf[0] >= 1 && nleaf[1] >= 1, "bad arguments");
    hps::Tree t;
    t.nx = nleaf[0];
    t.ny = nleaf[1];
    t.q = q;
    t.nh = t.nx * (t.ny + 1);
    std::vector<int> v;
    hps::box_boundary(t, 0, t.nx, 0, t.ny, v);
    if (n_bdry) *n_bdry = (int)v.size();
    if (ids) std::memcpy(ids, v.data(), v.size() * sizeof(int));
  });
}

hps_status hps_leaf_dtn(const double* coeffs, int nleaf, double hx, double hy, int p, int q,
                        double* T, void* stream) {
  return guard([&] {
    HPS_REQUIRE(coeffs && T && hx > 0 && hy > 0, "bad arguments");
    hps::leaf_dtn_batch(coeffs, nleaf, hx, hy, p, q, T, (hipStream_t)stream);
  });
}

hps_status hps_build_solution_operator(const double* coeffs, const double box[4],
                                       const int nleaf[2], int p, int q,
                                       const hps_build_opts* opts, hps_op** out) {
  if (out) *out = nullptr;
  return guard([&] {
    HPS_REQUIRE(out != nullptr, "out is null");
    HPS_REQUIRE(!opts || opts->mode == HPS_FP64 || opts->mode == HPS_MIXED_SPLIT32 ||
                    opts->mode == HPS_SURROGATE || opts->mode == HPS_MIXED_BF16X6,
                "unknown mode");
    HPS_REQUIRE(!opts || opts->mode != HPS_SURROGATE || opts->surrogate,
                "HPS_SURROGATE needs opts->surrogate");
    hps::BuildOptions bo = to_build_options(opts);
    auto op = hps::plan_operator(coeffs, box, nleaf, p, q, bo);
    std::vector<hps_op*> v{op.get()};
    hps::run_build(v, bo.stream);
    *out = op.release();
  });
}

hps_status hps_build_batch(const hps_problem* probs, int nprob, const hps_build_opts* opts,
                           hps_op** out) {
  return guard([&] {
    HPS_REQUIRE(probs && out && nprob >= 1, "bad arguments");
    for (int i = 0; i < nprob; ++i) out[i] = nullptr;
    HPS_REQUIRE(!opts || opts->mode == HPS_FP64 || opts->mode == HPS_MIXED_SPLIT32 ||
                    opts->mode == HPS_MIXED_BF16X6 ||
                    (opts->mode == HPS_SURROGATE && opts->surrogate),
                "unknown mode, or HPS_SURROGATE without a surrogate");
    hps::BuildOptions bo = to_build_options(opts);
    std::vector<std::unique_ptr<hps_op>> owned;
    std::vector<hps_op*> v;
    for (int i = 0; i < nprob; ++i) {
      owned.push_back(hps::plan_operator(probs[i].coeffs, probs[i].box, probs[i].nleaf,
                                         probs[i].p, probs[i].q, bo));
      v.push_back(owned.back().get());
    }
    hps::run_build(v, bo.stream);
    for (int i = 0; i < nprob; ++i) out[i] = owned[i].release();
  });
}

hps_status hps_gauss_nodes(const hps_op* op, double* xy, int* N) {
  return guard([&] {
    HPS_REQUIRE(op, "null operator");
    if (N) *N = op->tree().N;
    if (xy) {
      std::vector<double> v;
      hps::gauss_node_xy(op->tree(), op->box, v);
      std::memcpy(xy, v.data(), v.size() * sizeof(double));
    }
  });
}

hps_status hps_boundary_nodes(const hps_op* op, double* xy, int* n_bdry) {
  return guard([&] {
    HPS_REQUIRE(op, "null operator");
    if (n_bdry) *n_bdry = op->n_bdry;
    if (xy) {
      std::vector<double> v;
      std::vector<int> ids;
      hps::gauss_node_xy(op->tree(), op->box, v);
      hps::box_boundary(op->tree(), 0, op->nx, 0, op->ny, ids);
      for (size_t i = 0; i < ids.size(); ++i) {
        xy[2 * i] = v[2 * (size_t)ids[i]];
        xy[2 * i + 1] = v[2 * (size_t)ids[i] + 1];
      }
    }
  });
}

hps_status hps_solve(hps_op* op, const double* f, int nrhs, double* u, const hps_solve_opts* opts,
                     hps_solve_info* info) {
  return guard([&] {
    HPS_REQUIRE(op && f && u && nrhs >= 1, "bad arguments");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const bool dev = opts && opts->device_ptrs;
    const size_t nf = (size_t)op->n_bdry * nrhs, nu = (size_t)op->tree().N * nrhs;
    if (!dev)
      for (size_t i = 0; i < nf; ++i) HPS_REQUIRE(std::isfinite(f[i]), "non-finite boundary data");
    Staged F, U;
    stage_in(F, f, nf, dev, s);
    if (dev) {
      U.d = u;
    } else {
      U.d = (double*)hps::pool_alloc(nu * sizeof(double));
      U.owned = true;
    }
    if (info) std::memset(info, 0, sizeof(*info));
    hps::solve_device(op, F.d, nrhs, U.d, s);
    if (opts && opts->refine)
      hps::refine_device(op, F.d, nrhs, U.d, opts->refine_tol > 0 ? opts->refine_tol : 1e-12,
                         opts->max_iter > 0 ? opts->max_iter : 10, s, info);
    if (info) info->n_fallback_leaves = op->n_fallback;
    stage_out(U, u, nu, dev, s);
  });
}

hps_status hps_solve_batch(hps_op* const* ops, int nprob, const double* const* f, const int* nrhs,
                           double* const* u, const hps_solve_opts* opts) {
  return guard([&] {
    HPS_REQUIRE(ops && f && nrhs && u && nprob >= 1, "bad arguments");
    HPS_REQUIRE(opts && opts->device_ptrs, "hps_solve_batch takes device pointers");
    HPS_REQUIRE(!opts->refine, "refinement is per operator (hps_solve)");
    hipStream_t s = (hipStream_t)opts->stream;
    std::vector<hps_op*> v(ops, ops + nprob);
    std::vector<const double*> fv(f, f + nprob);
    std::vector<int> nv(nrhs, nrhs + nprob);
    std::vector<double*> uv(u, u + nprob);
    hps::solve_batch_device(v, fv, nv, uv, s);
    HPS_HIP(hipStreamSynchronize(s));
  });
}

hps_status hps_root_dtn_apply(const hps_op* op, const double* f, int nrhs, double* v,
                              const hps_solve_opts* opts) {
  return guard([&] {
    HPS_REQUIRE(op && f && v && nrhs >= 1, "bad arguments");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const bool dev = opts && opts->device_ptrs;
    const size_t n = (size_t)op->n_bdry * nrhs;
    Staged F, V;
    stage_in(F, f, n, dev, s);
    if (dev) {
      V.d = v;
    } else {
      V.d = (double*)hps::pool_alloc(n * sizeof(double));
      V.owned = true;
    }
    hps::root_apply_device(op, F.d, nrhs, V.d, s);
    stage_out(V, v, n, dev, s);
  });
}

hps_status hps_postprocess(const hps_op* op, const double* u, int nrhs, double* uc,
                           const hps_solve_opts* opts) {
  return guard([&] {
    HPS_REQUIRE(op && u && uc && nrhs >= 1, "bad arguments");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const bool dev = opts && opts->device_ptrs;
    const size_t nu = (size_t)op->tree().N * nrhs;
    const size_t nc = (size_t)nrhs * op->nx * op->ny * op->p * op->p;
    Staged U, V;
    stage_in(U, u, nu, dev, s);
    if (dev) {
      V.d = uc;
    } else {
      V.d = (double*)hps::pool_alloc(nc * sizeof(double));
      V.owned = true;
    }
    hps::postprocess_device(op, U.d, nrhs, V.d, s);
    stage_out(V, uc, nc, dev, s);
  });
}

hps_status hps_solve_body(hps_op* op, const double* f, const double* g, int nrhs, double* u,
                          double* uc, const hps_solve_opts* opts) {
  return guard([&] {
    HPS_REQUIRE(op && f && g && u && nrhs >= 1, "bad arguments");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    const bool dev = opts && opts->device_ptrs;
    const size_t nf = (size_t)op->n_bdry * nrhs, nu = (size_t)op->tree().N * nrhs;
    const size_t ng = (size_t)nrhs * op->nx * op->ny * op->p * op->p;
    if (!dev) {
      for (size_t i = 0; i < nf; ++i) HPS_REQUIRE(std::isfinite(f[i]), "non-finite boundary data");
      for (size_t i = 0; i < ng; ++i) HPS_REQUIRE(std::isfinite(g[i]), "non-finite body load");
    }
    Staged F, G, U, V;
    stage_in(F, f, nf, dev, s);
    stage_in(G, g, ng, dev, s);
    auto out = [&](Staged& st, double* p, size_t n) {
      if (dev) {
        st.d = p;
      } else {
        st.d = (double*)hps::pool_alloc(std::max<size_t>(n, 1) * sizeof(double));
        st.owned = true;
      }
    };
    out(U, u, nu);
    if (uc) out(V, uc, ng);
    hps::body_solve_device(op, F.d, G.d, nrhs, U.d, uc ? V.d : nullptr, s);
    stage_out(U, u, nu, dev, s);
    if (uc) stage_out(V, uc, ng, dev, s);
  });
}

hps_status hps_interface_residual(const hps_op* op, const double* u, int nrhs, double* r,
                                  void* stream) {
  return guard([&] {
    HPS_REQUIRE(op && u && r && nrhs >= 1, "bad arguments");
    hps::residual_device(op, u, nrhs, r, (hipStream_t)stream);
    HPS_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

hps_status hps_interface_residual_noalloc(const hps_op* op, const double* u, int nrhs, double* r,
                                          void* stream) {
  return guard([&] {
    HPS_REQUIRE(op && u && r && nrhs >= 1, "bad arguments");
    hps::residual_noalloc(op, u, nrhs, r, (hipStream_t)stream);
    HPS_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

hps_status hps_solve_with_sources(hps_op* op, const double* f, const double* s, int nrhs, double* u,
                                  void* stream) {
  return guard([&] {
    HPS_REQUIRE(op && f && s && u && nrhs >= 1, "bad arguments");
    hps::solve_with_sources_device(op, f, s, nrhs, u, (hipStream_t)stream);
    HPS_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

hps_status hps_op_query(const hps_op* op, hps_op_info* info) {
  return guard([&] {
    HPS_REQUIRE(op && info, "bad arguments");
    std::memset(info, 0, sizeof(*info));
    info->nx = op->nx;
    info->ny = op->ny;
    info->p = op->p;
    info->q = op->q;
    info->N = op->tree().N;
    info->n_bdry = op->n_bdry;
    info->n_boxes = (int)op->tree().boxes.size();
    info->n_levels = op->tree().depth + 1;
    info->mode = op->mode;
    info->n_fallback_leaves = op->n_fallback;
    std::memcpy(info->box, op->box, sizeof(info->box));
    info->bytes_S = op->bytes_S;
    info->bytes_total = (int64_t)op->mem.bytes;
    info->flops_build = op->flops;
    info->judge_worst = op->judge_worst;
    info->n_judged = op->n_judged;
  });
}

hps_status hps_box(const hps_op* op, int box, int rec[8]) {
  return guard([&] {
    HPS_REQUIRE(op && rec && box >= 0 && box < (int)op->tree().boxes.size(), "bad arguments");
    const hps::BoxRec& b = op->tree().boxes[box];
    int v[8] = {b.i0, b.i1, b.j0, b.j1, b.level, b.parent, b.ca, b.cb};
    std::memcpy(rec, v, sizeof(v));
  });
}

hps_status hps_export_S(const hps_op* op, int box, double* S, int* rows, int* cols) {
  return guard([&] {
    HPS_REQUIRE(op && box >= 0 && box < (int)op->tree().boxes.size(), "bad arguments");
    int lv = op->merge_level[box];
    HPS_REQUIRE(lv >= 0, "box is a leaf");
    const hps::MergeDesc& d = op->levels[lv].h[op->merge_index[box]];
    if (rows) *rows = d.m3;
    if (cols) *cols = d.me;
    if (S)
      HPS_HIP(hipMemcpy2D(S, d.me * sizeof(double), d.S, d.lds * sizeof(double),
                          d.me * sizeof(double), d.m3, hipMemcpyDeviceToHost));
  });
}

hps_status hps_level_conditions(const hps_op* op, double* cond_est, int* n_levels) {
  return guard([&] {
    HPS_REQUIRE(op && n_levels, "bad arguments");
    *n_levels = (int)op->level_cond.size();
    if (cond_est)
      for (size_t d = 0; d < op->level_cond.size(); ++d) cond_est[d] = op->level_cond[d];
  });
}

hps_status hps_export_root_dtn(const hps_op* op, double* T) {
  return guard([&] {
    HPS_REQUIRE(op && T, "bad arguments");
    HPS_REQUIRE(op->opt.root_dtn, "operator was built without the root DtN");
    HPS_HIP(hipMemcpy(T, op->rootT, (size_t)op->n_bdry * op->n_bdry * sizeof(double),
                      hipMemcpyDeviceToHost));
  });
}

hps_status hps_export_leaf_dtn(const hps_op* op, int leaf, double* T) {
  return guard([&] {
    HPS_REQUIRE(op && T && leaf >= 0 && leaf < op->nx * op->ny, "bad arguments");
    const size_t m = 4 * (size_t)op->q;
    HPS_HIP(hipMemcpy(T, op->leafT + (size_t)leaf * m * m, m * m * sizeof(double),
                      hipMemcpyDeviceToHost));
  });
}

hps_status hps_batched_solve(const double* M, const double* B, int n, int m, int nprob, double* X,
                             void* stream) {
  return guard([&] {
    HPS_REQUIRE(M && B && X && n >= 1 && m >= 1 && nprob >= 1, "bad arguments");
    HPS_REQUIRE(n <= hps::max_solve_rows(), "n too large");
    hipStream_t s = (hipStream_t)stream;
    hps::dense_init();
    hps::DeviceMem tmp;
    const int ld = n + m;
    double* W = tmp.alloc<double>((size_t)nprob * n * ld);
    int* piv = tmp.alloc<int>((size_t)nprob * n);
    int* st = tmp.alloc<int>(4);
    HPS_HIP(hipMemsetAsync(st, 0, 4 * sizeof(int), s));
    for (int i = 0; i < nprob; ++i) {
      HPS_HIP(hipMemcpy2DAsync(W + (size_t)i * n * ld, ld * sizeof(double), M + (size_t)i * n * n,
                               n * sizeof(double), n * sizeof(double), n, hipMemcpyDeviceToDevice,
                               s));
      HPS_HIP(hipMemcpy2DAsync(W + (size_t)i * n * ld + n, ld * sizeof(double),
                               B + (size_t)i * n * m, m * sizeof(double), m * sizeof(double), n,
                               hipMemcpyDeviceToDevice, s));
    }
    std::vector<hps::SolveDesc> hd(nprob);
    for (int i = 0; i < nprob; ++i)
      hd[i] = hps::SolveDesc{W + (size_t)i * n * ld, piv + (size_t)i * n,
                             W + (size_t)i * n * ld + n, n, m, ld, ld, i, 0};
    hps::SolveDesc* dd = tmp.upload(hd, s);
    hps::batched_solve(dd, hd, st, s, 32);
    for (int i = 0; i < nprob; ++i)
      HPS_HIP(hipMemcpy2DAsync(X + (size_t)i * n * m, m * sizeof(double),
                               W + (size_t)i * n * ld + n, ld * sizeof(double), m * sizeof(double),
                               n, hipMemcpyDeviceToDevice, s));
    int h[4];
    HPS_HIP(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    HPS_HIP(hipStreamSynchronize(s));
    if (h[0]) throw hps::Error(HPS_ESINGULAR, "zero or non-finite pivot in system " +
                                                  std::to_string(h[1]));
  });
}

hps_status hps_batched_gemm(const double* A, const double* B, double* C, int Mr, int Nc, int K,
                            int nprob, double alpha, int prec, void* stream) {
  return guard([&] {
    HPS_REQUIRE(A && B && C && Mr >= 1 && Nc >= 1 && K >= 1 && nprob >= 1, "bad arguments");
    HPS_REQUIRE(prec >= 0 && prec <= 2, "prec must be 0, 1 or 2");
    hipStream_t s = (hipStream_t)stream;
    hps::DeviceMem tmp;
    std::vector<hps::GemmDesc> hd(nprob);
    for (int i = 0; i < nprob; ++i)
      hd[i] = hps::GemmDesc{A + (size_t)i * Mr * K, B + (size_t)i * K * Nc, C + (size_t)i * Mr * Nc,
                            nullptr, Mr, Nc, K, K, Nc, Nc, 0, alpha};
    hps::GemmDesc* dd = tmp.upload(hd, s);
    hps::grouped_gemm(dd, hd, s, prec);
    HPS_HIP(hipStreamSynchronize(s));
  });
}

hps_status hps_hbs_sizes(int L, int m, int k, size_t* n_factors, size_t* n_inverse) {
  return guard([&] {
    hps::hbs_check(L, m, k);
    const hps::HbsLayout lo(L, m, k);
    if (n_factors) *n_factors = lo.nfac;
    if (n_inverse) *n_inverse = lo.ninv;
  });
}

hps_status hps_hbs_apply(int L, int m, int k, const double* factors, const double* x, double* y,
                         int nrhs, void* stream) {
  return guard([&] {
    hps::hbs_check(L, m, k);
    HPS_REQUIRE(factors && x && y && nrhs >= 1, "bad arguments");
    HPS_REQUIRE(x != y, "y must not overlap x");
    hps::hbs_apply(hps::HbsLayout(L, m, k), factors, x, y, nrhs, (hipStream_t)stream);
  });
}

hps_status hps_hbs_invert(int L, int m, int k, const double* factors, double* inverse,
                          void* stream) {
  return guard([&] {
    hps::hbs_check(L, m, k);
    HPS_REQUIRE(factors && inverse, "bad arguments");
    hps::hbs_invert(hps::HbsLayout(L, m, k), factors, inverse, (hipStream_t)stream);
  });
}

hps_status hps_hbs_solve(int L, int m, int k, const double* inverse, const double* x, double* y,
                         int nrhs, void* stream) {
  return guard([&] {
    hps::hbs_check(L, m, k);
    HPS_REQUIRE(inverse && x && y && nrhs >= 1, "bad arguments");
    HPS_REQUIRE(x != y, "y must not overlap x");
    hps::hbs_solve(hps::HbsLayout(L, m, k), inverse, x, y, nrhs, (hipStream_t)stream);
  });
}

hps_status hps_hbs_compress(int L, int m, int k, const double* H, int ldh, const double* omega,
                            const double* psit, double* factors, void* stream) {
  return guard([&] {
    hps::hbs_check(L, m, k);
    HPS_REQUIRE(k <= hps::hbs_max_compress_rank(m), "rank too large to compress (k <= 90, m k <= 16384)");
    HPS_REQUIRE(H && omega && psit && factors, "bad arguments");
    HPS_REQUIRE(ldh >= (m << L), "ldh smaller than the matrix");
    hps::hbs_compress(hps::HbsLayout(L, m, k), H, ldh, omega, psit, factors, (hipStream_t)stream);
  });
}

hps_status hps_root_dtn_compress(const hps_op* op, int L, int k, const double* omega,
                                 const double* psit, double* factors, void* stream) {
  return guard([&] {
    HPS_REQUIRE(op && omega && psit && factors, "bad arguments");
    HPS_REQUIRE(op->opt.root_dtn, "operator was built without the root DtN");
    HPS_REQUIRE(L >= 1 && L <= 14 && op->n_bdry % (1 << L) == 0,
                "2^L must divide the number of boundary nodes");
    const int m = op->n_bdry >> L;
    hps::hbs_check(L, m, k);
    HPS_REQUIRE(k <= hps::hbs_max_compress_rank(m), "rank too large to compress (k <= 90, m k <= 16384)");
    hps::hbs_compress(hps::HbsLayout(L, m, k), op->rootT, op->n_bdry, omega, psit, factors,
                      (hipStream_t)stream);
  });
}

hps_status hps_bgj_fallbacks(long long* count) {
  return guard([&] {
    HPS_REQUIRE(count != nullptr, "null count");
    *count = hps::bgj_fallbacks();
  });
}

hps_status hps_tune_set(const char* knob, int value) {
  return guard([&] {
    HPS_REQUIRE(knob != nullptr, "null knob");
    std::string k(knob);
    if (k == "leaf_variant") {
      HPS_REQUIRE(value >= -1 && value <= 4, "leaf_variant must be in [-1, 4]");
      hps::leaf_lu_set_variant(value);
    } else if (k == "leaf_mfma") {
      HPS_REQUIRE(value >= -1 && value <= 1, "leaf_mfma must be -1, 0 or 1");
      hps::leaf_set_mfma(value != 0);
    } else if (k == "bgj_min_rows") {
      HPS_REQUIRE(value >= -1, "bgj_min_rows must be >= -1");
      hps::set_bgj(value < 0 ? 256 : value, -1.0);
    } else if (k == "bgj_fallback_tol_exp") {
      HPS_REQUIRE(value >= -1 && value <= 300, "bgj_fallback_tol_exp must be in [-1, 300]");
      hps::set_bgj(-1, value < 0 ? 1e-6 : std::pow(10.0, -value));
    } else if (k == "gemm_variant") {
      HPS_REQUIRE(value >= -1 && value < hps::GEMM_VARIANTS, "gemm_variant out of range");
      hps::tune_force(hps::TUNE_GEMM, value);
    } else if (k == "solve_graph") {
      HPS_REQUIRE(value == 0 || value == 1, "solve_graph must be 0 or 1");
      hps::set_solve_graph(value != 0);
    } else if (k == "solve_mm_min_rhs") {
      HPS_REQUIRE(value >= -1, "solve_mm_min_rhs must be >= -1");
      hps::set_solve_mm_min_rhs(value < 0 ? 16 : value);
    } else if (k == "split_min_chunk") {
      HPS_REQUIRE(value == -1 || value >= 16, "split_min_chunk must be -1 or >= 16");
      hps::set_split_min_chunk(value < 0 ? 256 : value);
    } else if (k == "gj_lookahead") {
      HPS_REQUIRE(value >= -1 && value <= 1, "gj_lookahead must be -1, 0 or 1");
      hps::set_gj_lookahead(value == 1);
    } else if (k == "bf16x6_min_k") {
      HPS_REQUIRE(value >= -1, "bf16x6_min_k must be >= -1");
      hps::set_bf16x6_min_k(value);
    } else if (k == "post_rows") {
      hps::set_post_rows(value);
    } else if (k == "leaf_bgj") {
      HPS_REQUIRE(value >= -1 && value <= 1, "leaf_bgj must be -1, 0 or 1");
      hps::set_leaf_bgj(value != 0);
    } else if (k == "hbs_grid") {
      HPS_REQUIRE(value >= -1, "hbs_grid must be >= -1");
      hps::hbs_set_pass_grid(value < 0 ? 0 : value);
    } else if (k == "solve_persist") {
      HPS_REQUIRE(value >= -1 && value <= 1, "solve_persist must be -1, 0 or 1");
      hps::set_solve_persist(value == 1);
    } else if (k == "gemm_queue") {
      HPS_REQUIRE(value >= -1 && value <= 1, "gemm_queue must be -1, 0 or 1");
      hps::set_gemm_queue(value != 0);
    } else if (k == "merge_small") {
      HPS_REQUIRE(value >= -1 && value <= 1, "merge_small must be -1, 0 or 1");
      hps::set_merge_small(value != 0);
    } else if (k == "bgj_lookahead") {
      HPS_REQUIRE(value >= -1 && value <= 1, "bgj_lookahead must be -1, 0 or 1");
      hps::set_bgj_lookahead(value != 0);
    } else if (k == "parked_ops") {
      HPS_REQUIRE(value >= -1 && value <= 64, "parked_ops must be in [-1, 64]");
      hps::set_parked_limit(value < 0 ? 2 : value);
    } else if (k == "gj_variant") {
      HPS_REQUIRE(value >= -1 && value < 4 * hps::UPDATE_VARIANTS && (value < 0 || value % 4 < 3),
                  "gj_variant out of range");
      hps::tune_force(hps::TUNE_GJ, value);
    } else {
      throw hps::Error(HPS_EINVAL, "unknown knob " + k);
    }
  });
}

hps_status hps_autotune(const hps_problem* probs, int nprob, void* stream, double* seconds) {
  return guard([&] {
    HPS_REQUIRE(probs != nullptr && nprob >= 1, "bad arguments");
    std::vector<hps::TuneShape> shapes;
    for (int i = 0; i < nprob; ++i) {
      const hps_problem& p = probs[i];
      HPS_REQUIRE(p.nleaf[0] >= 1 && p.nleaf[1] >= 1 && p.box[1] > p.box[0] && p.box[3] > p.box[2],
                  "bad problem shape");
      shapes.push_back(hps::TuneShape{p.nleaf[0], p.nleaf[1], p.p, p.q,
                                      (p.box[1] - p.box[0]) / p.nleaf[0],
                                      (p.box[3] - p.box[2]) / p.nleaf[1]});
    }
    const double t = hps::autotune(shapes, (hipStream_t)stream);
    if (seconds) *seconds = t;
  });
}

hps_status hps_tune_save(const char* path) {
  return guard([&] {
    HPS_REQUIRE(path != nullptr, "null path");
    std::ofstream f(path);
    HPS_REQUIRE(f.good(), std::string("cannot write ") + path);
    f << hps::tune_json();
    HPS_REQUIRE(f.good(), std::string("write failed: ") + path);
  });
}

hps_status hps_tune_load(const char* path) {
  return guard([&] {
    HPS_REQUIRE(path != nullptr, "null path");
    std::ifstream f(path);
    HPS_REQUIRE(f.good(), std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    hps::tune_load_json(ss.str());
  });
}

hps_status hps_tune_reset(void) {
  return guard([&] { hps::tune_clear(); });
}

hps_status hps_leaf_tables(int p, int q, double hx, double hy, double* Dx, double* Dy, double* Dxx,
                           double* Dyy, double* G, double* P0, double* P1, int* Ji) {
  return guard([&] {
    HPS_REQUIRE(p >= 4 && p <= 24 && q >= 1 && q < p && hx > 0 && hy > 0,
                "bad arguments (need 4 <= p <= 24, 1 <= q <= p - 1, hx, hy > 0)");
    hps::LeafTables t = hps::make_leaf_tables(p, q, hx, hy);
    auto put = [](double* dst, const std::vector<double>& v) {
      if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
    };
    put(Dx, t.Dx);
    put(Dy, t.Dy);
    put(Dxx, t.Dxx);
    put(Dyy, t.Dyy);
    put(G, t.G);
    put(P0, t.P0);
    put(P1, t.P1);
    if (Ji) std::memcpy(Ji, t.Ji.data(), t.Ji.size() * sizeof(int));
  });
}

hps_status hps_plan_box(const int nleaf[2], int q, int box, int rec[8], int sizes[4], int* pmap,
                        int* a3, int* b3, int* Ie, int* Ii, int* n_boxes) {
  return guard([&] {
    HPS_REQUIRE(nleaf && nleaf[0] >= 1 && nleaf[1] >= 1 && q >= 1, "bad arguments");
    hps::Tree t = hps::build_tree(nleaf[0], nleaf[1], q);
    if (n_boxes) *n_boxes = (int)t.boxes.size();
    if (box < 0) return;
    HPS_REQUIRE(box < (int)t.boxes.size(), "box out of range");
    const hps::BoxRec& b = t.boxes[box];
    if (rec) {
      int v[8] = {b.i0, b.i1, b.j0, b.j1, b.level, b.parent, b.ca, b.cb};
      std::memcpy(rec, v, sizeof(v));
    }
    if (b.ca < 0) {
      if (sizes) sizes[0] = sizes[1] = sizes[2] = sizes[3] = 0;
      return;
    }
    hps::MergeMaps mm = hps::merge_maps(t, box);
    if (sizes) {
      sizes[0] = mm.me;
      sizes[1] = mm.m3;
      sizes[2] = mm.na;
      sizes[3] = mm.nb;
    }
    auto put = [](int* dst, const std::vector<int>& v) {
      if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(int));
    };
    put(pmap, mm.pmap);
    put(a3, mm.a3);
    put(b3, mm.b3);
    put(Ie, mm.Ie);
    put(Ii, mm.Ii);
  });
}

hps_status hps_surrogate_create(int p, int q, double hx, double hy, int hidden, int rank,
                                unsigned long long seed, void* stream, hps_surrogate** out) {
  if (out) *out = nullptr;
  return guard([&] {
    HPS_REQUIRE(out && hx > 0 && hy > 0, "bad arguments");
    *out = hps::surrogate_create(p, q, hx, hy, hidden, rank, seed, (hipStream_t)stream).release();
  });
}

hps_status hps_surrogate_train(hps_surrogate* s, const double* coeffs, const double* T, int n,
                               int epochs, int batch, double lr, unsigned long long seed,
                               void* stream, double* final_loss, double* history) {
  return guard([&] {
    HPS_REQUIRE(s && coeffs && T, "bad arguments");
    std::vector<double> hist;
    double L = hps::surrogate_train(s, coeffs, T, n, epochs, batch, lr, seed, (hipStream_t)stream,
                                    &hist);
    if (final_loss) *final_loss = L;
    if (history) std::memcpy(history, hist.data(), hist.size() * sizeof(double));
  });
}

hps_status hps_surrogate_grad(hps_surrogate* s, const double* coeffs, const double* T, int n,
                              float* grads, double* loss, void* stream) {
  return guard([&] {
    HPS_REQUIRE(s && coeffs && T && grads && n >= 1, "bad arguments");
    double L = hps::surrogate_grad(s, coeffs, T, n, grads, (hipStream_t)stream);
    if (loss) *loss = L;
  });
}

hps_status hps_surrogate_predict(hps_surrogate* s, const double* coeffs, int n, double* T,
                                 void* stream) {
  return guard([&] {
    HPS_REQUIRE(s && coeffs && T && n >= 1, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    hps::DeviceMem tmp;
    const size_t pp = (size_t)s->p * s->p, mm = (size_t)s->m * s->m;
    std::vector<const double*> cp(n);
    std::vector<double*> tp(n);
    for (int i = 0; i < n; ++i) {
      cp[i] = coeffs + i * 6 * pp;
      tp[i] = T + i * mm;
    }
    const double** dcp = tmp.upload(cp, st);
    double** dtp = tmp.upload(tp, st);
    hps::surrogate_predict(s, dcp, n, dtp, st);
    HPS_HIP(hipStreamSynchronize(st));
  });
}

hps_status hps_surrogate_info(const hps_surrogate* s, int dims[7], double* out_scale) {
  return guard([&] {
    HPS_REQUIRE(s, "null surrogate");
    if (dims) {
      int v[7] = {s->p, s->q, s->H, s->r, s->D, s->O, s->step};
      std::memcpy(dims, v, sizeof(v));
    }
    if (out_scale) *out_scale = s->out_scale;
  });
}

hps_status hps_surrogate_get_state(const hps_surrogate* s, void* buf, size_t* len) {
  return guard([&] {
    HPS_REQUIRE(s && len, "bad arguments");
    HPS_REQUIRE(s->fitted, "surrogate is not trained");
    std::vector<char> st = hps::surrogate_state(s);
    if (buf) {
      HPS_REQUIRE(*len >= st.size(), "buffer too small");
      std::memcpy(buf, st.data(), st.size());
    }
    *len = st.size();
  });
}

hps_status hps_surrogate_set_state(hps_surrogate* s, const void* buf, size_t len, void* stream) {
  return guard([&] {
    HPS_REQUIRE(s && buf, "bad arguments");
    hps::surrogate_set_state(s, (const char*)buf, len, (hipStream_t)stream);
  });
}

hps_status hps_surrogate_save(const hps_surrogate* s, const char* path) {
  return guard([&] {
    HPS_REQUIRE(s && path, "bad arguments");
    HPS_REQUIRE(s->fitted, "surrogate is not trained");
    std::vector<char> st = hps::surrogate_state(s);
    std::ofstream f(path, std::ios::binary);
    HPS_REQUIRE(f.good(), "cannot open file for writing");
    const char magic[8] = {'H', 'P', 'S', 'M', 'L', 'P', '1', 0};
    f.write(magic, 8);
    f.write(st.data(), (std::streamsize)st.size());
    HPS_REQUIRE(f.good(), "write failed");
  });
}

hps_status hps_surrogate_load(const char* path, void* stream, hps_surrogate** out) {
  if (out) *out = nullptr;
  return guard([&] {
    HPS_REQUIRE(path && out, "bad arguments");
    std::ifstream f(path, std::ios::binary);
    HPS_REQUIRE(f.good(), "cannot open file");
    std::vector<char> all((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    HPS_REQUIRE(all.size() > 8 + 14 * 8 && std::memcmp(all.data(), "HPSMLP1", 7) == 0,
                "not a surrogate file");
    double meta[14];
    std::memcpy(meta, all.data() + 8, sizeof(meta));
    auto sg = hps::surrogate_create((int)meta[0], (int)meta[1], meta[4], meta[5], (int)meta[2],
                                    (int)meta[3], 0, (hipStream_t)stream);
    hps::surrogate_set_state(sg.get(), all.data() + 8, all.size() - 8, (hipStream_t)stream);
    *out = sg.release();
  });
}

void hps_surrogate_destroy(hps_surrogate* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  delete s;
}

void hps_destroy(hps_op* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  try {
    hps::park_operator(op);
  } catch (...) {
  }
}

}  // extern "C"
