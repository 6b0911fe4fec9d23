// HBS matrices on the device (sections 6-8): brute-force compression of a
// dense matrix (Remark 8.2), the telescoping product (eq:tele1 - eq:tele3),
// Algorithm 3 and Algorithm 4.
//
// Compression and Algorithm 3 run level by level, each step a batch over the
// nodes of one tree level: products are grouped launches (one descriptor per
// node and block), the inverses of Algorithm 3 (Dt^-1 and Dhat) batched
// Gauss-Jordan solves with partial pivoting on [Dt | U | I] and
// [V* Dt^-1 U | I].  The product and Algorithm 4 are one persistent launch
// each (below).  Everything runs in order on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "dense.h"
#include "hbs.h"
#include "grid_sync.h"
#include "prof.h"
#include "solver.h"

namespace hps {

HbsLayout::HbsLayout(int L_, int m_, int k_) : L(L_), m(m_), k(k_) {
  const size_t nl = (size_t)1 << L;
  size_t o = 0;
  D = o;
  o += nl * m * m;
  U = o;
  o += nl * m * k;
  Vt = o;
  o += nl * k * m;
  Up.assign(L, 0);
  Vtp.assign(L, 0);
  B.assign(L, 0);
  for (int l = L - 1; l >= 1; --l) {
    Up[l] = o;
    o += ((size_t)1 << l) * 2 * k * k;
    Vtp[l] = o;
    o += ((size_t)1 << l) * k * 2 * k;
  }
  for (int l = L - 1; l >= 0; --l) {
    B[l] = o;
    o += ((size_t)1 << l) * 4 * k * k;
  }
  nfac = o;
  o = 0;
  E.assign(L + 1, 0);
  Fs.assign(L + 1, 0);
  G.assign(L + 1, 0);
  for (int l = L; l >= 1; --l) {
    const size_t nn = (size_t)1 << l, n = rows(l);
    E[l] = o;
    o += nn * n * k;
    Fs[l] = o;
    o += nn * k * n;
    G[l] = o;
    o += nn * n * n;
  }
  G[0] = o;
  o += 4 * (size_t)k * k;
  ninv = o;
}

int hbs_max_compress_rank(int m) { return std::min(90, 16384 / std::max(m, 1)); }

void hbs_check(int L, int m, int k) {
  // At most 2^14 leaves: a level's batched launches keep under 65536
  // descriptors (the limit of a grid's second and third dimensions).
  HPS_REQUIRE(L >= 1 && L <= 14, "HBS levels must be in [1, 14]");
  HPS_REQUIRE(k >= 1 && m >= k, "HBS sizes need 1 <= k <= m");
  HPS_REQUIRE(m <= max_solve_rows() && 2 * k <= max_solve_rows(), "HBS blocks too large");
  HPS_REQUIRE(((long long)m << L) <= (1LL << 30), "HBS matrix too large");
}

namespace {

// One block copy of a batch: dst[r][c] = src[r][c] (mode 0), the identity
// (mode 1), zero (mode 2) or src[c][r] (mode 3), for r < rows, c < cols.
struct CopyDesc {
  const double* src;
  double* dst;
  int lds, ldd, rows, cols, mode, pad;
};

__global__ void __launch_bounds__(256) k_block_copy(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  const long long tot = (long long)d.rows * d.cols;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int r = (int)(e / d.cols), c = (int)(e % d.cols);
    double v;
    if (d.mode == 0)
      v = d.src[(size_t)r * d.lds + c];
    else if (d.mode == 3)
      v = d.src[(size_t)c * d.lds + r];
    else
      v = (d.mode == 1 && r == c) ? 1.0 : 0.0;
    d.dst[(size_t)r * d.ldd + c] = v;
  }
}

void block_copies(DeviceMem& mem, const std::vector<CopyDesc>& h, hipStream_t s) {
  if (h.empty()) return;
  long long most = 1;
  for (auto& d : h) most = std::max(most, (long long)d.rows * d.cols);
  const CopyDesc* dd = mem.upload(h, s);
  const unsigned gx = (unsigned)std::min<long long>((most + 255) / 256, 64);
  hipLaunchKernelGGL(k_block_copy, dim3(gx, (unsigned)h.size()), dim3(256), 0, s, dd);
  HPS_HIP(hipGetLastError());
}

// C = A B (overwrite) or C += A B (accumulate); C0 given: C = C0 + alpha A B.
GemmDesc gd(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int M, int N,
            int K, bool overwrite, double alpha = 1.0, const double* C0 = nullptr, int ldc0 = 0) {
  GemmDesc g{A, B, C, C0, M, N, K, lda, ldb, ldc, ldc0, alpha};
  g.overwrite = overwrite ? 1 : 0;
  return g;
}

// Skinny products of compression and Algorithm 3 (N <= 8 columns, K N <= 4096):
// 16 lanes per row of C read the row of A in 128-byte segments against B
// staged in LDS, then reduce across the group; C = C0 or the old C (unless
// overwrite) plus alpha A B, as in the grouped GEMM.  Grid: (rows / 64,
// descriptors); each workgroup takes 64 rows.
constexpr int GEMV_MAX_N = 8, GEMV_LDS = 4096;

__global__ void __launch_bounds__(256) k_hbs_gemv(const GemmDesc* __restrict__ descs) {
  __shared__ double sB[GEMV_LDS];
  const GemmDesc d = descs[blockIdx.y];
  const int N = d.N, K = d.K;
  for (int e = threadIdx.x; e < K * N; e += 256) sB[e] = d.B[(size_t)(e / N) * d.ldb + e % N];
  __syncthreads();
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  for (int i = 0; i < 4; ++i) {
    const int r = blockIdx.x * 64 + g + 16 * i;
    if (r >= d.M) break;  // the same for the 16 lanes of a group
    double acc[GEMV_MAX_N];
#pragma unroll
    for (int c = 0; c < GEMV_MAX_N; ++c) acc[c] = 0.0;
    const double* a = d.A + (size_t)r * d.lda;
    for (int kk = l; kk < K; kk += 16) {
      const double av = a[kk];
#pragma unroll
      for (int c = 0; c < GEMV_MAX_N; ++c)
        if (c < N) acc[c] = fma(av, sB[kk * N + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < GEMV_MAX_N; ++c)
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 16);
    if (l == 0)
      for (int c = 0; c < N; ++c) {
        double* cp = d.C + (size_t)r * d.ldc + c;
        const double c0 = d.C0 ? d.C0[(size_t)r * d.ldc0 + c] : (d.overwrite ? 0.0 : *cp);
        *cp = c0 + d.alpha * acc[c];
      }
  }
}

// The launches of one operation, uploaded once: each launch is a grouped
// product over a contiguous range of the descriptors (the skinny kernel when
// every product of the launch fits it, else the grouped GEMM).
struct GemmPlan {
  std::vector<GemmDesc> all;
  std::vector<std::pair<size_t, size_t>> launches;
  void launch(const std::vector<GemmDesc>& g) {
    if (g.empty()) return;
    launches.push_back({all.size(), g.size()});
    all.insert(all.end(), g.begin(), g.end());
  }
  void enqueue(GemmDesc* d, hipStream_t s) const {
    for (auto& r : launches) {
      std::vector<GemmDesc> h(all.begin() + r.first, all.begin() + r.first + r.second);
      bool skinny = true;
      int mmax = 1;
      double fl = 0, by = 0;
      for (auto& g : h) {
        skinny = skinny && g.N <= GEMV_MAX_N && (long long)g.K * g.N <= GEMV_LDS;
        mmax = std::max(mmax, g.M);
        fl += 2.0 * g.M * g.N * g.K;
        by += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + 2.0 * g.M * g.N);
      }
      if (skinny) {
        ProfScope ps(PROF_HBS, s, fl, by);
        hipLaunchKernelGGL(k_hbs_gemv, dim3((unsigned)((mmax + 63) / 64), (unsigned)h.size()),
                           dim3(256), 0, s, d + r.first);
        HPS_HIP(hipGetLastError());
      } else {
        grouped_gemm(d + r.first, h, s, GEMM_F64, PROF_HBS);
      }
    }
  }
  void run(DeviceMem& mem, hipStream_t s) const {
    if (all.empty()) return;
    enqueue(mem.upload(all, s), s);
  }
};

// Orthonormalization of `cols` vectors of length `rows`, element i of vector
// c at A[i rs + c cs], by classical Gram-Schmidt with one re-orthogonalization
// pass (CGS2), one workgroup per descriptor, the vectors staged in LDS.  A
// vector that loses all but 1e-13 of its norm to the earlier ones (a sample
// of rank below `cols`) is replaced by a unit vector e_i orthogonalized the
// same way, trying i = c, c + 1, ... until one keeps over half of 1/rows of
// its squared norm, so the basis keeps full rank.
struct OrthDesc {
  double* A;
  int rows, cols, rs, cs;
};
constexpr int ORTH_LDS = 16384;  // doubles: rows * cols limit

// The vectors sit in LDS at an odd stride (rows, or rows + 1), so that the
// lanes that each take one earlier vector's dot product read different banks.
__global__ void __launch_bounds__(256) k_orth(const OrthDesc* __restrict__ descs) {
  __shared__ double Q[ORTH_LDS + 128];
  __shared__ double r[128];
  __shared__ double red[4];
  const OrthDesc d = descs[blockIdx.x];
  const int n = d.rows, ld = n | 1, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < n * d.cols; e += 256) {
    const int c = e / n, i = e % n;
    Q[c * ld + i] = d.A[(size_t)i * d.rs + (size_t)c * d.cs];
  }
  __syncthreads();
  auto norm2 = [&](const double* v) {
    double a = 0.0;
    for (int i = tid; i < n; i += 256) a += v[i] * v[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) red[w] = a;
    __syncthreads();
    const double t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
  };
  // v -= Q[0..c) (Q[0..c)^T v), twice: thread q takes the dot product with
  // vector q, then every thread updates its entries of v.
  auto project_out = [&](double* v, int c) {
    for (int pass = 0; pass < 2; ++pass) {
      // Four partial sums each, so the FMA chains overlap.
      if (tid < c) {
        const double* qv = Q + tid * ld;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = 0;
        for (; i + 4 <= n; i += 4) {
          a0 = fma(qv[i], v[i], a0);
          a1 = fma(qv[i + 1], v[i + 1], a1);
          a2 = fma(qv[i + 2], v[i + 2], a2);
          a3 = fma(qv[i + 3], v[i + 3], a3);
        }
        for (; i < n; ++i) a0 = fma(qv[i], v[i], a0);
        r[tid] = (a0 + a1) + (a2 + a3);
      }
      __syncthreads();
      for (int i = tid; i < n; i += 256) {
        double a0 = v[i], a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int q = 0;
        for (; q + 4 <= c; q += 4) {
          a0 = fma(-r[q], Q[q * ld + i], a0);
          a1 = fma(-r[q + 1], Q[(q + 1) * ld + i], a1);
          a2 = fma(-r[q + 2], Q[(q + 2) * ld + i], a2);
          a3 = fma(-r[q + 3], Q[(q + 3) * ld + i], a3);
        }
        for (; q < c; ++q) a0 = fma(-r[q], Q[q * ld + i], a0);
        v[i] = (a0 + a1) + (a2 + a3);
      }
      __syncthreads();
    }
  };
  for (int c = 0; c < d.cols; ++c) {
    double* v = Q + c * ld;
    const double n0 = norm2(v);
    project_out(v, c);
    double nv = norm2(v);
    // Some e_i keeps at least (n - c) / n of its squared norm outside the
    // span of the c earlier vectors, so the search ends.
    bool ok = nv > 1e-26 * n0 && nv > 0.0;
    for (int t = 0; t < n && !ok; ++t) {
      const int e = (c + t) % n;
      for (int i = tid; i < n; i += 256) v[i] = i == e ? 1.0 : 0.0;
      __syncthreads();
      project_out(v, c);
      nv = norm2(v);
      ok = nv > 0.5 / n;
    }
    const double inv = 1.0 / sqrt(nv);
    for (int i = tid; i < n; i += 256) v[i] *= inv;
    __syncthreads();
  }
  for (int e = tid; e < n * d.cols; e += 256) {
    const int c = e / n, i = e % n;
    d.A[(size_t)i * d.rs + (size_t)c * d.cs] = Q[c * ld + i];
  }
}

void orthonormalize(DeviceMem& mem, const std::vector<OrthDesc>& h, hipStream_t s) {
  if (h.empty()) return;
  for (auto& d : h) HPS_REQUIRE(d.rows >= d.cols && d.rows * d.cols <= ORTH_LDS, "basis too large");
  const OrthDesc* dd = mem.upload(h, s);
  hipLaunchKernelGGL(k_orth, dim3((unsigned)h.size()), dim3(256), 0, s, dd);
  HPS_HIP(hipGetLastError());
}

void solve_batch(DeviceMem& mem, const std::vector<SolveDesc>& h, int* st, hipStream_t s) {
  const SolveDesc* dd = mem.upload(h, s);
  batched_solve(dd, h, st, s, 32);
}

void check_status(const int* st, hipStream_t s, const char* what) {
  int h[4];
  HPS_HIP(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  if (h[0])
    throw Error(HPS_ESINGULAR, std::string("zero or non-finite pivot in ") + what + " of node " +
                                   std::to_string(h[1]));
}

}  // namespace

// Algorithm 3, one level at a time from the leaves: for every node,
// W = [Dt | U | I] gives Z = Dt^-1 U and Dt^-1; [V* Z | I] gives Dhat;
// then E = Z Dhat, P = V* Dt^-1, F* = Dhat P and G = Dt^-1 - E P.  A parent's
// Dt is [[Dhat_1, B_12], [B_21, Dhat_2]] from its children's Dhat and its own
// B; the root's G is the inverse of that block.
void hbs_invert(const HbsLayout& lo, const double* fac, double* inv, hipStream_t s) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k;
  DeviceMem mem;
  int* st = mem.alloc<int>(4);
  HPS_HIP(hipMemsetAsync(st, 0, 4 * sizeof(int), s));
  const double* dh_prev = nullptr;  // children's Dhat blocks, k x k at ld 2k, stride 2k k
  for (int l = L; l >= 0; --l) {
    const bool root = l == 0;
    const int nn = 1 << l, n = root ? k2 : lo.rows(l);
    const int wc = root ? 2 * n : 2 * n + k;  // columns of W
    double* W = mem.alloc<double>((size_t)nn * n * wc);
    int* piv = mem.alloc<int>((size_t)nn * n);
    std::vector<CopyDesc> cp;
    for (int j = 0; j < nn; ++j) {
      double* Wj = W + (size_t)j * n * wc;
      if (l == L) {
        cp.push_back({fac + lo.D + (size_t)j * m * m, Wj, m, wc, m, m, 0, 0});
      } else {
        const double* d1 = dh_prev + (size_t)(2 * j) * k2 * k;
        const double* d2 = dh_prev + (size_t)(2 * j + 1) * k2 * k;
        const double* Bj = fac + lo.B[l] + (size_t)j * 4 * k * k;
        cp.push_back({d1, Wj, k2, wc, k, k, 0, 0});
        cp.push_back({Bj + k, Wj + k, k2, wc, k, k, 0, 0});
        cp.push_back({Bj + (size_t)k * k2, Wj + (size_t)k * wc, k2, wc, k, k, 0, 0});
        cp.push_back({d2, Wj + (size_t)k * wc + k, k2, wc, k, k, 0, 0});
      }
      if (root) {
        cp.push_back({nullptr, Wj + n, 0, wc, n, n, 1, 0});
      } else {
        const double* Uj = l == L ? fac + lo.U + (size_t)j * m * k
                                  : fac + lo.Up[l] + (size_t)j * k2 * k;
        cp.push_back({Uj, Wj + n, k, wc, n, k, 0, 0});
        cp.push_back({nullptr, Wj + n + k, 0, wc, n, n, 1, 0});
      }
    }
    block_copies(mem, cp, s);
    std::vector<SolveDesc> sd(nn);
    for (int j = 0; j < nn; ++j) {
      double* Wj = W + (size_t)j * n * wc;
      sd[j] = SolveDesc{Wj, piv + (size_t)j * n, Wj + n, n, wc - n, wc, wc, j, 0};
    }
    solve_batch(mem, sd, st, s);
    if (root) {
      cp.clear();
      cp.push_back({W + n, inv + lo.G[0], wc, n, n, n, 0, 0});
      block_copies(mem, cp, s);
      break;
    }
    // Dhat = (V* Z)^-1 through [V* Z | I].
    double* W2 = mem.alloc<double>((size_t)nn * k * k2);
    int* piv2 = mem.alloc<int>((size_t)nn * k);
    double* Pm = mem.alloc<double>((size_t)nn * k * n);
    GemmPlan P;
    std::vector<GemmDesc> g;
    auto Vt_of = [&](int j) {
      return l == L ? fac + lo.Vt + (size_t)j * k * m : fac + lo.Vtp[l] + (size_t)j * k * k2;
    };
    for (int j = 0; j < nn; ++j)
      g.push_back(gd(Vt_of(j), n, W + (size_t)j * n * wc + n, wc, W2 + (size_t)j * k * k2, k2, k,
                     k, n, true));
    P.launch(g);
    P.run(mem, s);
    cp.clear();
    for (int j = 0; j < nn; ++j) cp.push_back({nullptr, W2 + (size_t)j * k * k2 + k, 0, k2, k, k, 1, 0});
    block_copies(mem, cp, s);
    for (int j = 0; j < nn; ++j) {
      double* Wj = W2 + (size_t)j * k * k2;
      sd[j] = SolveDesc{Wj, piv2 + (size_t)j * k, Wj + k, k, k, k2, k2, j, 0};
    }
    solve_batch(mem, sd, st, s);
    GemmPlan Q;
    std::vector<GemmDesc> ge, gp, gf, gg;
    for (int j = 0; j < nn; ++j) {
      const double* Z = W + (size_t)j * n * wc + n;  // Dt^-1 U
      const double* Di = Z + k;                      // Dt^-1
      const double* Dh = W2 + (size_t)j * k * k2 + k;
      double* Ej = inv + lo.E[l] + (size_t)j * n * k;
      double* Fj = inv + lo.Fs[l] + (size_t)j * k * n;
      double* Gj = inv + lo.G[l] + (size_t)j * n * n;
      double* Pj = Pm + (size_t)j * k * n;
      ge.push_back(gd(Z, wc, Dh, k2, Ej, k, n, k, k, true));
      gp.push_back(gd(Vt_of(j), n, Di, wc, Pj, n, k, n, n, true));
      gf.push_back(gd(Dh, k2, Pj, n, Fj, n, k, n, k, true));
      gg.push_back(gd(Ej, k, Pj, n, Gj, n, n, n, k, false, -1.0, Di, wc));
    }
    Q.launch(ge);
    Q.launch(gp);
    Q.launch(gf);
    Q.launch(gg);
    Q.run(mem, s);
    dh_prev = W2 + k;
  }
  check_status(st, s, "an HBS inversion block");
}

// ---------------------------------------------------------------------------
// The telescoping product and Algorithm 4 as one persistent launch each.
//
// Both passes are a fixed sequence of phases (one per tree level up, the
// root, one per level down, the leaves), and every phase is a set of rows
// c = A0[r] B0 + A1[r] B1 of small products whose right-hand factors are the
// caller's x or x-hat / y-hat blocks of earlier phases.  One cooperative
// launch runs all phases, separated by grid barriers; 16 lanes take one row
// (128-byte segments of A), up to 8 right-hand sides at a time.  The hat
// blocks pass between workgroups on different XCDs, so they are written and
// read with device-scope relaxed atomics (grid_sync.h), read once per node
// and workgroup into LDS; the factors and x are read with plain loads and the
// output y is written with plain stores.  A
// barrier that waits about a second sets the error flag (reported as a
// device error) and lets the workgroup go on, so the launch always ends.
// ---------------------------------------------------------------------------
struct RowDesc {
  const double* A0;
  const double* B0;
  const double* A1;
  const double* B1;
  double* C;
  int lda0, lda1, K0, K1;
  int plain0, plain1;  // 1: that B is the caller's x (plain loads)
};
struct Phase {
  int first, nodes, rows, out;  // out: C is the caller's y (plain stores)
};
constexpr int PASS_NC = 8;

// Each workgroup takes a contiguous share of a phase's rows.  For every node
// its share touches, the hat blocks that node reads (K x nrhs doubles each,
// written by other workgroups in the previous phases) are staged once in LDS
// with device-scope loads, so the rows then read them from LDS; a hat block
// larger than PASS_LDS doubles is read from memory row by row instead.
constexpr int PASS_LDS = 4096;

__global__ void __launch_bounds__(256) k_hbs_pass(const Phase* __restrict__ ph, int nph,
                                                  const RowDesc* __restrict__ rd, int N,
                                                  unsigned* bar, int* err) {
  __shared__ double sB[2][PASS_LDS];
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  unsigned gen = 0;
  for (int p = 0; p < nph; ++p) {
    const Phase P = ph[p];
    const long long rows = (long long)P.nodes * P.rows;
    const long long r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
    for (long long t = r0; t < r1;) {  // the same trip count for the whole workgroup
      const int node = (int)(t / P.rows);
      const long long te = min(r1, (long long)(node + 1) * P.rows);
      const RowDesc d = rd[P.first + node];
      const bool st0 = !d.plain0 && d.K0 * N <= PASS_LDS;
      const bool st1 = !d.plain1 && d.K1 * N <= PASS_LDS;
      __syncthreads();  // the previous node's rows are done with sB
      if (st0)
        for (int e = threadIdx.x; e < d.K0 * N; e += 256) sB[0][e] = ld_dev(d.B0 + e);
      if (st1)
        for (int e = threadIdx.x; e < d.K1 * N; e += 256) sB[1][e] = ld_dev(d.B1 + e);
      __syncthreads();
      for (long long row = t + g; row < te; row += 16) {
        const int r = (int)(row - (long long)node * P.rows);
        for (int c0 = 0; c0 < N; c0 += PASS_NC) {
          double acc[PASS_NC];
#pragma unroll
          for (int c = 0; c < PASS_NC; ++c) acc[c] = 0.0;
#pragma unroll
          for (int term = 0; term < 2; ++term) {
            const double* A = term ? d.A1 : d.A0;
            const double* B = term ? d.B1 : d.B0;
            const int K = term ? d.K1 : d.K0, lda = term ? d.lda1 : d.lda0;
            const bool plain = (term ? d.plain1 : d.plain0) != 0;
            const bool staged = term ? st1 : st0;
            const double* sb = sB[term];
            const double* a = A + (size_t)r * lda;
            for (int kk = l; kk < K; kk += 16) {
              const double av = a[kk];
              const size_t o = (size_t)kk * N + c0;
#pragma unroll
              for (int c = 0; c < PASS_NC; ++c)
                if (c0 + c < N) {
                  const double bv = staged ? sb[o + c] : (plain ? B[o + c] : ld_dev(B + o + c));
                  acc[c] = fma(av, bv, acc[c]);
                }
            }
          }
#pragma unroll
          for (int c = 0; c < PASS_NC; ++c)
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 16);
          if (l == 0) {
            double* cr = d.C + (size_t)r * N + c0;
#pragma unroll
            for (int c = 0; c < PASS_NC; ++c)
              if (c0 + c < N) {
                if (P.out)
                  cr[c] = acc[c];
                else
                  st_dev(cr + c, acc[c]);
              }
          }
        }
      }
      t = te;
    }
    if (p + 1 < nph) grid_barrier(bar, gridDim.x, gen, err);
  }
}

__global__ void k_hbs_pass_zero(unsigned* bar, int* err) {
  if (threadIdx.x < 9) bar[32 * threadIdx.x] = 0u;
  if (threadIdx.x == 0) *err = 0;
}

namespace {

RowDesc row(const double* A0, int lda0, const double* B0, int K0, bool plain0, double* C,
            const double* A1 = nullptr, int lda1 = 0, const double* B1 = nullptr, int K1 = 0,
            bool plain1 = false) {
  return RowDesc{A0, B0, A1, B1, C, lda0, lda1, K0, K1, plain0 ? 1 : 0, plain1 ? 1 : 0};
}

struct PassPlan {
  std::vector<Phase> ph;
  std::vector<RowDesc> rd;
  void phase(int rows, const std::vector<RowDesc>& nodes, bool out = false) {
    ph.push_back(Phase{(int)rd.size(), (int)nodes.size(), rows, out ? 1 : 0});
    rd.insert(rd.end(), nodes.begin(), nodes.end());
  }
};

// x-hat / y-hat pointers of a pass: level l (1 .. L) holds 2^l blocks of
// k x nrhs, node-major.
struct HatPtrs {
  std::vector<double*> x, y;
};

}  // namespace

// y = H x by the telescoping factorization: x-hat = V* x up the tree, the
// sibling blocks of each B, y-hat = U y-hat(parent) + B x-hat down the tree,
// and y = U y-hat + D x at the leaves.
static void apply_plan(const HbsLayout& lo, const double* fac, const double* x, double* y,
                       int nrhs, const HatPtrs& h, PassPlan& P) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k, NL = 1 << L;
  const size_t bx = (size_t)k * nrhs;
  std::vector<RowDesc> v;
  for (int j = 0; j < NL; ++j)
    v.push_back(row(fac + lo.Vt + (size_t)j * k * m, m, x + (size_t)j * m * nrhs, m, true,
                    h.x[L] + j * bx));
  P.phase(k, v);
  for (int l = L - 1; l >= 1; --l) {
    v.clear();
    for (int j = 0; j < (1 << l); ++j)
      v.push_back(row(fac + lo.Vtp[l] + (size_t)j * k * k2, k2, h.x[l + 1] + 2 * j * bx, k2,
                      false, h.x[l] + j * bx));
    P.phase(k, v);
  }
  // Root: y-hat of child h from the other child's x-hat through B's
  // off-diagonal block (upper right for h = 0, lower left for h = 1).
  v.clear();
  for (int hh = 0; hh < 2; ++hh)
    v.push_back(row(fac + lo.B[0] + (hh == 0 ? (size_t)k : (size_t)k * k2), k2,
                    h.x[1] + (1 - hh) * bx, k, false, h.y[1] + hh * bx));
  P.phase(k, v);
  for (int l = 1; l < L; ++l) {
    v.clear();
    for (int nd = 0; nd < (2 << l); ++nd) {
      const int j = nd / 2, hh = nd % 2;
      const double* Bj = fac + lo.B[l] + (size_t)j * 4 * k * k;
      v.push_back(row(fac + lo.Up[l] + (size_t)j * k2 * k + (size_t)hh * k * k, k,
                      h.y[l] + j * bx, k, false, h.y[l + 1] + nd * bx,
                      Bj + (hh == 0 ? (size_t)k : (size_t)k * k2), k2,
                      h.x[l + 1] + (2 * j + 1 - hh) * bx, k, false));
    }
    P.phase(k, v);
  }
  v.clear();
  for (int j = 0; j < NL; ++j)
    v.push_back(row(fac + lo.D + (size_t)j * m * m, m, x + (size_t)j * m * nrhs, m, true,
                    y + (size_t)j * m * nrhs, fac + lo.U + (size_t)j * m * k, k, h.y[L] + j * bx,
                    k, false));
  P.phase(m, v, true);
}

// Algorithm 4: x-hat = F* x up the tree, y-hat at the top from the root's G,
// then y-hat(children) = E y-hat + G x-hat(children) down the tree and
// y = E y-hat + G x at the leaves.
static void solve_plan(const HbsLayout& lo, const double* inv, const double* x, double* y,
                       int nrhs, const HatPtrs& h, PassPlan& P) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k, NL = 1 << L;
  const size_t bx = (size_t)k * nrhs;
  std::vector<RowDesc> v;
  for (int j = 0; j < NL; ++j)
    v.push_back(row(inv + lo.Fs[L] + (size_t)j * k * m, m, x + (size_t)j * m * nrhs, m, true,
                    h.x[L] + j * bx));
  P.phase(k, v);
  for (int l = L - 1; l >= 1; --l) {
    v.clear();
    for (int j = 0; j < (1 << l); ++j)
      v.push_back(row(inv + lo.Fs[l] + (size_t)j * k * k2, k2, h.x[l + 1] + 2 * j * bx, k2,
                      false, h.x[l] + j * bx));
    P.phase(k, v);
  }
  P.phase(k2, {row(inv + lo.G[0], k2, h.x[1], k2, false, h.y[1])});
  for (int l = 1; l < L; ++l) {
    v.clear();
    for (int j = 0; j < (1 << l); ++j)
      v.push_back(row(inv + lo.G[l] + (size_t)j * k2 * k2, k2, h.x[l + 1] + 2 * j * bx, k2, false,
                      h.y[l + 1] + 2 * j * bx, inv + lo.E[l] + (size_t)j * k2 * k, k,
                      h.y[l] + j * bx, k, false));
    P.phase(k2, v);
  }
  v.clear();
  for (int j = 0; j < NL; ++j)
    v.push_back(row(inv + lo.G[L] + (size_t)j * m * m, m, x + (size_t)j * m * nrhs, m, true,
                    y + (size_t)j * m * nrhs, inv + lo.E[L] + (size_t)j * m * k, k,
                    h.y[L] + j * bx, k, false));
  P.phase(m, v, true);
}

// A pass's phases, row descriptors, hat blocks and barrier counters are kept
// per (matrix buffer, x, y, nrhs, sizes, device) and reused by later calls
// (at most 16, least recently used first out; hps_mem_trim drops them).
namespace {

struct CachedPass {
  DeviceMem mem;
  Phase* ph = nullptr;
  RowDesc* rd = nullptr;
  int nph = 0;
  unsigned* bar = nullptr;
  int* err = nullptr;
  double flops = 0, bytes = 0;
};
using PassKey = std::tuple<int, int, const void*, const void*, const void*, int, int, int, int>;

std::mutex g_pass_mu;
std::map<PassKey, std::unique_ptr<CachedPass>> g_passes;
std::list<PassKey> g_pass_order;
constexpr size_t MAX_PASSES = 16;

int g_pass_grid_req = 0;  // knob hbs_grid: workgroups of a pass (0: two per CU)

int pass_grid() {
  static int cus = -1, per = 0;
  if (cus < 0) {
    int dev = 0;
    HPS_HIP(hipGetDevice(&dev));
    HPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_hbs_pass, 256, 0));
  }
  if (per < 1) return 0;
  return std::min(g_pass_grid_req > 0 ? g_pass_grid_req : 2 * cus, cus * per);
}

template <class Build>
void run_pass(int kind, const HbsLayout& lo, const double* mat, const double* x, const double* y,
              int nrhs, hipStream_t s, Build build) {
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  const int grid = pass_grid();
  HPS_REQUIRE(grid > 0, "HBS pass: no resident workgroups");
  std::lock_guard<std::mutex> lk(g_pass_mu);
  const PassKey key{kind, dev, mat, x, y, nrhs, lo.L, lo.m, lo.k};
  auto it = g_passes.find(key);
  if (it == g_passes.end()) {
    auto C = std::make_unique<CachedPass>();
    HatPtrs h{std::vector<double*>(lo.L + 1, nullptr), std::vector<double*>(lo.L + 1, nullptr)};
    for (int l = 1; l <= lo.L; ++l) {
      h.x[l] = C->mem.alloc<double>(((size_t)1 << l) * lo.k * nrhs);
      h.y[l] = C->mem.alloc<double>(((size_t)1 << l) * lo.k * nrhs);
    }
    PassPlan P;
    build(h, P);
    for (const Phase& q : P.ph)
      for (int n = 0; n < q.nodes; ++n) {
        const RowDesc& d = P.rd[q.first + n];
        C->flops += 2.0 * q.rows * nrhs * (d.K0 + d.K1);
        C->bytes += 8.0 * q.rows * (d.K0 + d.K1 + nrhs);
      }
    C->ph = C->mem.alloc<Phase>(P.ph.size());
    C->rd = C->mem.alloc<RowDesc>(P.rd.size());
    C->nph = (int)P.ph.size();
    C->bar = C->mem.alloc<unsigned>(9 * 32);
    C->err = C->mem.alloc<int>(1);
    HPS_HIP(hipMemcpy(C->ph, P.ph.data(), P.ph.size() * sizeof(Phase), hipMemcpyHostToDevice));
    HPS_HIP(hipMemcpy(C->rd, P.rd.data(), P.rd.size() * sizeof(RowDesc), hipMemcpyHostToDevice));
    if (g_passes.size() >= MAX_PASSES) {
      // Every call waits for its stream, so no evicted pass is still running.
      g_passes.erase(g_pass_order.front());
      g_pass_order.pop_front();
    }
    it = g_passes.emplace(key, std::move(C)).first;
    g_pass_order.push_back(key);
  } else {
    g_pass_order.remove(key);
    g_pass_order.push_back(key);
  }
  CachedPass& C = *it->second;
  hipLaunchKernelGGL(k_hbs_pass_zero, dim3(1), dim3(64), 0, s, C.bar, C.err);
  {
    ProfScope ps(PROF_HBS, s, C.flops, C.bytes);
    int N = nrhs;
    void* args[] = {(void*)&C.ph, (void*)&C.nph, (void*)&C.rd, (void*)&N, (void*)&C.bar,
                    (void*)&C.err};
    HPS_HIP(hipLaunchCooperativeKernel((const void*)k_hbs_pass, dim3(grid), dim3(256), args, 0, s));
  }
  int herr = 0;
  HPS_HIP(hipMemcpyAsync(&herr, C.err, sizeof(int), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  if (herr) throw Error(HPS_EDEVICE, "HBS pass: a grid barrier timed out");
}

}  // namespace

void hbs_set_pass_grid(int workgroups) { g_pass_grid_req = std::max(0, workgroups); }

void hbs_passes_clear() {
  std::lock_guard<std::mutex> lk(g_pass_mu);
  g_passes.clear();
  g_pass_order.clear();
}

void hbs_apply(const HbsLayout& lo, const double* fac, const double* x, double* y, int nrhs,
               hipStream_t s) {
  run_pass(0, lo, fac, x, y, nrhs, s,
           [&](const HatPtrs& h, PassPlan& P) { apply_plan(lo, fac, x, y, nrhs, h, P); });
}

void hbs_solve(const HbsLayout& lo, const double* inv, const double* x, double* y, int nrhs,
               hipStream_t s) {
  run_pass(1, lo, inv, x, y, nrhs, s,
           [&](const HatPtrs& h, PassPlan& P) { solve_plan(lo, inv, x, y, nrhs, h, P); });
}

// Brute-force compression (Remark 8.2) of a dense matrix into HBS factors of
// one rank k, with orthonormal nested bases taken from random samples
// Y = H Omega and Z* = Psi* H.  Level by level from the leaves: the samples
// of each node's off-diagonal block row and column are Y and Z* less the
// node's diagonal block times its part of Omega or Psi*; at a leaf they are
// orthonormalized into U and V*; at a parent they are first reduced to the
// children's bases (eq:def3) and then orthonormalized.  The bases in the
// original indices (Ubig* and Vbig, as k x M and M x k) follow from the
// children's; the children's interaction blocks of every parent are
// Ubig*(I_1) H(I_1, I_2) Vbig(I_2) and the reverse (eq:def6).
void hbs_compress(const HbsLayout& lo, const double* H, int ldh, const double* omega,
                  const double* psit, double* fac, hipStream_t s) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k;
  const long long M = lo.M();
  DeviceMem mem;
  double* Y = mem.alloc<double>((size_t)M * k);
  double* ZT = mem.alloc<double>((size_t)M * k);
  double* R = mem.alloc<double>((size_t)M * k);
  double* RT = mem.alloc<double>((size_t)M * k);
  double* UbT[2] = {mem.alloc<double>((size_t)M * k), mem.alloc<double>((size_t)M * k)};
  double* Vb[2] = {mem.alloc<double>((size_t)M * k), mem.alloc<double>((size_t)M * k)};
  double* T1 = mem.alloc<double>((size_t)M * k);
  double* Ut = mem.alloc<double>(((size_t)1 << L) * k * k);
  double* Vs = mem.alloc<double>(((size_t)1 << L) * k * k);
  {
    GemmPlan P;
    P.launch({gd(H, ldh, omega, k, Y, k, (int)M, k, (int)M, true)});
    P.launch({gd(psit, (int)M, H, ldh, ZT, (int)M, k, (int)M, (int)M, true)});
    P.run(mem, s);
  }
  std::vector<CopyDesc> cp;
  for (int j = 0; j < (1 << L); ++j)
    cp.push_back({H + (size_t)j * m * ldh + (size_t)j * m, fac + lo.D + (size_t)j * m * m, ldh, m,
                  m, m, 0, 0});
  block_copies(mem, cp, s);
  int cur = 0;  // UbT[cur], Vb[cur]: the bases of level l + 1
  for (int l = L; l >= 1; --l) {
    const int nn = 1 << l, nl = (int)(M >> l), nc = nl / 2;
    double* ubt = UbT[cur ^ 1];
    double* vb = Vb[cur ^ 1];
    const double* ubt_c = UbT[cur];
    const double* vb_c = Vb[cur];
    {
      GemmPlan P;
      std::vector<GemmDesc> g1, g2;
      for (int j = 0; j < nn; ++j) {
        const size_t i0 = (size_t)j * nl;
        const double* Hjj = H + i0 * ldh + i0;
        g1.push_back(gd(Hjj, ldh, omega + i0 * k, k, R + i0 * k, k, nl, k, nl, false, -1.0,
                        Y + i0 * k, k));
        g2.push_back(gd(psit + i0, (int)M, Hjj, ldh, RT + i0, (int)M, k, nl, nl, false, -1.0,
                        ZT + i0, (int)M));
      }
      P.launch(g1);
      P.launch(g2);
      P.run(mem, s);
    }
    std::vector<OrthDesc> od;
    cp.clear();
    if (l == L) {
      for (int j = 0; j < nn; ++j) {
        double* Uj = fac + lo.U + (size_t)j * m * k;
        double* Vtj = fac + lo.Vt + (size_t)j * k * m;
        cp.push_back({R + (size_t)j * m * k, Uj, k, k, m, k, 0, 0});
        cp.push_back({RT + (size_t)j * m, Vtj, (int)M, m, k, m, 0, 0});
        od.push_back({Uj, m, k, k, 1});
        od.push_back({Vtj, m, k, 1, m});
      }
      block_copies(mem, cp, s);
      orthonormalize(mem, od, s);
      cp.clear();
      for (int j = 0; j < nn; ++j) {
        cp.push_back({fac + lo.U + (size_t)j * m * k, ubt + (size_t)j * m, k, (int)M, k, m, 3, 0});
        cp.push_back({fac + lo.Vt + (size_t)j * k * m, vb + (size_t)j * m * k, m, k, m, k, 3, 0});
      }
      block_copies(mem, cp, s);
    } else {
      GemmPlan P;
      std::vector<GemmDesc> gu, gv;
      for (int j = 0; j < nn; ++j) {
        double* Uj = fac + lo.Up[l] + (size_t)j * k2 * k;
        double* Vtj = fac + lo.Vtp[l] + (size_t)j * k * k2;
        for (int h = 0; h < 2; ++h) {
          const size_t ic = (size_t)(2 * j + h) * nc;
          gu.push_back(gd(ubt_c + ic, (int)M, R + ic * k, k, Uj + (size_t)h * k * k, k, k, k, nc,
                          true));
          gv.push_back(gd(RT + ic, (int)M, vb_c + ic * k, k, Vtj + (size_t)h * k, k2, k, k, nc,
                          true));
        }
        od.push_back({Uj, k2, k, k, 1});
        od.push_back({Vtj, k2, k, 1, k2});
      }
      P.launch(gu);
      P.launch(gv);
      P.run(mem, s);
      orthonormalize(mem, od, s);
      for (int j = 0; j < nn; ++j) {
        cp.push_back({fac + lo.Up[l] + (size_t)j * k2 * k, Ut + (size_t)j * k * k2, k, k2, k, k2, 3, 0});
        cp.push_back({fac + lo.Vtp[l] + (size_t)j * k * k2, Vs + (size_t)j * k2 * k, k2, k, k2, k, 3, 0});
      }
      block_copies(mem, cp, s);
      GemmPlan Q;
      std::vector<GemmDesc> bu, bv;
      for (int j = 0; j < nn; ++j)
        for (int h = 0; h < 2; ++h) {
          const size_t ic = (size_t)(2 * j + h) * nc;
          bu.push_back(gd(Ut + (size_t)j * k * k2 + (size_t)h * k, k2, ubt_c + ic, (int)M, ubt + ic,
                          (int)M, k, nc, k, true));
          bv.push_back(gd(vb_c + ic * k, k, Vs + (size_t)j * k2 * k + (size_t)h * k * k, k,
                          vb + ic * k, k, nc, k, k, true));
        }
      Q.launch(bu);
      Q.launch(bv);
      Q.run(mem, s);
    }
    // The interaction blocks of the parents one level up: Ubig*(I_1) H(I_1, I_2) Vbig(I_2).
    {
      const int np = nn / 2;
      GemmPlan P;
      std::vector<GemmDesc> t1, tb;
      cp.clear();
      for (int j = 0; j < np; ++j) {
        const size_t i1 = (size_t)(2 * j) * nl, i2 = i1 + nl;
        double* Bj = fac + lo.B[l - 1] + (size_t)j * 4 * k * k;
        double* T1a = T1 + i1 * k;
        double* T1b = T1 + i2 * k;
        t1.push_back(gd(H + i1 * ldh + i2, ldh, vb + i2 * k, k, T1a, k, nl, k, nl, true));
        t1.push_back(gd(H + i2 * ldh + i1, ldh, vb + i1 * k, k, T1b, k, nl, k, nl, true));
        tb.push_back(gd(ubt + i1, (int)M, T1a, k, Bj + k, k2, k, k, nl, true));
        tb.push_back(gd(ubt + i2, (int)M, T1b, k, Bj + (size_t)k * k2, k2, k, k, nl, true));
        cp.push_back({nullptr, Bj, 0, k2, k, k, 2, 0});
        cp.push_back({nullptr, Bj + (size_t)k * k2 + k, 0, k2, k, k, 2, 0});
      }
      P.launch(t1);
      P.launch(tb);
      P.run(mem, s);
      block_copies(mem, cp, s);
    }
    cur ^= 1;
  }
  HPS_HIP(hipStreamSynchronize(s));
}

}  // namespace hps
