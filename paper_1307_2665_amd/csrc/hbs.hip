// HBS matrices on the device (sections 6-7): the telescoping product
// (eq:tele1 - eq:tele3), Algorithm 3 and Algorithm 4.
//
// Every step is a batch over the nodes of one tree level: the products are
// grouped FP64 GEMM launches (one descriptor per node and block), and the
// inverses of Algorithm 3 (Dt^-1 and Dhat) are batched Gauss-Jordan solves
// with partial pivoting on [Dt | U | I] and [V* Dt^-1 U | I].  The levels run
// in order on the caller's stream; nodes of a level are independent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dense.h"
#include "hbs.h"
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

void hbs_check(int L, int m, int k) {
  HPS_REQUIRE(L >= 1 && L <= 20, "HBS levels must be in [1, 20]");
  HPS_REQUIRE(k >= 1 && m >= k, "HBS sizes need 1 <= k <= m");
  HPS_REQUIRE(m <= max_solve_rows() && 2 * k <= max_solve_rows(), "HBS blocks too large");
  HPS_REQUIRE(((long long)m << L) <= (1LL << 30), "HBS matrix too large");
}

namespace {

// One block copy of a batch: dst[r][c] = src[r][c] (mode 0), the identity
// (mode 1) or zero (mode 2), for r < rows, c < cols.
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

// The launches of one operation, uploaded once: each launch is a grouped
// GEMM over a contiguous range of the descriptors.
struct GemmPlan {
  std::vector<GemmDesc> all;
  std::vector<std::pair<size_t, size_t>> launches;
  void launch(const std::vector<GemmDesc>& g) {
    if (g.empty()) return;
    launches.push_back({all.size(), g.size()});
    all.insert(all.end(), g.begin(), g.end());
  }
  void run(DeviceMem& mem, hipStream_t s) const {
    if (all.empty()) return;
    GemmDesc* d = mem.upload(all, s);
    for (auto& r : launches) {
      std::vector<GemmDesc> h(all.begin() + r.first, all.begin() + r.first + r.second);
      grouped_gemm(d + r.first, h, s, GEMM_F64);
    }
  }
};

// x-hat / y-hat buffers: level l (1 .. L) holds 2^l blocks of k x nrhs.
struct Hats {
  std::vector<double*> x, y;
  Hats(DeviceMem& mem, int L, int k, int nrhs) : x(L + 1, nullptr), y(L + 1, nullptr) {
    for (int l = 1; l <= L; ++l) {
      x[l] = mem.alloc<double>(((size_t)1 << l) * k * nrhs);
      y[l] = mem.alloc<double>(((size_t)1 << l) * k * nrhs);
    }
  }
};

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

// y = H x by the telescoping factorization: x-hat = V* x up the tree, the
// sibling blocks of each B, y-hat = U y-hat(parent) + B x-hat down the tree,
// and y = U y-hat + D x at the leaves.
void hbs_apply(const HbsLayout& lo, const double* fac, const double* x, double* y, int nrhs,
               hipStream_t s) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k;
  DeviceMem mem;
  Hats h(mem, L, k, nrhs);
  const size_t bx = (size_t)k * nrhs;  // one x-hat block
  GemmPlan P;
  std::vector<GemmDesc> g;
  const int NL = 1 << L;
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(fac + lo.Vt + (size_t)j * k * m, m, x + (size_t)j * m * nrhs, nrhs,
                   h.x[L] + j * bx, nrhs, k, nrhs, m, true));
  P.launch(g);
  for (int l = L - 1; l >= 1; --l) {
    g.clear();
    for (int j = 0; j < (1 << l); ++j)
      g.push_back(gd(fac + lo.Vtp[l] + (size_t)j * k * k2, k2, h.x[l + 1] + 2 * j * bx, nrhs,
                     h.x[l] + j * bx, nrhs, k, nrhs, k2, true));
    P.launch(g);
  }
  for (int l = 0; l < L; ++l) {
    const int nn = 1 << l;
    if (l > 0) {
      g.clear();
      for (int j = 0; j < nn; ++j)
        g.push_back(gd(fac + lo.Up[l] + (size_t)j * k2 * k, k, h.y[l] + j * bx, nrhs,
                       h.y[l + 1] + 2 * j * bx, nrhs, k2, nrhs, k, true));
      P.launch(g);
    }
    g.clear();
    for (int j = 0; j < nn; ++j) {
      const double* Bj = fac + lo.B[l] + (size_t)j * 4 * k * k;
      double* y1 = h.y[l + 1] + 2 * j * bx;
      const double* x1 = h.x[l + 1] + 2 * j * bx;
      // Upper-right block (rows of child 1, x-hat of child 2) and lower-left.
      g.push_back(gd(Bj + k, k2, x1 + bx, nrhs, y1, nrhs, k, nrhs, k, l == 0));
      g.push_back(gd(Bj + (size_t)k * k2, k2, x1, nrhs, y1 + bx, nrhs, k, nrhs, k, l == 0));
    }
    P.launch(g);
  }
  g.clear();
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(fac + lo.D + (size_t)j * m * m, m, x + (size_t)j * m * nrhs, nrhs,
                   y + (size_t)j * m * nrhs, nrhs, m, nrhs, m, true));
  P.launch(g);
  g.clear();
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(fac + lo.U + (size_t)j * m * k, k, h.y[L] + j * bx, nrhs,
                   y + (size_t)j * m * nrhs, nrhs, m, nrhs, k, false));
  P.launch(g);
  P.run(mem, s);
  HPS_HIP(hipStreamSynchronize(s));
}

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

// Algorithm 4: x-hat = F* x up the tree, y-hat at the top from the root's G,
// then y-hat(children) = E y-hat + G x-hat(children) down the tree and
// y = E y-hat + G x at the leaves.
void hbs_solve(const HbsLayout& lo, const double* inv, const double* x, double* y, int nrhs,
               hipStream_t s) {
  const int L = lo.L, m = lo.m, k = lo.k, k2 = 2 * k;
  DeviceMem mem;
  Hats h(mem, L, k, nrhs);
  const size_t bx = (size_t)k * nrhs;
  GemmPlan P;
  std::vector<GemmDesc> g;
  const int NL = 1 << L;
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(inv + lo.Fs[L] + (size_t)j * k * m, m, x + (size_t)j * m * nrhs, nrhs,
                   h.x[L] + j * bx, nrhs, k, nrhs, m, true));
  P.launch(g);
  for (int l = L - 1; l >= 1; --l) {
    g.clear();
    for (int j = 0; j < (1 << l); ++j)
      g.push_back(gd(inv + lo.Fs[l] + (size_t)j * k * k2, k2, h.x[l + 1] + 2 * j * bx, nrhs,
                     h.x[l] + j * bx, nrhs, k, nrhs, k2, true));
    P.launch(g);
  }
  g.clear();
  g.push_back(gd(inv + lo.G[0], k2, h.x[1], nrhs, h.y[1], nrhs, k2, nrhs, k2, true));
  P.launch(g);
  for (int l = 1; l < L; ++l) {
    const int nn = 1 << l;
    g.clear();
    for (int j = 0; j < nn; ++j)
      g.push_back(gd(inv + lo.G[l] + (size_t)j * k2 * k2, k2, h.x[l + 1] + 2 * j * bx, nrhs,
                     h.y[l + 1] + 2 * j * bx, nrhs, k2, nrhs, k2, true));
    P.launch(g);
    g.clear();
    for (int j = 0; j < nn; ++j)
      g.push_back(gd(inv + lo.E[l] + (size_t)j * k2 * k, k, h.y[l] + j * bx, nrhs,
                     h.y[l + 1] + 2 * j * bx, nrhs, k2, nrhs, k, false));
    P.launch(g);
  }
  g.clear();
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(inv + lo.G[L] + (size_t)j * m * m, m, x + (size_t)j * m * nrhs, nrhs,
                   y + (size_t)j * m * nrhs, nrhs, m, nrhs, m, true));
  P.launch(g);
  g.clear();
  for (int j = 0; j < NL; ++j)
    g.push_back(gd(inv + lo.E[L] + (size_t)j * m * k, k, h.y[L] + j * bx, nrhs,
                   y + (size_t)j * m * nrhs, nrhs, m, nrhs, k, false));
  P.launch(g);
  P.run(mem, s);
  HPS_HIP(hipStreamSynchronize(s));
}

}  // namespace hps
