// Batched dense FP64 kernels for gfx950: LU with partial pivoting of the
// augmented systems [M | B], the block-row triangular solve, the FP64 MFMA
// GEMM used for trailing updates and Schur products, the split-FP32 MFMA
// variant of the Schur product, and the blocked back substitution.
//
// These carry eq:leaf_solve (section 3.1: Z = A_ii^-1 R) and eq:U_parent
// (section 4: S = (T33a - T33b)^-1 [-T31a | T32b]); the Schur products carry
// eq:merge and the leaf's T = P0 - P1 Z.
#include "dense.h"

#include <algorithm>
#include <vector>

namespace hps {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Block-wide argmax of |v| (ties -> smallest index), 256 threads.
// ---------------------------------------------------------------------------
__device__ inline bool argmax_better(double v1, int i1, double v2, int i2) {
  // True when (v2, i2) should replace (v1, i1): valid beats invalid, larger
  // value wins, equal values go to the smaller row index.
  if (i2 < 0) return false;
  if (i1 < 0) return true;
  return v2 > v1 || (v2 == v1 && i2 < i1);
}

__device__ inline void block_argmax(double v, int idx, double* sv, int* si, double& bv, int& bi) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (argmax_better(v, idx, ov, oi)) { v = ov; idx = oi; }
  }
  if (lane == 0) { sv[wid] = v; si[wid] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sv[0];
    int i = si[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (argmax_better(b, i, sv[w], si[w])) { b = sv[w]; i = si[w]; }
    sv[0] = b;
    si[0] = i;
  }
  __syncthreads();
  bv = sv[0];
  bi = si[0];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Panel factorization: columns [k0, k0+kb) of rows [k0, n), partial pivoting.
// One workgroup per problem.  The panel is staged in LDS when it fits.
// Only panel columns are swapped here; ipiv records the pivot row per column.
// ---------------------------------------------------------------------------
constexpr int PANEL_LDS = 8192;  // doubles (64 KB)

__device__ void panel_factor(double* P, int st, int rows, int kb, int* ipiv_out, int k0,
                             int tag, int* status) {
  __shared__ double sv[16];
  __shared__ int si[16];
  for (int j = 0; j < kb; ++j) {
    double best = -1.0;
    int bidx = -1;
    for (int r = j + (int)threadIdx.x; r < rows; r += blockDim.x) {
      double v = fabs(P[(size_t)r * st + j]);
      if (v > best || (v != v)) { best = (v != v) ? INFINITY : v; bidx = r; }
    }
    double bv;
    int pr;
    block_argmax(best, bidx, sv, si, bv, pr);
    if (pr < 0) pr = j;
    if (pr != j) {
      for (int c = threadIdx.x; c < kb; c += blockDim.x) {
        double a = P[(size_t)j * st + c];
        P[(size_t)j * st + c] = P[(size_t)pr * st + c];
        P[(size_t)pr * st + c] = a;
      }
    }
    __syncthreads();
    const double piv = P[(size_t)j * st + j];
    if (threadIdx.x == 0) {
      ipiv_out[j] = k0 + pr;
      if (!(piv != 0.0) || piv != piv) {
        if (atomicCAS(status, 0, 1) == 0) status[1] = tag;
      }
    }
    const double inv = (piv != 0.0) ? 1.0 / piv : 0.0;
    for (int r = j + 1 + (int)threadIdx.x; r < rows; r += blockDim.x) {
      double l = P[(size_t)r * st + j] * inv;
      P[(size_t)r * st + j] = l;
      for (int c = j + 1; c < kb; ++c) P[(size_t)r * st + c] -= l * P[(size_t)j * st + c];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_lu_panel(const SolveDesc* __restrict__ descs, int k0,
                                                  int nb, int* status) {
  __shared__ double sp[PANEL_LDS];
  const SolveDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int kb = min(nb, d.n - k0);
  const int rows = d.n - k0;
  double* G = d.W + (size_t)k0 * d.ld + k0;
  if (rows * kb <= PANEL_LDS) {
    for (int e = threadIdx.x; e < rows * kb; e += blockDim.x) {
      int r = e / kb, c = e % kb;
      sp[e] = G[(size_t)r * d.ld + c];
    }
    __syncthreads();
    panel_factor(sp, kb, rows, kb, d.piv + k0, k0, d.tag, status);
    for (int e = threadIdx.x; e < rows * kb; e += blockDim.x) {
      int r = e / kb, c = e % kb;
      G[(size_t)r * d.ld + c] = sp[e];
    }
  } else {
    panel_factor(G, d.ld, rows, kb, d.piv + k0, k0, d.tag, status);
  }
}

// ---------------------------------------------------------------------------
// Apply the panel's row interchanges to columns [k0+kb, n+m) and solve
// L11 X = W[k0:k0+kb, cols] (unit lower) in place.  One thread per column.
// ---------------------------------------------------------------------------
constexpr int MAXNB = 32;

__global__ void __launch_bounds__(256) k_swap_trsm(const SolveDesc* __restrict__ descs, int k0,
                                                   int nb) {
  __shared__ double L[MAXNB * MAXNB];
  __shared__ int pv[MAXNB];
  const SolveDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int kb = min(nb, d.n - k0);
  const int c0 = k0 + kb;
  const int ncol = d.n + d.m - c0;
  if ((int)(blockIdx.x * blockDim.x) >= ncol) return;
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    int r = e / kb, c = e % kb;
    L[e] = d.W[(size_t)(k0 + r) * d.ld + k0 + c];
  }
  for (int e = threadIdx.x; e < kb; e += blockDim.x) pv[e] = d.piv[k0 + e];
  __syncthreads();
  const int col = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= d.n + d.m) return;
  double* W = d.W;
  const size_t ld = d.ld;
  for (int j = 0; j < kb; ++j) {
    int r2 = pv[j];
    if (r2 != k0 + j) {
      double a = W[(size_t)(k0 + j) * ld + col];
      W[(size_t)(k0 + j) * ld + col] = W[(size_t)r2 * ld + col];
      W[(size_t)r2 * ld + col] = a;
    }
  }
  double x[MAXNB];
#pragma unroll
  for (int j = 0; j < MAXNB; ++j)
    if (j < kb) x[j] = W[(size_t)(k0 + j) * ld + col];
#pragma unroll
  for (int j = 0; j < MAXNB; ++j) {
    if (j < kb) {
      double s = x[j];
#pragma unroll
      for (int i = 0; i < MAXNB; ++i)
        if (i < j) s -= L[j * kb + i] * x[i];
      x[j] = s;
      W[(size_t)(k0 + j) * ld + col] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 MFMA tile: 64x64 output tile per 256-thread workgroup, 4 waves in a
// 2x2 arrangement, each wave a 32x32 block = 2x2 MFMA 16x16x4 f64 blocks.
// Lane layout of v_mfma_f64_16x16x4f64: A operand lane l holds A[l%16][l/16],
// B operand B[l/16][l%16], result register r holds D[l/16 + 4r][l%16]
// (the f32 16x16x4 form instead holds D[4*(l/16) + r][l%16]).
// ---------------------------------------------------------------------------
constexpr int TBM = 64, TBN = 64, TBK = 16;

__device__ inline void gemm_tile_f64(const double* __restrict__ A, int lda,
                                     const double* __restrict__ B, int ldb, double* C, int ldc,
                                     const double* C0, int ldc0, int M, int N, int K, double alpha,
                                     int tm, int tn, double (*As)[TBM + 1],
                                     double (*Bs)[TBN + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int row0 = tm * TBM, col0 = tn * TBN;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kt = 0; kt < K; kt += TBK) {
#pragma unroll
    for (int e = 0; e < (TBM * TBK) / 256; ++e) {
      int idx = tid + 256 * e;
      int i = idx / TBK, k = idx % TBK;
      int gr = row0 + i, gk = kt + k;
      As[k][i] = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < (TBK * TBN) / 256; ++e) {
      int idx = tid + 256 * e;
      int k = idx / TBN, j = idx % TBN;
      int gk = kt + k, gc = col0 + j;
      Bs[k][j] = (gk < K && gc < N) ? B[(size_t)gk * ldb + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TBK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = row0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        int gc = col0 + wn * 32 + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double c0 = C0 ? C0[(size_t)gr * ldc0 + gc] : C[(size_t)gr * ldc + gc];
          C[(size_t)gr * ldc + gc] = c0 + alpha * acc[i][j][r];
        }
      }
}

// Trailing update of the blocked LU: W[k0+kb:n, k0+kb:n+m] -= L21 * U12.
__global__ void __launch_bounds__(256) k_lu_update(const SolveDesc* __restrict__ descs, int k0,
                                                   int nb) {
  __shared__ double As[TBK][TBM + 1];
  __shared__ double Bs[TBK][TBN + 1];
  const SolveDesc d = descs[blockIdx.z];
  if (k0 >= d.n) return;
  const int kb = min(nb, d.n - k0);
  const int r0 = k0 + kb;
  const int M = d.n - r0, N = d.n + d.m - r0;
  if ((int)blockIdx.y * TBM >= M || (int)blockIdx.x * TBN >= N) return;
  const size_t ld = d.ld;
  gemm_tile_f64(d.W + (size_t)r0 * ld + k0, d.ld, d.W + (size_t)k0 * ld + r0, d.ld,
                d.W + (size_t)r0 * ld + r0, d.ld, nullptr, 0, M, N, kb, -1.0, blockIdx.y,
                blockIdx.x, As, Bs);
}

// Grouped GEMM: one launch over problems, grid (tiles_n, tiles_m, nprob).
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc* __restrict__ descs) {
  __shared__ double As[TBK][TBM + 1];
  __shared__ double Bs[TBK][TBN + 1];
  const GemmDesc g = descs[blockIdx.z];
  if ((int)blockIdx.y * TBM >= g.M || (int)blockIdx.x * TBN >= g.N) return;
  gemm_tile_f64(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.C0, g.ldc0, g.M, g.N, g.K, g.alpha,
                blockIdx.y, blockIdx.x, As, Bs);
}

// ---------------------------------------------------------------------------
// Split-FP32 Schur product: A = Ah + Al, B = Bh + Bl with Ah = fl32(A),
// Al = fl32(A - Ah); C += alpha (Ah Bh + Ah Bl + Al Bh), the three products
// on FP32 MFMA 16x16x4 (same lane layout as the f64 form), each 16-deep
// k-slab accumulated in FP32 and then added into FP64 registers.  Result
// register r of lane l holds D[4*(l/16) + r][l%16] for this f32 form.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gemm_split32(const GemmDesc* __restrict__ descs) {
  __shared__ float Ah[TBK][TBM + 1], Al[TBK][TBM + 1];
  __shared__ float Bh[TBK][TBN + 1], Bl[TBK][TBN + 1];
  const GemmDesc g = descs[blockIdx.z];
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (tm * TBM >= g.M || tn * TBN >= g.N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int row0 = tm * TBM, col0 = tn * TBN;
  double acc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  for (int kt = 0; kt < g.K; kt += TBK) {
#pragma unroll
    for (int e = 0; e < (TBM * TBK) / 256; ++e) {
      int idx = tid + 256 * e;
      int i = idx / TBK, k = idx % TBK;
      int gr = row0 + i, gk = kt + k;
      double v = (gr < g.M && gk < g.K) ? g.A[(size_t)gr * g.lda + gk] : 0.0;
      float h = (float)v;
      Ah[k][i] = h;
      Al[k][i] = (float)(v - (double)h);
    }
#pragma unroll
    for (int e = 0; e < (TBK * TBN) / 256; ++e) {
      int idx = tid + 256 * e;
      int k = idx / TBN, j = idx % TBN;
      int gk = kt + k, gc = col0 + j;
      double v = (gk < g.K && gc < g.N) ? g.B[(size_t)gk * g.ldb + gc] : 0.0;
      float h = (float)v;
      Bh[k][j] = h;
      Bl[k][j] = (float)(v - (double)h);
    }
    __syncthreads();
    f4 hh[2][2], cr[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        hh[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        cr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
    for (int kk = 0; kk < TBK; kk += 4) {
      float ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int c = wm * 32 + i * 16 + (lane & 15);
        ah[i] = Ah[kk + (lane >> 4)][c];
        al[i] = Al[kk + (lane >> 4)][c];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int c = wn * 32 + j * 16 + (lane & 15);
        bh[j] = Bh[kk + (lane >> 4)][c];
        bl[j] = Bl[kk + (lane >> 4)][c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[i], bh[j], hh[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[i], bl[j], cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[i], bh[j], cr[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)hh[i][j][r] + (double)cr[i][j][r];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gr = row0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        int gc = col0 + wn * 32 + j * 16 + (lane & 15);
        if (gr < g.M && gc < g.N) {
          double c0 = g.C0 ? g.C0[(size_t)gr * g.ldc0 + gc] : g.C[(size_t)gr * g.ldc + gc];
          g.C[(size_t)gr * g.ldc + gc] = c0 + g.alpha * acc[i][j][r];
        }
      }
}

// ---------------------------------------------------------------------------
// Back substitution X = U^-1 Y on a column block of the right-hand sides,
// blocked by BS rows from the bottom; the Y block lives in LDS.
// ---------------------------------------------------------------------------
constexpr int BS = 32;
constexpr int BSUB_LDS = 16384;  // doubles (128 KB)

__global__ void __launch_bounds__(256) k_back_subst(const SolveDesc* __restrict__ descs, int cw) {
  extern __shared__ double smem[];
  const SolveDesc d = descs[blockIdx.y];
  const int c0 = blockIdx.x * cw;
  if (c0 >= d.m) return;
  const int w = min(cw, d.m - c0);
  const int n = d.n, ldy = cw + 1;
  double* Y = smem;                      // n x ldy
  double* Ud = smem + (size_t)n * ldy;   // BS x (BS+1)
  const size_t ld = d.ld;
  for (int e = threadIdx.x; e < n * w; e += blockDim.x) {
    int r = e / w, c = e % w;
    Y[r * ldy + c] = d.W[(size_t)r * ld + n + c0 + c];
  }
  __syncthreads();
  const int nblk = (n + BS - 1) / BS;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k = b * BS, kend = min(n, k + BS), kw = kend - k;
    for (int e = threadIdx.x; e < kw * kw; e += blockDim.x) {
      int r = e / kw, c = e % kw;
      Ud[r * (BS + 1) + c] = d.W[(size_t)(k + r) * ld + k + c];
    }
    __syncthreads();
    if ((int)threadIdx.x < w) {
      const int c = threadIdx.x;
      for (int r = kw - 1; r >= 0; --r) {
        double s = Y[(k + r) * ldy + c];
        for (int cc = r + 1; cc < kw; ++cc) s -= Ud[r * (BS + 1) + cc] * Y[(k + cc) * ldy + c];
        Y[(k + r) * ldy + c] = s / Ud[r * (BS + 1) + r];
      }
    }
    __syncthreads();
    // Rows above the block: Y[r] -= U[r, k:kend] X[k:kend].
    for (int r = threadIdx.x; r < k; r += blockDim.x) {
      double u[BS];
#pragma unroll
      for (int i = 0; i < BS; ++i) u[i] = (i < kw) ? d.W[(size_t)r * ld + k + i] : 0.0;
      for (int c = 0; c < w; ++c) {
        double s = Y[r * ldy + c];
#pragma unroll
        for (int i = 0; i < BS; ++i)
          if (i < kw) s -= u[i] * Y[(k + i) * ldy + c];
        Y[r * ldy + c] = s;
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * w; e += blockDim.x) {
    int r = e / w, c = e % w;
    d.X[(size_t)r * d.ldx + c0 + c] = Y[r * ldy + c];
  }
}

// ---------------------------------------------------------------------------
// Host drivers.
// ---------------------------------------------------------------------------

int back_subst_width(int n, int m) {
  // Largest column block whose Y tile plus the diagonal block fits in LDS.
  int cw = 64;
  while (cw > 1 && (size_t)n * (cw + 1) + BS * (BS + 1) > (size_t)BSUB_LDS) cw >>= 1;
  return std::max(1, std::min(cw, m));
}

void batched_solve(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                   hipStream_t stream, int nb) {
  if (h_desc.empty()) return;
  nb = std::min(nb, MAXNB);
  int nmax = 0, wmax = 0, mmax = 0, nfor_cw = 0;
  for (auto& d : h_desc) {
    nmax = std::max(nmax, d.n);
    wmax = std::max(wmax, d.n + d.m);
    mmax = std::max(mmax, d.m);
    nfor_cw = std::max(nfor_cw, d.n);
  }
  const int np = (int)h_desc.size();
  for (int k0 = 0; k0 < nmax; k0 += nb) {
    hipLaunchKernelGGL(k_lu_panel, dim3(np), dim3(256), 0, stream, d_desc, k0, nb, d_status);
    int rest = wmax - k0;
    if (rest > 0) {
      hipLaunchKernelGGL(k_swap_trsm, dim3((rest + 255) / 256, np), dim3(256), 0, stream, d_desc,
                         k0, nb);
      int mt = (nmax - k0 + TBM - 1) / TBM, nt = (rest + TBN - 1) / TBN;
      hipLaunchKernelGGL(k_lu_update, dim3(nt, mt, np), dim3(256), 0, stream, d_desc, k0, nb);
    }
  }
  const int cw = back_subst_width(nfor_cw, mmax);
  size_t shm = ((size_t)nfor_cw * (cw + 1) + BS * (BS + 1)) * sizeof(double);
  hipLaunchKernelGGL(k_back_subst, dim3((mmax + cw - 1) / cw, np), dim3(256), shm, stream, d_desc,
                     cw);
}

void grouped_gemm(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                  bool split32) {
  if (h_desc.empty()) return;
  int mmax = 0, nmax = 0;
  for (auto& g : h_desc) {
    mmax = std::max(mmax, g.M);
    nmax = std::max(nmax, g.N);
  }
  dim3 grid((nmax + TBN - 1) / TBN, (mmax + TBM - 1) / TBM, (unsigned)h_desc.size());
  if (split32)
    hipLaunchKernelGGL(k_gemm_split32, grid, dim3(256), 0, stream, d_desc);
  else
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, stream, d_desc);
}

void dense_init() {
  static bool done = false;
  if (done) return;
  HPS_HIP(hipFuncSetAttribute((const void*)k_back_subst,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(BSUB_LDS + BS * (BS + 1)) * (int)sizeof(double)));
  done = true;
}

}  // namespace hps
