// FP64 MFMA GEMM tile shared by the dense solver (trailing updates, Schur
// products) and the solution passes (downward pass and interface residual
// for many right-hand sides).  Device code only; included by .hip files.
#pragma once

#include <hip/hip_runtime.h>

namespace hps {

typedef double d4 __attribute__((ext_vector_type(4)));

// Row maps of the tile: row r of an operand lives at base + map(r) * ld.
struct RowsIdentity {
  __device__ int operator()(int r) const { return r; }
};
struct RowsIndexed {
  const int* idx;
  __device__ int operator()(int r) const { return idx[r]; }
};

// C0 given element by element (active = true), replacing C0 and acc_c.
struct NoC0Elem {
  static constexpr bool active = false;
  __device__ double operator()(int, int) const { return 0.0; }
};

// ---------------------------------------------------------------------------
// FP64 MFMA tiles.  A workgroup computes a BM x BN tile of C with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) block made of 16 x 16
// v_mfma_f64_16x16x4f64 blocks.  A and B stream through LDS in BK-deep
// slabs.  Lane layout of the instruction: A operand lane l holds A[l%16][l/16],
// B operand B[l/16][l%16], result register r holds D[l/16 + 4r][l%16]
// (the f32 16x16x4 form instead holds D[4*(l/16) + r][l%16]).
// Variants (index = tuning value): 0: 64x64x16 on 2x2 waves (the default),
// 1: 32x32x16 on one wave, 2: 128x128x16 on 4x2 waves, 3: 128x64x16 on 2x2,
// 4: 64x128x16 on 2x2, 5: 64x64x32 on 2x2.
// ---------------------------------------------------------------------------

template <int BM, int BN, int BK, int WM, int WN>
struct GemmTile {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
  static constexpr int SMEM = BK * (BM + 1) + BK * (BN + 1);  // doubles
  static_assert(FM >= 1 && FN >= 1 && BK % 4 == 0, "bad tile");
  static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "tile loads must divide evenly");
};

// Tile (row0.., col0..) of C = C0 (or C) + alpha * A (M x K) * B (K x N),
// row-major with the given leading dimensions, where B's row k lives at
// B + brow(k) * ldb, C's row r at C + crow(r) * ldc and C0's row r at
// C0 + c0row(r) * ldc0 (gathered operands, a scattered result; a negative
// c0row is a zero row; A rows are plain).  With C0 null the old C is added
// when acc_c is set and nothing otherwise (C is then not read).  An active
// c0elem gives C0 element by element instead.  PRE_C (with acc_c and no C0)
// loads the old C before the first product instead of after the last, one
// dependent round of global loads fewer; C must not overlap A or B.
template <int BM, int BN, int BK, int WM, int WN, class BRow, class CRow,
          class C0Row = RowsIdentity, class C0Elem = NoC0Elem, bool PRE_C = false, int DEPTH = 1>
__device__ inline void gemm_tile_map(const double* __restrict__ A, int lda,
                                     const double* B, int ldb, BRow brow, double* C, int ldc,
                                     CRow crow, const double* C0, int ldc0, int M, int N, int K,
                                     double alpha, int row0, int col0, double* sm, bool acc_c,
                                     C0Row c0row = C0Row{}, C0Elem c0elem = C0Elem{}) {
  using T = GemmTile<BM, BN, BK, WM, WN>;
  double(*As)[BM + 1] = reinterpret_cast<double(*)[BM + 1]>(sm);
  double(*Bs)[BN + 1] = reinterpret_cast<double(*)[BN + 1]>(sm + BK * (BM + 1));
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WN, wn = wid % WN;
  constexpr int WBM = BM / WM, WBN = BN / WN;
  d4 acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // The next slab's operands are loaded into registers while the current one
  // is multiplied out of LDS (one slab of global loads always in flight);
  // tiles whose accumulators leave no room for that load as they go.
  constexpr int EA = (BM * BK) / T::NT, EB = (BK * BN) / T::NT;
  constexpr bool PF = T::FM * T::FN <= 8;
  double ra[EA], rb[EB];
  auto load = [&](int kt) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + T::NT * e;
      const int i = idx / BK, k = idx % BK;
      const int gr = row0 + i, gk = kt + k;
      ra[e] = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + T::NT * e;
      const int k = idx / BN, j = idx % BN;
      const int gk = kt + k, gc = col0 + j;
      rb[e] = (gk < K && gc < N) ? B[(size_t)brow(gk) * ldb + gc] : 0.0;
    }
  };
  if (DEPTH == 1 && PF && K > 0) load(0);
  double pc[PRE_C ? T::FM : 1][PRE_C ? T::FN : 1][4];
  if constexpr (PRE_C) {
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gr = row0 + wm * WBM + i * 16 + (lane >> 4) + 4 * r;
          const int gc = col0 + wn * WBN + j * 16 + (lane & 15);
          pc[i][j][r] = (gr < M && gc < N) ? C[(size_t)crow(gr) * ldc + gc] : 0.0;
        }
  }
  if constexpr (DEPTH == 1) {
    for (int kt = 0; kt < K; kt += BK) {
      if (!PF) load(kt);
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int idx = tid + T::NT * e;
        As[idx % BK][idx / BK] = ra[e];
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int idx = tid + T::NT * e;
        Bs[idx / BN][idx % BN] = rb[e];
      }
      __syncthreads();
      if (PF && kt + BK < K) load(kt + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[T::FM], b[T::FN];
#pragma unroll
        for (int i = 0; i < T::FM; ++i) a[i] = As[kk + (lane >> 4)][wm * WBM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < T::FN; ++j) b[j] = Bs[kk + (lane >> 4)][wn * WBN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
          for (int j = 0; j < T::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  } else {
    // DEPTH slabs of global loads in flight: slab kt + DEPTH * BK is loaded
    // into the registers slab kt has just left (the slot index is a constant
    // of the unrolled inner loop).
    double qa[DEPTH][EA], qb[DEPTH][EB];
    auto load_slot = [&](int kt, double (&pa)[EA], double (&pb)[EB]) {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int idx = tid + T::NT * e;
        const int i = idx / BK, k = idx % BK;
        const int gr = row0 + i, gk = kt + k;
        pa[e] = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int idx = tid + T::NT * e;
        const int k = idx / BN, j = idx % BN;
        const int gk = kt + k, gc = col0 + j;
        pb[e] = (gk < K && gc < N) ? B[(size_t)brow(gk) * ldb + gc] : 0.0;
      }
    };
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
      if (d * BK < K) load_slot(d * BK, qa[d], qb[d]);
    for (int kt0 = 0; kt0 < K; kt0 += DEPTH * BK) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) {
        const int kt = kt0 + d * BK;
        if (kt < K) {
#pragma unroll
          for (int e = 0; e < EA; ++e) {
            const int idx = tid + T::NT * e;
            As[idx % BK][idx / BK] = qa[d][e];
          }
#pragma unroll
          for (int e = 0; e < EB; ++e) {
            const int idx = tid + T::NT * e;
            Bs[idx / BN][idx % BN] = qb[d][e];
          }
          __syncthreads();
          if (kt + DEPTH * BK < K) load_slot(kt + DEPTH * BK, qa[d], qb[d]);
#pragma unroll
          for (int kk = 0; kk < BK; kk += 4) {
            double a[T::FM], b[T::FN];
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
              a[i] = As[kk + (lane >> 4)][wm * WBM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < T::FN; ++j)
              b[j] = Bs[kk + (lane >> 4)][wn * WBN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
#pragma unroll
              for (int j = 0; j < T::FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
          }
          __syncthreads();
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * WBM + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wn * WBN + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double* cp = C + (size_t)crow(gr) * ldc + gc;
          double c0 = 0.0;
          if constexpr (C0Elem::active) {
            c0 = c0elem(gr, gc);
          } else if (C0) {
            const int r0 = c0row(gr);
            if (r0 >= 0) c0 = C0[(size_t)r0 * ldc0 + gc];
          } else if constexpr (PRE_C) {
            c0 = pc[i][j][r];
          } else if (acc_c) {
            c0 = *cp;
          }
          *cp = c0 + alpha * acc[i][j][r];
        }
      }
}

// gemm_tile_map with DEPTH k-slabs of global loads in flight and the row
// maps deduced from the arguments.
template <int BM, int BN, int BK, int WM, int WN, int DEPTH, class BRow, class CRow,
          class C0Row = RowsIdentity, class C0Elem = NoC0Elem>
__device__ inline void gemm_tile_map_d(const double* __restrict__ A, int lda, const double* B,
                                       int ldb, BRow brow, double* C, int ldc, CRow crow,
                                       const double* C0, int ldc0, int M, int N, int K,
                                       double alpha, int row0, int col0, double* sm, bool acc_c,
                                       C0Row c0row = C0Row{}, C0Elem c0elem = C0Elem{}) {
  gemm_tile_map<BM, BN, BK, WM, WN, BRow, CRow, C0Row, C0Elem, false, DEPTH>(
      A, lda, B, ldb, brow, C, ldc, crow, C0, ldc0, M, N, K, alpha, row0, col0, sm, acc_c, c0row,
      c0elem);
}

// C[row0.., col0..] (M x N valid) = C0 (or C) + alpha * A (M x K) * B (K x N);
// A, B, C, C0 point at the matrices' origins (row-major, given leading dims).
template <int BM, int BN, int BK, int WM, int WN>
__device__ inline void gemm_tile(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                 int ldb, double* C, int ldc, const double* C0, int ldc0, int M,
                                 int N, int K, double alpha, int row0, int col0, double* sm) {
  gemm_tile_map<BM, BN, BK, WM, WN>(A, lda, B, ldb, RowsIdentity{}, C, ldc, RowsIdentity{}, C0,
                                    ldc0, M, N, K, alpha, row0, col0, sm, true);
}

}  // namespace hps
