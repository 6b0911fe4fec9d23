// FP64 MFMA GEMM tile shared by the dense solver (trailing updates, Schur
// products) and the solution passes (downward pass and interface residual
// for many right-hand sides).  Device code only; included by .hip files.
#pragma once

#include <hip/hip_runtime.h>

namespace hps {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Global-memory view of a pointer.  Loads through it are global loads (vector
// memory counter only); through a plain pointer from a descriptor they are
// flat loads, which also count against the LDS counter, so that every wait
// for an LDS read would also wait for the global loads in flight.
template <class T>
using gptr = const T __attribute__((address_space(1)))*;
template <class T>
__device__ inline gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}

// Row maps of the tile: row r of an operand lives at base + map(r) * ld.
struct RowsIdentity {
  __device__ int operator()(int r) const { return r; }
};
struct RowsIndexed {
  const int* idx;
  __device__ int operator()(int r) const { return as_global(idx)[r]; }
};

// C0 given element by element (active = true), replacing C0 and acc_c:
// value(row(r), col(c)) = operator()(r, c), the row and column parts looked
// up separately so that a tile can load them once per row and column.
struct NoC0Elem {
  static constexpr bool active = false;
  __device__ double operator()(int, int) const { return 0.0; }
  __device__ int row(int) const { return 0; }
  __device__ int col(int) const { return 0; }
  __device__ double value(int, int) const { return 0.0; }
};

// ---------------------------------------------------------------------------
// FP64 MFMA tiles.  A workgroup computes a BM x BN tile of C with WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) block made of 16 x 16
// v_mfma_f64_16x16x4f64 blocks.  A and B stream through LDS in BK-deep
// slabs.  Lane layout of the instruction: A operand lane l holds A[l%16][l/16],
// B operand B[l/16][l%16], result register r holds D[l/16 + 4r][l%16]
// (the f32 16x16x4 form instead holds D[4*(l/16) + r][l%16]).
// Variants of the grouped GEMM (index = tuning value): 0: 64x64x16 on 2x2
// waves with three k-slabs of loads in flight (the default), 1: 32x32x16 on
// one wave, 2: 128x128x16 on 4x2 waves, 3: 128x64x16 on 2x2, 4: 64x128x16 on
// 2x2, 5: 64x64x32 on 2x2, 6: 64x64x16 on 2x2 (1-6 with one slab in flight);
// 7 is gemm128_tile below.
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
  const gptr<double> gA = as_global(A);
  const gptr<double> gB = as_global(B);
  auto load = [&](int kt) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + T::NT * e;
      const int i = idx / BK, k = idx % BK;
      const int gr = row0 + i, gk = kt + k;
      ra[e] = (gr < M && gk < K) ? gA[(size_t)gr * lda + gk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + T::NT * e;
      const int k = idx / BN, j = idx % BN;
      const int gk = kt + k, gc = col0 + j;
      rb[e] = (gk < K && gc < N) ? gB[(size_t)brow(gk) * ldb + gc] : 0.0;
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
          pc[i][j][r] = (gr < M && gc < N) ? as_global(C)[(size_t)crow(gr) * ldc + gc] : 0.0;
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
        pa[e] = (gr < M && gk < K) ? gA[(size_t)gr * lda + gk] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int idx = tid + T::NT * e;
        const int k = idx / BN, j = idx % BN;
        const int gk = kt + k, gc = col0 + j;
        pb[e] = (gk < K && gc < N) ? gB[(size_t)brow(gk) * ldb + gc] : 0.0;
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
  // Every old or pass-through value of this lane's elements first (loads
  // only, so they are all in flight together), then the stores.
  double c0v[T::FM][T::FN][4];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * WBM + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wn * WBN + j * 16 + (lane & 15);
        double c0 = 0.0;
        if (gr < M && gc < N) {
          if constexpr (C0Elem::active) {
            c0 = c0elem(gr, gc);
          } else if (C0) {
            const int r0 = c0row(gr);
            if (r0 >= 0) c0 = as_global(C0)[(size_t)r0 * ldc0 + gc];
          } else if constexpr (PRE_C) {
            c0 = pc[i][j][r];
          } else if (acc_c) {
            c0 = as_global(C)[(size_t)crow(gr) * ldc + gc];
          }
        }
        c0v[i][j][r] = c0;
      }
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * WBM + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wn * WBN + j * 16 + (lane & 15);
        if (gr < M && gc < N) C[(size_t)crow(gr) * ldc + gc] = c0v[i][j][r] + alpha * acc[i][j][r];
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

// ---------------------------------------------------------------------------
// Large FP64 tile: 128 x 128 on 2 x 2 waves, each wave 64 x 64 (4 x 4 MFMA
// blocks, 64 products per 16-deep slab against 8 operand reads per 4-deep
// step).  Two LDS buffers: slab s is multiplied out of one while slab s + 1,
// loaded into registers during slab s - 1, is stored into the other, so a
// slab costs one barrier.  A stays row-major in LDS with a row stride of 18
// doubles and B with 144: the MFMA operand reads (16 rows x 4 k of A, 4 k x
// 16 columns of B, 32 lanes per LDS pass) then hit 32 distinct bank pairs.
// VEC = 2 loads and stores pairs of doubles: A and B 16-byte aligned, lda,
// ldb, K and N even (a pair is then either wholly inside or wholly outside);
// VEC = 1 single doubles.
// ---------------------------------------------------------------------------
struct Gemm128 {
  static constexpr int BM = 128, BN = 128, BK = 16, SA = 18, SB = 144;
  static constexpr int ABUF = BM * SA, BBUF = BK * SB, BUF = ABUF + BBUF;
  static constexpr int SMEM = 2 * BUF;  // doubles (73,728 bytes)
};

template <int VEC, class C0Elem>
__device__ inline void gemm128_tile(const double* __restrict__ A, int lda,
                                    const double* __restrict__ B, int ldb, double* C, int ldc,
                                    const double* C0, int ldc0, int M, int N, int K, double alpha,
                                    int row0, int col0, double* sm, bool acc_c, C0Elem c0elem) {
  using G = Gemm128;
  constexpr int BM = G::BM, BN = G::BN, BK = G::BK, SA = G::SA, SB = G::SB;
  constexpr int NA = BM * BK / (256 * VEC), NB = BK * BN / (256 * VEC);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[NA][VEC], rb[NB][VEC];
  unsigned oka = 0, okb = 0;  // in-range bits of the loaded elements
  const gptr<double> gA = as_global(A);
  const gptr<double> gB = as_global(B);
  // Element e of this thread: A row (e * 256 + tid) / (BK / VEC), k offset
  // VEC * ((e * 256 + tid) % (BK / VEC)); B row (e * 256 + tid) / (BN / VEC),
  // column VEC * (... % (BN / VEC)).  Out-of-range elements load from the
  // operand's origin (a valid address) and are zeroed when stored to LDS, so
  // the loads carry no branches and nothing waits for them before the store.
  auto load = [&](int kt) {
    oka = okb = 0;
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int p = e * 256 + tid;
      const int i = p / (BK / VEC), k = VEC * (p % (BK / VEC));
      const int gr = row0 + i, gk = kt + k;
      const bool ok = gr < M && gk < K;
      oka |= (unsigned)ok << e;
      const size_t off = ok ? (size_t)gr * lda + gk : 0;
      if constexpr (VEC == 2) {
        const d2 v = *(gptr<d2>)(gA + off);
        ra[e][0] = v.x;
        ra[e][1] = v.y;
      } else {
        ra[e][0] = gA[off];
      }
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * 256 + tid;
      const int k = p / (BN / VEC), j = VEC * (p % (BN / VEC));
      const int gk = kt + k, gc = col0 + j;
      const bool ok = gk < K && gc < N;
      okb |= (unsigned)ok << e;
      const size_t off = ok ? (size_t)gk * ldb + gc : 0;
      if constexpr (VEC == 2) {
        const d2 v = *(gptr<d2>)(gB + off);
        rb[e][0] = v.x;
        rb[e][1] = v.y;
      } else {
        rb[e][0] = gB[off];
      }
    }
  };
  auto store = [&](double* buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int p = e * 256 + tid;
      const int i = p / (BK / VEC), k = VEC * (p % (BK / VEC));
      const bool ok = (oka >> e) & 1u;
      if constexpr (VEC == 2)
        *reinterpret_cast<double2*>(buf + i * SA + k) =
            double2{ok ? ra[e][0] : 0.0, ok ? ra[e][1] : 0.0};
      else
        buf[i * SA + k] = ok ? ra[e][0] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * 256 + tid;
      const int k = p / (BN / VEC), j = VEC * (p % (BN / VEC));
      const bool ok = (okb >> e) & 1u;
      if constexpr (VEC == 2)
        *reinterpret_cast<double2*>(buf + G::ABUF + k * SB + j) =
            double2{ok ? rb[e][0] : 0.0, ok ? rb[e][1] : 0.0};
      else
        buf[G::ABUF + k * SB + j] = ok ? rb[e][0] : 0.0;
    }
  };
  const int nslab = (K + BK - 1) / BK;
  if (nslab > 0) {
    load(0);
    store(sm);
    if (nslab > 1) load(BK);
  }
  __syncthreads();
  const int arow = (wm * 64 + (lane & 15)) * SA + (lane >> 4);
  const int bcol = (lane >> 4) * SB + wn * 64 + (lane & 15);
  for (int s = 0; s < nslab; ++s) {
    const double* buf = sm + (s & 1) * G::BUF;
    // Slab s + 1 into the other buffer (its last readers passed the barrier
    // that ended slab s - 1), then the loads of slab s + 2.
    if (s + 1 < nslab) {
      store(sm + ((s + 1) & 1) * G::BUF);
      if (s + 2 < nslab) load((s + 2) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = buf[arow + i * 16 * SA + kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = buf[G::ABUF + bcol + kk * SB + j * 16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // A pass-through's row and column map entries of every element this lane
  // writes first (one round of loads); then per 16-row block the old or
  // pass-through values (loads only, all in flight together) and the stores.
  int kr[4][4], kc[4];
  if constexpr (C0Elem::active) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * 64 + i * 16 + (lane >> 4) + 4 * r;
        kr[i][r] = gr < M ? c0elem.row(gr) : 0;
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + wn * 64 + j * 16 + (lane & 15);
      kc[j] = gc < N ? c0elem.col(gc) : 0;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double c0v[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * 64 + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wn * 64 + j * 16 + (lane & 15);
        double c0 = 0.0;
        if (gr < M && gc < N) {
          if constexpr (C0Elem::active) {
            c0 = c0elem.value(kr[i][r], kc[j]);
          } else if (C0) {
            c0 = as_global(C0)[(size_t)gr * ldc0 + gc];
          } else if (acc_c) {
            c0 = as_global(C)[(size_t)gr * ldc + gc];
          }
        }
        c0v[j][r] = c0;
      }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * 64 + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wn * 64 + j * 16 + (lane & 15);
        if (gr < M && gc < N)
          *(double __attribute__((address_space(1)))*)(C + (size_t)gr * ldc + gc) =
              c0v[j][r] + alpha * acc[i][j][r];
      }
  }
}

// Tile order of a launch's (tiles_n x tiles_m) grid for the 128 x 128 tile:
// workgroups go to the 8 XCDs in turn, so the linear index is first regrouped
// into 8 contiguous runs (one per XCD), and each run walks groups of 8 tile
// rows column by column, so that the tiles an XCD holds at once share A row
// panels and B column panels in its L2.  Grids whose size is not a multiple
// of 8 keep the plain order.
__device__ inline void gemm128_tile_order(int nx, int ny, int bx, int by, int& tx, int& ty) {
  const int total = nx * ny, lin = bx + nx * by;
  if (total % 8 != 0) {
    tx = bx;
    ty = by;
    return;
  }
  const int v = (lin % 8) * (total / 8) + lin / 8;
  constexpr int GR = 8;
  const int gid = v / (GR * nx), first = gid * GR;
  const int gsz = min(ny - first, GR);
  const int w = v - gid * GR * nx;
  ty = first + w % gsz;
  tx = w / gsz;
}

}  // namespace hps
