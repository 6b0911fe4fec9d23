// Batched dense FP64 kernels for gfx950: LU with partial pivoting of the
// augmented systems [M | B], the block-row triangular solve, the FP64 MFMA
// GEMM used for trailing updates and Schur products, the split-FP32 MFMA
// variant of the Schur product, and the blocked back substitution.
//
// These carry eq:leaf_solve (section 3.1: Z = A_ii^-1 R) and eq:U_parent
// (section 4: S = (T33a - T33b)^-1 [-T31a | T32b]); the Schur products carry
// eq:merge and the leaf's T = P0 - P1 Z.
#include "dense.h"
#include "mfma_tile.h"
#include "wave_ops.h"
#include "prof.h"
#include "tune.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

namespace hps {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Block Gauss-Jordan elimination of the augmented systems W = [M | B].
//
// For each panel of kb columns starting at k0:
//   1. k_gj_panel: LU with partial pivoting of W[k0:n, k0:k0+kb] in
//      registers (one workgroup per system, rows spread over the lanes, one
//      barrier per column).  piv[k0 + j] = row that moves to position k0 + j.
//      It writes L11\U11 into the pivot block rows and, for the positions
//      vacated below, the original panel values of the rows that move there.
//   2. k_gj_swap_trsm: applies the same row moves to every later column and
//      turns the pivot block rows into R = U11^-1 L11^-1 A12 (one thread per
//      column).
//   3. k_gj_update: every row outside the pivot block gets
//      A[i, k0+kb:] -= A[i, k0:k0+kb] R (FP64 MFMA tiles), which eliminates
//      the panel columns from the rows above and below alike.
// After the last panel the right-hand-side columns hold X = M^-1 B in natural
// row order, so no back substitution is needed; the extra cost over LU is
// n^3/3 flops, small next to the n^2 m of the right-hand sides.
//
// Row moves of a step: row pi[j] goes to position k0 + j; the rows at
// positions k0..k0+kb-1 that were not chosen (D, ascending) go to the
// positions of the chosen rows lying below the block (V, in pivot order).
// ---------------------------------------------------------------------------

// Row moves of a step from the chosen rows pi[0..kb) (run by one wave).  The
// block positions taken by a chosen row are marked in flag[0..kb) (LDS), so
// each lane learns whether its position was chosen in two LDS round trips.
__device__ inline void perm_lists(const int* pi, int kb, int k0, int* flag, int* sD, int* sV,
                                  int* nd) {
  const int lane = threadIdx.x & 63;
  const int myp = lane < kb ? pi[lane] : -1;
  if (lane < kb) flag[lane] = 0;
  wave_lds_sync();
  if (myp >= k0 && myp < k0 + kb) flag[myp - k0] = 1;
  wave_lds_sync();
  const bool chosen = lane < kb && flag[lane] != 0;
  const bool isd = lane < kb && !chosen, isv = lane < kb && myp >= k0 + kb;
  const unsigned long long md = __ballot(isd), mv = __ballot(isv);
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (isd) sD[__popcll(md & below)] = k0 + lane;
  if (isv) sV[__popcll(mv & below)] = myp;
  if (lane == 0) *nd = __popcll(md);
}

// End of a panel step, after the pivot rows' L \ U sits in sLU and the
// chosen rows in sPi[0..ns) (the caller has synchronised the workgroup):
// records the pivots and the status, then moves the panel rows.
template <int KB>
__device__ inline void panel_tail(const SolveDesc& d, int k0, int kb, int ns, bool bad,
                                  int* status, double (*sLU)[KB + 1], double (*sKeep)[KB + 1],
                                  int* sPi, int* sD, int* sV, int* sFlag, int* sNd) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const size_t ld = d.ld;
  double* P = d.W + (size_t)k0 * ld + k0;
  if (wid == 0) {
    // Fewer than kb pivots cannot happen (every live row has a nonzero key);
    // should it, the identity keeps every later access in bounds and the
    // status reports the system as singular.
    const bool short_ = ns < kb;
    if (short_ && lane < kb) sPi[lane] = k0 + lane;
    wave_lds_sync();
    perm_lists(sPi, kb, k0, sFlag, sD, sV, sNd);
    if (lane < kb) d.piv[k0 + lane] = sPi[lane];
    if (lane == 0 && (bad || short_))
      if (atomicCAS(status, 0, 1) == 0) status[1] = d.tag;
  }
  __syncthreads();
  // Original panel values of the displaced rows (they sit in the pivot block,
  // which is overwritten next), then the block's new rows.
  // The loops have a constant trip count (the workgroup has at least one
  // wave), so every thread issues all its loads before the first wait.
  constexpr int IT = KB * KB / 64;
  const int nd = *sNd, nkeep = nd * kb, bd = blockDim.x;
  double kv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * bd;
    kv[it] = e < nkeep ? P[(size_t)(sD[e / kb] - k0) * ld + e % kb] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * bd;
    if (e < nkeep) sKeep[e / kb][e % kb] = kv[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * bd;
    if (e < kb * kb) P[(size_t)(e / kb) * ld + e % kb] = sLU[e / kb][e % kb];
    if (e < nkeep) P[(size_t)(sV[e / kb] - k0) * ld + e % kb] = sKeep[e / kb][e % kb];
  }
}

constexpr int TP_MAXW = 8;  // waves of the panel workgroup (two per SIMD: 256 VGPRs each)

// Panel LU with partial pivoting, one workgroup barrier per column.  Local
// row i (absolute k0 + i) lives in wave i / (64 R), slot (i / 64) % R, lane
// i % 64; x holds its panel values.  For each column every wave finds its
// best candidate with DPP and its owner lane publishes that row before the
// barrier; after it every thread picks the workgroup's winner from the
// published keys and eliminates with the winner's row.  Buffers alternate
// between columns, so a single barrier per column suffices.  The column loop
// is unrolled in full, so that every row update covers only the columns
// still to the right (a compact loop over groups of columns, with the
// register file rotated between groups, measured slower: it must run every
// update over the whole panel width).
template <int R, int KB>
__global__ void __launch_bounds__(64 * TP_MAXW) k_gj_panel(const SolveDesc* __restrict__ descs,
                                                          int k0, int* status) {
  __shared__ unsigned sKey[2][TP_MAXW];
  __shared__ double sInvP[2][TP_MAXW];  // 1 / each wave's candidate pivot
  __shared__ double sRow[2][TP_MAXW][KB];
  __shared__ double sLU[KB][KB + 1];
  __shared__ double sKeep[KB][KB + 1];
  __shared__ int sPi[KB], sD[KB], sV[KB], sFlag[KB], sNd, sBad, sNs;
  const SolveDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int kb = min(KB, d.n - k0), rows = d.n - k0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const size_t ld = d.ld;
  double* P = d.W + (size_t)k0 * ld + k0;
  double x[R][KB];
  bool live[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = wid * 64 * R + r * 64 + lane;
    live[r] = lr < rows;
#pragma unroll
    for (int c = 0; c < KB; ++c) x[r][c] = (live[r] && c < kb) ? P[(size_t)lr * ld + c] : 0.0;
  }
  if (threadIdx.x == 0) {
    sBad = 0;
    sNs = 0;
  }
  // Keys of absent waves read as 0 (no candidate), so that every thread can
  // read all TP_MAXW keys at once.
  if (threadIdx.x < 2 * TP_MAXW) sKey[threadIdx.x / TP_MAXW][threadIdx.x % TP_MAXW] = 0;
  __syncthreads();
  int ns = 0;
  bool stop = false;
  double minp = INFINITY;  // smallest |pivot| of the panel (pivot statistics)
  // Step at which each of this lane's rows became a pivot row (-1: not yet).
  // A pivot row is no longer updated, so at the end its registers hold its
  // row of L \ U, which is then written out in one go.
  int sel[R];
#pragma unroll
  for (int r = 0; r < R; ++r) sel[r] = -1;
  // Constant trip count (columns past kb, or past the last candidate, are
  // skipped uniformly) so the loop unrolls and x stays in registers.
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (c >= kb || stop) continue;
    const int buf = c & 1;
    unsigned key = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (live[r]) key = max(key, pivot_key(x[r][c], wid * 64 * R + r * 64 + lane));
    const unsigned wkey = wave_max_u32(key);
    if (wkey != 0) {
      const int slot = 4095 - (int)(wkey & 4095u);
      const int wl = slot & 63, wr = (slot >> 6) % R;
      double cand = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (wr == r) {
          if (lane == wl) {
#pragma unroll
            for (int c2 = 0; c2 < KB; ++c2)
              if (c2 >= c) sRow[buf][wid][c2] = x[r][c2];
          }
          cand = __shfl(x[r][c], wl);
        }
      // The candidate's reciprocal is formed before the barrier, off the
      // critical path of the elimination that follows it.
      if (lane == 0) sInvP[buf][wid] = recip(cand);
    }
    if (lane == 0) sKey[buf][wid] = wkey;
    __syncthreads();
    unsigned g = 0;
#pragma unroll
    for (int w = 0; w < TP_MAXW; ++w) g = max(g, sKey[buf][w]);
    g = (unsigned)__builtin_amdgcn_readfirstlane((int)g);
    if (g == 0) {
      stop = true;
      continue;
    }
    const int gslot = 4095 - (int)(g & 4095u);
    const int gw = gslot / (64 * R), gr = (gslot >> 6) % R, gl = gslot & 63;
    const double* prow = sRow[buf][gw];
    if (wid == gw) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (gr == r && lane == gl) {
          live[r] = false;
          sel[r] = ns;
        }
    }
    if (threadIdx.x == 0) sPi[ns] = k0 + gslot;
    ++ns;
    const double piv = prow[c], invp = sInvP[buf][gw];
    const bool ok = (piv != 0.0) && (piv == piv) && fabs(piv) != INFINITY;
    if (!ok && threadIdx.x == 0) sBad = 1;
    minp = fmin(minp, fabs(piv));
    const double inv = ok ? invp : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (live[r]) {
        const double l = x[r][c] * inv;
        x[r][c] = l;
        // Runs over all KB columns (the test folds away once the column loop
        // is unrolled), so it unrolls and x stays in registers.
#pragma unroll
        for (int c2 = 0; c2 < KB; ++c2)
          if (c2 > c) x[r][c2] = fma(-l, prow[c2], x[r][c2]);
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (sel[r] >= 0) {
#pragma unroll
      for (int c2 = 0; c2 < KB; ++c2) sLU[sel[r]][c2] = x[r][c2];
    }
  if (threadIdx.x == 0) {
    sNs = ns;
    if (d.pstat && ns > 0) atomicMin(d.pstat + 1, abs_bits(minp));
  }
  __syncthreads();
  panel_tail<KB>(d, k0, kb, sNs, sBad != 0, status, sLU, sKeep, sPi, sD, sV, sFlag, &sNd);
}

// One-wave variant of k_gj_panel<2, KB> for panels of at most 128 rows:
// the same pivot keys, choices and arithmetic, but with no workgroup to
// synchronise the pivot row is read straight out of the winning lane's
// registers (readlane) instead of through LDS, so a column step holds no LDS
// round trip and no barrier.
template <int KB>
__global__ void __launch_bounds__(64) k_gj_panel_w1(const SolveDesc* __restrict__ descs, int k0,
                                                    int* status) {
  constexpr int R = 2;
  __shared__ double sLU[KB][KB + 1];
  __shared__ double sKeep[KB][KB + 1];
  __shared__ int sPi[KB], sD[KB], sV[KB], sFlag[KB], sNd;
  const SolveDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int kb = min(KB, d.n - k0), rows = d.n - k0;
  const int lane = threadIdx.x;
  const size_t ld = d.ld;
  const double* P = d.W + (size_t)k0 * ld + k0;
  double x[R][KB];
  bool live[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = r * 64 + lane;
    live[r] = lr < rows;
#pragma unroll
    for (int c = 0; c < KB; ++c) x[r][c] = (live[r] && c < kb) ? P[(size_t)lr * ld + c] : 0.0;
  }
  int ns = 0;
  bool stop = false, bad = false;
  double minp = INFINITY;  // smallest |pivot| of the panel (pivot statistics)
  int sel[R];
#pragma unroll
  for (int r = 0; r < R; ++r) sel[r] = -1;
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (c >= kb || stop) continue;
    unsigned key = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (live[r]) key = max(key, pivot_key(x[r][c], r * 64 + lane));
    const unsigned g = wave_max_u32(key);
    if (g == 0) {
      stop = true;
      continue;
    }
    const int gslot = 4095 - (int)(g & 4095u);
    const int gr = gslot >> 6, gl = gslot & 63;
    double prow[KB];
    if (gr == 0) {
#pragma unroll
      for (int c2 = 0; c2 < KB; ++c2)
        if (c2 >= c) prow[c2] = bcast_lane(x[0][c2], gl);
    } else {
#pragma unroll
      for (int c2 = 0; c2 < KB; ++c2)
        if (c2 >= c) prow[c2] = bcast_lane(x[1][c2], gl);
    }
    if (lane == gl) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (gr == r) {
          live[r] = false;
          sel[r] = ns;
        }
    }
    if (lane == 0) sPi[ns] = k0 + gslot;
    ++ns;
    const double piv = prow[c];
    const bool ok = (piv != 0.0) && (piv == piv) && fabs(piv) != INFINITY;
    bad |= !ok;
    minp = fmin(minp, fabs(piv));
    const double inv = ok ? recip(piv) : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (live[r]) {
        const double l = x[r][c] * inv;
        x[r][c] = l;
#pragma unroll
        for (int c2 = 0; c2 < KB; ++c2)
          if (c2 > c) x[r][c2] = fma(-l, prow[c2], x[r][c2]);
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (sel[r] >= 0) {
#pragma unroll
      for (int c2 = 0; c2 < KB; ++c2) sLU[sel[r]][c2] = x[r][c2];
    }
  if (lane == 0 && d.pstat && ns > 0) atomicMin(d.pstat + 1, abs_bits(minp));
  __syncthreads();
  panel_tail<KB>(d, k0, kb, ns, bad, status, sLU, sKeep, sPi, sD, sV, sFlag, &sNd);
}

// One thread per column to the right of the pivot block: apply the step's
// row moves to the column, then x <- U11^-1 L11^-1 x on the pivot block rows
// with L11 \ U11 (and the reciprocals of U11's diagonal) staged in LDS.
// Each row's dot product runs on four accumulators to shorten the dependent
// chain.  (Reading the factors from global memory instead measured 2.5x
// slower: every lane issues the same vector load.)
template <int KB>
__global__ void __launch_bounds__(256) k_gj_swap_trsm(const SolveDesc* __restrict__ descs, int k0) {
  __shared__ double LU[KB][KB + 1];
  __shared__ double rdiag[KB];
  __shared__ int pv[KB], sD[KB], sV[KB], sFlag[KB], sNd;
  const SolveDesc d = descs[blockIdx.y];
  if (k0 >= d.n) return;
  const int kb = min(KB, d.n - k0);
  const int c0 = k0 + kb;
  const int ncol = d.n + d.m - c0;
  if ((int)(blockIdx.x * blockDim.x) >= ncol) return;
  const size_t ld = d.ld;
  // Entries past kb are zero, so that the full-width loops below add exact
  // zeros for them.  Constant trip counts (the workgroup has at least one
  // wave): every thread issues all its loads before the first wait.
  constexpr int IT = KB * KB / 64;
  const int bd = blockDim.x, t = threadIdx.x;
  double lv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = t + it * bd, r = e / KB, c = e % KB;
    lv[it] = (e < KB * KB && r < kb && c < kb) ? d.W[(size_t)(k0 + r) * ld + k0 + c] : 0.0;
  }
  const double dg = t < kb ? d.W[(size_t)(k0 + t) * ld + k0 + t] : 0.0;
  const int pvt = t < kb ? d.piv[k0 + t] : 0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = t + it * bd;
    if (e < KB * KB) LU[e / KB][e % KB] = lv[it];
  }
  if (t < KB) {
    if (t < kb) pv[t] = pvt;
    rdiag[t] = t < kb ? 1.0 / dg : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 64) perm_lists(pv, kb, k0, sFlag, sD, sV, &sNd);
  __syncthreads();
  const int col = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= d.n + d.m) return;
  double* W = d.W;
  const int nd = sNd;
  double x[KB], y[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    x[j] = (j < kb) ? W[(size_t)pv[j] * ld + col] : 0.0;
    y[j] = (j < nd) ? W[(size_t)sD[j] * ld + col] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < KB; ++j)
    if (j < nd) W[(size_t)sV[j] * ld + col] = y[j];
#pragma unroll
  for (int j = 1; j < KB; ++j) {
    double s[4] = {x[j], 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < j; ++i) s[i & 3] = fma(-LU[j][i], x[i], s[i & 3]);
    x[j] = (j < kb) ? (s[0] + s[1]) + (s[2] + s[3]) : 0.0;
  }
#pragma unroll
  for (int j = KB - 1; j >= 0; --j) {
    double s[4] = {x[j], 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = j + 1; i < KB; ++i) s[i & 3] = fma(-LU[j][i], x[i], s[i & 3]);
    x[j] = (j < kb) ? ((s[0] + s[1]) + (s[2] + s[3])) * rdiag[j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < KB; ++j)
    if (j < kb) W[(size_t)(k0 + j) * ld + col] = x[j];
}

constexpr int TBM = 64, TBN = 64, TBK = 16;  // tile of the split-FP32 kernel

// Gauss-Jordan update: rows outside the pivot block [k0, k0+kb) get
// A[i, k0+kb:] -= A[i, k0:k0+kb] R.  Row tiles 0 .. ta-1 cover rows [0, k0),
// the rest cover rows [k0+kb, n).
template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) k_gj_update(const SolveDesc* __restrict__ descs,
                                                           int k0, int nb, int coff_lo,
                                                           int coff_hi) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const SolveDesc d = descs[blockIdx.z];
  if (k0 >= d.n) return;
  const int kb = min(nb, d.n - k0);
  const int ta = (k0 + BM - 1) / BM;
  int r0, M;
  if ((int)blockIdx.y < ta) {
    r0 = blockIdx.y * BM;
    M = min(BM, k0 - r0);
  } else {
    r0 = k0 + kb + (blockIdx.y - ta) * BM;
    M = min(BM, d.n - r0);
  }
  // Columns k0 + kb + [coff_lo, coff_hi) of this system (clipped to its width).
  const int c0 = k0 + kb + coff_lo + blockIdx.x * BN;
  const int N = min(BN, min(d.n + d.m, k0 + kb + coff_hi) - c0);
  if (M <= 0 || N <= 0) return;
  const size_t ld = d.ld;
  // The old values of the tile are loaded with the first operands (the tile
  // lies outside both the panel columns and the pivot-block rows).
  gemm_tile_map<BM, BN, BK, WM, WN, RowsIdentity, RowsIdentity, RowsIdentity, NoC0Elem, true>(
      d.W + (size_t)r0 * ld + k0, d.ld, d.W + (size_t)k0 * ld + c0, d.ld, RowsIdentity{},
      d.W + (size_t)r0 * ld + c0, d.ld, RowsIdentity{}, nullptr, 0, M, N, kb, -1.0, 0, 0, sm, true);
}

// The parent's pass-through diag(T11a, T22b) at (r, c) in parent order.
struct MergePass {
  static constexpr bool active = true;
  const int* __restrict__ pmap;
  const double* __restrict__ Ta;
  const double* __restrict__ Tb;
  int na, nb;
  __device__ int row(int r) const { return as_global(pmap)[r]; }
  __device__ int col(int c) const { return as_global(pmap)[c]; }
  __device__ double value(int pr, int pc) const {
    if (pr >= 0) return pc >= 0 ? as_global(Ta)[(size_t)pr * na + pc] : 0.0;
    return pc < 0 ? as_global(Tb)[(size_t)(-pr - 1) * nb + (-pc - 1)] : 0.0;
  }
  __device__ double operator()(int r, int c) const { return value(row(r), col(c)); }
};

__device__ inline MergePass merge_pass(const GemmDesc& g) {
  return MergePass{g.pmap, g.Ta, g.Tb, g.na, g.nb};
}

// Grouped GEMM: one launch over problems, grid (tiles_n, tiles_m, nprob).
// PASS: merge Schur products, C = diag(T11a, T22b) + alpha A B (descs with pmap).
template <int BM, int BN, int BK, int WM, int WN, bool PASS, int DEPTH = 1>
__global__ void __launch_bounds__(64 * WM * WN) k_gemm(const GemmDesc* __restrict__ descs) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const GemmDesc g = descs[blockIdx.z];
  if ((int)blockIdx.y * BM >= g.M || (int)blockIdx.x * BN >= g.N) return;
  if constexpr (PASS)
    gemm_tile_map<BM, BN, BK, WM, WN, RowsIdentity, RowsIdentity, RowsIdentity, MergePass, false,
                  DEPTH>(g.A, g.lda, g.B, g.ldb, RowsIdentity{}, g.C, g.ldc, RowsIdentity{},
                         nullptr, 0, g.M, g.N, g.K, g.alpha, blockIdx.y * BM, blockIdx.x * BN, sm,
                         false, RowsIdentity{}, merge_pass(g));
  else
    gemm_tile_map<BM, BN, BK, WM, WN, RowsIdentity, RowsIdentity, RowsIdentity, NoC0Elem, false,
                  DEPTH>(g.A, g.lda, g.B, g.ldb, RowsIdentity{}, g.C, g.ldc, RowsIdentity{}, g.C0,
                         g.ldc0, g.M, g.N, g.K, g.alpha, blockIdx.y * BM, blockIdx.x * BN, sm,
                         g.overwrite == 0);
}

// The 128 x 128 tile (gemm128_tile), tiles in XCD-grouped order.
template <int VEC, bool PASS>
__global__ void __launch_bounds__(256, 2) k_gemm128(const GemmDesc* __restrict__ descs) {
  __shared__ double sm[Gemm128::SMEM];
  const GemmDesc g = descs[blockIdx.z];
  int tx, ty;
  gemm128_tile_order(gridDim.x, gridDim.y, blockIdx.x, blockIdx.y, tx, ty);
  if (ty * Gemm128::BM >= g.M || tx * Gemm128::BN >= g.N) return;
  if constexpr (PASS)
    gemm128_tile<VEC>(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, nullptr, 0, g.M, g.N, g.K, g.alpha,
                      ty * Gemm128::BM, tx * Gemm128::BN, sm, false, merge_pass(g));
  else
    gemm128_tile<VEC>(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.C0, g.ldc0, g.M, g.N, g.K, g.alpha,
                      ty * Gemm128::BM, tx * Gemm128::BN, sm, g.overwrite == 0, NoC0Elem{});
}

// The 128 x 128 tile over a queue of tiles of many problems (one persistent
// launch): each workgroup takes the next tile from the counter until the
// queue is empty, so every workgroup exits once all tiles are taken.
template <int VEC, bool PASS>
__global__ void __launch_bounds__(256, 2) k_gemm128_queue(const GemmDesc* __restrict__ descs,
                                                          const TileRef* __restrict__ tiles,
                                                          int ntiles, int* counter) {
  __shared__ double sm[Gemm128::SMEM];
  __shared__ int s_t;
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_t;
    __syncthreads();  // every thread has read s_t before it is taken again
    if (t >= ntiles) return;
    const TileRef tr = tiles[t];
    const GemmDesc g = descs[tr.prob];
    if constexpr (PASS)
      gemm128_tile<VEC>(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, nullptr, 0, g.M, g.N, g.K, g.alpha,
                        tr.tm * Gemm128::BM, tr.tn * Gemm128::BN, sm, false, merge_pass(g));
    else
      gemm128_tile<VEC>(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.C0, g.ldc0, g.M, g.N, g.K, g.alpha,
                        tr.tm * Gemm128::BM, tr.tn * Gemm128::BN, sm, g.overwrite == 0,
                        NoC0Elem{});
  }
}

__global__ void k_set_int(int* p, int v) { *p = v; }

void set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
}

std::vector<TileRef> gemm_tile_queue(const std::vector<GemmDesc>& h_desc) {
  std::vector<int> order(h_desc.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  // Largest problems first (most work per tile, then most tiles), so the
  // last tiles taken are the small ones.
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const GemmDesc &x = h_desc[a], &y = h_desc[b];
    if (x.K != y.K) return x.K > y.K;
    return (long long)x.M * x.N > (long long)y.M * y.N;
  });
  std::vector<TileRef> q;
  for (int i : order) {
    const GemmDesc& g = h_desc[i];
    const int tm = (g.M + Gemm128::BM - 1) / Gemm128::BM, tn = (g.N + Gemm128::BN - 1) / Gemm128::BN;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) q.push_back(TileRef{i, a, b, 0});
  }
  return q;
}

void grouped_gemm_queue(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc,
                        const TileRef* d_tiles, int ntiles, int* d_counter, hipStream_t stream,
                        int prof_cls) {
  if (h_desc.empty() || ntiles == 0) return;
  double fl = 0, by = 0;
  bool v2 = true;
  const bool pass = h_desc[0].pmap != nullptr;
  for (auto& g : h_desc) {
    fl += 2.0 * g.M * g.N * g.K;
    by += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + 2.0 * g.M * g.N);
    v2 = v2 && g.lda % 2 == 0 && g.ldb % 2 == 0 && g.K % 2 == 0 && g.N % 2 == 0 &&
         ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0;
    HPS_REQUIRE((g.pmap != nullptr) == pass, "mixed GEMM descriptor kinds");
  }
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    HPS_HIP(hipGetDevice(&dev));
    HPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int grid = std::min(ntiles, 2 * cus);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_counter, 0);
  ProfScope ps(prof_cls, stream, fl, by);
  if (pass && v2)
    hipLaunchKernelGGL((k_gemm128_queue<2, true>), dim3(grid), dim3(256), 0, stream, d_desc, d_tiles,
                       ntiles, d_counter);
  else if (pass)
    hipLaunchKernelGGL((k_gemm128_queue<1, true>), dim3(grid), dim3(256), 0, stream, d_desc, d_tiles,
                       ntiles, d_counter);
  else if (v2)
    hipLaunchKernelGGL((k_gemm128_queue<2, false>), dim3(grid), dim3(256), 0, stream, d_desc,
                       d_tiles, ntiles, d_counter);
  else
    hipLaunchKernelGGL((k_gemm128_queue<1, false>), dim3(grid), dim3(256), 0, stream, d_desc,
                       d_tiles, ntiles, d_counter);
}

static bool g_gemm_queue = true;
void set_gemm_queue(bool on) { g_gemm_queue = on; }
bool gemm_queue_on() { return g_gemm_queue; }

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
  // Three 16-deep slabs of operand loads in flight: slab kt + 3 TBK goes into
  // the registers slab kt has just left (constant slot of the unrolled loop).
  constexpr int DEPTH = 3, EA = (TBM * TBK) / 256, EB = (TBK * TBN) / 256;
  double qa[DEPTH][EA], qb[DEPTH][EB];
  auto load_slot = [&](int kt, double (&pa)[EA], double (&pb)[EB]) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + 256 * e, i = idx / TBK, k = idx % TBK;
      const int gr = row0 + i, gk = kt + k;
      pa[e] = (gr < g.M && gk < g.K) ? g.A[(size_t)gr * g.lda + gk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + 256 * e, k = idx / TBN, j = idx % TBN;
      const int gk = kt + k, gc = col0 + j;
      pb[e] = (gk < g.K && gc < g.N) ? g.B[(size_t)gk * g.ldb + gc] : 0.0;
    }
  };
#pragma unroll
  for (int d = 0; d < DEPTH; ++d)
    if (d * TBK < g.K) load_slot(d * TBK, qa[d], qb[d]);
  for (int kt0 = 0; kt0 < g.K; kt0 += DEPTH * TBK) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int kt = kt0 + d * TBK;
      if (kt >= g.K) break;
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int idx = tid + 256 * e, i = idx / TBK, k = idx % TBK;
        const double v = qa[d][e];
        const float h = (float)v;
        Ah[k][i] = h;
        Al[k][i] = (float)(v - (double)h);
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int idx = tid + 256 * e, k = idx / TBN, j = idx % TBN;
        const double v = qb[d][e];
        const float h = (float)v;
        Bh[k][j] = h;
        Bl[k][j] = (float)(v - (double)h);
      }
      __syncthreads();
      if (kt + DEPTH * TBK < g.K) load_slot(kt + DEPTH * TBK, qa[d], qb[d]);
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
          double c0 = g.pmap ? merge_pass(g)(gr, gc)
                      : g.C0 ? g.C0[(size_t)gr * g.ldc0 + gc]
                      : g.overwrite ? 0.0 : g.C[(size_t)gr * g.ldc + gc];
          g.C[(size_t)gr * g.ldc + gc] = c0 + g.alpha * acc[i][j][r];
        }
      }
}

// ---------------------------------------------------------------------------
// Schur product on BF16 MFMA with three-slice splits.  Every FP64 operand
// value is written as h + m + l with h = bf16(v), m = bf16(v - h),
// l = bf16(v - h - m) (each remainder is exact in FP64); the product is
// formed from the six slice products of order 2^-16 or larger,
// hh + (hm + mh + hl + lh + mm).  BF16 products are exact in FP32; the two
// groups are summed in FP32 over one 32-deep step (v_mfma 16x16x32) and then
// added to FP64 accumulators, so the error is a few units of 2^-24 relative
// to |A||B|, like the split-FP32 form, at BF16 matrix-core rates.
//
// k_split3 writes the slices of an operand once per launch, k contiguous,
// rows and k zero-padded to multiples of 64 (B transposed on the way, through
// an LDS tile), so the GEMM reads each MFMA fragment (eight consecutive k of
// one row) with one 16-byte load and needs no bounds checks.  MFMA lane
// layout: A lane l holds A[l%16][8(l/16)..+7], B holds B[8(l/16)..+7][l%16],
// result register r holds D[4(l/16)+r][l%16].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline double bf16_val(unsigned short b) {
  return (double)__uint_as_float(((unsigned int)b) << 16);
}

// Slices of one operand: dst[s][r][k], s < 3, r < rows_pad, k < kpad, of the
// matrix element (r, k) = src[r * ld + k] (trans = 0) or src[k * ld + r]
// (trans = 1), zero outside rows x k.
struct SliceJob {
  const double* src;
  unsigned short* dst;
  int rows, k, ld, trans;
  int rows_pad, kpad;
};

__global__ void __launch_bounds__(256) k_split3(const SliceJob* __restrict__ jobs) {
  __shared__ double t[64][65];
  const SliceJob jb = jobs[blockIdx.z];
  const int r0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
  if (r0 >= jb.rows_pad || k0 >= jb.kpad) return;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int a = e / 64, b = e % 64;  // b runs along memory
    double v = 0.0;
    if (jb.trans) {
      const int k = k0 + a, r = r0 + b;
      if (k < jb.k && r < jb.rows) v = jb.src[(size_t)k * jb.ld + r];
      t[b][a] = v;
    } else {
      const int r = r0 + a, k = k0 + b;
      if (k < jb.k && r < jb.rows) v = jb.src[(size_t)r * jb.ld + k];
      t[a][b] = v;
    }
  }
  __syncthreads();
  const size_t per = (size_t)jb.rows_pad * jb.kpad;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int rl = e / 64, kl = e % 64;
    const double v = t[rl][kl];
    const unsigned short h = bf16_rne((float)v);
    const double r1 = v - bf16_val(h);
    const unsigned short m = bf16_rne((float)r1);
    const unsigned short l = bf16_rne((float)(r1 - bf16_val(m)));
    const size_t o = (size_t)(r0 + rl) * jb.kpad + k0 + kl;
    jb.dst[o] = h;
    jb.dst[per + o] = m;
    jb.dst[2 * per + o] = l;
  }
}

// Slices of one product's operands (from k_split3): A [3][mpad][kpad],
// B^T [3][npad][kpad].
struct SliceGemm {
  const unsigned short* a;
  const unsigned short* b;
  int mpad, npad, kpad, pad;
};

// Workgroup tile 128 x 64 (four waves stacked along M, 32 x 64 each, 2 x 4
// MFMA blocks), 32-deep steps.  The step's slices of A (128 rows) and B
// (64 columns) are staged in LDS with 16-byte copies, double-buffered, so
// each slice value is read from L2 once per workgroup; the small products
// accumulate in FP32 over the whole contraction (they are 2^-8 of the
// result), the hh products in FP32 over one step and then in FP64.
constexpr int XBM = 128, XBN = 64, XPAD = 40;  // XPAD: LDS row pitch in BF16 (80 bytes)

__global__ void __launch_bounds__(256) k_gemm_bf16x6(const GemmDesc* __restrict__ descs,
                                                     const SliceGemm* __restrict__ slices) {
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][3][XBM][XPAD];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][3][XBN][XPAD];
  const GemmDesc g = descs[blockIdx.z];
  const SliceGemm sg = slices[blockIdx.z];
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (tm * XBM >= g.M || tn * XBN >= g.N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int row0 = tm * XBM, col0 = tn * XBN, kq = 8 * (lane >> 4);
  const size_t sa = (size_t)sg.mpad * sg.kpad, sb = (size_t)sg.npad * sg.kpad;
  // Copy assignment: thread t moves 16 bytes (8 k values) of row t / 4,
  // k offset 8 (t % 4), for A rows t/4 and t/4 + 64 and B row t/4, per slice.
  const int cr = tid >> 2, ck = 8 * (tid & 3);
  // Rows past mpad/npad (a tile hanging over the padded edge) read row 0.
  const int ra0 = row0 + cr < sg.mpad ? row0 + cr : 0;
  const int ra1 = row0 + cr + 64 < sg.mpad ? row0 + cr + 64 : 0;
  const int rb0 = col0 + cr < sg.npad ? col0 + cr : 0;
  const unsigned short* ga0 = sg.a + (size_t)ra0 * sg.kpad + ck;
  const unsigned short* ga1 = sg.a + (size_t)ra1 * sg.kpad + ck;
  const unsigned short* gb0 = sg.b + (size_t)rb0 * sg.kpad + ck;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 ra[3][2], rbv[3];
  auto fetch = [&](int kt) {
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      ra[sl][0] = *reinterpret_cast<const u4*>(ga0 + sl * sa + kt);
      ra[sl][1] = *reinterpret_cast<const u4*>(ga1 + sl * sa + kt);
      rbv[sl] = *reinterpret_cast<const u4*>(gb0 + sl * sb + kt);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      *reinterpret_cast<u4*>(&sA[buf][sl][cr][ck]) = ra[sl][0];
      *reinterpret_cast<u4*>(&sA[buf][sl][cr + 64][ck]) = ra[sl][1];
      *reinterpret_cast<u4*>(&sB[buf][sl][cr][ck]) = rbv[sl];
    }
  };
  double acc[2][4][4];
  f4 small[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      small[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
    }
  fetch(0);
  stage(0);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < sg.kpad; kt += 32) {
    const bool more = kt + 32 < sg.kpad;
    if (more) fetch(kt + 32);  // in flight during this step's products
    bf16x8 a[3][2], b[3][4];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[sl][i] = *reinterpret_cast<const bf16x8*>(&sA[buf][sl][wid * 32 + i * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[sl][j] = *reinterpret_cast<const bf16x8*>(&sB[buf][sl][j * 16 + (lane & 15)][kq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        f4 big = f4{0.f, 0.f, 0.f, 0.f};
        big = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], big, 0, 0, 0);
        small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], small[i][j], 0, 0, 0);
        small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], small[i][j], 0, 0, 0);
        small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], small[i][j], 0, 0, 0);
        small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], small[i][j], 0, 0, 0);
        small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], small[i][j], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)big[r];
      }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wid * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + j * 16 + (lane & 15);
        if (gr < g.M && gc < g.N) {
          const double c0 = g.pmap ? merge_pass(g)(gr, gc)
                            : g.C0 ? g.C0[(size_t)gr * g.ldc0 + gc]
                            : g.overwrite ? 0.0 : g.C[(size_t)gr * g.ldc + gc];
          g.C[(size_t)gr * g.ldc + gc] =
              c0 + g.alpha * (acc[i][j][r] + (double)small[i][j][r]);
        }
      }
}

static int g_bf16x6_min_k = 384;
void set_bf16x6_min_k(int k) { g_bf16x6_min_k = k < 0 ? 384 : k; }
int bf16x6_min_k() { return g_bf16x6_min_k; }

// Slices for every product of a launch (stream-ordered scratch, released on
// the stream after the products), then the products.
static void gemm_bf16x6(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc,
                        hipStream_t s) {
  const int np = (int)h_desc.size();
  auto up64 = [](int x) { return (x + 63) / 64 * 64; };
  std::vector<SliceJob> jobs;
  std::vector<SliceGemm> sl(np);
  size_t total = 0;
  int mmax = 0, nmax = 0, rmax = 0, kmax = 0;
  for (const GemmDesc& g : h_desc) {
    const int mp = up64(g.M), npd = up64(g.N), kp = up64(g.K);
    total += (size_t)3 * ((size_t)mp + npd) * kp;
    mmax = std::max(mmax, g.M);
    nmax = std::max(nmax, g.N);
    rmax = std::max(rmax, std::max(mp, npd));
    kmax = std::max(kmax, kp);
  }
  unsigned short* buf = nullptr;
  HPS_HIP(hipMallocAsync((void**)&buf, total * sizeof(unsigned short), s));
  size_t off = 0;
  for (int i = 0; i < np; ++i) {
    const GemmDesc& g = h_desc[i];
    const int mp = up64(g.M), npd = up64(g.N), kp = up64(g.K);
    unsigned short* a = buf + off;
    off += (size_t)3 * mp * kp;
    unsigned short* b = buf + off;
    off += (size_t)3 * npd * kp;
    jobs.push_back(SliceJob{g.A, a, g.M, g.K, g.lda, 0, mp, kp});
    jobs.push_back(SliceJob{g.B, b, g.N, g.K, g.ldb, 1, npd, kp});
    sl[i] = SliceGemm{a, b, mp, npd, kp, 0};
  }
  SliceJob* djobs = nullptr;
  SliceGemm* dsl = nullptr;
  HPS_HIP(hipMallocAsync((void**)&djobs, jobs.size() * sizeof(SliceJob), s));
  HPS_HIP(hipMallocAsync((void**)&dsl, sl.size() * sizeof(SliceGemm), s));
  HPS_HIP(hipMemcpyAsync(djobs, jobs.data(), jobs.size() * sizeof(SliceJob),
                         hipMemcpyHostToDevice, s));
  HPS_HIP(hipMemcpyAsync(dsl, sl.data(), sl.size() * sizeof(SliceGemm), hipMemcpyHostToDevice, s));
  HPS_REQUIRE(jobs.size() <= 65535, "too many products in one launch");
  hipLaunchKernelGGL(k_split3, dim3(kmax / 64, rmax / 64, (unsigned)jobs.size()), dim3(256), 0, s,
                     djobs);
  hipLaunchKernelGGL(k_gemm_bf16x6, dim3((nmax + XBN - 1) / XBN, (mmax + XBM - 1) / XBM, np),
                     dim3(256), 0, s, d_desc, dsl);
  // The host vectors above were copied from pageable memory, so they may go.
  HPS_HIP(hipFreeAsync(dsl, s));
  HPS_HIP(hipFreeAsync(djobs, s));
  HPS_HIP(hipFreeAsync(buf, s));
}

// ---------------------------------------------------------------------------
// Host drivers.
// ---------------------------------------------------------------------------

// Panel launch: up to eight waves; two rows per lane for 32-wide panels
// (x[2][32] fits the 256 VGPRs of a wave at two waves per SIMD), six rows per
// lane for the 16-wide panels of systems beyond 1024 rows.
static void launch_panel(const SolveDesc* d_desc, int np, int k0, int rows, int nb, int* st,
                         hipStream_t s) {
  if (nb == 32) {
    HPS_REQUIRE(rows <= 64 * TP_MAXW * 2, "panel has too many rows");
    if (rows <= 128) {
      hipLaunchKernelGGL((k_gj_panel_w1<32>), dim3(np), dim3(64), 0, s, d_desc, k0, st);
      return;
    }
    const int nw = (rows + 127) / 128;
    hipLaunchKernelGGL((k_gj_panel<2, 32>), dim3(np), dim3(64 * nw), 0, s, d_desc, k0, st);
  } else {
    HPS_REQUIRE(rows <= 64 * TP_MAXW * 6, "panel has too many rows");
    const int nw = (rows + 383) / 384;
    hipLaunchKernelGGL((k_gj_panel<6, 16>), dim3(np), dim3(64 * nw), 0, s, d_desc, k0, st);
  }
}

int max_solve_rows() { return 3072; }

// Launch of one Gauss-Jordan update with tile variant v.
// Updates columns k0 + kb + [coff_lo, coff_lo + ncols) of every system.
static void launch_update(int v, const SolveDesc* d_desc, int np, int k0, int nb, int nmax,
                          int coff_lo, int ncols, hipStream_t s) {
  if (ncols <= 0) return;
  const int coff_hi = coff_lo + ncols;
#define HPS_UPD(BM, BN, BK, WM, WN)                                                        \
  {                                                                                         \
    const int ty = (k0 + BM - 1) / BM + (std::max(0, nmax - k0 - nb) + BM - 1) / BM;       \
    if (ty > 0)                                                                             \
      hipLaunchKernelGGL((k_gj_update<BM, BN, BK, WM, WN>), dim3((ncols + BN - 1) / BN, ty, np), \
                         dim3(64 * WM * WN), 0, s, d_desc, k0, nb, coff_lo, coff_hi);       \
    return;                                                                                 \
  }
  // Tile variants as listed at UPDATE_VARIANTS (tune.h).
  switch (v) {
    case 1: HPS_UPD(32, 32, 16, 1, 1)
    case 2: HPS_UPD(128, 128, 16, 4, 2)
    case 3: HPS_UPD(128, 64, 16, 2, 2)
    case 4: HPS_UPD(64, 128, 16, 2, 2)
    case 5: HPS_UPD(64, 64, 32, 2, 2)
    default: HPS_UPD(64, 64, 16, 2, 2)
  }
#undef HPS_UPD
}

// Side stream and events of the look-ahead, one set per device (default priority).
struct LookAhead {
  hipStream_t side = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
};
static const LookAhead& look_ahead() {
  static std::mutex mu;
  static std::map<int, LookAhead> per_device;
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  LookAhead& la = per_device[dev];
  if (!la.side) {
    HPS_HIP(hipStreamCreateWithFlags(&la.side, hipStreamNonBlocking));
    HPS_HIP(hipEventCreateWithFlags(&la.ready, hipEventDisableTiming));
    HPS_HIP(hipEventCreateWithFlags(&la.done, hipEventDisableTiming));
  }
  return la;
}
static bool g_gj_lookahead = false;
void set_gj_lookahead(bool on) { g_gj_lookahead = on; }

void batched_solve_v(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                     hipStream_t stream, int gj_variant) {
  if (h_desc.empty()) return;
  int nmax = 0, wmax = 0;
  for (auto& d : h_desc) {
    nmax = std::max(nmax, d.n);
    wmax = std::max(wmax, d.n + d.m);
  }
  HPS_REQUIRE(nmax <= max_solve_rows(), "dense system too large for the panel kernel");
  const int nb = nmax > 1024 ? 16 : 32;
  const int np = (int)h_desc.size();
  const int upd = gj_variant >= 0 ? gj_variant / 4 : 0;
  const int tb = TRSM_BLOCKS[gj_variant >= 0 ? std::min(gj_variant % 4, 2) : 0];
  const bool look = g_gj_lookahead && nmax > nb;
  const LookAhead& la = look ? look_ahead() : LookAhead{};
  bool pending = false;
  for (int k0 = 0; k0 < nmax; k0 += nb) {
    double fp = 0, ft = 0, fu = 0;
    for (auto& d : h_desc) {
      if (k0 >= d.n) continue;
      const double kb = std::min(nb, d.n - k0), rows = d.n - k0, rest = d.n + d.m - k0 - kb;
      fp += rows * kb * kb;
      ft += 2.0 * rest * kb * kb;
      fu += 2.0 * (d.n - kb) * rest * kb;
    }
    const int rows = nmax - k0;
    {
      ProfScope ps(PROF_LU_PANEL, stream, fp, 0);
      launch_panel(d_desc, np, k0, rows, nb, d_status, stream);
    }
    const int rest = wmax - k0 - std::min(nb, rows);
    if (rest <= 0) continue;
    if (pending) {  // the previous step's side-stream update must finish before these row moves
      HPS_HIP(hipStreamWaitEvent(stream, la.done, 0));
      pending = false;
    }
    {
      ProfScope ps(PROF_SWAP_TRSM, stream, ft, 0);
      dim3 g((rest + tb - 1) / tb, np);
      if (nb == 32)
        hipLaunchKernelGGL((k_gj_swap_trsm<32>), g, dim3(tb), 0, stream, d_desc, k0);
      else
        hipLaunchKernelGGL((k_gj_swap_trsm<16>), g, dim3(tb), 0, stream, d_desc, k0);
    }
    if (!look) {
      ProfScope ps(PROF_LU_UPDATE, stream, fu, 0);
      launch_update(upd, d_desc, np, k0, nb, nmax, 0, rest, stream);
      continue;
    }
    // Look-ahead: the next panel's columns are updated on the caller's
    // stream, so the next panel can start while the side stream updates the
    // remaining columns; the next step's row moves wait for that update.
    {
      ProfScope ps(PROF_LU_UPDATE, stream, fu, 0);
      launch_update(upd, d_desc, np, k0, nb, nmax, 0, std::min(nb, rest), stream);
      if (rest > nb) {
        HPS_HIP(hipEventRecord(la.ready, stream));
        HPS_HIP(hipStreamWaitEvent(la.side, la.ready, 0));
        launch_update(upd, d_desc, np, k0, nb, nmax, nb, rest - nb, la.side);
        HPS_HIP(hipEventRecord(la.done, la.side));
        pending = true;
      }
    }
  }
  if (pending) HPS_HIP(hipStreamWaitEvent(stream, la.done, 0));
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan with pivoting inside the diagonal block (large merge
// systems).  Step k0 of W = [M | I] (n = m3 rows, kb = min(64, n - k0)):
//   1. k_bgj_diag: B^-1 of the diagonal block B = W[K, K], K = [k0, k0 + kb),
//      by in-place Gauss-Jordan with partial pivoting among the kb rows of
//      the block (one workgroup per system: each of eight waves holds 8
//      columns of every row, the pivot row reaches each wave by readlane,
//      the multipliers through LDS; one barrier per column);
//   2. k_bgj_rows: the block's rows become B^-1 W[K, k0 + kb:] (FP64 MFMA);
//   3. k_gj_update: every other row gets W[i, :] -= W[i, K] W_new[K, :].
// No rows move, so the identity block ends up holding M^-1 in natural
// order, as with the partial-pivoting path.  The serial part of a step is a
// 64-column elimination of 64 rows, not of the whole remaining column, which
// is what makes the top merges (thousands of rows) fast.  Stability rests on
// the diagonal blocks: a block pivot below fb_tol max|M| (or a zero or
// non-finite one) raises status[3], and the caller redoes the level with
// partial pivoting.
// ---------------------------------------------------------------------------
constexpr int BGJ_NB = 64;
constexpr int BGJ_CPW = 8;  // diagonal-block columns per wave (eight waves)

__global__ void __launch_bounds__(64 * BGJ_NB / BGJ_CPW) k_bgj_diag(const SolveDesc* __restrict__ descs, int k0,
                                                  double* __restrict__ binv, double fb_tol,
                                                  int* status) {
  // Multipliers of the current column (double-buffered by column parity, so
  // one barrier per column suffices), its pivot row and pivot.
  __shared__ double sF[2][BGJ_NB];
  __shared__ double sPiv[2];
  __shared__ int sPr[2];
  __shared__ int sP[BGJ_NB], sPi[BGJ_NB];
  const SolveDesc d = descs[blockIdx.x];
  if (k0 >= d.n) return;
  const int kb = min(BGJ_NB, d.n - k0);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const size_t ld = d.ld;
  const double* Bk = d.W + (size_t)k0 * ld + k0;
  // Wave w holds columns CPW w .. CPW w + CPW - 1 of row `lane`; padding
  // (rows or columns >= kb) is the identity, which no real column can pick.
  constexpr int CPW = BGJ_CPW;
  double x[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = CPW * wid + j;
    x[j] = (lane < kb && c < kb) ? as_global(Bk)[(size_t)lane * ld + c] : (lane == c ? 1.0 : 0.0);
  }
  // Rows are scaled lazily: the true row is scale * x.  A pivot row keeps
  // its values and takes scale = 1 / pivot; only unchosen rows (scale 1)
  // are ever broadcast as pivot rows, so every update is one FMA per entry.
  double scale = 1.0;
  bool chosen = false, bad = false;
  double minp = INFINITY;
  for (int g = 0; g < (kb + CPW - 1) / CPW; ++g) {
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      const int c = CPW * g + cc;
      if (c >= kb) continue;  // uniform
      const int buf = c & 1;
      if (wid == g) {
        const unsigned key = chosen ? 0u : pivot_key(x[cc], lane);
        const unsigned gk = wave_max_u32(key);
        const int pr = 4095 - (int)(gk & 4095u);
        sF[buf][lane] = x[cc];
        if (lane == pr) sPiv[buf] = x[cc];
        if (lane == 0) {
          sPr[buf] = pr;
          sP[c] = pr;
        }
      }
      __syncthreads();
      const int pr = __builtin_amdgcn_readfirstlane(sPr[buf]);
      const double piv = uniform(sPiv[buf]);
      const double f = sF[buf][lane];
      const bool ok = piv != 0.0 && piv == piv && fabs(piv) != INFINITY;
      bad |= !ok;
      minp = fmin(minp, fabs(piv));
      const double inv = ok ? recip(piv) : 0.0;
      const bool me = lane == pr;
      const double gm = me ? 0.0 : -f * inv;
#pragma unroll
      for (int j = 0; j < CPW; ++j) x[j] = fma(gm, bcast_lane(x[j], pr), x[j]);
      if (wid == g) x[cc] = me ? 1.0 : gm;
      if (me) {
        scale = inv;
        chosen = true;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < CPW; ++j) x[j] *= scale;
  // Pivot statistics and the fall-back test (block pivots against max|M|);
  // a zero or non-finite block pivot also falls back (the partial-pivoting
  // path then decides whether M itself is singular).
  if (threadIdx.x == 0) {
    if (d.pstat && !bad) atomicMin(d.pstat + 1, abs_bits(minp));
    const double amax = d.pstat ? __longlong_as_double((long long)d.pstat[0]) : 0.0;
    if (bad || !(minp > fb_tol * amax)) atomicExch(status + 3, 1);
  }
  if (threadIdx.x < BGJ_NB) sPi[threadIdx.x] = 0;  // in range even for a failed block
  __syncthreads();
  if (threadIdx.x < kb) sPi[sP[threadIdx.x]] = threadIdx.x;
  __syncthreads();
  // In-place Gauss-Jordan with marked (unmoved) pivot rows leaves X with
  // B^-1[Pi[r]][P[c]] = X[r][c] (P: pivot row of each column, Pi its inverse).
  double* Bi = binv + (size_t)blockIdx.x * BGJ_NB * BGJ_NB;
  if (lane < kb) {
    const int a = sPi[lane];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int c = CPW * wid + j;
      if (c < kb) Bi[(size_t)a * BGJ_NB + sP[c]] = x[j];
    }
  }
}

// Rows K of every system: W[K, k0 + kb + c] = B^-1 W[K, k0 + kb + c] for the
// columns c of this tile (one 64-row tile covers all kb rows, so a tile reads
// its own columns of W[K, :] before it overwrites them).
__global__ void __launch_bounds__(256) k_bgj_rows(const SolveDesc* __restrict__ descs, int k0,
                                                  const double* __restrict__ binv, int ident) {
  __shared__ double sm[GemmTile<64, 64, 16, 2, 2>::SMEM];
  const SolveDesc d = descs[blockIdx.z];
  if (k0 >= d.n) return;
  const int kb = min(BGJ_NB, d.n - k0);
  // Columns past the block.  With W = [M | I] (ident): k0 + kb .. n + k0 + kb
  // - 1, the rest of M and the part of the identity block already touched
  // (its later columns are still unit vectors that no step changes before
  // its own); otherwise every column to the right.
  const int ncols = ident ? min(d.n, d.n + d.m - k0 - kb) : d.n + d.m - k0 - kb;
  if ((int)blockIdx.x * 64 >= ncols) return;
  double* Wk = d.W + (size_t)k0 * d.ld + k0 + kb;
  gemm_tile_map<64, 64, 16, 2, 2, RowsIdentity, RowsIdentity, RowsIdentity, NoC0Elem, false, 3>(
      binv + (size_t)blockIdx.z * BGJ_NB * BGJ_NB, BGJ_NB, Wk, (int)d.ld, RowsIdentity{}, Wk,
      (int)d.ld, RowsIdentity{}, nullptr, 0, kb, ncols, kb, 1.0, 0, blockIdx.x * 64, sm, false);
}

__global__ void k_pstat_reset_min(const SolveDesc* __restrict__ descs, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && descs[i].pstat) descs[i].pstat[1] = ~0ull;
}

void pstat_reset_min(const SolveDesc* d_desc, int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_pstat_reset_min, dim3((count + 255) / 256), dim3(256), 0, s, d_desc, count);
}

static double g_bgj_fb_tol = 1e-6;
static int g_bgj_min_rows = 256;
static bool g_bgj_lookahead = true;
void set_bgj_lookahead(bool on) { g_bgj_lookahead = on; }

void set_bgj(int min_rows, double fb_tol) {
  if (min_rows >= 0) g_bgj_min_rows = min_rows;
  if (fb_tol >= 0.0) g_bgj_fb_tol = fb_tol;
}

int bgj_min_rows() { return g_bgj_min_rows; }

void batched_solve_bgj(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                       double* binv, hipStream_t stream, bool ident) {
  if (h_desc.empty()) return;
  int nmax = 0, wmax = 0;
  for (auto& d : h_desc) {
    // Only the untouched columns of the identity block are skipped, so with
    // ident the right-hand block must be I (m == n).
    HPS_REQUIRE(!ident || d.m == d.n, "blocked Gauss-Jordan: W = [M | I] needs m == n");
    nmax = std::max(nmax, d.n);
    wmax = std::max(wmax, d.n + d.m);
  }
  const int np = (int)h_desc.size();
  const int upd = 0;
  // Look-ahead: each step updates the next diagonal block's columns first,
  // then the other columns on a side stream, so the next (latency-bound)
  // diagonal-block kernel runs beside that update; the next block-row kernel
  // waits for it.
  const bool look = g_bgj_lookahead && nmax > BGJ_NB;
  const LookAhead& la = look ? look_ahead() : LookAhead{};
  bool pending = false;
  for (int k0 = 0; k0 < nmax; k0 += BGJ_NB) {
    double fd = 0, fr = 0, fu = 0;
    for (auto& d : h_desc) {
      if (k0 >= d.n) continue;
      const double kb = std::min(BGJ_NB, d.n - k0),
                   rest = ident ? std::min<double>(d.n, d.n + d.m - k0 - kb) : d.n + d.m - k0 - kb;
      fd += 2.0 * kb * kb * kb;
      fr += 2.0 * kb * kb * rest;
      fu += 2.0 * (d.n - kb) * rest * kb;
    }
    {
      ProfScope ps(PROF_BGJ_DIAG, stream, fd, 0);
      hipLaunchKernelGGL(k_bgj_diag, dim3(np), dim3(64 * BGJ_NB / BGJ_CPW), 0, stream, d_desc, k0,
                         binv, g_bgj_fb_tol, d_status);
    }
    // Columns past the block (with ident: the rest of M and the touched part
    // of the identity block, n columns in all); k_bgj_rows and the update
    // clip them per system.
    const int rest = ident ? std::min(nmax, wmax - k0 - std::min(BGJ_NB, nmax - k0))
                           : wmax - k0 - std::min(BGJ_NB, nmax - k0);
    if (rest <= 0) continue;
    if (pending) {  // the previous step's side-stream update must finish first
      HPS_HIP(hipStreamWaitEvent(stream, la.done, 0));
      pending = false;
    }
    {
      ProfScope ps(PROF_BGJ_ROWS, stream, fr, 0);
      hipLaunchKernelGGL(k_bgj_rows, dim3((rest + 63) / 64, 1, np), dim3(256), 0, stream, d_desc,
                         k0, (const double*)binv, ident ? 1 : 0);
    }
    {
      ProfScope ps(PROF_BGJ_UPDATE, stream, fu, 0);
      if (!look || rest <= BGJ_NB) {
        launch_update(upd, d_desc, np, k0, BGJ_NB, nmax, 0, rest, stream);
      } else {
        launch_update(upd, d_desc, np, k0, BGJ_NB, nmax, 0, BGJ_NB, stream);
        HPS_HIP(hipEventRecord(la.ready, stream));
        HPS_HIP(hipStreamWaitEvent(la.side, la.ready, 0));
        launch_update(upd, d_desc, np, k0, BGJ_NB, nmax, BGJ_NB, rest - BGJ_NB, la.side);
        HPS_HIP(hipEventRecord(la.done, la.side));
        pending = true;
      }
    }
  }
  if (pending) HPS_HIP(hipStreamWaitEvent(stream, la.done, 0));
}

void batched_solve(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                   hipStream_t stream, int /*nb_hint*/) {
  if (h_desc.empty()) return;
  int nmax = 0, wmax = 0;
  for (auto& d : h_desc) {
    nmax = std::max(nmax, d.n);
    wmax = std::max(wmax, d.n + d.m);
  }
  const int v = tune_get(TUNE_GJ, tune_lg(nmax), tune_lg(wmax), tune_lg((long long)h_desc.size()), 0);
  batched_solve_v(d_desc, h_desc, d_status, stream, v);
}

void grouped_gemm_v(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                    int variant, int prec, int prof_cls) {
  if (h_desc.empty()) return;
  int mmax = 0, nmax = 0;
  for (auto& g : h_desc) {
    mmax = std::max(mmax, g.M);
    nmax = std::max(nmax, g.N);
  }
  double fl = 0, by = 0;
  for (auto& g : h_desc) {
    fl += 2.0 * g.M * g.N * g.K;
    by += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + 2.0 * g.M * g.N);
  }
  const unsigned np = (unsigned)h_desc.size();
  // Every descriptor of a launch is of one kind (merge Schur products or plain).
  const bool pass = h_desc[0].pmap != nullptr;
  for (auto& g : h_desc) {
    HPS_REQUIRE((g.pmap != nullptr) == pass, "mixed GEMM descriptor kinds");
    HPS_REQUIRE(!pass || (g.Ta != nullptr && g.Tb != nullptr && g.na > 0 && g.nb > 0),
                "merge Schur product without its children's DtNs");
  }
  HPS_REQUIRE(prec == GEMM_F64 || prec == GEMM_SPLIT32 || prec == GEMM_BF16X6,
              "unknown GEMM arithmetic");
  ProfScope ps(prec == GEMM_SPLIT32 ? PROF_GEMM_SPLIT32
                                    : (prec == GEMM_BF16X6 ? PROF_GEMM_BF16X6 : prof_cls),
               stream, fl, by);
  if (prec == GEMM_SPLIT32) {
    dim3 grid((nmax + TBN - 1) / TBN, (mmax + TBM - 1) / TBM, np);
    hipLaunchKernelGGL(k_gemm_split32, grid, dim3(256), 0, stream, d_desc);
    return;
  }
  if (prec == GEMM_BF16X6) {
    gemm_bf16x6(d_desc, h_desc, stream);
    return;
  }
#define HPS_GEMM(BM, BN, BK, WM, WN, D)                                                       \
  {                                                                                           \
    const dim3 grid((nmax + BN - 1) / BN, (mmax + BM - 1) / BM, np);                          \
    if (pass)                                                                                 \
      hipLaunchKernelGGL((k_gemm<BM, BN, BK, WM, WN, true, D>), grid, dim3(64 * WM * WN), 0,  \
                         stream, d_desc);                                                     \
    else                                                                                      \
      hipLaunchKernelGGL((k_gemm<BM, BN, BK, WM, WN, false, D>), grid, dim3(64 * WM * WN), 0, \
                         stream, d_desc);                                                     \
    return;                                                                                   \
  }
  if (variant == 7) {
    // Pairs of doubles when every operand row starts 16-byte aligned and no
    // pair straddles the K or N edge.
    bool v2 = true;
    for (auto& g : h_desc)
      v2 = v2 && g.lda % 2 == 0 && g.ldb % 2 == 0 && g.K % 2 == 0 && g.N % 2 == 0 &&
           ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0;
    const dim3 grid((nmax + 127) / 128, (mmax + 127) / 128, np);
    if (pass && v2)
      hipLaunchKernelGGL((k_gemm128<2, true>), grid, dim3(256), 0, stream, d_desc);
    else if (pass)
      hipLaunchKernelGGL((k_gemm128<1, true>), grid, dim3(256), 0, stream, d_desc);
    else if (v2)
      hipLaunchKernelGGL((k_gemm128<2, false>), grid, dim3(256), 0, stream, d_desc);
    else
      hipLaunchKernelGGL((k_gemm128<1, false>), grid, dim3(256), 0, stream, d_desc);
    return;
  }
  switch (variant) {
    case 1: HPS_GEMM(32, 32, 16, 1, 1, 1)
    case 2: HPS_GEMM(128, 128, 16, 4, 2, 1)
    case 3: HPS_GEMM(128, 64, 16, 2, 2, 1)
    case 4: HPS_GEMM(64, 128, 16, 2, 2, 1)
    case 5: HPS_GEMM(64, 64, 32, 2, 2, 1)
    case 6: HPS_GEMM(64, 64, 16, 2, 2, 1)
    default: HPS_GEMM(64, 64, 16, 2, 2, 3)
  }
#undef HPS_GEMM
}

int gemm_bucket_variant(const std::vector<GemmDesc>& h_desc) {
  int mmax = 0, nmax = 0, kmax = 0;
  for (auto& g : h_desc) {
    mmax = std::max(mmax, g.M);
    nmax = std::max(nmax, g.N);
    kmax = std::max(kmax, g.K);
  }
  return tune_get(TUNE_GEMM, tune_lg(mmax), tune_lg(nmax), tune_lg(kmax),
                  tune_lg((long long)h_desc.size()));
}

void grouped_gemm(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                  int prec, int prof_cls) {
  if (h_desc.empty()) return;
  grouped_gemm_v(d_desc, h_desc, stream, prec != GEMM_F64 ? 0 : gemm_bucket_variant(h_desc), prec,
                 prof_cls);
}

// ---------------------------------------------------------------------------
// Pivot statistics: max|M| of a system before its elimination, the smallest
// pivot magnitude after it, and the relative pivot test |pivot| <= tol max|M|.
// ---------------------------------------------------------------------------
__global__ void k_pstat_init(unsigned long long* __restrict__ pstat, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    pstat[2 * i] = 0ull;
    pstat[2 * i + 1] = ~0ull;
  }
}

__global__ void __launch_bounds__(256) k_sys_absmax(const SolveDesc* __restrict__ descs) {
  const SolveDesc d = descs[blockIdx.y];
  if (!d.pstat) return;
  const size_t tot = (size_t)d.n * d.n;
  double amax = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x)
    amax = fmax(amax, fabs(d.W[(e / d.n) * d.ld + e % d.n]));
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(d.pstat, abs_bits(m));
  }
}

__global__ void k_pivot_check(const SolveDesc* __restrict__ descs, int count, double tol,
                              int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const SolveDesc d = descs[i];
  if (!d.pstat) return;
  const double amax = __longlong_as_double((long long)d.pstat[0]);
  const unsigned long long pb = d.pstat[1];
  const double pmin = pb >= 0x7FF0000000000000ull ? INFINITY : __longlong_as_double((long long)pb);
  if (pmin <= tol * amax)
    if (atomicCAS(status, 0, 1) == 0) status[1] = d.tag;
}

void pstat_init(unsigned long long* pstat, size_t count, hipStream_t s) {
  if (count == 0) return;
  const int blocks = (int)std::min<size_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_pstat_init, dim3(blocks), dim3(256), 0, s, pstat, count);
}

void system_absmax(const SolveDesc* d_desc, int count, int nmax, hipStream_t s) {
  if (count == 0) return;
  const int bx = (int)std::min<size_t>(((size_t)nmax * nmax + 255) / 256, 64);
  hipLaunchKernelGGL(k_sys_absmax, dim3(bx, count), dim3(256), 0, s, d_desc);
}

void pivot_check(const SolveDesc* d_desc, int count, double tol, int* status, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_pivot_check, dim3((count + 255) / 256), dim3(256), 0, s, d_desc, count, tol,
                     status);
}

void dense_init() {}

}  // namespace hps
