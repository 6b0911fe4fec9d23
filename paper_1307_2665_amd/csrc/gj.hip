// Batched Gauss-Jordan eliminations for gfx950 (eq:leaf_solve, section 3.1:
// Z = A_ii^-1 R; eq:U_parent, section 4: M^-1 of M = T33a - T33b): the
// partial-pivoting block solver (panels, row moves with the block-row
// triangular solve, MFMA trailing updates), the blocked form with pivoting
// inside 64 x 64 diagonal blocks for large systems, and the pivot
// statistics of both.
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

}  // namespace hps
