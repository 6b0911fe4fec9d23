// Fused leaf solve (section 3.1, eq:leaf_solve): for one leaf per workgroup,
// assemble the augmented system [A_ii | R] (R = A_ie L1) directly in
// registers, run LU with partial pivoting on it (the elimination carries R
// along) and back-substitute, leaving Z = A_ii^-1 R in global memory.  The
// leaf DtN is then T = P0 - P1 Z (section 3.2), formed by the grouped GEMM.
//
// Register layout: a TR x TC thread grid (thread id = tr + TR * tc) owns the
// matrix cyclically: row i = tr + TR * s (s < NR), column j = tc + TC * t
// (t < NC), so each thread holds NR x NC doubles.  The TR threads owning a
// column are TR consecutive lanes of one wave, so the pivot search of a column
// is a shuffle reduction without barriers.  Step k of the elimination costs two
// workgroup barriers: one to publish the pivot, one to publish the pivot row
// and the multipliers (double-buffered in LDS).  The step loop is split as
// k = TR * ks + kk with ks unrolled, so the row slot ks of the pivot row and
// its column slot (TR * ks) / TC are compile-time register indices.
#include "leaf.h"
#include "prof.h"
#include "tune.h"
#include "mfma_tile.h"
#include "wave_ops.h"

namespace hps {

// Pivot threshold of a leaf system: tol * max|A_ii| over the workgroup (every
// thread passes its largest magnitude; all threads get the threshold), or 0
// when tol is 0 (then only exactly zero pivots are rejected).
__device__ inline double leaf_pivot_threshold(double mine, double tol, double* red) {
  if (!(tol > 0.0)) return 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mine = fmax(mine, __shfl_xor(mine, off));
  const int nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mine;
  __syncthreads();
  double m = 0.0;
  for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
  return tol * m;
}

template <int TR, int TC, int NR, int NC>
__global__ void __launch_bounds__(TR * TC) k_leaf_lu(const double* const* __restrict__ cptr,
                                                     const LeafDev tab, double* __restrict__ Z,
                                                     int* status, int tag0, double tol) {
  static_assert(TC % TR == 0, "column tile must be a multiple of the row tile");
  constexpr int NT = TR * TC;
  __shared__ double sD[4][24 * 24];
  __shared__ double sc[6][NR * TR];
  __shared__ double RowK[2][NC * TC], RowP[2][NC * TC], Lb[2][NR * TR];
  __shared__ double Ucol[2][NR * TR], Xr[2][NC * TC];
  __shared__ double dinv[NR * TR];
  __shared__ int pidx[2];
  __shared__ double pval[2];

  const int p = tab.p, n = tab.n, m = tab.m, pi = p - 2, w = n + m;
  const int tid = threadIdx.x, tr = tid % TR, tc = tid / TR;
  const double* cl = cptr[blockIdx.x];
  for (int e = tid; e < p * p; e += NT) {
    sD[0][e] = tab.Dx[e];
    sD[1][e] = tab.Dy[e];
    sD[2][e] = tab.Dxx[e];
    sD[3][e] = tab.Dyy[e];
  }
  for (int e = tid; e < 6 * n; e += NT) {
    int f = e / n, k = e % n;
    sc[f][k] = cl[(size_t)f * p * p + (1 + k % pi) + p * (1 + k / pi)];
  }
  __syncthreads();

  // ---- assembly (same formulas as the unfused path) ----
  double a[NR][NC];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = tr + TR * s;
    const bool rv = i < n;
    const int ia = rv ? 1 + i % pi : 1, ib = rv ? 1 + i / pi : 1;
    const double c11 = rv ? sc[0][i] : 0, c12 = rv ? sc[1][i] : 0, c22 = rv ? sc[2][i] : 0;
    const double c1 = rv ? sc[3][i] : 0, c2 = rv ? sc[4][i] : 0, c0 = rv ? sc[5][i] : 0;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int j = tc + TC * t;
      double v = 0.0;
      if (rv && j < n) {
        const int ja = 1 + j % pi, jb = 1 + j / pi;
        const double dx = sD[0][ia * p + ja], dy = sD[1][ib * p + jb];
        v = -2.0 * c12 * dx * dy;
        if (ib == jb) v += -c11 * sD[2][ia * p + ja] + c1 * dx;
        if (ia == ja) v += -c22 * sD[3][ib * p + jb] + c2 * dy;
        if (i == j) v += c0;
      } else if (rv && j < w) {
        const size_t o = (size_t)i * m + (j - n), st = (size_t)n * m;
        v = -c11 * tab.G[o] - 2.0 * c12 * tab.G[st + o] - c22 * tab.G[2 * st + o] +
            c1 * tab.G[3 * st + o] + c2 * tab.G[4 * st + o];
      }
      a[s][t] = v;
    }
  }
  __shared__ double sRed[16];
  double mine = 0.0;
#pragma unroll
  for (int s = 0; s < NR; ++s)
#pragma unroll
    for (int t = 0; t < NC; ++t)
      if (tr + TR * s < n && tc + TC * t < n) mine = fmax(mine, fabs(a[s][t]));
  const double thr = leaf_pivot_threshold(mine, tol, sRed);

  // ---- forward elimination with partial pivoting ----
#pragma unroll
  for (int ks = 0; ks < NR; ++ks) {
      const int ts = (TR * ks) / TC;
    for (int kk = 0; kk < TR; ++kk) {
      const int k = TR * ks + kk;
      if (k >= n) break;
      const int buf = k & 1;
      const int tck = (TR * ks) % TC + kk;
      if (tc == tck) {
        double best = -1.0, bval = 0.0;
        int bidx = -1;
#pragma unroll
        for (int s = ks; s < NR; ++s) {
          const int i = tr + TR * s;
          const double v = a[s][ts];
          const double av = (v != v) ? INFINITY : fabs(v);
          if (i >= k && i < n && av > best) {
            best = av;
            bidx = i;
            bval = v;
          }
        }
#pragma unroll
        for (int off = TR / 2; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, TR);
          const double ov = __shfl_xor(bval, off, TR);
          const int oi = __shfl_xor(bidx, off, TR);
          if (oi >= 0 && (bidx < 0 || ob > best || (ob == best && oi < bidx))) {
            best = ob;
            bval = ov;
            bidx = oi;
          }
        }
        if (tr == 0) {
          pidx[buf] = bidx < 0 ? k : bidx;
          pval[buf] = bval;
        }
      }
      __syncthreads();
      // The pivot row is the same for the whole workgroup: keep it in scalar
      // registers so the slot selection below is a scalar branch.
      const int pr = __builtin_amdgcn_readfirstlane(pidx[buf]);
      const double piv = pval[buf];
      const int trp = pr % TR, sp = pr / TR;
      if (tr == kk) {
#pragma unroll
        for (int t = 0; t < NC; ++t) RowK[buf][tc + TC * t] = a[ks][t];
      }
#pragma unroll
      for (int s = 0; s < NR; ++s)
        if (s == sp) {
          if (tr == trp) {
#pragma unroll
            for (int t = 0; t < NC; ++t) RowP[buf][tc + TC * t] = a[s][t];
          }
        }
      const double inv = (piv != 0.0 && piv == piv) ? 1.0 / piv : 0.0;
      // Multipliers of every row slot s >= ks (zero for rows <= k and padding
      // rows), so the update below needs no row or column masks: rows <= k are
      // left unchanged, and column k of the rows below becomes exactly 0.
      if (tc == tck) {
#pragma unroll
        for (int s = ks; s < NR; ++s) {
          const int i = tr + TR * s;
          double l = (i > k && i < n && i != pr) ? a[s][ts] * inv : 0.0;
          Lb[buf][i] = l;
        }
        if (tr == kk && pr != k) Lb[buf][pr] = a[ks][ts] * inv;  // old row k moves to pr
        if (tr == 0) dinv[k] = inv;
      }
      if (tid == 0 && (piv == 0.0 || piv != piv || fabs(piv) <= thr))
        if (atomicCAS(status, 0, 1) == 0) status[1] = tag0 - (int)blockIdx.x;
      __syncthreads();
      if (pr != k) {
        // Row k takes the pivot row, row pr takes the old row k.
        if (tr == kk) {
#pragma unroll
          for (int t = 0; t < NC; ++t) a[ks][t] = RowP[buf][tc + TC * t];
        }
#pragma unroll
        for (int s = 0; s < NR; ++s)
          if (s == sp) {
            if (tr == trp) {
#pragma unroll
              for (int t = 0; t < NC; ++t) a[s][t] = RowK[buf][tc + TC * t];
            }
          }
      }
#pragma unroll
      for (int t = ts; t < NC; ++t) {
        const double ut = RowP[buf][tc + TC * t];
#pragma unroll
        for (int s = ks; s < NR; ++s) a[s][t] = fma(-Lb[buf][tr + TR * s], ut, a[s][t]);
      }
    }
  }

  // ---- back substitution on the right-hand-side columns ----
  // Row k's RHS entries are final once rows > k are done; x_k = y_k / u_kk,
  // then y_i -= u_ik x_k for i < k.
  __syncthreads();
#pragma unroll
  for (int ks = NR - 1; ks >= 0; --ks) {
    const int ts = (TR * ks) / TC;
    for (int kk = TR - 1; kk >= 0; --kk) {
      const int k = TR * ks + kk;
      if (k >= n) continue;
      const int buf = k & 1;
      const int tck = (TR * ks) % TC + kk;
      if (tr == kk) {
        const double di = dinv[k];
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const int j = tc + TC * t;
          if (j >= n && j < w) {
            a[ks][t] *= di;
            Xr[buf][j - n] = a[ks][t];
          }
        }
      }
      if (tc == tck) {
#pragma unroll
        for (int s = 0; s <= ks; ++s) {
          const int i = tr + TR * s;
          if (i < k) Ucol[buf][i] = a[s][ts];
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s <= ks; ++s) {
        const int i = tr + TR * s;
        if (i < k) {
          const double uk = Ucol[buf][i];
#pragma unroll
          for (int t = 0; t < NC; ++t) {
            const int j = tc + TC * t;
            if (j >= n && j < w) a[s][t] -= uk * Xr[buf][j - n];
          }
        }
      }
    }
  }

  // ---- Z out: [n][m] per leaf ----
  double* Zl = Z + (size_t)blockIdx.x * n * m;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = tr + TR * s;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int j = tc + TC * t;
      if (i < n && j >= n && j < w) Zl[(size_t)i * m + (j - n)] = a[s][t];
    }
  }
}

// ---------------------------------------------------------------------------
// Gauss-Jordan leaf solve with one workgroup barrier per column.  Same result
// as k_leaf_lu (Z = A_ii^-1 R) without its back substitution.
//
// Register layout: thread (tr, tc) = (tid % 16, tid / 16) holds rows
// i = tr + 16 s (s < NR) and the NC consecutive columns j = NC tc + t
// (t < NC).  The 16 threads of one tc are one DPP row (16 lanes) of a wave,
// so column k lives in a single DPP row and row i's values in the columns of
// any tc live in that tc's DPP row.
//
// Column k (owner tc = k / NC): the owner lanes store the column a[., k]
// to LDS and find the pivot row p with a DPP max (rows stay in place; chosen
// rows are only marked); that and one barrier is all the serial work of a
// column.  After the barrier every thread reads a[p][k], fetches row p's
// values for its own columns from lane p % 16 of its DPP row and scales them
// by 1 / a[p][k] (giving r_j = a[p][j] / a[p][k], row p's new values), and
// applies a[i][j] -= a[i][k] r_j, which eliminates column k from every other
// row (above and below: Gauss-Jordan); the lane holding row p then stores
// r_j in it.  Threads whose columns all precede k + 1 have nothing left to
// update.  After the last column, row p_k holds row k of A_ii^-1 R in its
// right-hand-side columns.
// ---------------------------------------------------------------------------

// Search key of a pivot candidate: the high word of |v| (exponent and the
// top 20 mantissa bits, an order-preserving image of |v|) with the low 8
// bits replaced by 255 - slot, so one unsigned max gives the largest
// magnitude (to 2^-12 relative) and its place.  NaN sorts above every
// number and is then reported as a bad pivot.  Every slot gives a nonzero
// key (slots are below 256 - 48).
__device__ inline unsigned leaf_key(double v, int slot) {
  const unsigned hi = (unsigned)(__double_as_longlong(v) >> 32) & 0x7FFFFFFFu;
  return (hi & ~255u) | (unsigned)(255 - slot);
}

// Max over the 16 lanes of a DPP row (all 16 must be active).
__device__ inline unsigned row16_max(unsigned k) {
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x124, 0xF, 0xF, false));  // row_ror:4
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x128, 0xF, 0xF, false));  // row_ror:8
  return k;
}

template <int TC, int NR, int NC>
__global__ void __launch_bounds__(16 * TC) k_leaf_gj(const double* const* __restrict__ cptr,
                                                     const LeafDev tab, double* __restrict__ Z,
                                                     int* status, int tag0, double tol) {
  constexpr int TR = 16, NT = TR * TC, NROW = NR * TR;
  static_assert(NROW <= 208, "pivot keys hold slots below 208");
  __shared__ double sD[4][24 * 24];
  __shared__ double sc[6][NROW];
  // The current column a[., k], stored by row slot: row tr + 16 s at
  // sA[buf][tr][s], so that every lane reads its NR values as one
  // contiguous run (rows padded to an odd count of doubles against bank
  // conflicts).
  constexpr int NRP = NR | 1;
  __shared__ double sA[2][TR][NRP];
  __shared__ int sP[2];           // its pivot row
  __shared__ int sInv[NROW];      // row -> column whose pivot it is
  __shared__ double sRowP[TC][NC];  // the pivot row's values, one line per DPP row

  const int p = tab.p, n = tab.n, m = tab.m, pi = p - 2, w = n + m;
  const int tid = threadIdx.x, tr = tid % TR, tc = tid / TR;
  const int lane = tid & 63, rowlane = lane & ~15;
  const double* cl = cptr[blockIdx.x];
  for (int e = tid; e < p * p; e += NT) {
    sD[0][e] = tab.Dx[e];
    sD[1][e] = tab.Dy[e];
    sD[2][e] = tab.Dxx[e];
    sD[3][e] = tab.Dyy[e];
  }
  for (int e = tid; e < 6 * n; e += NT) {
    int f = e / n, k = e % n;
    sc[f][k] = cl[(size_t)f * p * p + (1 + k % pi) + p * (1 + k / pi)];
  }
  __syncthreads();

  // ---- assembly of [A_ii | R] (same formulas as k_leaf_lu) ----
  double a[NR][NC];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = tr + TR * s;
    const bool rv = i < n;
    const int ia = rv ? 1 + i % pi : 1, ib = rv ? 1 + i / pi : 1;
    const double c11 = rv ? sc[0][i] : 0, c12 = rv ? sc[1][i] : 0, c22 = rv ? sc[2][i] : 0;
    const double c1 = rv ? sc[3][i] : 0, c2 = rv ? sc[4][i] : 0, c0 = rv ? sc[5][i] : 0;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int j = NC * tc + t;
      double v = 0.0;
      if (rv && j < n) {
        const int ja = 1 + j % pi, jb = 1 + j / pi;
        const double dx = sD[0][ia * p + ja], dy = sD[1][ib * p + jb];
        v = -2.0 * c12 * dx * dy;
        if (ib == jb) v += -c11 * sD[2][ia * p + ja] + c1 * dx;
        if (ia == ja) v += -c22 * sD[3][ib * p + jb] + c2 * dy;
        if (i == j) v += c0;
      } else if (rv && j < w) {
        const size_t o = (size_t)i * m + (j - n), st = (size_t)n * m;
        v = -c11 * tab.G[o] - 2.0 * c12 * tab.G[st + o] - c22 * tab.G[2 * st + o] +
            c1 * tab.G[3 * st + o] + c2 * tab.G[4 * st + o];
      }
      a[s][t] = v;
    }
  }

  __shared__ double sRed[16];
  double mine = 0.0;
#pragma unroll
  for (int s = 0; s < NR; ++s)
#pragma unroll
    for (int t = 0; t < NC; ++t)
      if (tr + TR * s < n && NC * tc + t < n) mine = fmax(mine, fabs(a[s][t]));
  const double thr = leaf_pivot_threshold(mine, tol, sRed);

  // Rows already chosen as pivots (bit s: row tr + 16 s); padding rows count as chosen.
  unsigned done = 0;
#pragma unroll
  for (int s = 0; s < NR; ++s)
    if (tr + TR * s >= n) done |= 1u << s;

  const int nblk = (n + NC - 1) / NC;
  for (int kb = 0; kb < nblk; ++kb) {
    // Constant trip count over the block's columns (t is a register index).
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int k = NC * kb + t;
      if (k >= n) continue;
      const int buf = k & 1;
      if (tc == kb) {
        unsigned key = 0;
#pragma unroll
        for (int s = 0; s < NR; ++s) {
          sA[buf][tr][s] = a[s][t];
          if (!((done >> s) & 1u)) key = max(key, leaf_key(a[s][t], TR * s + tr));
        }
        key = row16_max(key);
        if (tr == 0) {
          const int slot = 255 - (int)(key & 255u);
          sP[buf] = slot;
          sInv[slot] = k;
        }
      }
      __syncthreads();
      const int slot = __builtin_amdgcn_readfirstlane(sP[buf]);
      const int sp = slot / TR, trp = slot % TR;
      if (tr == trp) done |= 1u << sp;
      const double piv = sA[buf][slot % TR][slot / TR];
      const bool ok = (piv != 0.0) && (piv == piv) && fabs(piv) != INFINITY && fabs(piv) > thr;
      if (!ok && tid == 0)
        if (atomicCAS(status, 0, 1) == 0) status[1] = tag0 - (int)blockIdx.x;
      // Columns of this thread that are still to be updated: j > k.
      if (NC * tc + NC - 1 > k) {
        const double inv = ok ? recip(piv) : 0.0;
        // Row p's values in my columns (lane trp of my DPP row, slot sp),
        // divided by the pivot.
        // Lane trp of each DPP row stores row p's values of its columns to
        // the row's LDS line, which the row's lanes read back: all within
        // one wave, whose LDS operations complete in program order.
        if (tr == trp) {
#pragma unroll
          for (int s = 0; s < NR; ++s)
            if (s == sp) {
#pragma unroll
              for (int t2 = 0; t2 < NC; ++t2) sRowP[tc][t2] = a[s][t2];
            }
        }
        __builtin_amdgcn_wave_barrier();
        double prow[NC];
#pragma unroll
        for (int t2 = 0; t2 < NC; ++t2) prow[t2] = sRowP[tc][t2] * inv;
#pragma unroll
        for (int s = 0; s < NR; ++s) {
          const double lv = sA[buf][tr][s];
#pragma unroll
          for (int t2 = 0; t2 < NC; ++t2) a[s][t2] = fma(-lv, prow[t2], a[s][t2]);
        }
        if (tr == trp) {
#pragma unroll
          for (int s = 0; s < NR; ++s)
            if (s == sp) {
#pragma unroll
              for (int t2 = 0; t2 < NC; ++t2) a[s][t2] = prow[t2];
            }
        }
      }
    }
  }

  // ---- Z out: row p_k holds row k of A_ii^-1 R ----
  double* Zl = Z + (size_t)blockIdx.x * n * m;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = tr + TR * s;
    if (i >= n) continue;
    const int k = sInv[i];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int j = NC * tc + t;
      if (j >= n && j < w) Zl[(size_t)k * m + (j - n)] = a[s][t];
    }
  }
}

// ---------------------------------------------------------------------------
// Leaf solve and DtN on FP64 MFMA (sections 3.1-3.2): blocked Gauss-Jordan on
// W = [A_ii | R] (R = A_ie L1) with partial pivoting, rank-16 updates on
// v_mfma_f64_16x16x4f64, and T = P0 - P1 Z formed before the leaf leaves the
// CU (Z = A_ii^-1 R never goes to memory).
//
// W is padded to NR = 16 NTI rows and 16 (NTI + NTR) columns: padding rows and
// columns of A_ii are identity, padding of R is zero.  Tile wave ti (< NTI)
// holds row tile ti of W as NTI + NTR 16 x 16 MFMA accumulator tiles (lane l,
// register r: row 16 ti + l/16 + 4r, column l%16 of the tile); wave NTI is the
// panel wave.  Rows stay in place; a row chosen as a pivot is only marked.
//
// Step k eliminates the columns of block K = [16k, 16k + 16).  With P the 16
// rows chosen as pivots and B = W[P, K], Gauss-Jordan takes W[P] to B^-1 W[P]
// and every other row i to W[i] - W[i, K] B^-1 W[P]:
//   1. the tile waves store their block-K tiles (the panel X) to LDS;
//   2. the panel wave runs in-place Gauss-Jordan with partial pivoting on X
//      (candidates: rows not chosen at an earlier step; every row is
//      eliminated, earlier pivot rows included).  Column c of X ends up
//      holding the multipliers of column c's step, so X becomes Z = E[:, P],
//      the columns P of the step's elimination matrix E: Z[P] = B^-1 and
//      Z[i] = -W[i, K] B^-1 elsewhere;
//   3. each tile wave loads its rows of Z (in the MFMA A-operand layout),
//      stages the chosen rows' values W[P, :] that it holds and sets those
//      rows to zero;
//   4. every tile (ti, tj) with tj past block K gets C += Z(ti) W[P, tj]
//      (four MFMAs): the chosen rows become B^-1 W[P] from zero, with no
//      cancellation between a row and its own update; block K itself is
//      finished (it is not needed again).
// After the last step row p of the R block holds row j of A_ii^-1 R, where p
// is the pivot row of column j; the R block is staged in LDS in the order of
// j, and T = P0 - P1 (A_ii^-1 R) is one more MFMA product.
// Pivot search keys compare magnitudes rounded to float (ties to the lowest
// row), so a pivot may differ from exact partial pivoting among candidates
// within 2^-11 of each other; the results agree to rounding.
// ---------------------------------------------------------------------------
constexpr int LMF_XS = 17;  // LDS row stride of 16-wide blocks (odd: spreads banks)

template <int NTI, int NTR>
struct LeafMfmaShape {
  static constexpr int NR = 16 * NTI;           // padded rows (and A_ii columns)
  static constexpr int NTC = NTI + NTR;         // column tiles of W
  static constexpr int NC = 16 * NTC;
  static constexpr int NS = (NR + 63) / 64;     // row slots per lane of the panel wave
  static constexpr int NW = NTI + 1;            // waves
  static constexpr int LDR = 16 * NTR + 1;      // row stride of the staged R block
  // LDS doubles: panel X, rows of Z, staged pivot rows (rows of W[P, :]);
  // the R block reuses the same space at the end.
  static constexpr int STEP = 2 * NR * LMF_XS + 16 * NC;
  static constexpr int TAIL = NR * LDR;
  static constexpr int BUF = STEP > TAIL ? STEP : TAIL;
};

template <int NTI, int NTR>
__global__ void __launch_bounds__(64 * (NTI + 1), 4) k_leaf_mfma(
    const double* const* __restrict__ cptr, const LeafDev tab, const double* __restrict__ P0,
    const double* __restrict__ P1, double* const* __restrict__ tdst, int* status, int tag0,
    double tol) {
  using S = LeafMfmaShape<NTI, NTR>;
  constexpr int NR = S::NR, NTC = S::NTC, NC = S::NC, NS = S::NS, XS = LMF_XS;
  __shared__ double sD[4][256];
  __shared__ double sc[6][NR];
  __shared__ double sbuf[S::BUF];
  __shared__ int sInv[NR];        // row -> column whose pivot it is
  __shared__ int sIdx[NR];        // interior node j -> (1 + j % (p-2)) | (1 + j / (p-2)) << 8
  __shared__ double sRed[S::NW];
  __shared__ double sPiv[16];     // the current pivot row (panel wave only)
  double* sX = sbuf;                      // [NR][XS] panel block
  double* sL = sbuf + NR * XS;            // [NR][XS] rows of Z (the step's multipliers)
  double* sWP = sbuf + 2 * NR * XS;       // [16][NC] the chosen rows' values

  const int p = tab.p, n = tab.n, m = tab.m, pi = p - 2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool panel_wave = wid == NTI;
  const int ti = wid;
  const double* cl = cptr[blockIdx.x];
  for (int e = tid; e < p * p; e += 64 * S::NW) {
    sD[0][e] = tab.Dx[e];
    sD[1][e] = tab.Dy[e];
    sD[2][e] = tab.Dxx[e];
    sD[3][e] = tab.Dyy[e];
  }
  for (int e = tid; e < 6 * NR; e += 64 * S::NW) {
    const int f = e / NR, k = e % NR;
    sc[f][k] = k < n ? cl[(size_t)f * p * p + (1 + k % pi) + p * (1 + k / pi)] : 0.0;
  }
  for (int e = tid; e < NR; e += 64 * S::NW) {
    sInv[e] = 1 << 20;  // not chosen yet
    sIdx[e] = e < n ? (1 + e % pi) | ((1 + e / pi) << 8) : 0;
  }
  __syncthreads();

  // The panel wave and the tile waves run separate loops with the same
  // sequence of workgroup barriers (three per step), so neither keeps the
  // other's registers live.
  if (panel_wave) {
    __syncthreads();  // the tile waves' assembly (and their max|A_ii|)
    double thr = 0.0;
    if (tol > 0.0) {
      double mx = 0.0;
#pragma unroll
      for (int w = 0; w < NTI; ++w) mx = fmax(mx, sRed[w]);
      thr = uniform(tol * mx);
    }
    bool cand[NS];  // rows not chosen as a pivot yet
#pragma unroll
    for (int s = 0; s < NS; ++s) cand[s] = s * 64 + lane < NR;
    bool bad = false;
    for (int k = 0; k < NTI; ++k) {
      int chosen[NS];  // column of this step whose pivot the slot's row became, or -1
#pragma unroll
      for (int s = 0; s < NS; ++s) chosen[s] = -1;
      __syncthreads();  // (1) the panel block is in LDS
      double x[NS][16];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int row = s * 64 + lane;
#pragma unroll
        for (int c = 0; c < 16; ++c) x[s][c] = row < NR ? sX[row * XS + c] : 0.0;
      }
      // Rows are scaled lazily: the true row is scl * stored, a row chosen as
      // pivot keeps its stored values and takes scl = 1 / pivot, so a column
      // costs one FMA per entry and the pivot row needs no rewrite; the
      // scales are applied once after the 16 columns.  Candidates are never
      // scaled (scl = 1), so the search sees true magnitudes.
      double scl[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) scl[s] = 1.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        unsigned key = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          key = cand[s] ? max(key, pivot_key(x[s][c], s * 64 + lane)) : key;
        const unsigned g = wave_max_u32(key);
        // Every step leaves at least 16 candidates (NR - 16 k rows), so g != 0.
        const int slot = 4095 - (int)(g & 4095u);
        const int gs = slot >> 6, gl = slot & 63;
        // The pivot row (all 16 columns: those left of c hold its multipliers
        // of earlier columns, which Gauss-Jordan carries along) goes through
        // LDS: lane gl of slot gs (gs is the same for the whole wave) writes
        // it and every lane reads it back, so it stays in vector registers
        // (as 32 readlanes it filled the scalar registers, which spilled).
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (gs == s && lane == gl) {
#pragma unroll
            for (int c2 = 0; c2 < 16; ++c2) sPiv[c2] = x[s][c2];
          }
        wave_lds_sync();
        double prow[16];
#pragma unroll
        for (int c2 = 0; c2 < 16; ++c2) prow[c2] = sPiv[c2];
        bool mine[NS];  // this lane's slot s holds the pivot row
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          mine[s] = gs == s && lane == gl;
          cand[s] = cand[s] && !mine[s];  // chosen: no longer a candidate
          chosen[s] = mine[s] ? 16 * k + c : chosen[s];
        }
        const double piv = prow[c];
        const bool ok = g != 0 && piv != 0.0 && piv == piv && fabs(piv) != INFINITY &&
                        fabs(piv) > thr;
        bad |= !ok;
        const double inv = uniform(ok ? recip(piv) : 0.0);
        // Gauss-Jordan step on column c: every other row loses f times the
        // scaled pivot row and column c takes the multipliers (-f / pivot);
        // the pivot row keeps its values (1 in column c) and its scale
        // becomes 1 / pivot.  In stored form the update does not depend on a
        // row's scale.
        double f[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) f[s] = mine[s] ? 0.0 : x[s][c];
#pragma unroll
        for (int c2 = 0; c2 < 16; ++c2)
          if (c2 != c) {
            const double pr = prow[c2] * inv;
#pragma unroll
            for (int s = 0; s < NS; ++s) x[s][c2] = fma(-f[s], pr, x[s][c2]);
          }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          x[s][c] = mine[s] ? 1.0 : -f[s] * inv;
          scl[s] = mine[s] ? inv : scl[s];
        }
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c2 = 0; c2 < 16; ++c2) x[s][c2] *= scl[s];
      // Pivot marks of this step (read by the tile waves after barrier 2).
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (chosen[s] >= 0) sInv[s * 64 + lane] = chosen[s];
      // Row i of the panel now holds row i of Z = E[:, P]: the update is
      // W_new = W + Z W[P] with the chosen rows W[P] set to zero first.
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int row = s * 64 + lane;
        if (row < NR) {
#pragma unroll
          for (int c2 = 0; c2 < 16; ++c2) sL[row * XS + c2] = x[s][c2];
        }
      }
      __syncthreads();  // (2) factors out
      __syncthreads();  // (3) the chosen rows' values are staged
    }
    if (bad && lane == 0)
      if (atomicCAS(status, 0, 1) == 0) status[1] = tag0 - (int)blockIdx.x;
    __syncthreads();  // before the tile waves reuse the step buffers for R
  } else {
    // ---- assembly of row tile ti of A_ii (formulas of k_leaf_lu); the R
    // tiles are assembled during step 0's panel, when this wave waits ----
    d4 acc[NTC];
    double mine = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // One row at a time: keeps the assembly's temporaries from piling up
      // on top of the accumulator tiles.
      __builtin_amdgcn_sched_barrier(0);
      const int i = 16 * ti + (lane >> 4) + 4 * r;
      const bool rv = i < n;
      const int ii = sIdx[i], ia = ii & 255, ib = ii >> 8;
      const double c11 = sc[0][i], c12 = sc[1][i], c22 = sc[2][i];
      const double c1 = sc[3][i], c2 = sc[4][i], c0 = sc[5][i];
#pragma unroll
      for (int tj = 0; tj < NTI; ++tj) {
        const int j = 16 * tj + (lane & 15);
        double v = 0.0;
        if (rv && j < n) {
          const int jj = sIdx[j], ja = jj & 255, jb = jj >> 8;
          const double dx = sD[0][ia * p + ja], dy = sD[1][ib * p + jb];
          v = -2.0 * c12 * dx * dy;
          if (ib == jb) v += -c11 * sD[2][ia * p + ja] + c1 * dx;
          if (ia == ja) v += -c22 * sD[3][ib * p + jb] + c2 * dy;
          if (i == j) v += c0;
          mine = fmax(mine, fabs(v));
        } else if (i == j) {
          v = 1.0;  // padding: identity
        }
        acc[tj][r] = v;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine = fmax(mine, __shfl_xor(mine, off));
    if (lane == 0) sRed[wid] = mine;
    __syncthreads();

    for (int k = 0; k < NTI; ++k) {
      // (1) the panel block to LDS
#pragma unroll
      for (int tj = 0; tj < NTI; ++tj)
        if (tj == k) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            sX[(16 * ti + (lane >> 4) + 4 * r) * XS + (lane & 15)] = acc[tj][r];
        }
      __syncthreads();
      if (k == 0) {
        // R = A_ie L1 (five coefficient-free tables weighted by the row's
        // coefficients), overlapping the first panel.
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          __builtin_amdgcn_sched_barrier(0);  // one row's loads in flight at a time
          const int i = 16 * ti + (lane >> 4) + 4 * r;
          const bool rv = i < n;
          const double c11 = sc[0][i], c12 = sc[1][i], c22 = sc[2][i];
          const double c1 = sc[3][i], c2 = sc[4][i];
#pragma unroll
          for (int tr = 0; tr < NTR; ++tr) {
            const int jr = 16 * tr + (lane & 15);
            double v = 0.0;
            if (rv && jr < m) {
              const size_t o = (size_t)i * m + jr, st = (size_t)n * m;
              v = -c11 * tab.G[o] - 2.0 * c12 * tab.G[st + o] - c22 * tab.G[2 * st + o] +
                  c1 * tab.G[3 * st + o] + c2 * tab.G[4 * st + o];
            }
            acc[NTI + tr][r] = v;
          }
        }
      }
      __syncthreads();  // (2) the panel wave's factors
      // (3) this row tile's rows of Z (the A operands of the update) and the
      // chosen rows' values held by this wave
      double la[4];
#pragma unroll
      for (int st = 0; st < 4; ++st)
        la[st] = sL[(16 * ti + (lane & 15)) * XS + 4 * st + (lane >> 4)];
      int cr[4];  // column of this step whose pivot each of my rows is, or -1
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = sInv[16 * ti + (lane >> 4) + 4 * r] - 16 * k;
        cr[r] = (c >= 0 && c < 16) ? c : -1;
      }
#pragma unroll
      for (int tj = 0; tj < NTC; ++tj)
        if (tj > k) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (cr[r] >= 0) {
              sWP[cr[r] * NC + 16 * tj + (lane & 15)] = acc[tj][r];
              acc[tj][r] = 0.0;  // the update then writes B^-1 W[P, :] into this row
            }
        }
      __syncthreads();
      // (4) rank-16 update of every tile right of block K
#pragma unroll
      for (int tj = 0; tj < NTC; ++tj)
        if (tj > k) {
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const double b = sWP[(4 * st + (lane >> 4)) * NC + 16 * tj + (lane & 15)];
            acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[st], b, acc[tj], 0, 0, 0);
          }
          // Tile by tile: the next tile's operand loads are not hoisted above
          // this one's products (they would not fit next to the accumulators).
          __builtin_amdgcn_sched_barrier(0);
        }
    }
    // The R block to LDS for T, row j of A_ii^-1 R (held by the pivot row
    // of column j) at row j.
    __syncthreads();  // every wave is done with the step buffers
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = sInv[16 * ti + (lane >> 4) + 4 * r];
#pragma unroll
      for (int tr = 0; tr < NTR; ++tr) sbuf[j * S::LDR + 16 * tr + (lane & 15)] = acc[NTI + tr][r];
    }
  }
  __syncthreads();  // the R block is staged

  // ---- T = P0 - P1' W_R ----
  const double* sR = sbuf;  // [NR][LDR]
  double* T = tdst[blockIdx.x];
  for (int tt = wid; tt < NTR * NTR; tt += S::NW) {
    const int ta = tt / NTR, tb = tt % NTR;
    const int trow = 16 * ta + (lane & 15);
    // P1 operands a chunk at a time, the chunk's loads in flight together
    // (clamped addresses and a select, no branches), then its products.
    constexpr int KS = NR / 4, CH = (KS + 1) / 2;
    const int tr_c = min(trow, m - 1);
    d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < KS; k0 += CH) {
      double af[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int kk = 4 * (k0 + j) + (lane >> 4);
        const double v = as_global(P1)[(size_t)tr_c * n + min(kk, n - 1)];
        af[j] = (k0 + j < KS && trow < m && kk < n) ? v : 0.0;
      }
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (k0 + j < KS) {
          const int kk = 4 * (k0 + j) + (lane >> 4);
          const double b = sR[kk * S::LDR + 16 * tb + (lane & 15)];
          t = __builtin_amdgcn_mfma_f64_16x16x4f64(af[j], b, t, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ta + (lane >> 4) + 4 * r, col = 16 * tb + (lane & 15);
      if (row < m && col < m) T[(size_t)row * m + col] = P0[(size_t)row * m + col] - t[r];
    }
  }
}

static bool g_leaf_mfma = true;
static int g_leaf_variant = -1;  // -1: default choice; else forced leaf_lu variant index

void leaf_set_mfma(bool on) { g_leaf_mfma = on; }

bool leaf_mfma_fits(int n, int m) {
  const int nti = (n + 15) / 16, ntr = (m + 15) / 16;
  // A forced leaf_lu variant (leaf_variant knob) selects the older kernels.
  return g_leaf_mfma && g_leaf_variant < 0 && ((nti == 7 && ntr == 3) || (nti == 4 && ntr == 2) ||
                         (nti == 3 && ntr == 2) || (nti == 1 && ntr == 1) ||
                         (nti == 2 && ntr == 2) || (nti == 5 && ntr == 2) ||
                         (nti == 6 && ntr == 3));
}

void leaf_dtn_mfma(const double* const* cptr, const LeafDev& tab, const double* P0,
                   const double* P1, double* const* tdst, int count, int* status, int tag0,
                   hipStream_t s, double tol) {
  const double n = tab.n, m = tab.m;
  ProfScope ps(PROF_LEAF_LU, s, count * (2.0 * n * n * n / 3.0 + 2.0 * n * n * m + 2.0 * m * m * n),
               8.0 * count * (6.0 * tab.p * tab.p + m * m));
  const int nti = (tab.n + 15) / 16, ntr = (tab.m + 15) / 16;
#define HPS_LMF(A, B)                                                                           \
  if (nti == A && ntr == B) {                                                                   \
    hipLaunchKernelGGL((k_leaf_mfma<A, B>), dim3(count), dim3(64 * (A + 1)), 0, s, cptr, tab, P0, \
                       P1, tdst, status, tag0, tol);                                            \
    return;                                                                                     \
  }
  HPS_LMF(7, 3)
  HPS_LMF(4, 2)
  HPS_LMF(3, 2)
  HPS_LMF(1, 1)
  HPS_LMF(2, 2)
  HPS_LMF(5, 2)
  HPS_LMF(6, 3)
#undef HPS_LMF
  HPS_REQUIRE(false, "leaf shape without an MFMA leaf kernel");
}

// Register variants: rows <= NR*TR, columns (n + m) <= NC*TC.
bool leaf_lu_fits(int n, int m) {
  return (n <= 13 * 16 && n + m <= 8 * 32) || (n <= 7 * 16 && n + m <= 9 * 16);
}

void leaf_lu_set_variant(int v) { g_leaf_variant = v; }

void leaf_lu(const double* const* cptr, const LeafDev& tab, int count, double* Z, int* status,
             int tag0, hipStream_t s, double tol) {
  const double n = tab.n, m = tab.m;
  ProfScope ps(PROF_LEAF_LU, s, count * (2.0 * n * n * n / 3.0 + 2.0 * n * n * m), 0);
  const bool small = tab.n <= 7 * 16 && tab.n + tab.m <= 9 * 16;
  // Variants: 0-2 step-by-step LU (k_leaf_lu), 3-4 blocked Gauss-Jordan (k_leaf_gj).
  int v = g_leaf_variant >= 0 ? g_leaf_variant : tune_get(TUNE_LEAF, tab.n, tab.m, 0, 0);
  if (v < 0) v = small ? 3 : 4;
  if ((v == 0 || v == 3) && !small) v = (v == 0) ? 1 : 4;
  switch (v) {
    case 0:
      hipLaunchKernelGGL((k_leaf_lu<16, 16, 7, 9>), dim3(count), dim3(256), 0, s, cptr, tab, Z,
                         status, tag0, tol);
      break;
    case 1:
      hipLaunchKernelGGL((k_leaf_lu<16, 64, 13, 4>), dim3(count), dim3(1024), 0, s, cptr, tab, Z,
                         status, tag0, tol);
      break;
    case 2:
      hipLaunchKernelGGL((k_leaf_lu<16, 32, 13, 8>), dim3(count), dim3(512), 0, s, cptr, tab, Z,
                         status, tag0, tol);
      break;
    case 3:
      hipLaunchKernelGGL((k_leaf_gj<16, 7, 9>), dim3(count), dim3(256), 0, s, cptr, tab, Z, status,
                         tag0, tol);
      break;
    default:
      hipLaunchKernelGGL((k_leaf_gj<32, 13, 8>), dim3(count), dim3(512), 0, s, cptr, tab, Z,
                         status, tag0, tol);
      break;
  }
}

}  // namespace hps
