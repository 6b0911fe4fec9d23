// Problem-specific kernels: leaf assembly (section 3), merge gather
// (section 4), downward pass (Algorithm 2), interface residual and the
// upward source pass used by iterative refinement.
#include "mfma_tile.h"
#include "ops.h"
#include "prof.h"
#include "wave_ops.h"
#include "grid_sync.h"

#include <algorithm>
#include <mutex>

namespace hps {

// ---------------------------------------------------------------------------
// Leaf assembly (section 3.1): for every leaf build the augmented system
// W = [A_ii | R], R = A_ie L1, with n = (p-2)^2 rows and ld = n + 4q.
// A_ii[k][k'] with k = (a, b), k' = (a', b') interior:
//   -c11 Dxx[a][a'] d_bb' - 2 c12 Dx[a][a'] Dy[b][b'] - c22 Dyy[b][b'] d_aa'
//   + c1 Dx[a][a'] d_bb' + c2 Dy[b][b'] d_aa' + c d_kk'
// R[k][:] = -c11 G11[k] - 2 c12 G12[k] - c22 G22[k] + c1 G1[k] + c2 G2[k].
// With a body load the system is W = [A_ii | G] instead (ld = n + nrhs): G
// holds the load of every right-hand side at the leaf's interior nodes.  For
// the kept body operator it is W = [A_ii^T | P1^T] (ld = n + m), whose
// solution is (P1 A_ii^-1)^T.
// ---------------------------------------------------------------------------
constexpr int PMAX = 24;

__global__ void __launch_bounds__(256) k_leaf_assemble(const double* const* __restrict__ cptr,
                                                       const LeafDev tab,
                                                       double* __restrict__ W,
                                                       const double* __restrict__ body, int nrhs,
                                                       int nl, int leaf0,
                                                       const double* __restrict__ P1) {
  __shared__ double Dx[PMAX * PMAX], Dy[PMAX * PMAX], Dxx[PMAX * PMAX], Dyy[PMAX * PMAX];
  __shared__ double cf[6][(PMAX - 2) * (PMAX - 2)];
  const int p = tab.p, n = tab.n, m = tab.m, pi = p - 2;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    Dx[e] = tab.Dx[e];
    Dy[e] = tab.Dy[e];
    Dxx[e] = tab.Dxx[e];
    Dyy[e] = tab.Dyy[e];
  }
  const double* cl = cptr[blockIdx.x];
  for (int e = threadIdx.x; e < 6 * n; e += blockDim.x) {
    int f = e / n, k = e % n;
    int a = 1 + k % pi, b = 1 + k / pi;
    cf[f][k] = cl[(size_t)f * p * p + a + p * b];
  }
  __syncthreads();
  const int ld = body ? n + nrhs : n + m;
  double* Wl = W + (size_t)blockIdx.x * n * ld;
  for (int e = threadIdx.x; e < n * ld; e += blockDim.x) {
    const int k = e / ld, col = e % ld;
    const double c11 = cf[0][k], c12 = cf[1][k], c22 = cf[2][k];
    const double c1 = cf[3][k], c2 = cf[4][k];
    double v;
    if (col < n) {
      // A_ii[i][j] (row i carries the coefficients); transposed for the body operator.
      const int i = P1 ? col : k, j = P1 ? k : col;
      const int a = 1 + i % pi, b = 1 + i / pi;
      const int a2 = 1 + j % pi, b2 = 1 + j / pi;
      const double dx = Dx[a * p + a2], dy = Dy[b * p + b2];
      v = -2.0 * cf[1][i] * dx * dy;
      if (b == b2) v += -cf[0][i] * Dxx[a * p + a2] + cf[3][i] * dx;
      if (a == a2) v += -cf[2][i] * Dyy[b * p + b2] + cf[4][i] * dy;
      if (i == j) v += cf[5][i];
    } else if (P1) {  // P1^T[k][col - n]
      v = P1[(size_t)(col - n) * n + k];
    } else if (body) {  // load of right-hand side col - n at interior node k
      const int a = 1 + k % pi, b = 1 + k / pi;
      v = body[((size_t)(col - n) * nl + leaf0 + blockIdx.x) * p * p + a + p * b];
    } else {
      const int c = col - n;
      const size_t o = (size_t)k * m + c, s = (size_t)n * m;
      v = -c11 * tab.G[o] - 2.0 * c12 * tab.G[s + o] - c22 * tab.G[2 * s + o] +
          c1 * tab.G[3 * s + o] + c2 * tab.G[4 * s + o];
    }
    Wl[e] = v;
  }
}

void leaf_assemble(const double* const* cptr, const LeafDev& tab, int count, double* W,
                   hipStream_t s) {
  HPS_REQUIRE(tab.p <= PMAX, "p too large");
  ProfScope ps(PROF_LEAF_ASSEMBLE, s, 0, 8.0 * count * ((double)tab.n * (tab.n + tab.m) + 6.0 * tab.p * tab.p));
  hipLaunchKernelGGL(k_leaf_assemble, dim3(count), dim3(256), 0, s, cptr, tab, W, nullptr, 0, 0,
                     0, nullptr);
}

void leaf_assemble_body_operator(const double* const* cptr, const LeafDev& tab, int count,
                                 double* W, const double* P1, hipStream_t s) {
  HPS_REQUIRE(tab.p <= PMAX, "p too large");
  ProfScope ps(PROF_LEAF_ASSEMBLE, s, 0,
               8.0 * count * ((double)tab.n * (tab.n + tab.m) + 6.0 * tab.p * tab.p));
  hipLaunchKernelGGL(k_leaf_assemble, dim3(count), dim3(256), 0, s, cptr, tab, W, nullptr, 0, 0,
                     0, P1);
}

void leaf_assemble_body(const double* const* cptr, const LeafDev& tab, int count, double* W,
                        const double* body, int nrhs, int nl, int leaf0, hipStream_t s) {
  HPS_REQUIRE(tab.p <= PMAX, "p too large");
  ProfScope ps(PROF_LEAF_ASSEMBLE, s, 0,
               8.0 * count * ((double)tab.n * (tab.n + nrhs) + 6.0 * tab.p * tab.p));
  hipLaunchKernelGGL(k_leaf_assemble, dim3(count), dim3(256), 0, s, cptr, tab, W, body, nrhs, nl,
                     leaf0, nullptr);
}

// Body loads: for leaves leaf0 .. leaf0 + count - 1, X = W + n (ld) holds the
// particular solutions w_i of every right-hand side ([n][nrhs]).  Writes
// their fluxes h = P1 w_i ([m][n] times [n][nrhs]) to
// hbuf[(hoff + leaf m) nrhs + k m + r] (the upward pass's per-box layout) and,
// when wpart is not null, w_i to wpart[k][leaf][i].
__global__ void __launch_bounds__(256) k_body_flux(const double* __restrict__ W, int n, int m,
                                                   int ld, int nrhs, const double* __restrict__ P1,
                                                   double* __restrict__ hbuf, long long hoff,
                                                   double* __restrict__ wpart, int nl, int leaf0) {
  const int leaf = leaf0 + blockIdx.x;
  const double* X = W + (size_t)blockIdx.x * n * ld + n;
  for (int e = threadIdx.x; e < nrhs * m; e += blockDim.x) {
    const int k = e / m, r = e % m;
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc = fma(P1[(size_t)r * n + c], X[(size_t)c * ld + k], acc);
    hbuf[(size_t)(hoff + (long long)leaf * m) * nrhs + (size_t)k * m + r] = acc;
  }
  if (wpart)
    for (int e = threadIdx.x; e < nrhs * n; e += blockDim.x) {
      const int k = e / n, i = e % n;
      wpart[((size_t)k * nl + leaf) * n + i] = X[(size_t)i * ld + k];
    }
}

void body_flux(const double* W, int count, int n, int m, int ld, int nrhs, const double* P1,
               double* hbuf, long long hoff, double* wpart, int nl, int leaf0, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_body_flux, dim3(count), dim3(256), 0, s, W, n, m, ld, nrhs, P1, hbuf, hoff,
                     wpart, nl, leaf0);
}

// Body loads with the kept operator: h = K g_i for every leaf and right-hand
// side, K^T = Kt [nl][n][m], g [nrhs][nl][p*p] read at the interior nodes.
// One workgroup per leaf: wave w takes a quarter of the interior nodes c,
// lane r the flux row r (64 rows per pass), so each step reads one row of
// K^T (up to 64 consecutive doubles) across the wave, eight rows in flight
// per lane; the four partial sums meet in LDS in a fixed order.  Up to BRC
// right-hand sides share each pass over K.
constexpr int BRC = 4;

__global__ void __launch_bounds__(256) k_body_flux_kept(const double* __restrict__ Kt,
                                                        const double* __restrict__ g, int nrhs,
                                                        int n, int m, int p, int nl,
                                                        double* __restrict__ hbuf,
                                                        long long hoff) {
  extern __shared__ double sh[];  // gi [BRC][n], then part [4][BRC][64]
  double* gi = sh;
  double* part = sh + BRC * n;
  const int leaf = blockIdx.x, pi = p - 2, pp = p * p;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double* K = Kt + (size_t)leaf * n * m;
  const int q4 = (n + 3) / 4, c0 = wid * q4, c1 = min(n, c0 + q4);
  for (int k0 = 0; k0 < nrhs; k0 += BRC) {
    const int nk = min(BRC, nrhs - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < nk * n; e += blockDim.x) {
      const int k = e / n, c = e % n;
      gi[e] = g[((size_t)(k0 + k) * nl + leaf) * pp + (1 + c % pi) + p * (1 + c / pi)];
    }
    for (int rb = 0; rb < m; rb += 64) {
      __syncthreads();
      const int r = rb + lane < m ? rb + lane : m - 1;
      double acc[BRC];
#pragma unroll
      for (int k = 0; k < BRC; ++k) acc[k] = 0.0;
      int c = c0;
      for (; c + 8 <= c1; c += 8) {
        double kv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) kv[t] = K[(size_t)(c + t) * m + r];
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
          for (int k = 0; k < BRC; ++k)
            if (k < nk) acc[k] = fma(kv[t], gi[k * n + c + t], acc[k]);
      }
      for (; c < c1; ++c) {
        const double kv = K[(size_t)c * m + r];
#pragma unroll
        for (int k = 0; k < BRC; ++k)
          if (k < nk) acc[k] = fma(kv, gi[k * n + c], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < BRC; ++k) part[(wid * BRC + k) * 64 + lane] = acc[k];
      __syncthreads();
      const int mr = min(64, m - rb);
      for (int e = threadIdx.x; e < nk * mr; e += blockDim.x) {
        const int k = e / mr, rr = e % mr;
        const double* ps = part + k * 64 + rr;
        const double v = ((ps[0] + ps[BRC * 64]) + ps[2 * BRC * 64]) + ps[3 * BRC * 64];
        const size_t o = (size_t)(hoff + (long long)leaf * m) * nrhs + (size_t)(k0 + k) * m;
        hbuf[o + rb + rr] = v;
      }
    }
  }
}

void body_flux_kept(const double* Kt, const double* g, int nrhs, int n, int m, int p, int nl,
                    double* hbuf, long long hoff, hipStream_t s) {
  const double cells = (double)nl * n * m;
  ProfScope ps(PROF_BODY_FLUX, s, 2.0 * nrhs * cells,
               8.0 * (cells + (double)nrhs * nl * (n + m)));
  const size_t lds = sizeof(double) * (BRC * n + 4 * BRC * 64);
  hipLaunchKernelGGL(k_body_flux_kept, dim3(nl), dim3(256), lds, s, Kt, g, nrhs, n, m, p, nl,
                     hbuf, hoff);
}

__global__ void __launch_bounds__(256) k_copy_rows(const double* const* src, double* const* dst,
                                                   int rows, int cols, int lds) {
  const double* a = src[blockIdx.x];
  double* b = dst[blockIdx.x];
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x)
    b[e] = a[(size_t)(e / cols) * lds + e % cols];
}

void copy_rows_batch(const double* const* src, double* const* dst, int count, int rows, int cols,
                     int lds, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy_rows, dim3(count), dim3(256), 0, s, src, dst, rows, cols, lds);
}

// uc[k][leaf][post_node[i]] += wpart[k][leaf][i] for the n interior rows.
__global__ void k_add_particular(double* __restrict__ uc, const double* __restrict__ wpart,
                                 const int* __restrict__ post_node, int n, int pp, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t kl = e / n;
    const int i = (int)(e % n);
    uc[kl * pp + post_node[i]] += wpart[e];
  }
}

void add_particular(double* uc, const double* wpart, const int* post_node, int n, int pp,
                    int nleaf, int nrhs, hipStream_t s) {
  const size_t count = (size_t)nrhs * nleaf * n;
  const int blocks = (int)std::min<size_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(k_add_particular, dim3(std::max(blocks, 1)), dim3(256), 0, s, uc, wpart,
                     post_node, n, pp, count);
}

// ---------------------------------------------------------------------------
// Merge gather (section 4, eq:premerge blocks): for each merge build
//   W = [T33a - T33b | I] (m3 x 2 m3), whose elimination leaves M^-1,
//   B = [-T31a, T32b]     (m3 x me, columns in parent order),
//   Q = [T13a; T23b]      (me x m3, rows in parent order),
// and record max|M| in the merge's pivot statistics.  The parent's
// diag(T11a, T22b) is not formed: the Schur product reads it from the
// children's DtNs as it writes T = diag(T11a, T22b) + Q S.
// ---------------------------------------------------------------------------
// Rows of W (m3), B (m3) and Q (me) are taken in turn by groups of LPR
// lanes (64 / LPR rows per wave, four waves per workgroup), each group
// walking its row in strides of LPR columns: the row's own lookups (a3, b3,
// pmap of the row) are one load per group, writes are contiguous, and no
// element index is divided.
template <int LPR>
__global__ void __launch_bounds__(256) k_merge_gather(const MergeDesc* __restrict__ descs) {
  const MergeDesc d = descs[blockIdx.y];
  const int m3 = d.m3, me = d.me, ldw = d.ldw;
  const int sub = threadIdx.x % LPR;
  constexpr int GROUPS = 256 / LPR;
  const int nrows = 2 * m3 + me;
  const gptr<double> Ta = as_global(d.Ta), Tb = as_global(d.Tb);
  const gptr<int> a3 = as_global(d.a3), b3 = as_global(d.b3), pmap = as_global(d.pmap);
  double amax = 0.0;
  for (int row = blockIdx.x * GROUPS + (int)threadIdx.x / LPR; row < nrows;
       row += gridDim.x * GROUPS) {
    if (row < m3) {
      // W row i = [T33a(i, :) - T33b(i, :) | e_i].
      const int i = row;
      const size_t ra = (size_t)a3[i] * d.na, rb = (size_t)b3[i] * d.nb;
      double* w = d.W + (size_t)i * ldw;
      for (int j = sub; j < ldw; j += LPR) {
        double v;
        if (j < m3) {
          v = Ta[ra + a3[j]] - Tb[rb + b3[j]];
          amax = fmax(amax, fabs(v));
        } else {
          v = (j - m3 == i) ? 1.0 : 0.0;
        }
        w[j] = v;
      }
    } else if (row < 2 * m3) {
      // B row i = [-T31a(i, :) | T32b(i, :)] in parent column order.
      const int i = row - m3;
      const size_t ra = (size_t)a3[i] * d.na, rb = (size_t)b3[i] * d.nb;
      double* bp = d.B + (size_t)i * me;
      for (int j = sub; j < me; j += LPR) {
        const int pm = pmap[j];
        bp[j] = pm >= 0 ? -Ta[ra + pm] : Tb[rb + (-pm - 1)];
      }
    } else {
      // Q row r = T13a(r, :) or T23b(r, :) (parent row order).
      const int r = row - 2 * m3;
      const int pm = pmap[r];
      double* qp = d.Q + (size_t)r * m3;
      if (pm >= 0) {
        const size_t ra = (size_t)pm * d.na;
        for (int j = sub; j < m3; j += LPR) qp[j] = Ta[ra + a3[j]];
      } else {
        const size_t rb = (size_t)(-pm - 1) * d.nb;
        for (int j = sub; j < m3; j += LPR) qp[j] = Tb[rb + b3[j]];
      }
    }
  }
  if (d.pstat) {
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
}

void merge_gather(const MergeDesc* d_desc, const std::vector<MergeDesc>& h_desc, hipStream_t s) {
  if (h_desc.empty()) return;
  int m3 = 0, me = 0;
  double bytes = 0;
  for (const MergeDesc& d : h_desc) {
    m3 = std::max(m3, d.m3);
    me = std::max(me, d.me);
    // Written: W (m3 x 2 m3), B, Q; read: two entries per M entry, one per B and Q entry.
    bytes += 8.0 * (4.0 * d.m3 * d.m3 + 4.0 * d.m3 * d.me);
  }
  const int rows = 2 * m3 + me;
  const int np = (int)h_desc.size();
  ProfScope ps(PROF_MERGE_GATHER, s, 0, bytes);
  // Lanes per row by the typical row length (rows of W are 2 m3 long, of B
  // me, of Q m3); workgroups per merge so that a level has about 4096
  // workgroups in all (many small merges: one workgroup walks a whole merge).
  const int typ = (2 * m3 * m3 + 2 * m3 * me) / std::max(rows, 1);
  const int cap = std::max(1, 4096 / np);
#define HPS_GATHER(LPR)                                                                      \
  {                                                                                          \
    const int gx = std::min((rows + 256 / LPR - 1) / (256 / LPR), cap);                      \
    hipLaunchKernelGGL(k_merge_gather<LPR>, dim3(gx, np), dim3(256), 0, s, d_desc);          \
  }
  if (typ <= 24)
    HPS_GATHER(16)
  else if (typ <= 48)
    HPS_GATHER(32)
  else
    HPS_GATHER(64)
#undef HPS_GATHER
}

// ---------------------------------------------------------------------------
// Small merges in one launch (section 4 for one merge, Algorithm 1 for a
// level): one workgroup per merge gathers M = T33a - T33b next to I in LDS,
// eliminates [M | I] by Gauss-Jordan with partial pivoting (rows stay in
// place, pivots are marked), forms S = M^-1 [-T31a | T32b] and
// T = diag(T11a, T22b) + [T13a; T23b] S on FP64 MFMA, with the right-hand
// sides and Q gathered from the children's DtNs as operand fragments.  Only
// S and T (and, with the factors kept, M^-1 and Q) reach HBM.  The same
// statistics as the level-wise path: max|M| and the smallest pivot, and a
// zero or non-finite pivot in status (tag: the merge's box).
// LDS: Wl [m3][2 m3 + 1] and Sl [m3][me + 1] doubles, m3 <= 64.  One to
// four waves per workgroup (blockDim.x = 64 nw).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_merge_small(const MergeDesc* __restrict__ descs, int keep,
                                                     int root_T, int* status) {
  extern __shared__ double smem[];
  __shared__ int sP[64], sPr;
  __shared__ unsigned char sChosen[64];
  __shared__ double sF[64], sRed[4];
  const MergeDesc d = descs[blockIdx.x];
  const int m3 = d.m3, me = d.me;
  const int lw = 2 * m3 + 1, ls = me + 1;
  double* Wl = smem;
  double* Sl = smem + (size_t)m3 * lw;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nw = blockDim.x >> 6, nthr = blockDim.x;
  const gptr<double> Ta = as_global(d.Ta), Tb = as_global(d.Tb);
  const gptr<int> a3 = as_global(d.a3), b3 = as_global(d.b3), pmap = as_global(d.pmap);
  // Stores through global-address-space pointers (flat stores would also
  // count against the LDS wait counter).
  typedef double __attribute__((address_space(1))) * gout;
  const gout gS = (gout)d.S, gT = (gout)d.Tp, gW = (gout)d.W, gQ = (gout)d.Q;
  // 1. [M | I] into LDS, max|M|.
  double amax = 0.0;
  for (int i = wid; i < m3; i += nw) {
    const size_t ra = (size_t)a3[i] * d.na, rb = (size_t)b3[i] * d.nb;
    for (int j = lane; j < 2 * m3; j += 64) {
      double v;
      if (j < m3) {
        v = Ta[ra + a3[j]] - Tb[rb + b3[j]];
        amax = fmax(amax, fabs(v));
      } else {
        v = (j - m3 == i) ? 1.0 : 0.0;
      }
      Wl[i * lw + j] = v;
    }
  }
  if (tid < 64) sChosen[tid] = 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  if (lane == 0) sRed[wid] = amax;
  __syncthreads();
  // 2. Gauss-Jordan on [M | I]: wave 0 picks the pivot row (lanes are rows)
  // and publishes the column's multipliers; then each thread owns columns of
  // W and walks their rows (no other thread touches its columns in a step).
  bool bad = false;
  double minp = INFINITY;
  for (int c = 0; c < m3; ++c) {
    if (wid == 0) {
      const double v = lane < m3 ? Wl[lane * lw + c] : 0.0;
      const unsigned key = (lane < m3 && !sChosen[lane]) ? pivot_key(v, lane) : 0u;
      const unsigned g = wave_max_u32(key);
      const int pr = g != 0 ? 4095 - (int)(g & 4095u) : 0;
      if (lane < m3) sF[lane] = v;
      if (lane == 0) {
        sPr = pr;
        sP[c] = pr;
        sChosen[pr] = 1;
      }
    }
    __syncthreads();
    const int pr = sPr;
    const double piv = sF[pr];
    const bool ok = piv != 0.0 && piv == piv && fabs(piv) != INFINITY;
    bad |= !ok;
    minp = fmin(minp, fabs(piv));
    const double inv = ok ? recip(piv) : 0.0;
    for (int j = tid; j < 2 * m3; j += nthr) {
      if (j == c) {
        for (int i = 0; i < m3; ++i) Wl[i * lw + j] = i == pr ? 1.0 : 0.0;
        continue;
      }
      const double pj = Wl[pr * lw + j] * inv;
      for (int i = 0; i < m3; ++i)
        Wl[i * lw + j] = i == pr ? pj : fma(-sF[i], pj, Wl[i * lw + j]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double m = sRed[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, sRed[w]);
    if (d.pstat) {
      if (m > 0.0) atomicMax(d.pstat, abs_bits(m));
      if (!bad) atomicMin(d.pstat + 1, abs_bits(minp));
    }
    if (bad)
      if (atomicCAS(status, 0, 1) == 0) status[1] = d.box;
  }
  // Row r of M^-1 is row sP[r] of the right block.
  if (keep)
    for (int r = wid; r < m3; r += nw)
      for (int j = lane; j < m3; j += 64)
        gW[(size_t)r * d.ldw + m3 + j] = Wl[sP[r] * lw + m3 + j];
  // 3. S = M^-1 B, B[k][col] = -T31a or T32b gathered per fragment.
  const int nt3 = (m3 + 15) / 16, nte = (me + 15) / 16;
  for (int t = wid; t < nt3 * nte; t += nw) {
    const int ti = t / nte, tj = t % nte;
    const int row = ti * 16 + (lane & 15), col = tj * 16 + (lane & 15);
    const int pc = col < me ? pmap[col] : 0;
    // Every B fragment of the tile first (all gathers in flight together).
    double bf[16];
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4) {
      const int k = 4 * s4 + (lane >> 4);
      double b = 0.0;
      if (k < m3 && col < me)
        b = pc >= 0 ? -Ta[(size_t)a3[k] * d.na + pc] : Tb[(size_t)b3[k] * d.nb + (-pc - 1)];
      bf[s4] = b;
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4) {
      if (4 * s4 >= m3) break;
      const int k = 4 * s4 + (lane >> 4);
      const double a = (row < m3 && k < m3) ? Wl[sP[row] * lw + m3 + k] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[s4], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti * 16 + (lane >> 4) + 4 * r;
      if (i < m3 && col < me) {
        Sl[i * ls + col] = acc[r];
        gS[(size_t)i * d.lds + col] = acc[r];
      }
    }
  }
  __syncthreads();
  if (d.box == 0 && !root_T) return;
  // 4. T = diag(T11a, T22b) + Q S, one 16-row block of T per wave at a time:
  // its Q fragments (gathered once) against every 16-column block of S.
  for (int ti = wid; ti < nte; ti += nw) {
    const int row = ti * 16 + (lane & 15);
    const int prow = row < me ? pmap[row] : 0;
    double qa[16];
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4) {
      const int k = 4 * s4 + (lane >> 4);
      double v = 0.0;
      if (row < me && k < m3)
        v = prow >= 0 ? Ta[(size_t)prow * d.na + a3[k]] : Tb[(size_t)(-prow - 1) * d.nb + b3[k]];
      qa[s4] = v;
      if (keep && row < me && k < m3) gQ[(size_t)row * m3 + k] = v;
    }
    int pr4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti * 16 + (lane >> 4) + 4 * r;
      pr4[r] = i < me ? pmap[i] : 0;
    }
    for (int tj = 0; tj < nte; ++tj) {
      const int col = tj * 16 + (lane & 15);
      // The pass-through values first, in flight during the products.
      const int pcol = col < me ? pmap[col] : 0;
      double pass[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 16 + (lane >> 4) + 4 * r;
        double v = 0.0;
        if (i < me && col < me) {
          const int pr = pr4[r];
          if (pr >= 0 && pcol >= 0) v = Ta[(size_t)pr * d.na + pcol];
          else if (pr < 0 && pcol < 0) v = Tb[(size_t)(-pr - 1) * d.nb + (-pcol - 1)];
        }
        pass[r] = v;
      }
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        if (4 * s4 >= m3) break;
        const int k = 4 * s4 + (lane >> 4);
        const double b = (k < m3 && col < me) ? Sl[k * ls + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[s4], b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 16 + (lane >> 4) + 4 * r;
        if (i < me && col < me) gT[(size_t)i * me + col] = pass[r] + acc[r];
      }
    }
  }
}

static bool g_merge_small = true;
void set_merge_small(bool on) { g_merge_small = on; }
bool merge_small_on() { return g_merge_small; }

size_t merge_small_lds(int m3, int me) {
  return 8 * ((size_t)m3 * (2 * m3 + 1) + (size_t)m3 * (me + 1));
}

void merge_small(const MergeDesc* d_desc, const std::vector<MergeDesc>& h_desc, bool keep,
                 bool root_T, int* status, hipStream_t s) {
  if (h_desc.empty()) return;
  int m3 = 0, me = 0;
  double flops = 0, bytes = 0;
  for (const MergeDesc& d : h_desc) {
    m3 = std::max(m3, d.m3);
    me = std::max(me, d.me);
    flops += 2.0 * d.m3 * d.m3 * d.m3 + 2.0 * d.m3 * d.m3 * d.me + 2.0 * d.me * d.me * d.m3;
    bytes += 8.0 * (2.0 * d.m3 * d.m3 + 2.0 * d.m3 * d.me + 1.5 * d.me * d.me + d.m3 * d.me);
  }
  HPS_REQUIRE(m3 <= 64, "merge_small: interface longer than 64 nodes");
  const size_t lds = merge_small_lds(m3, me);
  HPS_REQUIRE(lds <= MERGE_SMALL_MAX_LDS, "merge_small: merge too large for LDS");
  static std::once_flag once;
  std::call_once(once, [] {
    HPS_HIP(hipFuncSetAttribute((const void*)k_merge_small,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)MERGE_SMALL_MAX_LDS));
  });
  ProfScope ps(PROF_MERGE_SMALL, s, flops, bytes);
  // One wave per merge for interfaces of at most 16 nodes (more merges in
  // flight per CU), four waves for longer ones.
  const int threads = m3 <= 16 ? 64 : 256;
  hipLaunchKernelGGL(k_merge_small, dim3((unsigned)h_desc.size()), dim3(threads), lds, s, d_desc,
                     keep ? 1 : 0, root_T ? 1 : 0, status);
}

// ---------------------------------------------------------------------------
// Row-parallel passes of a level: for every merge, y_r = A_r . x (one row of a
// stored matrix against a gathered vector, per right-hand side).  Every wave
// first issues the loads of all the matrix entries it will use (16 per lane
// at most), then gathers the matching vector entries (lane l of a wave always
// owns columns l, l + 64, ... of its rows, so it needs the vector at those
// columns only), so a level costs about two memory latencies instead of one
// per row.  Two shapes:
//  - whole rows (row length <= 1024): wave w of a workgroup owns RPW
//    consecutive rows, L = ceil(length/64) loads per lane and row;
//  - split rows (longer): the four waves of a workgroup take a quarter of one
//    row each, in pieces of 1024 columns, and add their four sums in a fixed
//    order through LDS.
// Up to DRHS right-hand sides share each pass over the loaded rows.  The
// operation (which matrix, which vector, where the result goes) is a small
// functor (Algorithm 2 itself runs on k_downward below, the same scheme
// written out for that pass):
//  - RowUpZ, the upward pass: z = M^-1 (s3 - h3a + h3b);
//  - RowUpH, the upward pass: h_parent = [h1a ; h2b] (parent order) + Q z.
// (The two upward steps follow from the third block row of eq:premerge with
// a source term; M^-1 is the explicit inverse the elimination of [M | B | I]
// leaves in W.)
// ---------------------------------------------------------------------------
constexpr int DRHS = 4, DSU = 16;

struct RowUpZ {
  struct Args {
    const MergeDesc* descs;
    const double* s;
    int N, nrhs;
    const double* hbase;
    const long long* ha_off;
    const long long* hb_off;
    double* zbuf;
    const long long* z_off;
  };
  MergeDesc d;
  const double* s;
  int N, nrhs;
  const double* ha;  // [nrhs][na] or null (a leaf child: h = 0)
  const double* hb;
  double* z;         // [nrhs][m3]
  __device__ RowUpZ(const Args& a, int mi) : d(a.descs[mi]), s(a.s), N(a.N), nrhs(a.nrhs) {
    ha = a.ha_off[mi] < 0 ? nullptr : a.hbase + a.ha_off[mi] * nrhs;
    hb = a.hb_off[mi] < 0 ? nullptr : a.hbase + a.hb_off[mi] * nrhs;
    z = a.zbuf + a.z_off[mi] * nrhs;
  }
  __device__ int rows() const { return d.m3; }
  __device__ int cols() const { return d.m3; }
  __device__ const double* row(int r) const { return d.W + d.m3 + (size_t)r * d.ldw; }
  struct Key {
    int g, a, b;
  };
  __device__ Key key(int c) const { return Key{d.Ii[c], d.a3[c], d.b3[c]}; }
  __device__ double vec(int k, Key e) const {
    return (s ? s[(size_t)k * N + e.g] : 0.0) - (ha ? ha[(size_t)k * d.na + e.a] : 0.0) +
           (hb ? hb[(size_t)k * d.nb + e.b] : 0.0);
  }
  __device__ void out(int k, int r, double v) const { z[(size_t)k * d.m3 + r] = v; }
};

struct RowUpH {
  struct Args {
    const MergeDesc* descs;
    double* hbase;
    const long long* ha_off;
    const long long* hb_off;
    const long long* hp_off;
    const double* zbuf;
    const long long* z_off;
    int nrhs;
  };
  MergeDesc d;
  int nrhs;
  const double* ha;
  const double* hb;
  double* hp;       // [nrhs][me]
  const double* z;  // [nrhs][m3]
  __device__ RowUpH(const Args& a, int mi) : d(a.descs[mi]), nrhs(a.nrhs) {
    ha = a.ha_off[mi] < 0 ? nullptr : a.hbase + a.ha_off[mi] * nrhs;
    hb = a.hb_off[mi] < 0 ? nullptr : a.hbase + a.hb_off[mi] * nrhs;
    hp = a.hbase + a.hp_off[mi] * nrhs;
    z = a.zbuf + a.z_off[mi] * nrhs;
  }
  __device__ int rows() const { return d.me; }
  __device__ int cols() const { return d.m3; }
  __device__ const double* row(int r) const { return d.Q + (size_t)r * d.m3; }
  using Key = int;
  __device__ Key key(int c) const { return c; }
  __device__ double vec(int k, Key c) const { return z[(size_t)k * d.m3 + c]; }
  __device__ void out(int k, int r, double v) const {
    const int pm = d.pmap[r];
    v += (pm >= 0) ? (ha ? ha[(size_t)k * d.na + pm] : 0.0)
                   : (hb ? hb[(size_t)k * d.nb + (-pm - 1)] : 0.0);
    hp[(size_t)k * d.me + r] = v;
  }
};

// Dense y[k] = A x[k]: A [rows][cols] row-major, x [nrhs][cols], y [nrhs][rows]
// (the root DtN apply).  One "merge" (blockIdx.y = 0).
struct RowMat {
  struct Args {
    const double* A;
    int rows, cols, nrhs;
    const double* x;
    double* y;
  };
  const double* A;
  int nr, nc, nrhs;
  const double* x;
  double* y;
  __device__ RowMat(const Args& a, int) : A(a.A), nr(a.rows), nc(a.cols), nrhs(a.nrhs), x(a.x),
                                           y(a.y) {}
  __device__ int rows() const { return nr; }
  __device__ int cols() const { return nc; }
  __device__ const double* row(int r) const { return A + (size_t)r * nc; }
  using Key = int;
  __device__ Key key(int c) const { return c; }
  __device__ double vec(int k, Key c) const { return x[(size_t)k * nc + c]; }
  __device__ void out(int k, int r, double v) const { y[(size_t)k * nr + r] = v; }
};

template <class Op, int L, bool SPLIT>
__global__ void __launch_bounds__(256) k_rowdot(const typename Op::Args args) {
  constexpr int RPW = SPLIT ? 1 : (DSU / L < 4 ? DSU / L : 4);
  __shared__ double part[4][DRHS];
  const Op op(args, blockIdx.y);
  const int nrows = op.rows(), ncols = op.cols();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rbase = SPLIT ? blockIdx.x : (blockIdx.x * 4 + wid) * RPW;
  if (SPLIT ? rbase >= nrows : blockIdx.x * 4 * RPW >= nrows) return;  // whole workgroup
  const int nrhs = op.nrhs;
  // Columns of this wave: [c0, c1).
  const int seg = SPLIT ? ((ncols + 255) / 256) * 64 : ncols;
  const int c0 = SPLIT ? wid * seg : 0, c1 = SPLIT ? min(ncols, c0 + seg) : ncols;

  for (int rb = 0; rb < nrhs; rb += DRHS) {
    const int nr = min(DRHS, nrhs - rb);
    double acc[RPW][DRHS];
#pragma unroll
    for (int g = 0; g < RPW; ++g)
#pragma unroll
      for (int j = 0; j < DRHS; ++j) acc[g][j] = 0.0;
    for (int cb = c0; cb < c1; cb += 64 * L) {
      double sv[RPW][L];
#pragma unroll
      for (int g = 0; g < RPW; ++g) {
        const int r = rbase + g;
        const double* Arow = op.row(r < nrows ? r : 0);
#pragma unroll
        for (int l = 0; l < L; ++l) {
          const int c = cb + lane + 64 * l;
          sv[g][l] = (r < nrows && c < c1) ? Arow[c] : 0.0;
        }
      }
      typename Op::Key key[L];
      bool live[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const int c = cb + lane + 64 * l;
        live[l] = c < c1;
        key[l] = op.key(live[l] ? c : c0);
      }
#pragma unroll
      for (int j = 0; j < DRHS; ++j) {
        if (j < nr) {
          double xv[L];
#pragma unroll
          for (int l = 0; l < L; ++l) xv[l] = live[l] ? op.vec(rb + j, key[l]) : 0.0;
#pragma unroll
          for (int g = 0; g < RPW; ++g)
#pragma unroll
            for (int l = 0; l < L; ++l) acc[g][j] = fma(sv[g][l], xv[l], acc[g][j]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < RPW; ++g)
#pragma unroll
      for (int j = 0; j < DRHS; ++j) {
        if (j < nr) {
          double v = acc[g][j];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
          acc[g][j] = v;
        }
      }
    if (SPLIT) {
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < DRHS; ++j) part[wid][j] = acc[0][j];
      }
      __syncthreads();
      if (threadIdx.x < nr) {
        const int j = threadIdx.x;
        op.out(rb + j, rbase, ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j]);
      }
      __syncthreads();
    } else if (lane == 0) {
#pragma unroll
      for (int g = 0; g < RPW; ++g) {
        const int r = rbase + g;
        if (r < nrows) {
#pragma unroll
          for (int j = 0; j < DRHS; ++j)
            if (j < nr) op.out(rb + j, r, acc[g][j]);
        }
      }
    }
  }
}

// One launch of a row-parallel pass over nmerge merges whose longest rows
// have len_max entries and whose row count is at most rows_max.
template <class Op>
static void launch_rowdot(const typename Op::Args& a, int nmerge, int rows_max, int len_max,
                          hipStream_t s) {
  if (nmerge <= 0 || rows_max <= 0) return;
  if (len_max > 64 * DSU) {
    hipLaunchKernelGGL((k_rowdot<Op, DSU, true>), dim3(rows_max, nmerge), dim3(256), 0, s, a);
    return;
  }
  const int L = std::max(1, (len_max + 63) / 64);
  const int rpw = std::min(4, DSU / L);
  const dim3 grid((rows_max + 4 * rpw - 1) / (4 * rpw), nmerge);
  switch (L) {
#define HPS_ROWDOT(LL) \
  case LL: hipLaunchKernelGGL((k_rowdot<Op, LL, false>), grid, dim3(256), 0, s, a); break;
    HPS_ROWDOT(1) HPS_ROWDOT(2) HPS_ROWDOT(3) HPS_ROWDOT(4) HPS_ROWDOT(5) HPS_ROWDOT(6)
    HPS_ROWDOT(7) HPS_ROWDOT(8) HPS_ROWDOT(9) HPS_ROWDOT(10) HPS_ROWDOT(11) HPS_ROWDOT(12)
    HPS_ROWDOT(13) HPS_ROWDOT(14) HPS_ROWDOT(15) HPS_ROWDOT(16)
#undef HPS_ROWDOT
    default:
      HPS_REQUIRE(false, "row pass: bad row length");
  }
}

// ---------------------------------------------------------------------------
// Downward pass (Algorithm 2): u(I_i) = S u(I_e) (+ z) for every merge of one
// level, u [nrhs][N]: the row-pass scheme above with S against the
// gathered u(I_e), written out for this pass (it measured about 15% faster
// per level than the functor form).
// ---------------------------------------------------------------------------
template <int L, bool SPLIT>
__global__ void __launch_bounds__(256) k_downward(const MergeDesc* __restrict__ descs,
                                                  const SolveIO* __restrict__ io,
                                                  const SolveIO io0, int io_shared,
                                                  const double* __restrict__ zbase,
                                                  const long long* __restrict__ zoff) {
  constexpr int RPW = SPLIT ? 1 : (DSU / L < 4 ? DSU / L : 4);
  __shared__ double part[4][DRHS];
  const MergeDesc d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rbase = SPLIT ? blockIdx.x : (blockIdx.x * 4 + wid) * RPW;
  if (SPLIT ? rbase >= d.m3 : blockIdx.x * 4 * RPW >= d.m3) return;  // whole workgroup
  const SolveIO b = io ? io[io_shared ? 0 : blockIdx.y] : io0;
  double* u = b.u;
  const int N = b.N, nrhs = b.nrhs, me = d.me, m3 = d.m3;
  const double* z = zbase ? zbase + zoff[blockIdx.y] * nrhs : nullptr;
  // Columns of this wave: [c0, c1).
  const int seg = SPLIT ? ((me + 255) / 256) * 64 : me;
  const int c0 = SPLIT ? wid * seg : 0, c1 = SPLIT ? min(me, c0 + seg) : me;

  for (int rb = 0; rb < nrhs; rb += DRHS) {
    const int nr = min(DRHS, nrhs - rb);
    double acc[RPW][DRHS];
#pragma unroll
    for (int g = 0; g < RPW; ++g)
#pragma unroll
      for (int j = 0; j < DRHS; ++j) acc[g][j] = 0.0;
    for (int cb = c0; cb < c1; cb += 64 * L) {
      double sv[RPW][L];
#pragma unroll
      for (int g = 0; g < RPW; ++g) {
        const int r = rbase + g;
        const double* Srow = d.S + (size_t)r * d.lds;
#pragma unroll
        for (int l = 0; l < L; ++l) {
          const int c = cb + lane + 64 * l;
          sv[g][l] = (r < m3 && c < c1) ? Srow[c] : 0.0;
        }
      }
      int ie[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const int c = cb + lane + 64 * l;
        ie[l] = c < c1 ? d.Ie[c] : -1;
      }
#pragma unroll
      for (int j = 0; j < DRHS; ++j) {
        if (j < nr) {
          double uv[L];
#pragma unroll
          for (int l = 0; l < L; ++l) uv[l] = ie[l] >= 0 ? u[(size_t)(rb + j) * N + ie[l]] : 0.0;
#pragma unroll
          for (int g = 0; g < RPW; ++g)
#pragma unroll
            for (int l = 0; l < L; ++l) acc[g][j] = fma(sv[g][l], uv[l], acc[g][j]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < RPW; ++g)
#pragma unroll
      for (int j = 0; j < DRHS; ++j) {
        if (j < nr) {
          double v = acc[g][j];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
          acc[g][j] = v;
        }
      }
    if (SPLIT) {
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < DRHS; ++j) part[wid][j] = acc[0][j];
      }
      __syncthreads();
      if (threadIdx.x < nr) {
        const int j = threadIdx.x, k = rb + j, r = rbase;
        double v = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
        if (z) v += z[(size_t)k * m3 + r];
        u[(size_t)k * N + d.Ii[r]] = v;
      }
      __syncthreads();
    } else if (lane == 0) {
#pragma unroll
      for (int g = 0; g < RPW; ++g) {
        const int r = rbase + g;
        if (r < m3) {
#pragma unroll
          for (int j = 0; j < DRHS; ++j) {
            if (j < nr) {
              const int k = rb + j;
              double v = acc[g][j];
              if (z) v += z[(size_t)k * m3 + r];
              u[(size_t)k * N + d.Ii[r]] = v;
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 as one persistent launch: every level of one operator in a
// single cooperative kernel, the levels separated by a grid-wide barrier.  Rows are dealt
// to waves (rows up to 1024 long) or to workgroups (longer rows, split over
// the four waves and summed through LDS in a fixed order) exactly as in
// k_downward, so the result is bit for bit the level-by-level one.  A
// barrier that waits longer than about a second sets *err and lets the
// workgroup go on (the host then reports a device error): every workgroup
// always reaches the end.
// ---------------------------------------------------------------------------
// The solution u is the only data passed between levels, and every access
// to it here is a device-scope relaxed atomic (coherent across the XCDs,
// whose L2 caches are not coherent with each other for plain accesses).  So
// the barrier needs no cache write-back or invalidation: each thread waits
// for its own stores, the workgroup meets, thread 0 counts it in and spins.
__global__ void __launch_bounds__(256) k_downward_persist(const PersistLevel* __restrict__ levels,
                                                          int nlev, const double* __restrict__ f,
                                                          const int* __restrict__ gamma, int nb,
                                                          double* u, int N, int nrhs,
                                                          unsigned* bar, int* err) {
  __shared__ double part[4][DRHS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned nblk = gridDim.x;
  unsigned gen = 0;
  // Boundary data onto Gamma.
  const size_t tot = (size_t)nb * nrhs, nthr = (size_t)nblk * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += nthr) {
    const int r = (int)(e / nb), i = (int)(e % nb);
    st_dev(u + (size_t)r * N + gamma[i], f[e]);
  }
  for (int lev = 0; lev < nlev; ++lev) {
    grid_barrier(bar, nblk, gen, err);
    const PersistLevel P = levels[lev];
    const int m3 = P.m3, me = P.me;
    const long long rows = (long long)P.nmerge * m3;
    if (me <= 64 * DSU) {
      // One row per wave and task (k_downward<L, false> with L = ceil(me / 64)).
      const int Lc = (me + 63) / 64;
      for (long long rr = (long long)blockIdx.x * 4 + wid; rr < rows; rr += (long long)nblk * 4) {
        const int mi = (int)(rr / m3), r = (int)(rr % m3);
        const MergeDesc& d = P.d[mi];
        const gptr<double> Srow = as_global(d.S + (size_t)r * d.lds);
        const gptr<int> Ie = as_global(d.Ie);
        double sv[DSU];
        int ie[DSU];
#pragma unroll
        for (int l = 0; l < DSU; ++l) {
          const int c = lane + 64 * l;
          const bool in = l < Lc && c < me;
          sv[l] = in ? Srow[c] : 0.0;
          ie[l] = in ? Ie[c] : -1;
        }
        const int out = d.Ii[r];
        for (int rb = 0; rb < nrhs; rb += DRHS) {
          const int nr = min(DRHS, nrhs - rb);
          double acc[DRHS];
#pragma unroll
          for (int j = 0; j < DRHS; ++j) {
            acc[j] = 0.0;
            if (j < nr) {
#pragma unroll
              for (int l = 0; l < DSU; ++l) {
                if (l < Lc) {
                  const double uv = ie[l] >= 0 ? ld_dev(u + (size_t)(rb + j) * N + ie[l]) : 0.0;
                  acc[j] = fma(sv[l], uv, acc[j]);
                }
              }
#pragma unroll
              for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
            }
          }
          if (lane == 0)
#pragma unroll
            for (int j = 0; j < DRHS; ++j)
              if (j < nr) st_dev(u + (size_t)(rb + j) * N + out, acc[j]);
        }
      }
    } else {
      // One row per workgroup and task, the four waves on quarters of it
      // (k_downward<DSU, true>).
      const int seg = ((me + 255) / 256) * 64;
      const int c0 = wid * seg, c1 = min(me, c0 + seg);
      for (long long rr = blockIdx.x; rr < rows; rr += nblk) {
        const int mi = (int)(rr / m3), r = (int)(rr % m3);
        const MergeDesc& d = P.d[mi];
        const gptr<double> Srow = as_global(d.S + (size_t)r * d.lds);
        const gptr<int> Ie = as_global(d.Ie);
        for (int rb = 0; rb < nrhs; rb += DRHS) {
          const int nr = min(DRHS, nrhs - rb);
          double acc[DRHS];
#pragma unroll
          for (int j = 0; j < DRHS; ++j) acc[j] = 0.0;
          for (int cb = c0; cb < c1; cb += 64 * DSU) {
            double sv[DSU];
            int ie[DSU];
#pragma unroll
            for (int l = 0; l < DSU; ++l) {
              const int c = cb + lane + 64 * l;
              sv[l] = c < c1 ? Srow[c] : 0.0;
              ie[l] = c < c1 ? Ie[c] : -1;
            }
#pragma unroll
            for (int j = 0; j < DRHS; ++j) {
              if (j < nr) {
                double uv[DSU];
#pragma unroll
                for (int l = 0; l < DSU; ++l)
                  uv[l] = ie[l] >= 0 ? ld_dev(u + (size_t)(rb + j) * N + ie[l]) : 0.0;
#pragma unroll
                for (int l = 0; l < DSU; ++l) acc[j] = fma(sv[l], uv[l], acc[j]);
              }
            }
          }
#pragma unroll
          for (int j = 0; j < DRHS; ++j) {
            if (j < nr) {
              double v = acc[j];
#pragma unroll
              for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
              acc[j] = v;
            }
          }
          if (lane == 0)
#pragma unroll
            for (int j = 0; j < DRHS; ++j) part[wid][j] = acc[j];
          __syncthreads();
          if (threadIdx.x < nr) {
            const int j = threadIdx.x;
            st_dev(u + (size_t)(rb + j) * N + d.Ii[r],
                   ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j]);
          }
          __syncthreads();
        }
      }
    }
  }
}

__global__ void k_zero_persist(unsigned* bar, int* err) {
  if (threadIdx.x < 9) bar[32 * threadIdx.x] = 0u;
  if (threadIdx.x == 0) *err = 0;
}

int downward_persist_grid() {
  static int grid = -1;
  if (grid < 0) {
    int dev = 0, cus = 0, per = 0;
    HPS_HIP(hipGetDevice(&dev));
    HPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_downward_persist, 256, 0));
    grid = std::max(0, std::min(per, 4)) * cus;
  }
  return grid;
}

void downward_persist(const PersistLevel* d_levels, int nlev, const double* f, const int* gamma,
                      int nb, double* u, int N, int nrhs, unsigned* d_bar, int* d_err,
                      hipStream_t s) {
  const int grid = downward_persist_grid();
  HPS_REQUIRE(grid > 0, "persistent downward pass: no resident workgroups");
  hipLaunchKernelGGL(k_zero_persist, dim3(1), dim3(64), 0, s, d_bar, d_err);
  void* args[] = {(void*)&d_levels, (void*)&nlev, (void*)&f, (void*)&gamma, (void*)&nb,
                  (void*)&u, (void*)&N, (void*)&nrhs, (void*)&d_bar, (void*)&d_err};
  HPS_HIP(hipLaunchCooperativeKernel((const void*)k_downward_persist, dim3(grid), dim3(256), args,
                                     0, s));
}

template <int L>
static void launch_down_rows(dim3 grid, hipStream_t s, const MergeDesc* d_desc,
                             const SolveIO* d_io, const SolveIO& io0, bool io_shared,
                             const double* zbase, const long long* zoff) {
  hipLaunchKernelGGL((k_downward<L, false>), grid, dim3(256), 0, s, d_desc, d_io, io0,
                     io_shared ? 1 : 0, zbase, zoff);
}

void downward(const MergeDesc* d_desc, const SolveIO* d_io, const SolveIO& io0, int nmerge,
              int m3_max, int me_max, int nrhs_max, const double* zbase, const long long* zoff,
              hipStream_t s, double s_bytes, bool io_shared) {
  ProfScope ps(PROF_DOWNWARD, s, 2.0 * nrhs_max * s_bytes / 8.0, s_bytes);
  if (nmerge <= 0 || m3_max <= 0) return;
  if (me_max > 64 * DSU) {
    hipLaunchKernelGGL((k_downward<DSU, true>), dim3(m3_max, nmerge), dim3(256), 0, s, d_desc,
                       d_io, io0, io_shared ? 1 : 0, zbase, zoff);
    return;
  }
  const int L = std::max(1, (me_max + 63) / 64);
  const int rpw = std::min(4, DSU / L);
  const dim3 grid((m3_max + 4 * rpw - 1) / (4 * rpw), nmerge);
  switch (L) {
#define HPS_DOWN(LL) \
  case LL: launch_down_rows<LL>(grid, s, d_desc, d_io, io0, io_shared, zbase, zoff); break;
    HPS_DOWN(1) HPS_DOWN(2) HPS_DOWN(3) HPS_DOWN(4) HPS_DOWN(5) HPS_DOWN(6) HPS_DOWN(7)
    HPS_DOWN(8) HPS_DOWN(9) HPS_DOWN(10) HPS_DOWN(11) HPS_DOWN(12) HPS_DOWN(13) HPS_DOWN(14)
    HPS_DOWN(15) HPS_DOWN(16)
#undef HPS_DOWN
    default:
      HPS_REQUIRE(false, "downward pass: bad row length");
  }
}

// Boundary data into u: u[r][gamma[i]] = f[r][i].
__global__ void k_set_boundary(const double* __restrict__ f, const int* __restrict__ gamma,
                               int nb, double* __restrict__ u, int N, int nrhs) {
  size_t tot = (size_t)nb * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int r = (int)(e / nb), i = (int)(e % nb);
    u[(size_t)r * N + gamma[i]] = f[e];
  }
}

// The same with f, u, N and nrhs read from a device-side SolveIO (graph replay).
__global__ void k_set_boundary_io(const SolveIO* __restrict__ io, const int* __restrict__ gamma,
                                  int nb) {
  const SolveIO b = *io;
  size_t tot = (size_t)nb * b.nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int r = (int)(e / nb), i = (int)(e % nb);
    b.u[(size_t)r * b.N + gamma[i]] = b.f[e];
  }
}

void set_boundary_io(const SolveIO* io, const int* gamma, int nb, int nrhs, hipStream_t s) {
  size_t tot = (size_t)nb * nrhs;
  int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_set_boundary_io, dim3(std::max(blocks, 1)), dim3(256), 0, s, io, gamma, nb);
}

void set_boundary(const double* f, const int* gamma, int nb, double* u, int N, int nrhs,
                  hipStream_t s) {
  size_t tot = (size_t)nb * nrhs;
  int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_set_boundary, dim3(std::max(blocks, 1)), dim3(256), 0, s, f, gamma, nb, u,
                     N, nrhs);
}

// ---------------------------------------------------------------------------
// Interface residual: v_leaf = T_leaf u(I_e^leaf) for every leaf, then the
// jump v_alpha - v_beta at every interior Gauss node (0 on the boundary).
// ---------------------------------------------------------------------------
__device__ inline int leaf_bdry_id(int i, int j, int nx, int nh, int q, int k) {
  int side = k / q, t = k % q;
  switch (side) {
    case 0: return (j * nx + i) * q + t;                  // S: hedge (i, j)
    case 1: return (nh + j * (nx + 1) + i + 1) * q + t;   // E: vedge (i+1, j)
    case 2: return ((j + 1) * nx + i) * q + t;            // N: hedge (i, j+1)
    default: return (nh + j * (nx + 1) + i) * q + t;      // W: vedge (i, j)
  }
}

__global__ void __launch_bounds__(256) k_leaf_flux(const double* __restrict__ T,
                                                   const double* __restrict__ u, int N, int nrhs,
                                                   int nx, int ny, int q,
                                                   double* __restrict__ v) {
  __shared__ double ue[8][96];
  const int leaf = blockIdx.x;
  const int i = leaf % nx, j = leaf / nx;
  const int m = 4 * q, nh = nx * (ny + 1);
  const double* Tl = T + (size_t)leaf * m * m;
  for (int rb = 0; rb < nrhs; rb += 8) {
    const int nr = min(8, nrhs - rb);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * m; e += blockDim.x) {
      int k = e / m, c = e % m;
      ue[k][c] = u[(size_t)(rb + k) * N + leaf_bdry_id(i, j, nx, nh, q, c)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * m; e += blockDim.x) {
      int k = e / m, r = e % m;
      double acc = 0.0;
      for (int c = 0; c < m; ++c) acc += Tl[(size_t)r * m + c] * ue[k][c];
      v[((size_t)(rb + k) * nx * ny + leaf) * m + r] = acc;
    }
  }
}

__global__ void k_jump(const double* __restrict__ v, int nx, int ny, int q, int nrhs,
                       double* __restrict__ r, int N) {
  const int nh = nx * (ny + 1), m = 4 * q;
  const size_t nl = (size_t)nx * ny;
  size_t tot = (size_t)N * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int rh = (int)(e / N), g = (int)(e % N);
    int edge = g / q, k = g % q;
    double val = 0.0;
    const double* vr = v + (size_t)rh * nl * m;
    if (edge < nh) {
      int i = edge % nx, j = edge / nx;
      if (j > 0 && j < ny)  // alpha = south leaf (its N side), beta = north leaf (its S side)
        val = vr[((size_t)(i + nx * (j - 1))) * m + 2 * q + k] - vr[((size_t)(i + nx * j)) * m + k];
    } else {
      int ve = edge - nh;
      int i = ve % (nx + 1), j = ve / (nx + 1);
      if (i > 0 && i < nx)  // alpha = west leaf (its E side), beta = east leaf (its W side)
        val = vr[((size_t)(i - 1 + nx * j)) * m + q + k] - vr[((size_t)(i + nx * j)) * m + 3 * q + k];
    }
    r[e] = val;
  }
}

void interface_residual(const double* leafT, const double* u, int N, int nrhs, int nx, int ny,
                        int q, double* vbuf, double* r, hipStream_t s) {
  HPS_REQUIRE(4 * q <= 96, "q too large for the residual kernel");
  ProfScope ps(PROF_RESIDUAL, s, 2.0 * nrhs * nx * ny * 16.0 * q * q, 8.0 * nx * ny * 16.0 * q * q);
  hipLaunchKernelGGL(k_leaf_flux, dim3(nx * ny), dim3(256), 0, s, leafT, u, N, nrhs, nx, ny, q,
                     vbuf);
  size_t tot = (size_t)N * nrhs;
  int blocks = (int)std::min<size_t>((tot + 255) / 256, 8192);
  hipLaunchKernelGGL(k_jump, dim3(blocks), dim3(256), 0, s, vbuf, nx, ny, q, nrhs, r, N);
}

// ---------------------------------------------------------------------------
// Post-processing (section 5.3).  Row list of a leaf: the (p-2)^2 rows of -Z
// (interior nodes), then the 4(p-1) rows of L1 (grid-boundary nodes);
// post_node[rho] is the Chebyshev node that row rho produces.  Z and L1 are
// stored transposed (column-major), so lanes that own consecutive rows read
// consecutive addresses.  Workgroup (leaf, chunk of 64 R rows, group of
// right-hand sides): lane l owns rows 64 r + l of the chunk and wave w the q
// columns that act on side w's Gauss values, kept in registers.  A side's
// Gauss values are q consecutive entries of u, the same for the whole wave,
// so they are read as wave-uniform (scalar) loads and every multiply-add takes
// them as a scalar operand; the four side sums meet in LDS in a fixed order.
// ---------------------------------------------------------------------------
constexpr int POST_QMAX = 24, POST_ROWS = 64, POST_RG = 48;

// R rows per lane (64 R rows per workgroup): each wave-uniform value of u then
// feeds R multiply-adds.  RC right-hand sides share one round of side sums.
template <int Q, int R>
__global__ void __launch_bounds__(256) k_leaf_post(const double* __restrict__ Zt,
                                                   const double* __restrict__ L1t,
                                                   const int* __restrict__ post_node,
                                                   const double* __restrict__ u, int N, int nrhs,
                                                   int nx, int ny, int p,
                                                   double* __restrict__ uc) {
  constexpr int q = Q, m = 4 * Q, RC = 12 / R, ROWS = POST_ROWS * R;
  extern __shared__ double sbuf[];  // [min(RC, nrhs)][4][ROWS] side sums
  const int leaf = blockIdx.x, i = leaf % nx, j = leaf / nx;
  const int nh = nx * (ny + 1), pp = p * p, n = (p - 2) * (p - 2);
  const int lane = threadIdx.x & 63;
  const int side = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t nl = (size_t)nx * ny;

  // Column c of the leaf's Z^T (and of L1^T) is contiguous over rows, so
  // every load below reads 64 consecutive doubles across the wave.
  const int ne = pp - n;
  double z[R][Q];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = blockIdx.y * ROWS + r * POST_ROWS + lane;
    if (row < n) {
      const double* src = Zt + (size_t)leaf * n * m + (size_t)side * q * n + row;
#pragma unroll
      for (int c = 0; c < Q; ++c) z[r][c] = -src[(size_t)c * n];
    } else if (row < pp) {
      const double* src = L1t + (size_t)side * q * ne + (row - n);
#pragma unroll
      for (int c = 0; c < Q; ++c) z[r][c] = src[c * ne];
    } else {
#pragma unroll
      for (int c = 0; c < Q; ++c) z[r][c] = 0.0;
    }
  }

  const int base = __builtin_amdgcn_readfirstlane(leaf_bdry_id(i, j, nx, nh, q, side * q));
  const int g0 = blockIdx.z * POST_RG, g1 = min(g0 + POST_RG, nrhs);
  for (int rb = g0; rb < g1; rb += RC) {
    const int nr = min(RC, g1 - rb);
    for (int k = 0; k < nr; ++k) {
      const double* us = u + (size_t)(rb + k) * N + base;
      double acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const double uv = us[c];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(z[r][c], uv, acc[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) sbuf[(k * 4 + side) * ROWS + r * POST_ROWS + lane] = acc[r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ROWS; e += 256) {
      const int k = e / ROWS, l = e % ROWS, row = blockIdx.y * ROWS + l;
      if (row < pp) {
        const double* ps = sbuf + k * 4 * ROWS + l;
        uc[((size_t)(rb + k) * nl + leaf) * pp + post_node[row]] =
            ((ps[0] + ps[ROWS]) + ps[2 * ROWS]) + ps[3 * ROWS];
      }
    }
    __syncthreads();
  }
}

static int g_post_rows = 0;  // rows per lane: 0 = by right-hand-side count (2, or 4 from 16 on)
void set_post_rows(int r) {
  HPS_REQUIRE(r == -1 || r == 0 || r == 1 || r == 2 || r == 4, "post_rows must be 1, 2 or 4");
  g_post_rows = r < 0 ? 0 : r;
}

template <int R>
static void launch_post(const double* Zt, const double* L1t, const int* post_node, const double* u,
                        int N, int nrhs, int nx, int ny, int p, int q, double* uc, hipStream_t s) {
  const int rows = POST_ROWS * R, rc = 12 / R;
  const dim3 grid(nx * ny, (p * p + rows - 1) / rows, (nrhs + POST_RG - 1) / POST_RG);
  const size_t lds = sizeof(double) * std::min(rc, nrhs) * 4 * rows;
  switch (q) {
#define HPS_POST(QQ)                                                                            \
  case QQ:                                                                                      \
    hipLaunchKernelGGL((k_leaf_post<QQ, R>), grid, dim3(256), lds, s, Zt, L1t, post_node, u, N, \
                       nrhs, nx, ny, p, uc);                                                    \
    break;
    HPS_POST(1) HPS_POST(2) HPS_POST(3) HPS_POST(4) HPS_POST(5) HPS_POST(6) HPS_POST(7)
    HPS_POST(8) HPS_POST(9) HPS_POST(10) HPS_POST(11) HPS_POST(12) HPS_POST(13) HPS_POST(14)
    HPS_POST(15) HPS_POST(16) HPS_POST(17) HPS_POST(18) HPS_POST(19) HPS_POST(20) HPS_POST(21)
    HPS_POST(22) HPS_POST(23) HPS_POST(24)
#undef HPS_POST
    default:
      HPS_REQUIRE(false, "q too large for the post-processing kernel");
  }
}

void leaf_postprocess(const double* Zt, const double* L1t, const int* post_node, const double* u,
                      int N, int nrhs, int nx, int ny, int p, int q, double* uc, hipStream_t s) {
  HPS_REQUIRE(q >= 1 && q <= POST_QMAX, "q out of range for the post-processing kernel");
  HPS_REQUIRE(nrhs >= 1 && (nrhs + POST_RG - 1) / POST_RG <= 65535, "bad right-hand-side count");
  const double nl = (double)nx * ny, n = (double)(p - 2) * (p - 2), m = 4.0 * q;
  ProfScope ps(PROF_POSTPROCESS, s, 2.0 * nrhs * nl * p * p * m,
               8.0 * (nl * n * m + nrhs * nl * (m + (double)p * p)));
  const int R = g_post_rows ? g_post_rows : (nrhs >= 16 ? 4 : 2);
  if (R == 4)
    launch_post<4>(Zt, L1t, post_node, u, N, nrhs, nx, ny, p, q, uc, s);
  else if (R == 2)
    launch_post<2>(Zt, L1t, post_node, u, N, nrhs, nx, ny, p, q, uc, s);
  else
    launch_post<1>(Zt, L1t, post_node, u, N, nrhs, nx, ny, p, q, uc, s);
}

// Batched transpose through LDS, 64 source rows per workgroup: loads run along
// a source row, stores along a destination row.
__global__ void __launch_bounds__(256) k_transpose_rows(const double* const* src,
                                                        double* const* dst, int rows, int cols,
                                                        int lds) {
  extern __shared__ double tile[];  // [64][cols + 1]
  const double* a = src[blockIdx.x];
  double* b = dst[blockIdx.x];
  const int r0 = blockIdx.y * 64, nr = min(64, rows - r0);
  for (int e = threadIdx.x; e < nr * cols; e += 256) {
    const int rl = e / cols, c = e - rl * cols;
    tile[rl * (cols + 1) + c] = a[(size_t)(r0 + rl) * lds + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nr * cols; e += 256) {
    const int c = e / nr, rl = e - c * nr;
    b[(size_t)c * rows + r0 + rl] = tile[rl * (cols + 1) + c];
  }
}

void transpose_rows_batch(const double* const* src, double* const* dst, int count, int rows,
                          int cols, int lds, hipStream_t s) {
  if (count <= 0 || rows <= 0) return;
  HPS_REQUIRE(count <= 0x7fffffff && (rows + 63) / 64 <= 65535, "transpose too large");
  hipLaunchKernelGGL(k_transpose_rows, dim3(count, (rows + 63) / 64), dim3(256),
                     sizeof(double) * 64 * (cols + 1), s, src, dst, rows, cols, lds);
}

// ---------------------------------------------------------------------------
// Upward source pass for one level: z = M^-1 (s3 - h3a + h3b), then
// h_parent = [h1a ; h2b] + Q z (row passes RowUpZ and RowUpH above).
// ---------------------------------------------------------------------------
void upward_level(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, const double* s,
                  int N, double* hbase, const long long* ha_off, const long long* hb_off,
                  const long long* hp_off, double* zbuf, const long long* z_off, int nrhs,
                  double flops, hipStream_t st) {
  ProfScope ps(PROF_UPWARD, st, flops, 8.0 * flops / 2.0);
  const RowUpZ::Args az{d_desc, s, N, nrhs, hbase, ha_off, hb_off, zbuf, z_off};
  launch_rowdot<RowUpZ>(az, nmerge, m3_max, m3_max, st);
  const RowUpH::Args ah{d_desc, hbase, ha_off, hb_off, hp_off, zbuf, z_off, nrhs};
  launch_rowdot<RowUpH>(ah, nmerge, me_max, m3_max, st);
}

// ---------------------------------------------------------------------------
// Small elementwise helpers.
// ---------------------------------------------------------------------------
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

void axpy(double* y, const double* x, double a, size_t n, hipStream_t s) {
  int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_axpy, dim3(std::max(blocks, 1)), dim3(256), 0, s, y, x, a, n);
}

// max |x| per block into out[block]; host finishes.  Used for refinement norms.
__global__ void k_absmax(const double* __restrict__ x, size_t n, double* __restrict__ out) {
  __shared__ double sm[4];
  double m = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    m = x[e] != x[e] ? INFINITY : fmax(m, fabs(x[e]));  // NaN counts as infinite
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

void absmax_partial(const double* x, size_t n, double* out, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(blocks), dim3(256), 0, s, x, n, out);
}

// y[r][i] = sum_j A[i][j] x[r][j] on the row-pass kernel (loads first, long rows
// split over four waves, up to four right-hand sides per pass over A).
void matvec(const double* A, int rows, int cols, const double* x, int nrhs, double* y,
            hipStream_t s) {
  const RowMat::Args a{A, rows, cols, nrhs, x, y};
  launch_rowdot<RowMat>(a, 1, rows, cols, s);
}

// flag[0] = 1 if any entry is NaN or infinite.
__global__ void k_nonfinite(const double* __restrict__ x, size_t n, int* flag) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[e])) flag[0] = 1;
}

void nonfinite(const double* x, size_t n, int* flag, hipStream_t s) {
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_nonfinite, dim3(std::max(blocks, 1)), dim3(256), 0, s, x, n, flag);
}

// flag[l] = 1 when a leaf's c11, c22 or c leaves [lo - margin*w, hi + margin*w]
// (w = hi - lo) of the surrogate's training data.  lohi = {lo[3], hi[3]}.
__global__ void __launch_bounds__(256) k_range_flags(const double* const* __restrict__ cptr, int pp,
                                                     const double* __restrict__ lohi, double margin,
                                                     int* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const double* c = cptr[blockIdx.x];
  const int field[3] = {0, 2, 5};
  int my = 0;
  for (int e = threadIdx.x; e < 3 * pp; e += blockDim.x) {
    const int f = e / pp;
    const double v = c[(size_t)field[f] * pp + e % pp];
    const double w = lohi[3 + f] - lohi[f];
    if (!(v >= lohi[f] - margin * w && v <= lohi[3 + f] + margin * w)) my = 1;
  }
  if (my) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) flag[blockIdx.x] = bad;
}

void leaf_range_flags(const double* const* cptr, int nl, int pp, const double* lohi, double margin,
                      int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_range_flags, dim3(nl), dim3(256), 0, s, cptr, pp, lohi, margin, flag);
}

// ---------------------------------------------------------------------------
// Solution passes for many right-hand sides on node-major arrays: U is
// [N][nrhs] (the nrhs values of one node are contiguous), so the boundary
// values of a box are whole rows and every pass is a grouped FP64 MFMA GEMM
// with gathered and scattered rows.  Per box the upward-pass arrays h are
// [boundary size][nrhs] and z is [m3][nrhs].
// ---------------------------------------------------------------------------
// Tiles of these passes: BM x BN outputs (BM = 16, 32 or 64 rows, so that
// the short interfaces of the lowest depths do not run mostly padded tiles;
// BN = 16, 32 or 64 right-hand sides), BK = 16, WM x WN waves.
template <int BM, int BN>
struct MmCfg {
  static constexpr int WM = BM == 16 ? 1 : (BM == 32 ? 2 : (BN == 16 ? 4 : 2));
  static constexpr int WN =
      BM == 16 ? BN / 16 : (BM == 32 ? (BN == 64 ? 2 : 1) : (BN == 16 ? 1 : 2));
  static constexpr int NT = 64 * WM * WN;
};
#define HPS_MMT(BM, BN) BM, BN, 16, MmCfg<BM, BN>::WM, MmCfg<BM, BN>::WN
#define HPS_MM_TILE(BN) HPS_MMT(64, BN)

// Row-tile height for a launch whose output blocks have at most rows rows.
static int mm_rows(int rows) { return rows <= 16 ? 16 : (rows <= 32 ? 32 : 64); }

// Algorithm 2 for one depth: U[Ii[r]][:] = S[r][:] U[Ie[:]][:] (+ z[r][:]).
// Depths with few merges split the contraction over me into ks chunks
// (grid z = merge * ks + chunk) whose partial products go to P
// ([merge][ks][m3_max][nrhs]) and are summed in chunk order by
// k_down_reduce, so that the few large S of the top levels are streamed by
// enough workgroups to fill the chip.
template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) k_down_mm(const MergeDesc* __restrict__ descs,
                                                         double* U, int nrhs,
                                                         const double* __restrict__ zbase,
                                                         const long long* __restrict__ zoff,
                                                         const SolveIO* __restrict__ io, int ks,
                                                         double* __restrict__ P, int m3_max) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const int mi = blockIdx.z / ks, kc = blockIdx.z % ks;
  const MergeDesc d = descs[mi];
  if (io) {
    U = io[mi].u;
    nrhs = io[mi].nrhs;
  }
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  if (row0 >= d.m3 || col0 >= nrhs) return;
  if (ks == 1) {
    const double* z = zbase ? zbase + zoff[mi] * nrhs : nullptr;
    gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(d.S, d.lds, U, nrhs, RowsIndexed{d.Ie}, U, nrhs,
                                      RowsIndexed{d.Ii}, z, nrhs, d.m3, nrhs, d.me, 1.0, row0,
                                      col0, sm, false);
    return;
  }
  const int kchunk = ((d.me + ks - 1) / ks + BK - 1) / BK * BK;
  const int k0 = min(d.me, kc * kchunk), K = min(kchunk, d.me - k0);
  gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(d.S + k0, d.lds, U, nrhs, RowsIndexed{d.Ie + k0},
                                    P + (size_t)blockIdx.z * m3_max * nrhs, nrhs, RowsIdentity{},
                                    nullptr, 0, d.m3, nrhs, K, 1.0, row0, col0, sm, false);
}

__global__ void k_down_reduce(const MergeDesc* __restrict__ descs, double* __restrict__ U,
                              int nrhs, const double* __restrict__ zbase,
                              const long long* __restrict__ zoff, int ks,
                              const double* __restrict__ P, int m3_max) {
  const int mi = blockIdx.y;
  const MergeDesc d = descs[mi];
  const double* z = zbase ? zbase + zoff[mi] * nrhs : nullptr;
  const double* Pm = P + (size_t)mi * ks * m3_max * nrhs;
  const int tot = d.m3 * nrhs;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int r = e / nrhs, c = e % nrhs;
    double v = z ? z[e] : 0.0;
    for (int j = 0; j < ks; ++j) v += Pm[((size_t)j * m3_max + r) * nrhs + c];
    U[(size_t)d.Ii[r] * nrhs + c] = v;
  }
}

// Number of contraction chunks for a launch of `tiles` output tiles with
// contraction length K: enough workgroups to fill the chip (about 1024),
// chunks of at least g_split_min (256 by default).
static int g_split_min = 256;

void set_split_min_chunk(int v) { g_split_min = std::max(16, v); }

static int split_chunks(long long tiles, int K) {
  if (tiles >= 512) return 1;
  const long long want = (1024 + tiles - 1) / tiles;
  return (int)std::max<long long>(1, std::min<long long>(want, K / g_split_min));
}

template <int BM, int BN>
static void launch_down_mm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max,
                           double* U, int nrhs, const double* zbase, const long long* zoff,
                           const SolveIO* io, hipStream_t s) {
  const long long tiles = (long long)((nrhs + BN - 1) / BN) * ((m3_max + BM - 1) / BM) * nmerge;
  const int ks = io ? 1 : split_chunks(tiles, me_max);
  HPS_REQUIRE((long long)nmerge * ks <= 65535, "downward pass: too many merges at one depth");
  double* P = nullptr;
  if (ks > 1)
    HPS_HIP(hipMallocAsync((void**)&P, (size_t)nmerge * ks * m3_max * nrhs * sizeof(double), s));
  dim3 grid((nrhs + BN - 1) / BN, (m3_max + BM - 1) / BM, nmerge * ks);
  hipLaunchKernelGGL((k_down_mm<HPS_MMT(BM, BN)>), grid, dim3(MmCfg<BM, BN>::NT), 0, s, d_desc, U,
                     nrhs, zbase, zoff, io, ks, P, m3_max);
  if (ks > 1) {
    // One thread per output element: the top levels (one to a few merges)
    // would otherwise leave most of the chip idle while summing the chunks.
    const int bx = std::max(1, (m3_max * nrhs + 255) / 256);
    hipLaunchKernelGGL(k_down_reduce, dim3(bx, nmerge), dim3(256), 0, s, d_desc, U, nrhs, zbase,
                       zoff, ks, P, m3_max);
    HPS_HIP(hipFreeAsync(P, s));
  }
}

template <int BM>
static void launch_down_mm_bn(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max,
                              double* U, int nrhs, const double* zbase, const long long* zoff,
                              const SolveIO* io, hipStream_t s) {
  if (nrhs > 32)
    launch_down_mm<BM, 64>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
  else if (nrhs > 16)
    launch_down_mm<BM, 32>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
  else
    launch_down_mm<BM, 16>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
}

void downward_mm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, double* U, int nrhs,
                 const double* zbase, const long long* zoff, hipStream_t s, double s_bytes,
                 const SolveIO* io) {
  if (nmerge == 0) return;
  ProfScope ps(PROF_DOWNWARD, s, 2.0 * nrhs * s_bytes / 8.0, s_bytes);
  const int bm = mm_rows(m3_max);
  if (bm == 16)
    launch_down_mm_bn<16>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
  else if (bm == 32)
    launch_down_mm_bn<32>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
  else
    launch_down_mm_bn<64>(d_desc, nmerge, m3_max, me_max, U, nrhs, zbase, zoff, io, s);
}

// Node-major boundary data: U[gamma[i]][r] = f[r][i].
__global__ void k_set_boundary_nm(const double* __restrict__ f, const int* __restrict__ gamma,
                                  int nb, int nrhs, double* __restrict__ U) {
  const size_t tot = (size_t)nb * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / nrhs), r = (int)(e % nrhs);
    U[(size_t)gamma[i] * nrhs + r] = f[(size_t)r * nb + i];
  }
}

void set_boundary_nm(const double* f, const int* gamma, int nb, int nrhs, double* U,
                     hipStream_t s) {
  const size_t tot = (size_t)nb * nrhs;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_set_boundary_nm, dim3(std::max(blocks, 1)), dim3(256), 0, s, f, gamma, nb,
                     nrhs, U);
}

// out[c][r] = in[r][c] for an R x C row-major in (64 x 64 tiles through LDS).
__global__ void __launch_bounds__(256) k_transpose(const double* __restrict__ in, int R, int C,
                                                   double* __restrict__ out) {
  __shared__ double t[64][65];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int r = r0 + i, c = c0 + tx;
    if (r < R && c < C) t[i][tx] = in[(size_t)r * C + c];
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int c = c0 + i, r = r0 + tx;
    if (r < R && c < C) out[(size_t)c * R + r] = t[tx][i];
  }
}

void transpose(const double* in, int R, int C, double* out, hipStream_t s) {
  if (R == 0 || C == 0) return;
  HPS_REQUIRE((R + 63) / 64 <= 65535, "transpose: too many row tiles");
  dim3 grid((C + 63) / 64, (R + 63) / 64);
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, in, R, C, out);
}

// Interface residual, node-major: v_leaf = T_leaf U(I_e^leaf) for every leaf
// (one GEMM tile per leaf and column block), then the jump at every interior
// Gauss node.
struct LeafRows {
  int i, j, nx, nh, q;
  __device__ int operator()(int c) const { return leaf_bdry_id(i, j, nx, nh, q, c); }
};

template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) k_flux_mm(const double* __restrict__ T,
                                                         const double* __restrict__ U, int nrhs,
                                                         int nx, int ny, int q,
                                                         double* __restrict__ v) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const int leaf = blockIdx.z, m = 4 * q;
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  const LeafRows rows{leaf % nx, leaf / nx, nx, nx * (ny + 1), q};
  gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(T + (size_t)leaf * m * m, m, U, nrhs, rows,
                                    v + (size_t)leaf * m * nrhs, nrhs, RowsIdentity{}, nullptr, 0,
                                    m, nrhs, m, 1.0, row0, col0, sm, false);
}

__global__ void k_jump_nm(const double* __restrict__ v, int nx, int ny, int q, int nrhs,
                          double* __restrict__ r, int N) {
  const int nh = nx * (ny + 1), m = 4 * q;
  const size_t tot = (size_t)N * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int g = (int)(e / nrhs), rh = (int)(e % nrhs);
    const int edge = g / q, k = g % q;
    double val = 0.0;
    if (edge < nh) {
      const int i = edge % nx, j = edge / nx;
      if (j > 0 && j < ny)  // alpha = south leaf (its N side), beta = north leaf (its S side)
        val = v[((size_t)(i + nx * (j - 1)) * m + 2 * q + k) * nrhs + rh] -
              v[((size_t)(i + nx * j) * m + k) * nrhs + rh];
    } else {
      const int ve = edge - nh;
      const int i = ve % (nx + 1), j = ve / (nx + 1);
      if (i > 0 && i < nx)  // alpha = west leaf (its E side), beta = east leaf (its W side)
        val = v[((size_t)(i - 1 + nx * j) * m + q + k) * nrhs + rh] -
              v[((size_t)(i + nx * j) * m + 3 * q + k) * nrhs + rh];
    }
    r[e] = val;
  }
}

void interface_residual_nm(const double* leafT, const double* U, int N, int nrhs, int nx, int ny,
                           int q, double* vbuf, double* r, hipStream_t s) {
  const int m = 4 * q;
  HPS_REQUIRE(nx * ny <= 65535, "residual: too many leaves for one launch");
  ProfScope ps(PROF_RESIDUAL, s, 2.0 * nrhs * nx * ny * (double)m * m, 8.0 * nx * ny * (double)m * m);
  if (nrhs > 32) {
    dim3 grid((nrhs + 63) / 64, (m + 63) / 64, nx * ny);
    hipLaunchKernelGGL((k_flux_mm<HPS_MM_TILE(64)>), grid, dim3(MmCfg<64, 64>::NT), 0, s, leafT,
                       U, nrhs, nx, ny, q, vbuf);
  } else if (nrhs > 16) {
    dim3 grid((nrhs + 31) / 32, (m + 63) / 64, nx * ny);
    hipLaunchKernelGGL((k_flux_mm<HPS_MM_TILE(32)>), grid, dim3(MmCfg<64, 32>::NT), 0, s, leafT,
                       U, nrhs, nx, ny, q, vbuf);
  } else {
    dim3 grid((nrhs + 15) / 16, (m + 63) / 64, nx * ny);
    hipLaunchKernelGGL((k_flux_mm<HPS_MM_TILE(16)>), grid, dim3(MmCfg<64, 16>::NT), 0, s, leafT,
                       U, nrhs, nx, ny, q, vbuf);
  }
  const size_t tot = (size_t)N * nrhs;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 8192);
  hipLaunchKernelGGL(k_jump_nm, dim3(blocks), dim3(256), 0, s, vbuf, nx, ny, q, nrhs, r, N);
}

// Upward source pass for one depth, node-major (same equations as the row
// passes RowUpZ / RowUpH): rhs = s3 - h3a + h3b gathered per merge, then
// z = M^-1 rhs and h_parent = [h1a ; h2b] + Q z as grouped GEMMs.
// Rows of merge blockIdx.y: rhs[i][:] = src[Ii[i]][:] - ha[a3[i]][:] +
// hb[b3[i]][:]; thread (x, y) of a (64, 4) block takes column x (+ 64 j) of
// rows y + 4 k.  A leaf child (offset -1) contributes zero.
__global__ void __launch_bounds__(256) k_up_gather_nm(const MergeDesc* __restrict__ descs,
                                                      const double* __restrict__ src,
                                                      const double* __restrict__ hbase,
                                                      const long long* __restrict__ ha_off,
                                                      const long long* __restrict__ hb_off,
                                                      const long long* __restrict__ z_off,
                                                      int nrhs, double* __restrict__ rbuf) {
  const int mi = blockIdx.y;
  const MergeDesc d = descs[mi];
  const double* ha = ha_off[mi] < 0 ? nullptr : hbase + ha_off[mi] * nrhs;
  const double* hb = hb_off[mi] < 0 ? nullptr : hbase + hb_off[mi] * nrhs;
  double* rr = rbuf + z_off[mi] * nrhs;
  for (int i = blockIdx.x * 4 + threadIdx.y; i < d.m3; i += gridDim.x * 4) {
    const double* sr = src + (size_t)d.Ii[i] * nrhs;
    const double* ar = ha ? ha + (size_t)d.a3[i] * nrhs : nullptr;
    const double* br = hb ? hb + (size_t)d.b3[i] * nrhs : nullptr;
    for (int k = threadIdx.x; k < nrhs; k += 64)
      rr[(size_t)i * nrhs + k] = sr[k] - (ar ? ar[k] : 0.0) + (br ? br[k] : 0.0);
  }
}

// Row r of the pass-through [h1a ; h2b] of a parent, as a row of the h
// array (rows of nrhs values): alpha's row pmap[r] or beta's row
// -pmap[r] - 1; -1 (zero) for a leaf child.
struct PassRows {
  const int* pmap;
  long long ha, hb;
  __device__ int operator()(int r) const {
    const int pm = pmap[r];
    if (pm >= 0) return ha < 0 ? -1 : (int)(ha + pm);
    return hb < 0 ? -1 : (int)(hb - pm - 1);
  }
};

// z = M^-1 rhs (M^-1 at W + m3 + me) and h_parent += Q z for every merge of a
// depth; with ks > 1 the contraction over m3 is split as in k_down_mm and the
// partial products are summed in chunk order by k_up_reduce.
template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) k_up_z_mm(const MergeDesc* __restrict__ descs,
                                                         const double* __restrict__ rbuf,
                                                         double* __restrict__ zbuf,
                                                         const long long* __restrict__ z_off,
                                                         int nrhs, int ks, double* __restrict__ P,
                                                         int rows_max) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const int mi = blockIdx.z / ks, kc = blockIdx.z % ks;
  const MergeDesc d = descs[mi];
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  if (row0 >= d.m3 || col0 >= nrhs) return;
  const size_t o = z_off[mi] * nrhs;
  const int kchunk = ((d.m3 + ks - 1) / ks + BK - 1) / BK * BK;
  const int k0 = min(d.m3, kc * kchunk), K = min(kchunk, d.m3 - k0);
  double* C = ks == 1 ? zbuf + o : P + (size_t)blockIdx.z * rows_max * nrhs;
  gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(d.W + d.m3 + k0, d.ldw, rbuf + o + (size_t)k0 * nrhs,
                                    nrhs, RowsIdentity{}, C, nrhs, RowsIdentity{}, nullptr, 0,
                                    d.m3, nrhs, K, 1.0, row0, col0, sm, false);
}

template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) k_up_h_mm(const MergeDesc* __restrict__ descs,
                                                         const double* __restrict__ zbuf,
                                                         const long long* __restrict__ z_off,
                                                         double* __restrict__ hbase,
                                                         const long long* __restrict__ ha_off,
                                                         const long long* __restrict__ hb_off,
                                                         const long long* __restrict__ hp_off,
                                                         int nrhs, int ks, double* __restrict__ P,
                                                         int rows_max) {
  __shared__ double sm[GemmTile<BM, BN, BK, WM, WN>::SMEM];
  const int mi = blockIdx.z / ks, kc = blockIdx.z % ks;
  const MergeDesc d = descs[mi];
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  if (row0 >= d.me || col0 >= nrhs) return;
  const int kchunk = ((d.m3 + ks - 1) / ks + BK - 1) / BK * BK;
  const int k0 = min(d.m3, kc * kchunk), K = min(kchunk, d.m3 - k0);
  const double* B = zbuf + z_off[mi] * nrhs + (size_t)k0 * nrhs;
  if (ks == 1)
    gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(d.Q, d.m3, B, nrhs, RowsIdentity{},
                                      hbase + hp_off[mi] * nrhs, nrhs, RowsIdentity{}, hbase, nrhs,
                                      d.me, nrhs, d.m3, 1.0, row0, col0, sm, false,
                                      PassRows{d.pmap, ha_off[mi], hb_off[mi]});
  else
    gemm_tile_map_d<BM, BN, BK, WM, WN, 3>(d.Q + k0, d.m3, B, nrhs, RowsIdentity{},
                                      P + (size_t)blockIdx.z * rows_max * nrhs, nrhs,
                                      RowsIdentity{}, nullptr, 0, d.me, nrhs, K, 1.0, row0, col0,
                                      sm, false);
}

// dst rows of merge mi from the ks partial products: z (m3 rows) or, with
// to_h, h_parent (me rows) with its pass-through rows added.
__global__ void k_up_reduce(const MergeDesc* __restrict__ descs, double* __restrict__ base,
                            const long long* __restrict__ off, int nrhs, int ks,
                            const double* __restrict__ P, int rows_max, int to_h,
                            const double* __restrict__ hbase, const long long* __restrict__ ha_off,
                            const long long* __restrict__ hb_off) {
  const int mi = blockIdx.y;
  const MergeDesc d = descs[mi];
  const int rows = to_h ? d.me : d.m3;
  double* dst = base + off[mi] * nrhs;
  const double* Pm = P + (size_t)mi * ks * rows_max * nrhs;
  const PassRows pass{d.pmap, to_h ? ha_off[mi] : -1, to_h ? hb_off[mi] : -1};
  const int tot = rows * nrhs;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    double v = 0.0;
    if (to_h) {
      const int pr = pass(e / nrhs);
      if (pr >= 0) v = hbase[(size_t)pr * nrhs + e % nrhs];
    }
    for (int j = 0; j < ks; ++j) v += Pm[(size_t)j * rows_max * nrhs + e];
    dst[e] = v;
  }
}

template <int BMZ, int BN>
static void launch_up_mm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max,
                         double* hbase, const long long* ha_off, const long long* hb_off,
                         const long long* hp_off, double* rbuf, double* zbuf,
                         const long long* z_off, int nrhs, hipStream_t st) {
  const int ct = (nrhs + BN - 1) / BN;
  const int ksz = split_chunks((long long)ct * ((m3_max + BMZ - 1) / BMZ) * nmerge, m3_max);
  const int ksh = split_chunks((long long)ct * ((me_max + 63) / 64) * nmerge, m3_max);
  HPS_REQUIRE((long long)nmerge * std::max(ksz, ksh) <= 65535,
              "upward pass: too many merges at one depth");
  double* P = nullptr;
  const size_t pz = (size_t)nmerge * ksz * m3_max * nrhs, ph = (size_t)nmerge * ksh * me_max * nrhs;
  if (ksz > 1 || ksh > 1)
    HPS_HIP(hipMallocAsync((void**)&P, std::max(ksz > 1 ? pz : 0, ksh > 1 ? ph : 0) *
                                           sizeof(double), st));
  // Chunk sums: one thread per output element (see launch_down_mm).
  const int bx = std::max(1, ((m3_max + me_max) * nrhs + 255) / 256);
  dim3 gz(ct, (m3_max + BMZ - 1) / BMZ, nmerge * ksz);
  hipLaunchKernelGGL((k_up_z_mm<HPS_MMT(BMZ, BN)>), gz, dim3(MmCfg<BMZ, BN>::NT), 0, st, d_desc,
                     rbuf, zbuf, z_off, nrhs, ksz, P, m3_max);
  if (ksz > 1)
    hipLaunchKernelGGL(k_up_reduce, dim3(bx, nmerge), dim3(256), 0, st, d_desc, zbuf, z_off, nrhs,
                       ksz, P, m3_max, 0, hbase, ha_off, hb_off);
  dim3 gh(ct, (me_max + 63) / 64, nmerge * ksh);
  hipLaunchKernelGGL((k_up_h_mm<HPS_MM_TILE(BN)>), gh, dim3(MmCfg<64, BN>::NT), 0, st, d_desc, zbuf,
                     z_off, hbase, ha_off, hb_off, hp_off, nrhs, ksh, P, me_max);
  if (ksh > 1)
    hipLaunchKernelGGL(k_up_reduce, dim3(bx, nmerge), dim3(256), 0, st, d_desc, hbase, hp_off, nrhs,
                       ksh, P, me_max, 1, hbase, ha_off, hb_off);
  if (P) HPS_HIP(hipFreeAsync(P, st));
}

template <int BMZ>
static void launch_up_mm_bn(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max,
                            double* hbase, const long long* ha_off, const long long* hb_off,
                            const long long* hp_off, double* rbuf, double* zbuf,
                            const long long* z_off, int nrhs, hipStream_t st) {
  if (nrhs > 32)
    launch_up_mm<BMZ, 64>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                          zbuf, z_off, nrhs, st);
  else if (nrhs > 16)
    launch_up_mm<BMZ, 32>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                          zbuf, z_off, nrhs, st);
  else
    launch_up_mm<BMZ, 16>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                          zbuf, z_off, nrhs, st);
}

void upward_level_nm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, const double* src,
                     double* hbase, const long long* ha_off, const long long* hb_off,
                     const long long* hp_off, double* rbuf, double* zbuf, const long long* z_off,
                     int nrhs, double flops, hipStream_t st) {
  if (nmerge == 0) return;
  ProfScope ps(PROF_UPWARD, st, flops, 8.0 * flops / (2.0 * nrhs));
  const int bx = std::max(1, (m3_max + 3) / 4);  // one row per group of 64 threads
  hipLaunchKernelGGL(k_up_gather_nm, dim3(bx, nmerge), dim3(64, 4), 0, st, d_desc, src, hbase,
                     ha_off, hb_off, z_off, nrhs, rbuf);
  const int bm = mm_rows(m3_max);
  if (bm == 16)
    launch_up_mm_bn<16>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                        zbuf, z_off, nrhs, st);
  else if (bm == 32)
    launch_up_mm_bn<32>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                        zbuf, z_off, nrhs, st);
  else
    launch_up_mm_bn<64>(d_desc, nmerge, m3_max, me_max, hbase, ha_off, hb_off, hp_off, rbuf,
                        zbuf, z_off, nrhs, st);
}

void ops_init() {
  static bool done = false;
  if (done) return;
  done = true;
}

}  // namespace hps
