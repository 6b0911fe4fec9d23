// Batched FP64 products for gfx950: the grouped MFMA GEMM tiles (Schur
// products T = diag(T11a, T22b) + Q S of eq:merge, S = M^-1 B of
// eq:U_parent, the leaf's T = P0 - P1 Z), the persistent tile-queue form for
// batches, and the split-FP32 and BF16 three-slice variants of the Schur
// product.  The eliminations live in gj.hip.
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

constexpr int TBM = 64, TBN = 64, TBK = 16;  // tile of the split-FP32 kernel

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

// The old values of a plain product for the 128 tile, through the same
// row / column form as the pass-through: C0 if given, else C itself when
// accumulating, else zero (row offsets fit an int for matrices under 2^31
// elements).
struct PlainOld {
  static constexpr bool active = true;
  const double* __restrict__ src;
  int ld, use;
  __device__ int row(int r) const { return r * ld; }
  __device__ int col(int c) const { return c; }
  __device__ double value(int pr, int pc) const { return use ? as_global(src)[pr + pc] : 0.0; }
  __device__ double operator()(int r, int c) const { return value(row(r), col(c)); }
};

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
  else  // old values through PlainOld: the NoC0Elem form of this tile spills registers
    gemm128_tile<VEC>(g.A, g.lda, g.B, g.ldb, g.C, g.ldc, nullptr, 0, g.M, g.N, g.K, g.alpha,
                      ty * Gemm128::BM, tx * Gemm128::BN, sm, false,
                      PlainOld{g.C0 ? g.C0 : g.C, g.C0 ? g.ldc0 : g.ldc,
                               (g.C0 || g.overwrite == 0) ? 1 : 0});
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

void dense_init() {}

}  // namespace hps
