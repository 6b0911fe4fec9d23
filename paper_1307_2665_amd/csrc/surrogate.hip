// Learned leaf-DtN surrogate: a small MLP trained on (coefficient samples ->
// FP64 leaf DtN) pairs produced by the leaf solver itself, used in place of the
// leaf computation of section 3 for fields A u = -c11 u_11 - c22 u_22 + c u.
//
//   x  = ((c11, c22, c) at the p^2 Chebyshev nodes - mu) / sigma   (D = 3p^2)
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), o = W3 h2 + b3    (O = 2 m r)
//   T  = T_ref + s U V^T with U = o[:mr], V = o[mr:] (m x r, row-major)
//
// T_ref is the Laplace leaf DtN of the same leaf size.  Weights are held in
// BF16 for the GEMMs (FP32 master copies, FP32 Adam moments); every GEMM runs
// on BF16 MFMA 16x16x16 with FP32 accumulation.  The FP64 leaf solve is both
// the source of training targets and the judge of the surrogate's error.
#include "surrogate.h"

#include <cmath>
#include <cstring>
#include <fstream>
#include <random>

#include "prof.h"

namespace hps {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float x) {
  // round to nearest even
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

template <class T>
__device__ inline unsigned short to_bf(T v);
template <>
__device__ inline unsigned short to_bf<float>(float v) { return f2bf(v); }
template <>
__device__ inline unsigned short to_bf<unsigned short>(unsigned short v) { return v; }

// ---------------------------------------------------------------------------
// C[i][j] (FP32, ldc) = sum_k A(i,k) B(k,j) with A(i,k) = A[i*sai + k*sak],
// B(k,j) = B[k*sbk + j*sbj]; operands converted to BF16 when staged in LDS.
// EPI 0: C = acc (+ C if accum); 1: C = tanh(acc + bias[j]); 2: C = acc + bias[j].
// 64x64 tile per 256-thread workgroup, 4 waves of 2x2 MFMA 16x16x16 blocks.
// MFMA lane layout: A lane l holds A[l%16][4(l/16)..+3], B holds
// B[4(l/16)..+3][l%16], result register r holds D[4(l/16)+r][l%16].
// ---------------------------------------------------------------------------
template <class TA, class TB, int EPI>
__global__ void __launch_bounds__(256) k_bgemm(const TA* __restrict__ A, long sai, long sak,
                                               const TB* __restrict__ B, long sbk, long sbj,
                                               float* __restrict__ C, int ldc, int M, int N, int K,
                                               const float* __restrict__ bias, int accum) {
  __shared__ unsigned short As[64][16 + 4];
  __shared__ unsigned short Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      const int i = idx / 16, k = idx % 16;
      const int gi = row0 + i, gk = k0 + k;
      As[i][k] = (gi < M && gk < K) ? to_bf<TA>(A[gi * sai + gk * sak]) : (unsigned short)0;
      const int kk = idx / 64, j = idx % 64;
      const int gk2 = k0 + kk, gj = col0 + j;
      Bs[kk][j] = (gk2 < K && gj < N) ? to_bf<TB>(B[gk2 * sbk + gj * sbj]) : (unsigned short)0;
    }
    __syncthreads();
    s4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + i * 16 + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) a[i][t] = (short)As[r][4 * (lane >> 4) + t];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) b[j][t] = (short)Bs[4 * (lane >> 4) + t][c];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gj = col0 + wn * 32 + j * 16 + (lane & 15);
        if (gi < M && gj < N) {
          float v = acc[i][j][r];
          float* c = C + (size_t)gi * ldc + gj;
          if (EPI == 1)
            v = tanhf(v + bias[gj]);
          else if (EPI == 2)
            v += bias[gj];
          else if (accum)
            v += *c;
          *c = v;
        }
      }
}

template <class TA, class TB, int EPI>
static void bgemm(const TA* A, long sai, long sak, const TB* B, long sbk, long sbj, float* C,
                  int ldc, int M, int N, int K, const float* bias, hipStream_t s) {
  dim3 g((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_bgemm<TA, TB, EPI>), g, dim3(256), 0, s, A, sai, sak, B, sbk, sbj, C, ldc,
                     M, N, K, bias, 0);
}

// ---------------------------------------------------------------------------
// Elementwise pieces.
// ---------------------------------------------------------------------------
__global__ void k_features(const double* const* __restrict__ cptr, int pp,
                           const float* __restrict__ mu, const float* __restrict__ sig,
                           float* __restrict__ X, int B) {
  const int D = 3 * pp;
  const size_t tot = (size_t)B * D;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / D), d = (int)(e % D);
    const int f = d / pp, node = d % pp;
    const int field = (f == 0) ? 0 : (f == 1 ? 2 : 5);  // c11, c22, c
    const double v = cptr[b][(size_t)field * pp + node];
    X[e] = mu ? (float)((v - mu[d]) / sig[d]) : (float)v;
  }
}

// dA = dH * (1 - H^2) in place on dH.
__global__ void k_tanh_back(float* __restrict__ dH, const float* __restrict__ Hv, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    dH[e] *= 1.0f - Hv[e] * Hv[e];
}

// db[j] = sum_b dA[b][j].
__global__ void k_colsum(const float* __restrict__ dA, int Bn, int N, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int b = 0; b < Bn; ++b) s += dA[(size_t)b * N + j];
  db[j] = s;
}

// Per sample: R = U V^T - Y with Y = (T - Tref)/s; loss partial; dU = g R V,
// dV = g R^T U, g = 2 / (m^2 B).  One workgroup per sample.
__global__ void __launch_bounds__(256) k_lowrank_loss(const float* __restrict__ O, int m, int r,
                                                      const double* const* __restrict__ Tt,
                                                      const double* __restrict__ Tref, double s,
                                                      float* __restrict__ dO,
                                                      double* __restrict__ lossp, int Bn) {
  extern __shared__ float sm[];
  const int b = blockIdx.x, O_ = 2 * m * r;
  float* U = sm;
  float* V = sm + m * r;
  float* R = sm + 2 * m * r;
  const float* o = O + (size_t)b * O_;
  for (int e = threadIdx.x; e < O_; e += blockDim.x) sm[e] = o[e];
  __syncthreads();
  const double* T = Tt[b];
  double lp = 0.0;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    float acc = 0.f;
    for (int k = 0; k < r; ++k) acc += U[i * r + k] * V[j * r + k];
    const float y = (float)((T[e] - Tref[e]) / s);
    const float res = acc - y;
    R[e] = res;
    lp += (double)res * res;
  }
  __shared__ double red[256];
  red[threadIdx.x] = lp;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[b] = red[0] / ((double)m * m * Bn);
  const float g = 2.0f / ((float)m * m * Bn);
  float* d = dO + (size_t)b * O_;
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) {
    const int i = e / r, k = e % r;
    float su = 0.f, sv = 0.f;
    for (int j = 0; j < m; ++j) {
      su += R[i * m + j] * V[j * r + k];
      sv += R[j * m + i] * U[j * r + k];
    }
    d[e] = g * su;
    d[m * r + e] = g * sv;
  }
}

__global__ void k_adam(float* __restrict__ w, unsigned short* __restrict__ wb,
                       const float* __restrict__ g, float* __restrict__ mm, float* __restrict__ vv,
                       size_t n, float lr, float c1, float c2) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float m1 = 0.9f * mm[e] + 0.1f * ge;
    const float v1 = 0.999f * vv[e] + 0.001f * ge * ge;
    mm[e] = m1;
    vv[e] = v1;
    const float nw = w[e] - lr * (m1 / c1) / (sqrtf(v1 / c2) + 1e-8f);
    w[e] = nw;
    if (wb) wb[e] = f2bf(nw);
  }
}

__global__ void k_to_bf16(const float* __restrict__ w, unsigned short* __restrict__ wb, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    wb[e] = f2bf(w[e]);
}

// T[leaf] = Tref + s U V^T in FP64; one workgroup per leaf.
__global__ void __launch_bounds__(256) k_expand(const float* __restrict__ O, int m, int r,
                                                const double* __restrict__ Tref, double s,
                                                double* const* __restrict__ Tout) {
  extern __shared__ float sm[];
  const int b = blockIdx.x, O_ = 2 * m * r;
  const float* o = O + (size_t)b * O_;
  for (int e = threadIdx.x; e < O_; e += blockDim.x) sm[e] = o[e];
  __syncthreads();
  const float* U = sm;
  const float* V = sm + m * r;
  double* T = Tout[b];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    float acc = 0.f;
    for (int k = 0; k < r; ++k) acc += U[i * r + k] * V[j * r + k];
    T[e] = Tref[e] + s * (double)acc;
  }
}

// err[b] = max |A_b - B_b| / max |B_b| for m x m blocks.
__global__ void __launch_bounds__(256) k_block_err(double* const* __restrict__ A,
                                                   const double* __restrict__ Bv, int mm,
                                                   double* __restrict__ err) {
  __shared__ double sd[256], sb[256];
  const int b = blockIdx.x;
  const double* a = A[b];
  const double* bb = Bv + (size_t)b * mm;
  double md = 0, mb = 0;
  for (int e = threadIdx.x; e < mm; e += blockDim.x) {
    md = fmax(md, fabs(a[e] - bb[e]));
    mb = fmax(mb, fabs(bb[e]));
  }
  sd[threadIdx.x] = md;
  sb[threadIdx.x] = mb;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + st]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[b] = sd[0] / fmax(sb[0], 1e-300);
}

// Copy judged FP64 blocks into place where flagged.
__global__ void k_replace(double* const* __restrict__ A, const double* __restrict__ Bv, int mm,
                          const double* __restrict__ err, double tol) {
  const int b = blockIdx.x;
  if (!(err[b] <= tol)) {
    double* a = A[b];
    for (int e = threadIdx.x; e < mm; e += blockDim.x) a[e] = Bv[(size_t)b * mm + e];
  }
}

static inline int nblk(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 8192); }

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
}  // namespace hps

using namespace hps;

hps_surrogate::~hps_surrogate() = default;

namespace hps {

static void upload_f(float* d, const std::vector<double>& v, hipStream_t s) {
  std::vector<float> f(v.begin(), v.end());
  HPS_HIP(hipMemcpyAsync(d, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HPS_HIP(hipStreamSynchronize(s));
}

std::unique_ptr<hps_surrogate> surrogate_create(int p, int q, double hx, double hy, int hidden,
                                                int rank, unsigned long long seed, hipStream_t s) {
  HPS_REQUIRE(p >= 4 && p <= 24 && q >= 1 && q < p && hidden >= 8 && rank >= 1 && rank <= 4 * q,
              "bad surrogate shape");
  auto sg = std::make_unique<hps_surrogate>();
  sg->p = p;
  sg->q = q;
  sg->m = 4 * q;
  sg->r = rank;
  sg->D = 3 * p * p;
  sg->H = hidden;
  sg->O = 2 * sg->m * rank;
  sg->hx = hx;
  sg->hy = hy;
  const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
  const int bs[3] = {sg->H, sg->H, sg->O};
  const int fan[3] = {sg->D, sg->H, sg->H};
  std::mt19937_64 rng(seed);
  for (int l = 0; l < 3; ++l) {
    sg->W[l] = sg->mem.alloc<float>(sz[l]);
    sg->Wb[l] = sg->mem.alloc<unsigned short>(sz[l]);
    sg->b[l] = sg->mem.alloc<float>(bs[l]);
    sg->mW[l] = sg->mem.alloc<float>(sz[l]);
    sg->vW[l] = sg->mem.alloc<float>(sz[l]);
    sg->mb[l] = sg->mem.alloc<float>(bs[l]);
    sg->vb[l] = sg->mem.alloc<float>(bs[l]);
    std::uniform_real_distribution<double> U(-1.0 / std::sqrt(fan[l]), 1.0 / std::sqrt(fan[l]));
    std::vector<double> w(sz[l]);
    for (auto& x : w) x = U(rng);
    if (l == 2)  // small output layer: start near T = T_ref
      for (auto& x : w) x *= 0.1;
    upload_f(sg->W[l], w, s);
    HPS_HIP(hipMemsetAsync(sg->b[l], 0, bs[l] * sizeof(float), s));
    HPS_HIP(hipMemsetAsync(sg->mW[l], 0, sz[l] * sizeof(float), s));
    HPS_HIP(hipMemsetAsync(sg->vW[l], 0, sz[l] * sizeof(float), s));
    HPS_HIP(hipMemsetAsync(sg->mb[l], 0, bs[l] * sizeof(float), s));
    HPS_HIP(hipMemsetAsync(sg->vb[l], 0, bs[l] * sizeof(float), s));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(sz[l])), dim3(256), 0, s, sg->W[l], sg->Wb[l],
                       (size_t)sz[l]);
  }
  sg->mu = sg->mem.alloc<float>(sg->D);
  sg->sig = sg->mem.alloc<float>(sg->D);
  sg->Tref = sg->mem.alloc<double>((size_t)sg->m * sg->m);
  // T_ref: the Laplace leaf DtN of this leaf size, from the FP64 leaf solver.
  std::vector<double> lap((size_t)6 * p * p, 0.0);
  for (int k = 0; k < p * p; ++k) lap[k] = lap[2 * p * p + k] = 1.0;
  DeviceMem tmp;
  double* dlap = tmp.upload(lap, s);
  leaf_dtn_batch(dlap, 1, hx, hy, p, q, sg->Tref, s);
  HPS_HIP(hipStreamSynchronize(s));
  return sg;
}

// Forward pass for B samples given coefficient pointers; fills the activations.
static void forward(hps_surrogate* sg, const double* const* dcp, int B, float* X, float* H1,
                    float* H2, float* O, hipStream_t s) {
  const int D = sg->D, H = sg->H, Ot = sg->O;
  hipLaunchKernelGGL(k_features, dim3(nblk((size_t)B * D)), dim3(256), 0, s, dcp, sg->p * sg->p,
                     sg->mu, sg->sig, X, B);
  // H1[b][h] = tanh(sum_d X[b][d] W1[h][d] + b1[h]): B(k=d, j=h) = W1[h*D + d].
  bgemm<float, unsigned short, 1>(X, D, 1, sg->Wb[0], 1, D, H1, H, B, H, D, sg->b[0], s);
  bgemm<float, unsigned short, 1>(H1, H, 1, sg->Wb[1], 1, H, H2, H, B, H, H, sg->b[1], s);
  bgemm<float, unsigned short, 2>(H2, H, 1, sg->Wb[2], 1, H, O, Ot, B, Ot, H, sg->b[2], s);
}

struct Work {
  DeviceMem mem;
  float *X, *H1, *H2, *O, *dO, *dH2, *dH1, *gW[3], *gb[3];
  double* lossp;
  const double** cp;
  const double** tp;
  Work(const hps_surrogate* sg, int B) {
    X = mem.alloc<float>((size_t)B * sg->D);
    H1 = mem.alloc<float>((size_t)B * sg->H);
    H2 = mem.alloc<float>((size_t)B * sg->H);
    O = mem.alloc<float>((size_t)B * sg->O);
    dO = mem.alloc<float>((size_t)B * sg->O);
    dH2 = mem.alloc<float>((size_t)B * sg->H);
    dH1 = mem.alloc<float>((size_t)B * sg->H);
    const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
    const int bs[3] = {sg->H, sg->H, sg->O};
    for (int l = 0; l < 3; ++l) {
      gW[l] = mem.alloc<float>(sz[l]);
      gb[l] = mem.alloc<float>(bs[l]);
    }
    lossp = mem.alloc<double>(B);
    cp = mem.alloc<const double*>(B);
    tp = mem.alloc<const double*>(B);
  }
};

// One forward + backward over B samples: gradients into w.gW / w.gb, loss returned.
static double forward_backward(hps_surrogate* sg, Work& w, int B, hipStream_t s) {
  const int D = sg->D, H = sg->H, Ot = sg->O, m = sg->m, r = sg->r;
  ProfScope ps(PROF_MLP_TRAIN, s, 6.0 * B * ((double)D * H + (double)H * H + (double)H * Ot), 0);
  forward(sg, w.cp, B, w.X, w.H1, w.H2, w.O, s);
  const size_t shm = ((size_t)2 * m * r + (size_t)m * m) * sizeof(float);
  hipLaunchKernelGGL(k_lowrank_loss, dim3(B), dim3(256), shm, s, w.O, m, r, w.tp, sg->Tref,
                     sg->out_scale, w.dO, w.lossp, B);
  // dW3[o][h] = sum_b dO[b][o] H2[b][h]: A(i=o,k=b) = dO[b*Ot + o], B(k=b,j=h) = H2[b*H + h].
  bgemm<float, float, 0>(w.dO, 1, Ot, w.H2, H, 1, w.gW[2], H, Ot, H, B, nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((Ot + 255) / 256), dim3(256), 0, s, w.dO, B, Ot, w.gb[2]);
  // dH2[b][h] = sum_o dO[b][o] W3[o][h].
  bgemm<float, unsigned short, 0>(w.dO, Ot, 1, sg->Wb[2], H, 1, w.dH2, H, B, H, Ot, nullptr, s);
  hipLaunchKernelGGL(k_tanh_back, dim3(nblk((size_t)B * H)), dim3(256), 0, s, w.dH2, w.H2,
                     (size_t)B * H);
  bgemm<float, float, 0>(w.dH2, 1, H, w.H1, H, 1, w.gW[1], H, H, H, B, nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, w.dH2, B, H, w.gb[1]);
  bgemm<float, unsigned short, 0>(w.dH2, H, 1, sg->Wb[1], H, 1, w.dH1, H, B, H, H, nullptr, s);
  hipLaunchKernelGGL(k_tanh_back, dim3(nblk((size_t)B * H)), dim3(256), 0, s, w.dH1, w.H1,
                     (size_t)B * H);
  bgemm<float, float, 0>(w.dH1, 1, H, w.X, D, 1, w.gW[0], D, H, D, B, nullptr, s);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, w.dH1, B, H, w.gb[0]);
  std::vector<double> lp(B);
  HPS_HIP(hipMemcpyAsync(lp.data(), w.lossp, B * sizeof(double), hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  double L = 0;
  for (double v : lp) L += v;
  return L;
}

static void set_ptrs(const double** dst, const double* base, size_t stride, const int* idx, int B,
                     hipStream_t s) {
  std::vector<const double*> v(B);
  for (int i = 0; i < B; ++i) v[i] = base + stride * (size_t)idx[i];
  HPS_HIP(hipMemcpyAsync(dst, v.data(), B * sizeof(void*), hipMemcpyHostToDevice, s));
  HPS_HIP(hipStreamSynchronize(s));
}

// Feature statistics and output scale from the whole training set (host, FP64).
static void fit_normalisation(hps_surrogate* sg, const double* coeffs, const double* T, int n,
                              hipStream_t s) {
  const int pp = sg->p * sg->p, D = sg->D, mm = sg->m * sg->m;
  std::vector<double> hc((size_t)n * 6 * pp), ht((size_t)n * mm), tref(mm);
  HPS_HIP(hipMemcpyAsync(hc.data(), coeffs, hc.size() * 8, hipMemcpyDeviceToHost, s));
  HPS_HIP(hipMemcpyAsync(ht.data(), T, ht.size() * 8, hipMemcpyDeviceToHost, s));
  HPS_HIP(hipMemcpyAsync(tref.data(), sg->Tref, mm * 8, hipMemcpyDeviceToHost, s));
  HPS_HIP(hipStreamSynchronize(s));
  std::vector<double> mu(D, 0.0), sd(D, 0.0);
  const int field[3] = {0, 2, 5};
  sg->lo.assign(3, 1e300);
  sg->hi.assign(3, -1e300);
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < D; ++d) {
      const int f = d / pp;
      const double v = hc[((size_t)i * 6 + field[f]) * pp + d % pp];
      mu[d] += v;
      sd[d] += v * v;
      sg->lo[f] = std::min(sg->lo[f], v);
      sg->hi[f] = std::max(sg->hi[f], v);
    }
  for (int d = 0; d < D; ++d) {
    mu[d] /= n;
    sd[d] = std::sqrt(std::max(sd[d] / n - mu[d] * mu[d], 0.0));
    if (sd[d] < 1e-12) sd[d] = 1.0;
  }
  double s2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int e = 0; e < mm; ++e) {
      const double dlt = ht[(size_t)i * mm + e] - tref[e];
      s2 += dlt * dlt;
    }
  sg->out_scale = std::sqrt(s2 / ((double)n * mm));
  if (!(sg->out_scale > 0)) sg->out_scale = 1.0;
  // Y = U V^T is a product of two factors of size ~1 each at initialisation.
  upload_f(sg->mu, mu, s);
  upload_f(sg->sig, sd, s);
  sg->fitted = true;
}

double surrogate_train(hps_surrogate* sg, const double* coeffs, const double* T, int n, int epochs,
                       int batch, double lr, unsigned long long seed, hipStream_t s,
                       std::vector<double>* history) {
  HPS_REQUIRE(n >= 1 && epochs >= 1 && batch >= 1, "bad training arguments");
  if (!sg->fitted) fit_normalisation(sg, coeffs, T, n, s);
  const int B = std::min(batch, n);
  Work w(sg, B);
  std::mt19937_64 rng(seed);
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  const int pp = sg->p * sg->p, mm = sg->m * sg->m;
  const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
  const int bs[3] = {sg->H, sg->H, sg->O};
  double last = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    double el = 0.0;
    int nb = 0;
    for (int i0 = 0; i0 + B <= n; i0 += B) {
      set_ptrs(w.cp, coeffs, (size_t)6 * pp, perm.data() + i0, B, s);
      set_ptrs(w.tp, T, (size_t)mm, perm.data() + i0, B, s);
      el += forward_backward(sg, w, B, s);
      ++nb;
      ++sg->step;
      const float c1 = 1.0f - std::pow(0.9f, (float)sg->step);
      const float c2 = 1.0f - std::pow(0.999f, (float)sg->step);
      for (int l = 0; l < 3; ++l) {
        hipLaunchKernelGGL(k_adam, dim3(nblk(sz[l])), dim3(256), 0, s, sg->W[l], sg->Wb[l],
                           w.gW[l], sg->mW[l], sg->vW[l], (size_t)sz[l], (float)lr, c1, c2);
        hipLaunchKernelGGL(k_adam, dim3(nblk(bs[l])), dim3(256), 0, s, sg->b[l],
                           (unsigned short*)nullptr, w.gb[l], sg->mb[l], sg->vb[l], (size_t)bs[l],
                           (float)lr, c1, c2);
      }
    }
    last = el / std::max(nb, 1);
    if (history) history->push_back(last);
  }
  HPS_HIP(hipStreamSynchronize(s));
  return last;
}

double surrogate_grad(hps_surrogate* sg, const double* coeffs, const double* T, int n,
                      float* grads, hipStream_t s) {
  HPS_REQUIRE(sg->fitted, "surrogate has no normalisation yet (train it or set its state)");
  Work w(sg, n);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  set_ptrs(w.cp, coeffs, (size_t)6 * sg->p * sg->p, idx.data(), n, s);
  set_ptrs(w.tp, T, (size_t)sg->m * sg->m, idx.data(), n, s);
  const double L = forward_backward(sg, w, n, s);
  const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
  const int bs[3] = {sg->H, sg->H, sg->O};
  size_t o = 0;
  for (int l = 0; l < 3; ++l) {
    HPS_HIP(hipMemcpyAsync(grads + o, w.gW[l], sz[l] * sizeof(float), hipMemcpyDeviceToHost, s));
    o += sz[l];
    HPS_HIP(hipMemcpyAsync(grads + o, w.gb[l], bs[l] * sizeof(float), hipMemcpyDeviceToHost, s));
    o += bs[l];
  }
  HPS_HIP(hipStreamSynchronize(s));
  return L;
}

void surrogate_predict(hps_surrogate* sg, const double* const* dcp, int n, double* const* dT,
                       hipStream_t s) {
  HPS_REQUIRE(sg->fitted, "surrogate is not trained");
  const int B = std::min(n, 16384);
  Work w(sg, B);
  ProfScope ps(PROF_MLP_INFER, s,
               2.0 * n * ((double)sg->D * sg->H + (double)sg->H * sg->H + (double)sg->H * sg->O +
                          (double)sg->m * sg->m * sg->r), 0);
  for (int i0 = 0; i0 < n; i0 += B) {
    const int cnt = std::min(B, n - i0);
    forward(sg, dcp + i0, cnt, w.X, w.H1, w.H2, w.O, s);
    hipLaunchKernelGGL(k_expand, dim3(cnt), dim3(256), 2 * sg->m * sg->r * sizeof(float), s, w.O,
                       sg->m, sg->r, sg->Tref, sg->out_scale, dT + i0);
  }
}

void block_errors(double* const* dA, const double* B, int n, int mm, double* err, hipStream_t s) {
  hipLaunchKernelGGL(k_block_err, dim3(n), dim3(256), 0, s, dA, B, mm, err);
}

void block_replace(double* const* dA, const double* B, int n, int mm, const double* err, double tol,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_replace, dim3(n), dim3(256), 0, s, dA, B, mm, err, tol);
}

// State: [meta doubles][mu][sig][W1 b1 W2 b2 W3 b3] all as FP32 after the meta block.
std::vector<char> surrogate_state(const hps_surrogate* sg) {
  std::vector<double> meta = {(double)sg->p, (double)sg->q, (double)sg->H, (double)sg->r,
                              sg->hx, sg->hy, sg->out_scale, (double)sg->step,
                              sg->lo[0], sg->lo[1], sg->lo[2], sg->hi[0], sg->hi[1], sg->hi[2]};
  std::vector<char> out(meta.size() * 8);
  std::memcpy(out.data(), meta.data(), out.size());
  auto add = [&](const float* d, size_t n) {
    size_t o = out.size();
    out.resize(o + n * 4);
    HPS_HIP(hipMemcpy(out.data() + o, d, n * 4, hipMemcpyDeviceToHost));
  };
  add(sg->mu, sg->D);
  add(sg->sig, sg->D);
  const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
  const int bs[3] = {sg->H, sg->H, sg->O};
  for (int l = 0; l < 3; ++l) {
    add(sg->W[l], sz[l]);
    add(sg->b[l], bs[l]);
  }
  return out;
}

void surrogate_set_state(hps_surrogate* sg, const char* buf, size_t len, hipStream_t s) {
  const size_t meta = 14 * 8;
  const int sz[3] = {sg->H * sg->D, sg->H * sg->H, sg->O * sg->H};
  const int bs[3] = {sg->H, sg->H, sg->O};
  size_t need = meta + (size_t)2 * sg->D * 4;
  for (int l = 0; l < 3; ++l) need += (size_t)(sz[l] + bs[l]) * 4;
  HPS_REQUIRE(len == need, "surrogate state has the wrong size");
  double m[14];
  std::memcpy(m, buf, meta);
  HPS_REQUIRE((int)m[0] == sg->p && (int)m[1] == sg->q && (int)m[2] == sg->H && (int)m[3] == sg->r,
              "surrogate state shape mismatch");
  sg->out_scale = m[6];
  sg->step = (int)m[7];
  sg->lo = {m[8], m[9], m[10]};
  sg->hi = {m[11], m[12], m[13]};
  size_t o = meta;
  auto put = [&](float* d, size_t n) {
    HPS_HIP(hipMemcpy(d, buf + o, n * 4, hipMemcpyHostToDevice));
    o += n * 4;
  };
  put(sg->mu, sg->D);
  put(sg->sig, sg->D);
  for (int l = 0; l < 3; ++l) {
    put(sg->W[l], sz[l]);
    put(sg->b[l], bs[l]);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(sz[l])), dim3(256), 0, s, sg->W[l], sg->Wb[l],
                       (size_t)sz[l]);
  }
  HPS_HIP(hipStreamSynchronize(s));
  sg->fitted = true;
}

}  // namespace hps
