// Learned leaf-DtN surrogate (MLP with BF16 weights) -- host entry points.
#pragma once

#include <memory>
#include <vector>

#include "common.h"
#include "solver.h"

struct hps_surrogate {
  int p = 0, q = 0, m = 0, r = 0, D = 0, H = 0, O = 0;
  double hx = 0, hy = 0;
  double out_scale = 1.0;           // s in T = T_ref + s U V^T
  int step = 0;                     // Adam step count
  bool fitted = false;              // normalisation known
  std::vector<double> lo, hi;       // training ranges of c11, c22, c (judge flags leaves outside)
  float* W[3] = {};                 // FP32 master weights W1 (H x D), W2 (H x H), W3 (O x H)
  unsigned short* Wb[3] = {};       // BF16 copies used by the GEMMs
  float* b[3] = {};
  float *mW[3] = {}, *vW[3] = {}, *mb[3] = {}, *vb[3] = {};
  float* mu = nullptr;              // input normalisation
  float* sig = nullptr;
  double* Tref = nullptr;           // Laplace leaf DtN, m x m
  hps::DeviceMem mem;
  ~hps_surrogate();
};

namespace hps {

std::unique_ptr<hps_surrogate> surrogate_create(int p, int q, double hx, double hy, int hidden,
                                                int rank, unsigned long long seed, hipStream_t s);
// Trains on n samples: coefficients [n][6][p*p], FP64 leaf DtNs T [n][m][m] (device).
double surrogate_train(hps_surrogate* sg, const double* coeffs, const double* T, int n, int epochs,
                       int batch, double lr, unsigned long long seed, hipStream_t s,
                       std::vector<double>* history);
// Loss and all parameter gradients (W1 b1 W2 b2 W3 b3, FP32, host) of one batch.
double surrogate_grad(hps_surrogate* sg, const double* coeffs, const double* T, int n,
                      float* grads, hipStream_t s);
// T[i] = T_ref + s U V^T for n leaves with coefficient pointers dcp (device arrays of pointers).
void surrogate_predict(hps_surrogate* sg, const double* const* dcp, int n, double* const* dT,
                       hipStream_t s);
void block_errors(double* const* dA, const double* B, int n, int mm, double* err, hipStream_t s);
void block_replace(double* const* dA, const double* B, int n, int mm, const double* err, double tol,
                   hipStream_t s);
std::vector<char> surrogate_state(const hps_surrogate* sg);
void surrogate_set_state(hps_surrogate* sg, const char* buf, size_t len, hipStream_t s);

}  // namespace hps
