// Batched dense FP64 kernels (LU solve, grouped GEMM) -- host entry points.
#pragma once

#include <vector>

#include "common.h"

namespace hps {

// Solves every system of the batch in place: LU with partial pivoting of M,
// forward elimination of B during the factorization, then back substitution
// into X.  Panel width nb (<= 32).  d_status[0] becomes 1 (and d_status[1]
// the tag) if a pivot is exactly zero or not finite.
void batched_solve(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                   hipStream_t stream, int nb);

// C += alpha A B for every descriptor, FP64 MFMA (or the split-FP32 form).
void grouped_gemm(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                  bool split32);

void dense_init();

}  // namespace hps
