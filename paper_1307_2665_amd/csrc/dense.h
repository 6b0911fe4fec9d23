// Batched dense FP64 kernels (LU solve, grouped GEMM) -- host entry points.
#pragma once

#include <vector>

#include "common.h"

namespace hps {

// Solves every system of the batch in place by block Gauss-Jordan elimination
// with partial pivoting: afterwards W[:, n:n+m] holds X = M^-1 B (X must be
// W + n with ldx = ld).  d_status[0] becomes 1 (and d_status[1] the tag) if a
// pivot is exactly zero or not finite.  n <= max_solve_rows().
void batched_solve(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                   hipStream_t stream, int nb);

// C += alpha A B for every descriptor, FP64 MFMA (or the split-FP32 form).
void grouped_gemm(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                  bool split32);

// The same with explicit kernel variants (the autotuner times them):
// gj_variant = update tile * 4 + TRSM block code (see tune.h), -1 = default;
// variant = FP64 MFMA tile of gemm_tile (0..5), -1 = default.
void batched_solve_v(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                     hipStream_t stream, int gj_variant);
void grouped_gemm_v(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                    int variant, bool split32);

void dense_init();
int max_solve_rows();

}  // namespace hps
