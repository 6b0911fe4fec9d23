// Fused register-resident leaf solve (section 3.1) -- host entry points.
#pragma once

#include "common.h"
#include "ops.h"

namespace hps {

// True when the augmented leaf system (n rows, n + m columns) fits a register variant.
bool leaf_lu_fits(int n, int m);

// Z[leaf] = A_ii^-1 R for count leaves (coefficients cptr[leaf]); Z is [count][n][m].
// status[0] becomes 1 and status[1] = tag0 - leaf on a zero or non-finite pivot,
// or (tol > 0) on a pivot with |pivot| <= tol max|A_ii|.
// Kernel variant: 0-2 step-by-step LU (16x16 threads for p <= 12, 16x64, 16x32), 3-4
// blocked Gauss-Jordan (16x16 threads, 9-column blocks; 16x32 threads, 8-column blocks).
void leaf_lu_set_variant(int v);

// MFMA leaf solve with the DtN formed in-kernel: T[leaf] = P0 - P1 A_ii^-1 R
// (P0 [m][m], P1 [m][n], tdst[leaf] -> [m][m]) for leaf shapes where
// leaf_mfma_fits(n, m); statuses as leaf_lu.
// (leaf_set_mfma(false) turns the MFMA path off: leaves then take leaf_lu and
// a separate T product.)
bool leaf_mfma_fits(int n, int m);
void leaf_set_mfma(bool on);
void leaf_dtn_mfma(const double* const* cptr, const LeafDev& tab, const double* P0,
                   const double* P1, double* const* tdst, int count, int* status, int tag0,
                   hipStream_t s, double tol = 0.0);

void leaf_lu(const double* const* cptr, const LeafDev& tab, int count, double* Z, int* status,
             int tag0, hipStream_t s, double tol = 0.0);

}  // namespace hps
