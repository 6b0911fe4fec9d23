// HBS matrices (sections 6-7) on the device: the telescoping product,
// Algorithm 3 (inversion) and Algorithm 4 (application of the inverse).
#pragma once

#include <vector>

#include "common.h"

namespace hps {

// Offsets (in doubles) of the blocks of an HBS matrix of M = m 2^L rows with
// one rank k at every node, in the buffer layouts documented in hps.h.
// rows(l): m at the leaves (l = L), 2k at a parent.
struct HbsLayout {
  int L = 0, m = 0, k = 0;
  size_t D = 0, U = 0, Vt = 0;          // leaves
  std::vector<size_t> Up, Vtp, B;       // Up/Vtp: l = 1 .. L-1; B: l = 0 .. L-1
  size_t nfac = 0;
  std::vector<size_t> E, Fs, G;         // l = 1 .. L; G[0]: the root's block
  size_t ninv = 0;
  HbsLayout(int L, int m, int k);
  int rows(int l) const { return l == L ? m : 2 * k; }
  long long M() const { return (long long)m << L; }
};

// Checks the sizes (HPS_EINVAL otherwise).
void hbs_check(int L, int m, int k);
// y = H x (x, y: M x nrhs row-major, device; y must not overlap x).
void hbs_apply(const HbsLayout& lo, const double* fac, const double* x, double* y, int nrhs,
               hipStream_t s);
// Algorithm 3: the factors E, F*, G of H^-1 into inv.  Raises HPS_ESINGULAR
// when a block it inverts has a zero or non-finite pivot.
void hbs_invert(const HbsLayout& lo, const double* fac, double* inv, hipStream_t s);
// Algorithm 4: y = H^-1 x from the factors of hbs_invert.
void hbs_solve(const HbsLayout& lo, const double* inv, const double* x, double* y, int nrhs,
               hipStream_t s);

// Brute-force compression of the dense M x M matrix H (row stride ldh, device)
// into factors of rank k from the caller's random samples omega (M x k) and
// psit (k x M).  k <= 90 and m k <= 16384 (the bases are orthonormalized in
// LDS).
void hbs_compress(const HbsLayout& lo, const double* H, int ldh, const double* omega,
                  const double* psit, double* fac, hipStream_t s);
int hbs_max_compress_rank(int m);
// Drops the recorded apply / solve passes (the device must be idle).
void hbs_passes_clear();
// Workgroups of the persistent apply / solve launch (0: two per CU).
void hbs_set_pass_grid(int workgroups);

}  // namespace hps
