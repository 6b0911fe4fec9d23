// Shared definitions of the HIP library: error plumbing, device descriptors.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/hps.h"

namespace hps {

// Error carried from deep inside the library to the C ABI, where it becomes a
// status code plus a thread-local message.  Exceptions never cross the ABI.
struct Error : std::runtime_error {
  hps_status status;
  Error(hps_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define HPS_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::hps::Error(e_ == hipErrorOutOfMemory ? HPS_ENOMEM : HPS_EDEVICE,          \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define HPS_REQUIRE(cond, msg)                                                          \
  do {                                                                                  \
    if (!(cond)) throw ::hps::Error(HPS_EINVAL, msg);                                   \
  } while (0)

// One dense system of the batched solver: the augmented row-major matrix
// W = [M | B] (n rows, n + m columns used, leading dimension ld) is factored in
// place (LU with partial pivoting of M, forward elimination applied to B) and
// X = M^-1 B is written to X (n rows, leading dimension ldx).
struct SolveDesc {
  double* W;
  int* piv;        // n pivot rows (absolute row index chosen at each column)
  double* X;
  int n, m, ld, ldx;
  int tag;         // caller's id (box or leaf), reported on singular pivots
  int pad;
};

// C (M x N, ldc) = C0 + alpha * A (M x K, lda) * B (K x N, ldb), all row-major
// FP64, where C0 is the matrix at C0 (leading dimension ldc0) when C0 is not
// null and the old contents of C otherwise.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  const double* C0;
  int M, N, K;
  int lda, ldb, ldc, ldc0;
  double alpha;
  // Merge Schur product (eq:merge): with pmap set, C0 is the parent's
  // block-diagonal pass-through diag(T11a, T22b), read from the children's
  // DtNs through the parent-order map pmap (>= 0: row/column of Ta, < 0:
  // -(row/column of Tb) - 1); C0 and the old C are then not read.
  const int* pmap = nullptr;
  const double* Ta = nullptr;
  const double* Tb = nullptr;
  int na = 0, nb = 0;
};

// One tile of a grouped GEMM launch: problem index and tile coordinates.
struct TileRef {
  int prob, tm, tn, pad;
};

// One merge of two sibling boxes (section 4).  alpha = west/south child,
// beta = east/north child.  Maps are child-local boundary positions.
struct MergeDesc {
  const double* Ta;   // alpha's DtN, na x na
  const double* Tb;   // beta's DtN, nb x nb
  double* Tp;         // parent DtN, me x me (me = m1 + m2)
  double* W;          // augmented [M | B (| I)], m3 x ldw; after the solve
                      // [* | S (| M^-1)]
  double* S;          // solution operator, m3 x me, leading dimension ldw (inside W)
  double* Q;          // [T13a; T23b] in parent order, me x m3
  int* piv;           // m3 pivots
  const int* pmap;    // me entries: >= 0 position in alpha, < 0: -(position in beta) - 1
  const int* a3;      // m3 positions of the shared edge in alpha
  const int* b3;      // m3 positions of the shared edge in beta
  const int* Ie;      // me global ids (parent boundary, S,E,N,W)
  const int* Ii;      // m3 global ids (shared edge)
  int na, nb, me, m3;
  int box, ldw;       // ldw = m3 + me (+ m3 when M^-1 is kept)
  int inv, pad;       // inv = 1: W carries the identity block, giving M^-1 at W + m3 + me
};

// Solution array of the problem a merge belongs to (downward pass), and its
// boundary data (used by the graph-captured solve, which reads both here).
struct SolveIO {
  double* u;       // [nrhs][N]
  int N, nrhs;
  const double* f = nullptr;  // [nrhs][n_bdry]
};

}  // namespace hps
