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
  // Pivot statistics of this system, or null: pstat[0] = max|M| and
  // pstat[1] = min |pivot|, both as the bit patterns of non-negative doubles
  // (which order like the integers), kept with atomicMax / atomicMin.
  unsigned long long* pstat = nullptr;
};

// Bit pattern of |x| for the pivot statistics (NaN counts as +inf).
__host__ __device__ inline unsigned long long abs_bits(double x) {
  if (x != x) return 0x7FF0000000000000ull;
  union {
    double d;
    unsigned long long u;
  } c;
  c.d = x < 0 ? -x : x;
  return c.u;
}

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
  // 1: C = alpha A B (the old C is neither read nor kept); 0: as above.
  int overwrite = 0;
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
  double* W;          // merge system [M | I], m3 x ldw (ldw = 2 m3), M = T33a - T33b;
                      // after the elimination W + m3 holds M^-1 (leading dimension ldw)
  double* B;          // gathered right-hand sides [-T31a | T32b], m3 x me (leading dimension me)
  double* S;          // solution operator S = M^-1 B (eq:U_parent), m3 x me, leading dimension lds
  double* Q;          // [T13a; T23b] in parent order, me x m3
  int* piv;           // m3 pivots
  const int* pmap;    // me entries: >= 0 position in alpha, < 0: -(position in beta) - 1
  const int* a3;      // m3 positions of the shared edge in alpha
  const int* b3;      // m3 positions of the shared edge in beta
  const int* Ie;      // me global ids (parent boundary, S,E,N,W)
  const int* Ii;      // m3 global ids (shared edge)
  int na, nb, me, m3;
  int box, ldw;       // ldw = 2 m3
  int lds, pad;       // lds = me
  unsigned long long* pstat = nullptr;  // the merge system's pivot statistics (SolveDesc)
};

// One level of the persistent downward pass: nmerge merges of one shape.
struct PersistLevel {
  const MergeDesc* d;
  int nmerge, m3, me, pad;
};

// Solution array of the problem a merge belongs to (downward pass), and its
// boundary data (used by the graph-captured solve, which reads both here).
struct SolveIO {
  double* u;       // [nrhs][N]
  int N, nrhs;
  const double* f = nullptr;  // [nrhs][n_bdry]
};

}  // namespace hps
