// Launch-level timing of kernel classes with HIP events on the launch stream,
// plus the algorithmic FLOPs and bytes of each timed launch.  Off unless a
// class is enabled through hps_prof_enable.
#pragma once

#include <hip/hip_runtime.h>

namespace hps {

enum ProfClass {
  PROF_LEAF_ASSEMBLE = 0,
  PROF_LU_PANEL = 1,
  PROF_SWAP_TRSM = 2,
  PROF_LU_UPDATE = 3,
  PROF_BACK_SUBST = 4,
  PROF_GEMM = 5,
  PROF_GEMM_SPLIT32 = 6,
  PROF_MERGE_GATHER = 7,
  PROF_DOWNWARD = 8,
  PROF_RESIDUAL = 9,
  PROF_UPWARD = 10,
  PROF_LEAF_LU = 11,
  PROF_MLP_TRAIN = 12,
  PROF_MLP_INFER = 13,
  PROF_POSTPROCESS = 14,
  PROF_GEMM_BF16X6 = 15,
  PROF_BODY_FLUX = 16,
  PROF_LEAF_GEMM = 17,   // leaf T = P0 - P1 Z products (section 3.2, step 4)
  PROF_MERGE_S = 18,     // S = M^-1 B products of the merges (eq:U_parent)
  PROF_BGJ_DIAG = 19,    // blocked Gauss-Jordan: diagonal-block inverses
  PROF_BGJ_ROWS = 20,    // blocked Gauss-Jordan: block rows times the inverse
  PROF_BGJ_UPDATE = 21,  // blocked Gauss-Jordan: updates of the other rows
  PROF_MERGE_SMALL = 22, // whole small merges in one launch
  PROF_HBS = 23,         // HBS passes: telescoping product, Algorithms 3-4, compression
  PROF_NCLASS = 24
};

bool prof_on(int cls);

// While alive, this thread records no events (used around graph capture,
// whose launches are timed as a whole when the graph is replayed).
class ProfPause {
 public:
  ProfPause();
  ~ProfPause();
};

// Records a start event on construction and a stop event on destruction when
// the class is enabled; flops/bytes are the launch's algorithmic work.
class ProfScope {
 public:
  ProfScope(int cls, hipStream_t s, double flops, double bytes);
  ~ProfScope();

 private:
  int rec_ = -1;
  hipStream_t s_;
};

}  // namespace hps
