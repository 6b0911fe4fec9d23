// Kernel-variant selection per shape bucket, and the autotuner that fills it.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace hps {

enum TuneKnob {
  TUNE_LEAF = 0,  // leaf kernel variant; key (n, m)
  TUNE_GEMM = 1,  // FP64 MFMA tile variant; key (lg M, lg N, lg K, lg count)
  TUNE_GJ = 2,    // Gauss-Jordan update tile * 4 + TRSM block code; key (lg n, lg n+m, lg count)
  TUNE_NKNOBS = 3
};

constexpr int GEMM_VARIANTS = 8;   // tiles of grouped_gemm_v (dense.hip)
// Tiles of the Gauss-Jordan trailing update (launch_update in gj.hip):
// 0: 64x64x16 on 2x2 waves, 1: 32x32x16 on one wave, 2: 128x128x16 on 4x2
// waves, 3: 128x64x16, 4: 64x128x16, 5: 64x64x32; each loads its tile's old
// values with the first operands and keeps one k-slab of loads in flight.
constexpr int UPDATE_VARIANTS = 6;
constexpr int TRSM_BLOCKS[3] = {256, 128, 64};

// ceil(log2(x)) for x >= 1.
int tune_lg(long long x);

// Variant for a shape key: a forced value (hps_tune_set) first, then the
// table, else -1 (callers fall back to their default).
int tune_get(int knob, int a, int b, int c, int d);
void tune_force(int knob, int variant);  // -1 removes the force
// all: every candidate's time, in variant order (GEMM buckets; kept in the
// cache as "all_ms").
void tune_put(int knob, int a, int b, int c, int d, int variant, double ms, double ms_default,
              const std::vector<double>& all = {});
void tune_clear();
std::string tune_json();
void tune_load_json(const std::string& text);

// Shape of a problem to tune for (coefficients are not needed).
struct TuneShape {
  int nx, ny, p, q;
  double hx, hy;
};
// Times the variants of every kernel the builds of these shapes launch, on
// synthetic data of the same shapes, and records the fastest per bucket.
// Returns the seconds spent.
double autotune(const std::vector<TuneShape>& shapes, hipStream_t s);

}  // namespace hps
