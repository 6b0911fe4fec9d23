// Interface residual that allocates nothing (for callers that cannot call
// hipMalloc: code under graph capture, tight serving loops).
//
// The per-leaf flux scratch of the residual (section 4: the flux-jump
// equations the merges solve exactly) lives in a file-scope device array of
// fixed size.  Each GPU the library runs on holds its own copy for the life of
// the process; its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels (the
// array's name in host code is not a device address).  Every call on a GPU
// shares that GPU's array: calls that overlap on one GPU (two streams or two
// threads) race on it.  The kernels write every scratch entry they read, so
// nothing has to be cleared between calls.
#include <cstdio>
#include <mutex>

#include "../../include/hps.h"
#include "common.h"
#include "ops.h"
#include "prof.h"
#include "solver.h"

namespace hps {

namespace {

constexpr size_t kScratchDoubles = (size_t)HPS_NOALLOC_SCRATCH_BYTES / sizeof(double);

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
double* scratch_ptr() {
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  HPS_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    HPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HPS_REQUIRE(p != nullptr, "no device address for the scratch array");
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}

}  // namespace

void residual_noalloc(const hps_op* op, const double* u, int nrhs, double* r, hipStream_t s) {
  HPS_REQUIRE(op->opt.keep_leaf && op->leafT, "operator was built without keep_leaf_ops");
  HPS_REQUIRE(op->q <= 24, "q too large for the residual kernel");
  const size_t need = (size_t)nrhs * op->nx * op->ny * 4 * op->q;
  if (need > kScratchDoubles) {
    char buf[200];
    std::snprintf(buf, sizeof(buf),
                  "hps_interface_residual_noalloc: %d right-hand sides need %zu bytes of scratch, "
                  "above the %zu-byte limit", nrhs, need * sizeof(double),
                  (size_t)HPS_NOALLOC_SCRATCH_BYTES);
    throw Error(HPS_EINVAL, buf);
  }
  double* v = scratch_ptr();
  ProfPause pause;  // no profiling events (their creation could allocate)
  interface_residual(op->leafT, u, op->tree().N, nrhs, op->nx, op->ny, op->q, v, r, s);
  HPS_HIP(hipGetLastError());
}

}  // namespace hps
