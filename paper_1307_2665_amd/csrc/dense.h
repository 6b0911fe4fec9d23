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

// Arithmetic of a grouped GEMM: FP64 MFMA; FP32 MFMA on hi/lo splits of the
// operands (three products); BF16 MFMA on three-slice splits (six products).
enum GemmPrec { GEMM_F64 = 0, GEMM_SPLIT32 = 1, GEMM_BF16X6 = 2 };

// Merge levels whose longest contraction is shorter than this run their
// Schur products in FP64 even in the BF16 mode (slicing costs more than it
// saves there); default 384.
void set_bf16x6_min_k(int k);
int bf16x6_min_k();

// C = C0 + alpha A B for every descriptor, in the given arithmetic.
// prof_cls: the profiling class its FP64 launches are timed under.
void grouped_gemm(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                  int prec, int prof_cls = 5 /* PROF_GEMM */);

// Heterogeneous grouped FP64 products (the merges of many problems at one
// depth) as one persistent launch of the 128 x 128 tile: gemm_tile_queue
// lists every tile, largest problems first; the caller uploads it and
// passes one int of device scratch for the queue counter.  Workgroups take
// tiles until the queue is empty.  Knob "gemm_queue" (default on) lets
// run_build use it for batches.
std::vector<TileRef> gemm_tile_queue(const std::vector<GemmDesc>& h_desc);
void grouped_gemm_queue(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc,
                        const TileRef* d_tiles, int ntiles, int* d_counter, hipStream_t stream,
                        int prof_cls = 5 /* PROF_GEMM */);
void set_gemm_queue(bool on);
bool gemm_queue_on();

// The same with explicit kernel variants (the autotuner times them):
// gj_variant = update tile * 4 + TRSM block code (see tune.h), -1 = default;
// variant = FP64 MFMA tile of gemm_tile (0..5), -1 = default.
void batched_solve_v(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                     hipStream_t stream, int gj_variant);
void grouped_gemm_v(const GemmDesc* d_desc, const std::vector<GemmDesc>& h_desc, hipStream_t stream,
                    int variant, int prec, int prof_cls = 5 /* PROF_GEMM */);

// Look-ahead in the block Gauss-Jordan solver (default off): each step updates
// the next panel's columns first, and the remaining columns on a side stream
// while the next panel is factored.  Measured slower on config 2: the side
// stream's update fills the CUs, and the next panel's lone workgroup waits.
void set_gj_lookahead(bool on);

// Pivot statistics of the systems (SolveDesc::pstat): pstat_init clears count
// pairs (max|M| = 0, min |pivot| = none); system_absmax records max|M| of the
// n x n block of every system with statistics before it is eliminated (nmax:
// the largest n); after the elimination pivot_check sets status[0] = 1 and
// status[1] = the tag of a system whose smallest pivot is <= tol max|M|.
void pstat_init(unsigned long long* pstat, size_t count, hipStream_t s);
void system_absmax(const SolveDesc* d_desc, int count, int nmax, hipStream_t s);
void pivot_check(const SolveDesc* d_desc, int count, double tol, int* status, hipStream_t s);
void dense_init();

// Blocked Gauss-Jordan with pivoting inside 64 x 64 diagonal blocks (see
// gj.hip); binv: scratch of 64 x 64 doubles per system.  Raises
// status[3] when a block pivot is not above fb_tol max|M|: the caller then
// redoes the systems with batched_solve.  Used for systems of at least
// bgj_min_rows() rows (set_bgj: -1 keeps a value).
// *p = v on the stream (a one-thread kernel, not a memset node).
void set_int(int* p, int v, hipStream_t s);

// ident: W = [M | I] (m == n), whose identity columns right of the touched
// part are skipped; otherwise every column right of the block is updated.
void batched_solve_bgj(const SolveDesc* d_desc, const std::vector<SolveDesc>& h_desc, int* d_status,
                       double* binv, hipStream_t stream, bool ident = true);
void set_bgj(int min_rows, double fb_tol);
// On (default): each step's update of the columns past the next diagonal
// block runs on a side stream beside the next diagonal-block kernel.
void set_bgj_lookahead(bool on);
// Clears the smallest-pivot statistic of every system (before a redo).
void pstat_reset_min(const SolveDesc* d_desc, int count, hipStream_t s);
int bgj_min_rows();
int max_solve_rows();

}  // namespace hps
