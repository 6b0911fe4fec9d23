// Problem-specific kernels (leaf assembly, merge gather, downward and upward
// passes, interface residual) -- host entry points.
#pragma once

#include <cstddef>

#include "common.h"

namespace hps {

// Device copies of the coefficient-independent leaf tables (see LeafTables).
struct LeafDev {
  const double* Dx;
  const double* Dy;
  const double* Dxx;
  const double* Dyy;
  const double* G;   // 5 x n x m
  int p, n, m, pad;
};

void leaf_assemble(const double* const* cptr, const LeafDev& tab, int count, double* W,
                   hipStream_t s);
// Body loads: W = [A_ii | G] per leaf (ld = n + nrhs), G[k][r] = body[r][leaf][node k]
// with body [nrhs][nl][p*p] and leaf = leaf0 + position in the batch.
void leaf_assemble_body(const double* const* cptr, const LeafDev& tab, int count, double* W,
                        const double* body, int nrhs, int nl, int leaf0, hipStream_t s);
// Fluxes P1 w_i of the particular solutions left in W + n by the solve, into
// the upward pass's h buffer at unit offset hoff + leaf m; optionally w_i
// itself into wpart [nrhs][nl][n].
void body_flux(const double* W, int count, int n, int m, int ld, int nrhs, const double* P1,
               double* hbuf, long long hoff, double* wpart, int nl, int leaf0, hipStream_t s);
// Kept body operator: W = [A_ii^T | P1^T] per leaf (ld = n + m), P1 [m][n].
void leaf_assemble_body_operator(const double* const* cptr, const LeafDev& tab, int count,
                                 double* W, const double* P1, hipStream_t s);
// Body-load fluxes with the kept operator: h = K g_i, Kt [nl][n][m] = K^T per
// leaf, g [nrhs][nl][p*p]; h into the upward pass's buffer as body_flux does.
void body_flux_kept(const double* Kt, const double* g, int nrhs, int n, int m, int p, int nl,
                    double* hbuf, long long hoff, hipStream_t s);
// dst[i][r * cols + c] = src[i][r * lds + c] for r < rows, c < cols, i < count.
void copy_rows_batch(const double* const* src, double* const* dst, int count, int rows, int cols,
                     int lds, hipStream_t s);
// uc [nrhs][nleaf][pp]: adds wpart [nrhs][nleaf][n] at the interior nodes post_node[0..n).
void add_particular(double* uc, const double* wpart, const int* post_node, int n, int pp,
                    int nleaf, int nrhs, hipStream_t s);
// W = [M | I], B and Q of every merge (max_elems: the largest merge's element
// count of the three), and max|M| into each merge's pivot statistics.
void merge_gather(const MergeDesc* d_desc, const std::vector<MergeDesc>& h_desc, hipStream_t s);
// A whole level of small merges (interfaces of at most 64 nodes) in one
// launch: gather, elimination of [M | I], S and (unless the root's is not
// wanted) T, all in one workgroup per merge; with keep, M^-1 and Q too.
// merge_small_lds: the dynamic LDS bytes a merge of that shape needs.
constexpr size_t MERGE_SMALL_MAX_LDS = 150 * 1024;
size_t merge_small_lds(int m3, int me);
// Levels whose interfaces have at most MERGE_SMALL_MAX_M3 nodes use
// merge_small while it is on (knob "merge_small", default on).  Longer
// interfaces were measured slower in one workgroup per merge than on the
// level-wise path (256 x 256 leaves, q = 10: 3.2-3.5 ms against 1.6-1.7 ms
// for interfaces of 40 nodes), whose kernels spread each merge over the GPU.
constexpr int MERGE_SMALL_MAX_M3 = 20;
void set_merge_small(bool on);
bool merge_small_on();
void merge_small(const MergeDesc* d_desc, const std::vector<MergeDesc>& h_desc, bool keep,
                 bool root_T, int* status, hipStream_t s);
// Downward pass of one depth; io[i] gives merge i's solution array (io null:
// every merge uses io0).  s_bytes: bytes of all S of the launch (its
// algorithmic traffic per RHS chunk).
// d_io: per-merge SolveIO array, or (io_shared) one SolveIO for all merges;
// null: io0 (passed by value) for all merges.
void downward(const MergeDesc* d_desc, const SolveIO* d_io, const SolveIO& io0, int nmerge,
              int m3_max, int me_max, int nrhs_max, const double* zbase, const long long* zoff,
              hipStream_t s, double s_bytes, bool io_shared = false);
// Algorithm 2 for one operator as one cooperative launch (levels root
// first, each with merges of one shape; nrhs <= 15; f [nrhs][nb], u
// [nrhs][N]); d_bar: 9 x 32 words, d_err: one word, zeroed by the call;
// *d_err becomes 1 if a level barrier timed out.
void downward_persist(const PersistLevel* d_levels, int nlev, const double* f, const int* gamma,
                      int nb, double* u, int N, int nrhs, unsigned* d_bar, int* d_err,
                      hipStream_t s);
void set_boundary(const double* f, const int* gamma, int nb, double* u, int N, int nrhs,
                  hipStream_t s);
// u[r][gamma[i]] = f[r][i] with f, u, N, nrhs read from *io on the device.
void set_boundary_io(const SolveIO* io, const int* gamma, int nb, int nrhs, hipStream_t s);
void interface_residual(const double* leafT, const double* u, int N, int nrhs, int nx, int ny,
                        int q, double* vbuf, double* r, hipStream_t s);
// Section 5.3 post-processing: every leaf's p x p Chebyshev grid values from u
// at its 4q boundary Gauss nodes.  A leaf's rows are the (p-2)^2 rows of -Z
// (Z = A_ii^-1 A_ie L1) for the interior nodes, then the 4(p-1) rows of L1
// (the Gauss-to-Chebyshev edge interpolation) for the grid-boundary nodes;
// post_node[rho] is the node row rho produces.  Both are given transposed:
// Zt [nleaf][4q][(p-2)^2], L1t [4q][4(p-1)].  uc is [nrhs][nx*ny][p*p].
void leaf_postprocess(const double* Zt, const double* L1t, const int* post_node, const double* u,
                      int N, int nrhs, int nx, int ny, int p, int q, double* uc, hipStream_t s);
// dst[i][c * rows + r] = src[i][r * lds + c] for r < rows, c < cols, i < count.
void transpose_rows_batch(const double* const* src, double* const* dst, int count, int rows,
                          int cols, int lds, hipStream_t s);
// Rows per lane of the post-processing kernel: 1, 2, 4, or 0/-1 (by count).
void set_post_rows(int r);
// Upward source pass of one depth, per right-hand side (s, [nrhs][N], may be
// null: no interface sources).
void upward_level(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, const double* s,
                  int N, double* hbase, const long long* ha_off, const long long* hb_off,
                  const long long* hp_off, double* zbuf, const long long* z_off, int nrhs,
                  double flops, hipStream_t st);
// Node-major solution passes for many right-hand sides: arrays are
// [nodes][nrhs].  Algorithm 2 for one depth (z: upward-pass terms, [m3][nrhs]
// per merge, or null); d_io, when not null, gives merge i's array and count
// (U and nrhs then give only the launch shape: U unused, nrhs the largest).
void downward_mm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, double* U, int nrhs,
                 const double* zbase, const long long* zoff, hipStream_t s, double s_bytes,
                 const SolveIO* d_io = nullptr);
void set_boundary_nm(const double* f, const int* gamma, int nb, int nrhs, double* U,
                     hipStream_t s);
// Depths with few merges split the GEMM contractions of these passes into
// chunks of at least v (default 256, at least 16) summed in a fixed order.
void set_split_min_chunk(int v);
// out[c][r] = in[r][c], in being R x C row-major.
void transpose(const double* in, int R, int C, double* out, hipStream_t s);
void interface_residual_nm(const double* leafT, const double* U, int N, int nrhs, int nx, int ny,
                           int q, double* vbuf, double* r, hipStream_t s);
// rbuf: scratch of the size of zbuf.
void upward_level_nm(const MergeDesc* d_desc, int nmerge, int m3_max, int me_max, const double* src,
                     double* hbase, const long long* ha_off, const long long* hb_off,
                     const long long* hp_off, double* rbuf, double* zbuf, const long long* z_off,
                     int nrhs, double flops, hipStream_t st);
void axpy(double* y, const double* x, double a, size_t n, hipStream_t s);
void absmax_partial(const double* x, size_t n, double* out, int blocks, hipStream_t s);
void matvec(const double* A, int rows, int cols, const double* x, int nrhs, double* y,
            hipStream_t s);
void nonfinite(const double* x, size_t n, int* flag, hipStream_t s);
void leaf_range_flags(const double* const* cptr, int nl, int pp, const double* lohi, double margin,
                      int* flag, hipStream_t s);
void ops_init();

}  // namespace hps
