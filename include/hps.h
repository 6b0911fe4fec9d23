/*
 * hps.h -- C ABI of the MI355X composite spectral direct solver.
 *
 * Method: Gillman & Martinsson, "A direct solver with O(N) complexity for
 * variable coefficient elliptic PDEs discretized via a high-order composite
 * spectral collocation method" (arXiv:1307.2665), dense path of sections 2-5:
 *   - leaf DtN maps by p x p Chebyshev collocation with q Gauss nodes per leaf
 *     edge (section 3, T = L4 L3 L2 L1),
 *   - level-by-level merges of sibling DtNs (section 4, eq:U_parent and
 *     eq:merge; Algorithm 1),
 *   - the downward solve (Algorithm 2).
 *
 * Problem (section 1.1, eq:basic and eq:defA): A u = 0 on a rectangle, u = f on
 * its boundary, with
 *   A u = -c11 u_11 - 2 c12 u_12 - c22 u_22 + c1 u_1 + c2 u_2 + c u.
 *
 * Conventions shared by every entry point:
 *   - Leaves: nx-by-ny equal leaves; leaf index i + nx*j, i along x1.
 *   - Chebyshev nodes of a leaf: Chebyshev-Lobatto points, ascending in each
 *     direction; node (a, b) has index a + p*b.
 *   - Coefficients: double [nx*ny][6][p*p], the six fields in the order
 *     c11, c12, c22, c1, c2, c, sampled at each leaf's Chebyshev nodes.
 *   - Gauss nodes: q Gauss-Legendre points per leaf edge.  Global numbering:
 *     horizontal edge (i, j), i < nx, j <= ny, has id j*nx + i; vertical edge
 *     (i, j), i <= nx, j < ny, has id nx*(ny+1) + j*(nx+1) + i; node k of an
 *     edge is id*q + k, ascending along the edge.  N = q*(nx*(ny+1)+(nx+1)*ny).
 *   - Box boundaries (including the domain boundary Gamma) are ordered S (x1
 *     ascending), E (x2 ascending), N (x1 ascending), W (x2 ascending);
 *     n_bdry = 2*q*(nx+ny).
 *   - Fluxes follow section 2: v = du/dx2 on horizontal edges, du/dx1 on
 *     vertical edges (so a DtN here is not the outward-normal map).
 *   - Tree: the root is the whole rectangle; a box is split across its longer
 *     side (in leaf units) at floor(n/2), x1 first on ties; boxes are numbered
 *     breadth first (root 0, children 2k+1... in creation order), so every
 *     parent precedes its children (section 2).  alpha = west/south child.
 *   - All matrices are row-major FP64 unless stated otherwise.
 *
 * Memory: pointers are host pointers unless the options say device_ptrs = 1,
 * in which case they are device pointers on the current HIP device.  The
 * library never keeps a caller pointer after a call returns.  An hps_op owns
 * all of its device memory until hps_destroy; see hps_destroy for the
 * buffers it then keeps for the next build of the same shape.
 *
 * Streams: all device work is enqueued on the given hipStream_t (NULL means
 * the default stream) and every call synchronizes that stream before it
 * returns, so outputs are ready on return.
 *
 * Errors: no C++ exception crosses this ABI.  A non-OK status leaves output
 * handles NULL, and hps_last_error() returns a thread-local message.
 *
 * Threading: one hps_op must not be used from two threads at once.
 */
#ifndef HPS_H
#define HPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hps_op hps_op;
typedef struct hps_surrogate hps_surrogate;

typedef enum {
  HPS_OK = 0,
  HPS_EINVAL = 1,      /* bad argument: sizes, q >= p, p < 4, non-finite data, ... */
  HPS_ESINGULAR = 2,   /* a pivot of a leaf or merge elimination fell below pivot_tol */
  HPS_ENOMEM = 3,      /* device allocation failed */
  HPS_EDEVICE = 4,     /* HIP runtime error (no device, launch failure) */
  HPS_ENOTCONV = 5,    /* iterative refinement did not reach refine_tol in max_iter */
  HPS_ESURROGATE = 6   /* surrogate unusable for this problem (shape mismatch) */
} hps_status;

typedef enum {
  HPS_FP64 = 0,           /* every step in FP64 */
  HPS_MIXED_SPLIT32 = 1,  /* Schur products on FP32 MFMA with hi/lo splits; LU and TRSM FP64 */
  HPS_SURROGATE = 2,      /* leaf DtNs from a trained surrogate, judged by the FP64 leaf build */
  HPS_MIXED_BF16X6 = 3    /* Schur products on BF16 MFMA from three-slice splits (six products);
                             LU and TRSM FP64; refinement as in HPS_MIXED_SPLIT32 */
} hps_mode;

typedef struct {
  int mode;                        /* hps_mode */
  void* stream;                    /* hipStream_t */
  int device_ptrs;                 /* coeffs is a device pointer */
  int keep_leaf_ops;               /* keep leaf DtNs (needed by refinement; forced on in the mixed modes) */
  int keep_factors;                /* keep LU(M), pivots and Q = [T13a; T23b] per merge (upward pass)
                                      and a copy of the coefficients (body loads) */
  int compute_root_dtn;            /* 1: form T^1 at the root (default), 0: skip its Schur product */
  double pivot_tol;                /* in [0, 1): a leaf whose elimination meets a pivot with
                                      |pivot| <= pivot_tol * max|A_ii|, or a merge whose smallest
                                      pivot is <= pivot_tol * max|T33a - T33b|, makes the build
                                      fail with HPS_ESINGULAR naming the leaf or the merge's box
                                      and depth; 0: only zero or non-finite pivots fail */
  const hps_surrogate* surrogate;  /* mode HPS_SURROGATE only */
  int judge_samples;               /* surrogate: number of leaves re-built in FP64 to judge it */
  double judge_tol;                /* surrogate: max rel. leaf-DtN error before fallback */
  int keep_leaf_solution;          /* keep each leaf's Z = A_ii^-1 A_ie L1 ((p-2)^2 x 4q doubles
                                      per leaf, stored transposed) for hps_postprocess; not in
                                      surrogate mode */
  int keep_body_operator;          /* keep K = P1 A_ii^-1 per leaf ((p-2)^2 x 4q doubles, stored
                                      transposed; P1: interior values to leaf flux), so that
                                      hps_solve_body needs no leaf factorization; implies
                                      keep_factors */
} hps_build_opts;

typedef struct {
  void* stream;          /* hipStream_t */
  int device_ptrs;       /* f and u are device pointers */
  int refine;            /* iterative refinement against the FP64 leaf DtNs */
  double refine_tol;     /* stop when max|delta| <= refine_tol * max|u| */
  int max_iter;          /* refinement sweeps allowed */
} hps_solve_opts;

typedef struct {
  int iters;                 /* refinement sweeps done */
  double last_update_rel;    /* max|delta| / max|u| of the last sweep */
  double first_update_rel;   /* same for the first sweep */
  int n_fallback_leaves;     /* surrogate leaves replaced by the FP64 leaf build */
} hps_solve_info;

typedef struct {
  int nx, ny, p, q;
  int N;              /* Gauss nodes */
  int n_bdry;         /* nodes on Gamma */
  int n_boxes;        /* boxes in the tree */
  int n_levels;       /* tree depth + 1 */
  int mode;
  int n_fallback_leaves;
  double box[4];
  int64_t bytes_S;    /* device bytes of all solution operators S */
  int64_t bytes_total;
  int64_t flops_build;/* algorithmic FP64 FLOPs of the build (leaf + LU + TRSM + Schur) */
  double judge_worst; /* surrogate mode: worst relative leaf-DtN error in the judged sample */
  int n_judged;       /* surrogate mode: leaves re-solved by the FP64 leaf solver */
} hps_op_info;

/* One problem of a heterogeneous batch (hps_build_batch). */
typedef struct {
  const double* coeffs;   /* [nx*ny][6][p*p] */
  double box[4];
  int nleaf[2];
  int p, q;
} hps_problem;

/* ---- discretization helpers (host outputs) ------------------------------ */

/* Chebyshev node coordinates of every leaf: xy[nx*ny][p*p][2] (section 3.1). */
hps_status hps_cheb_nodes(const double box[4], const int nleaf[2], int p, double* xy);

/* Coordinates of all N Gauss nodes in the global numbering: xy[N][2] (section 2).
   Also returns N. */
hps_status hps_gauss_nodes_grid(const double box[4], const int nleaf[2], int q, double* xy, int* N);

/* Global ids of the nodes on Gamma in S,E,N,W order: ids[n_bdry]. */
hps_status hps_boundary_ids(const int nleaf[2], int q, int* ids, int* n_bdry);

/* ---- leaf stage (section 3) --------------------------------------------- */

/* Leaf DtN maps of nleaf equal leaves of size hx-by-hy (section 3.2):
   coeffs [nleaf][6][p*p] -> T [nleaf][4q][4q].  Both device pointers.
   Requires 4 <= p <= 24 and 1 <= q <= p - 1 (HPS_EINVAL otherwise). */
hps_status hps_leaf_dtn(const double* coeffs, int nleaf, double hx, double hy, int p, int q,
                        double* T, void* stream);

/* ---- build (Algorithm 1) and solve (Algorithm 2) ------------------------ */

/* Builds every S^tau and the root DtN T^1 for one problem.  coeffs as above;
   box = {x0, x1, y0, y1}; nleaf = {nx, ny}; requires 4 <= p <= 24 and
   1 <= q <= p - 1, else HPS_EINVAL.  (Section 3.2 step 1 maps the 4q Gauss
   values of a leaf onto its 4(p-1) boundary Chebyshev nodes, averaging the
   two sides at each corner; for q >= p that map has a null space, and at
   every interior cross point the four edges carry a mode +a, -a, +a, -a that
   no leaf sees, so T33a - T33b is singular for every merge whose shared edge
   passes a cross point.)  opts may be NULL. */
hps_status hps_build_solution_operator(const double* coeffs, const double box[4],
                                       const int nleaf[2], int p, int q,
                                       const hps_build_opts* opts, hps_op** out);

/* Gauss node coordinates of an operator's grid: xy[N][2]. */
hps_status hps_gauss_nodes(const hps_op* op, double* xy, int* N);

/* Coordinates of the n_bdry boundary nodes in S,E,N,W order: xy[n_bdry][2]. */
hps_status hps_boundary_nodes(const hps_op* op, double* xy, int* n_bdry);

/* Algorithm 2: f [nrhs][n_bdry] -> u [nrhs][N] (u on Gamma equals f).
   With opts->refine, corrections from the interface residual of the FP64
   leaf DtNs are added until max|delta| <= refine_tol*max|u|. */
hps_status hps_solve(hps_op* op, const double* f, int nrhs, double* u,
                     const hps_solve_opts* opts, hps_solve_info* info);

/* Root DtN apply: v = T^1 f, f [nrhs][n_bdry] -> v [nrhs][n_bdry] (Table 1's T_apply). */
hps_status hps_root_dtn_apply(const hps_op* op, const double* f, int nrhs, double* v,
                              const hps_solve_opts* opts);

/* Post-processing (section 5.3): the solution on every leaf's p x p Chebyshev
   grid from u at the Gauss nodes (the output of hps_solve).  Grid-boundary
   nodes interpolate the leaf's edge values (corner nodes average their two
   edges); interior nodes apply the leaf solution operator -A_ii^-1 A_ie that
   the build kept (Remark 3.2).  u [nrhs][N] -> uc [nrhs][nx*ny][p*p], node
   (a, b) of leaf i + nx*j at uc[r][i + nx*j][a + p*b].  Needs an operator
   built with keep_leaf_solution (HPS_EINVAL otherwise).  Uses opts->stream
   and opts->device_ptrs (u and uc both host or both device); the refinement
   fields are ignored.  Exact only for A u = 0 inside the leaves, which is
   the problem hps_solve answers. */
hps_status hps_postprocess(const hps_op* op, const double* u, int nrhs, double* uc,
                           const hps_solve_opts* opts);

/* Body loads: A u = g in the domain, u = f on its boundary (an extension of
   eq:basic, whose right-hand side is zero).  In every leaf u = v + w: w solves
   the leaf's interior collocation equations with the load and zero boundary
   values (section 3.1's A_ii w_i = g_i), v the homogeneous ones; the flux of
   w joins the leaf's DtN relation (flux = T v + L4 L3 w), these particular
   fluxes ride the merges' interface-source recursion up the tree (third
   block row of eq:premerge), and Algorithm 2 adds the resulting interface
   terms.  f [nrhs][n_bdry]; g [nrhs][nx*ny][p*p] at every leaf's Chebyshev
   nodes (only interior nodes are used); u [nrhs][N] at the Gauss nodes; uc
   (may be NULL) [nrhs][nx*ny][p*p], the solution on every leaf grid.  Needs
   an operator built with keep_factors (and keep_leaf_solution for uc),
   HPS_EINVAL otherwise; HPS_ESINGULAR if a leaf's A_ii is singular.  With
   keep_body_operator and uc NULL the particular fluxes are one batched
   product with the kept P1 A_ii^-1; otherwise every call eliminates
   [A_ii | g] for all leaves (the particular solutions w_i are needed for uc).  Uses
   opts->stream and opts->device_ptrs (f, g, u, uc all host or all device);
   the refinement fields are ignored.  Exact up to rounding for the FP64
   operator; a mixed-precision operator gives its unrefined accuracy. */
hps_status hps_solve_body(hps_op* op, const double* f, const double* g, int nrhs, double* u,
                          double* uc, const hps_solve_opts* opts);

/* ---- iterative-refinement building blocks (device pointers) ------------- */

/* Flux jump v_alpha - v_beta of the FP64 leaf DtNs at every Gauss node
   (0 on Gamma): u [nrhs][N] -> r [nrhs][N]. */
hps_status hps_interface_residual(const hps_op* op, const double* u, int nrhs, double* r,
                                  void* stream);

/* For callers that cannot allocate (code under graph capture, tight serving
   loops): hps_interface_residual without any allocation.  The per-leaf flux
   scratch (nrhs * nleaf * 4q doubles) comes from a fixed device array of
   HPS_NOALLOC_SCRATCH_BYTES that each GPU holds for the life of the process;
   calls that need more return HPS_EINVAL and launch nothing.  u and r are
   device pointers ([nrhs][N]); the operator needs its leaf DtNs (every build
   keeps them).  Waits for the stream before returning, like every call.
   Every call on one GPU shares that GPU's array: calls that overlap on one
   GPU (two streams, two threads) race and must be serialised by the caller. */
#define HPS_NOALLOC_SCRATCH_BYTES (64ull << 20)
hps_status hps_interface_residual_noalloc(const hps_op* op, const double* u, int nrhs, double* r,
                                          void* stream);

/* Solution of "jump = s at interior nodes, u = f on Gamma": upward pass for the
   sources s [nrhs][N], then the downward pass.  Needs keep_factors. */
hps_status hps_solve_with_sources(hps_op* op, const double* f, const double* s, int nrhs,
                                  double* u, void* stream);

/* ---- learned leaf surrogate (not in the paper) -------------------------- */
/* A small MLP maps (c11, c22, c) at a leaf's p^2 Chebyshev nodes (fields with
   c12 = c1 = c2 = 0) to low-rank factors U, V (4q x rank) of
   T = T_Laplace(h) + s U V^T, with T_Laplace(h) the leaf DtN of the Laplace
   operator for the same leaf size.  Two tanh layers of width `hidden`; weights
   are BF16 for every GEMM (BF16 MFMA, FP32 accumulation) with FP32 master
   copies and Adam moments.  Training pairs come from hps_leaf_dtn.  A build in
   mode HPS_SURROGATE infers every leaf DtN, then re-solves opts->judge_samples
   seeded leaves plus every leaf whose coefficients leave the training ranges
   with the FP64 leaf solver; judged leaves whose relative error exceeds
   opts->judge_tol are replaced (counted in n_fallback_leaves), and if more than
   a quarter of the random sample fails every leaf is rebuilt in FP64. */

hps_status hps_surrogate_create(int p, int q, double hx, double hy, int hidden, int rank,
                                unsigned long long seed, void* stream, hps_surrogate** out);
/* Adam training on n device samples: coeffs [n][6][p*p], T [n][4q][4q] (FP64
   leaf DtNs).  The first call also fixes the input normalisation and output
   scale from these samples.  history (host, may be NULL) gets the mean loss of
   every epoch; final_loss the last one. */
hps_status hps_surrogate_train(hps_surrogate* s, const double* coeffs, const double* T, int n,
                               int epochs, int batch, double lr, unsigned long long seed,
                               void* stream, double* final_loss, double* history);
/* Loss and gradients (host float [W1 b1 W2 b2 W3 b3]) of one batch; no update. */
hps_status hps_surrogate_grad(hps_surrogate* s, const double* coeffs, const double* T, int n,
                              float* grads, double* loss, void* stream);
/* T [n][4q][4q] (device, FP64) from coeffs [n][6][p*p] (device). */
hps_status hps_surrogate_predict(hps_surrogate* s, const double* coeffs, int n, double* T,
                                 void* stream);
/* dims = {p, q, hidden, rank, D, O, step}; out_scale = s. */
hps_status hps_surrogate_info(const hps_surrogate* s, int dims[7], double* out_scale);
/* Serialized state (shape, normalisation, scale, training ranges, FP32 weights). */
hps_status hps_surrogate_get_state(const hps_surrogate* s, void* buf, size_t* len);
hps_status hps_surrogate_set_state(hps_surrogate* s, const void* buf, size_t len, void* stream);
hps_status hps_surrogate_save(const hps_surrogate* s, const char* path);
hps_status hps_surrogate_load(const char* path, void* stream, hps_surrogate** out);
void hps_surrogate_destroy(hps_surrogate* s);

/* ---- heterogeneous batches --------------------------------------------- */

/* Builds nprob operators; leaves of equal (p, q, h) and merges at equal tree depth
   of all problems share launches.  out[nprob]. */
hps_status hps_build_batch(const hps_problem* probs, int nprob, const hps_build_opts* opts,
                           hps_op** out);

/* Solves every problem of a batch: f[i] [nrhs[i]][n_bdry_i] -> u[i] [nrhs[i]][N_i];
   the downward passes of all problems share one launch per depth. */
hps_status hps_solve_batch(hps_op* const* ops, int nprob, const double* const* f,
                           const int* nrhs, double* const* u, const hps_solve_opts* opts);

/* ---- introspection for tests ------------------------------------------- */

hps_status hps_op_query(const hps_op* op, hps_op_info* info);

/* Box record: {i0, i1, j0, j1, level, parent, child_alpha, child_beta} (children -1 for leaves). */
hps_status hps_box(const hps_op* op, int box, int rec[8]);

/* S^tau = (T33a - T33b)^-1 [-T31a | T32b] of a parent box (host copy):
   [m3][m1+m2], rows in I_i order, columns in I_e order.  The build forms it
   as M^-1 B: Gauss-Jordan elimination with partial pivoting of [M | I], then
   an FP64 MFMA product. */
hps_status hps_export_S(const hps_op* op, int box, double* S, int* rows, int* cols);

/* Conditioning of the merges (section 4; the interface systems
   (T33a - T33b) u3 = ... that eq:U_parent solves): for every tree depth d < n
   (n = *n_levels, the tree depth + 1), cond_est[d] is the largest over the
   depth's merges of max|M| / min |pivot| of M = T33a - T33b, from the
   elimination with partial pivoting; a lower estimate of cond(M) up to a
   modest factor.  The deepest depth holds only leaves: 0.  cond_est may be
   NULL (only *n_levels is returned). */
hps_status hps_level_conditions(const hps_op* op, double* cond_est, int* n_levels);

/* Root DtN T^1 (host copy), [n_bdry][n_bdry]. */
hps_status hps_export_root_dtn(const hps_op* op, double* T);

/* Leaf DtN of leaf index i + nx*j (host copy), [4q][4q]; needs keep_leaf_ops. */
hps_status hps_export_leaf_dtn(const hps_op* op, int leaf, double* T);

/* ---- batched dense layer (device pointers) ------------------------------- */

/* X_i = M_i^-1 B_i for nprob independent systems by LU with partial pivoting
   (the elimination used for eq:leaf_solve and eq:U_parent).  M [nprob][n][n],
   B [nprob][n][m], X [nprob][n][m]; inputs are not modified.  A zero or
   non-finite pivot gives HPS_ESINGULAR (X is then unspecified). */
hps_status hps_batched_solve(const double* M, const double* B, int n, int m, int nprob, double* X,
                             void* stream);

/* C_i = C_i + alpha A_i B_i for nprob products, A [nprob][Mr][K], B [nprob][K][Nc],
   C [nprob][Mr][Nc].  prec selects the arithmetic of the Schur products:
   0 FP64 MFMA; 1 split-FP32 MFMA (three FP32 products of hi/lo halves, FP64
   accumulation per 16-deep slab); 2 BF16 MFMA on three-slice splits (six
   BF16 products, FP64 accumulation per 32-deep slab).  Other values give
   HPS_EINVAL.  C_i must not overlap A_j or B_j (tiles of C are written while
   other tiles still read the operands). */
hps_status hps_batched_gemm(const double* A, const double* B, double* C, int Mr, int Nc, int K,
                            int nprob, double alpha, int prec, void* stream);

/* ---- HBS matrices (sections 6-7) -----------------------------------------
   An HBS matrix H of M = m 2^L rows on the uniform binary tree of section 6.3:
   node (l, j), 0 <= j < 2^l, owns rows and columns [j M/2^l, (j+1) M/2^l); its
   children are (l+1, 2j) and (l+1, 2j+1).  One rank k at every node
   (1 <= k <= m).  Device buffers of doubles, every block row-major and
   contiguous, the blocks of one level in node order.

   Factors (section 6.4, the factor table there), in this order:
     D    2^L blocks m x m     leaf diagonal blocks H(I_j, I_j)   (eq:def5)
     U    2^L blocks m x k     leaf column bases
     Vt   2^L blocks k x m     leaf row bases, as V* (transposed)
     for l = L-1 down to 1:
       U_l  2^l blocks 2k x k  parent column bases (eq:def4)
       Vt_l 2^l blocks k x 2k  parent row bases, as V*
     for l = L-1 down to 0:
       B_l  2^l blocks 2k x 2k interaction of the node's children (eq:def6);
                               the two diagonal k x k blocks are not read.
   so that H = U(L) Ht(L) V(L)* + D(L) with Ht(l+1) = U(l) Ht(l) V(l)* + B(l)
   and Ht(1) = B(0) (eq:tele1 - eq:tele3).

   Inverse factors (Algorithm 3), in this order:
     for l = L down to 1 (n = m at the leaves, 2k above):
       E_l  2^l blocks n x k;  F_l  2^l blocks k x n (as F*);  G_l  2^l blocks n x n
     G_0  one block 2k x 2k (the root's).

   Vectors x, y: M x nrhs row-major.  All pointers are device memory owned by
   the caller; the calls allocate their scratch (the library's pool), run on
   `stream` and return after it has finished.  hps_hbs_apply and
   hps_hbs_solve record their launches for one (buffer, x, y, nrhs, sizes)
   into a HIP graph on the first call and replay it afterwards (the last 16
   such passes are kept; hps_mem_trim drops them): the buffers' contents may
   change between calls, their addresses are part of the record.  Sizes outside the limits
   (L in [1, 14], 1 <= k <= m, m and 2k at most 3072) give HPS_EINVAL. */

/* Numbers of doubles in the factor and inverse buffers (either may be null). */
hps_status hps_hbs_sizes(int L, int m, int k, size_t* n_factors, size_t* n_inverse);
/* y = H x through the telescoping factorization (eq:tele1 - eq:tele3): x-hat up
   the tree through V*, the children's blocks of each B, y-hat down through U,
   and D at the leaves.  y must not overlap x. */
hps_status hps_hbs_apply(int L, int m, int k, const double* factors, const double* x, double* y,
                         int nrhs, void* stream);
/* Algorithm 3: the factors {E, F, G} of H^-1 (section 7.1; the blocks it
   inverts use Gauss-Jordan with partial pivoting).  A zero or non-finite
   pivot gives HPS_ESINGULAR (inverse is then unspecified). */
hps_status hps_hbs_invert(int L, int m, int k, const double* factors, double* inverse,
                          void* stream);
/* Algorithm 4: y = H^-1 x from the factors of hps_hbs_invert.  E multiplies
   the parent's y-hat in the downward and leaf steps.  y must not overlap x. */
hps_status hps_hbs_solve(int L, int m, int k, const double* inverse, const double* x, double* y,
                         int nrhs, void* stream);

/* Brute-force compression (Remark 8.2) of the dense M x M matrix H (device,
   row stride ldh >= M) into the factor layout above with rank k, from random
   samples that the caller draws: omega [M][k] and psit [k][M], i.i.d.
   standard normal (passed in so that a run can be repeated).  Bases are
   orthonormal and nested: each node's samples of its off-diagonal block row
   (H Omega less its diagonal block's part) and column (Psi* H likewise) are
   reduced to the children's bases at a parent (eq:def3) and orthonormalized
   by Gram-Schmidt with re-orthogonalization; B holds the children's
   projected interaction blocks (eq:def6).  The error is that of rank-k
   randomized range finding on every block row and column: choose k above
   the numerical rank (section 8 reports 10 to 80 at 1e-10 for
   non-oscillatory problems).  Limits: k <= 90 and m k <= 16384, else
   HPS_EINVAL. */
hps_status hps_hbs_compress(int L, int m, int k, const double* H, int ldh, const double* omega,
                            const double* psit, double* factors, void* stream);
/* The same for the root DtN T^1 of a built operator (M = n_bdry, m = n_bdry / 2^L;
   2^L must divide n_bdry): the HBS form that makes T_apply O(M k). */
hps_status hps_root_dtn_compress(const hps_op* op, int L, int k, const double* omega,
                                 const double* psit, double* factors, void* stream);

/* ---- host-side planner queries (no device work; used by CPU tests) ------ */

/* Coefficient-independent leaf tables for a hx-by-hy leaf (section 3.2),
   n = (p-2)^2, m = 4q: Dx, Dy, Dxx, Dyy [p][p]; G [5][n][m] (the images of L1
   under D1^2, D1 D2, D2^2, D1, D2 restricted to interior rows); P0 = L4 L3e L1
   [m][m]; P1 = L4 L3i [m][n]; Ji [n] interior node indices.  Any output may be
   NULL.  Requires 4 <= p <= 24, 1 <= q <= p - 1, hx, hy > 0 (HPS_EINVAL
   otherwise). */
hps_status hps_leaf_tables(int p, int q, double hx, double hy, double* Dx, double* Dy, double* Dxx,
                           double* Dyy, double* G, double* P0, double* P1, int* Ji);

/* Tree and merge maps of an nx-by-ny grid without building anything.
   rec as in hps_box; for a parent box sizes = {m1+m2, m3, n_alpha, n_beta} and
   pmap [m1+m2] (>= 0: position in alpha's boundary list, < 0: -(position in
   beta's) - 1), a3/b3 [m3] (shared-edge positions in alpha/beta), Ie [m1+m2]
   and Ii [m3] (global ids).  Returns the number of boxes in *n_boxes. */
hps_status hps_plan_box(const int nleaf[2], int q, int box, int rec[8], int sizes[4], int* pmap,
                        int* a3, int* b3, int* Ie, int* Ii, int* n_boxes);

/* ---- tuning knobs and the autotuner --------------------------------------- */

/* Forces a kernel variant for later launches in this process (-1 returns the
   choice to the tuning table, else the built-in default):
   "leaf_variant": fused leaf solve, 0-2 step-by-step LU (16x16 threads for
     p <= 12, 16x64, 16x32), 3-4 Gauss-Jordan (16x16 threads for p <= 12,
     16x32 threads);
   "gemm_variant": FP64 MFMA GEMM tile (0: 64x64x16 on 2x2 waves with three
     k-slabs of loads in flight, 1: 32x32x16 on one wave, 2: 128x128x16 on
     eight waves, 3: 128x64x16, 4: 64x128x16, 5: 64x64x32, 6: 64x64x16 with
     one slab in flight; 1-6 keep one slab in flight; 7: 128x128x16 on 2x2
     waves of 64x64, two LDS buffers, tiles in XCD-grouped order);
   "gj_variant": merge solver, 4 * (update tile) + TRSM block (0: 256, 1: 128,
     2: 64 threads); update tiles 0: 64x64x16 on 2x2 waves, 1: 32x32x16 on
     one wave, 2: 128x128x16 on 4x2 waves, 3: 128x64x16, 4: 64x128x16,
     5: 64x64x32 (one k-slab of loads in flight each);
   "solve_graph": 1 (default) runs plain solves as a captured HIP graph per
     operator and right-hand-side count, 0 launches kernel by kernel;
   "solve_mm_min_rhs": solves, source solves and refinement with at least
     this many right-hand sides keep the solution node by node ([N][nrhs],
     transposed on entry and exit) and run every pass as grouped FP64 MFMA
     GEMMs (-1: the default, 16; 0: never);
   "split_min_chunk": in those passes, depths with too few merges to fill
     the GPU split each GEMM contraction into chunks of at least this length
     (-1: the default, 256; else at least 16), summed in a fixed order;
   "parked_ops": how many destroyed operators keep their device buffers and
     descriptors for the next build of the same shape (0 frees at once; -1:
     the default, 2);
   "post_rows": Chebyshev-grid rows per lane in hps_postprocess (1, 2 or 4;
     -1: the default, 4 from 16 right-hand sides on, else 2);
   "gj_lookahead": 1 lets the merge solver update the next panel's columns
     first and the remaining columns on a second stream while the next panel
     is factored; 0 (default, also -1) runs every step on the caller's stream
     (faster on MI355X: the side stream's update delays the next panel);
   "bf16x6_min_k": in HPS_MIXED_BF16X6 builds, merge levels whose longest
     contraction (interface length m3) is below this run their Schur
     products in FP64 (-1: the default, 384; 0: BF16 on every level);
   "leaf_mfma": 1 (default, also -1) runs leaves with (p-2)^2 <= 112 on the
     MFMA leaf kernel (T formed in the kernel), 0 on leaf_variant's kernels;
   "bgj_min_rows": merge levels whose largest system (M = T33a - T33b, m3
     rows) has at least this many rows eliminate [M | I] by blocked
     Gauss-Jordan with pivoting inside 64 x 64 diagonal blocks (-1: the
     default, 256; 0: never), the others by partial pivoting;
   "bgj_fallback_tol_exp": e; a level whose blocked elimination meets a
     block pivot of at most 10^-e max|M| (or a zero or non-finite one) is
     gathered again and eliminated with partial pivoting (-1: the default,
     e = 6; 0 makes every level fall back);
   "leaf_bgj": 1 (default, also -1) eliminates the leaf systems the MFMA
     leaf kernel does not take (p > 12, or with keep_leaf_solution) by
     blocked Gauss-Jordan on the assembled [A_ii | R], pivoting inside 64 x 64
     diagonal blocks; a chunk of leaves with a block pivot at or below
     10^-e max|A_ii| ("bgj_fallback_tol_exp") is assembled again and
     eliminated with partial pivoting; 0 keeps the register kernels and the
     panel solver;
   "hbs_grid": workgroups of the persistent HBS apply / solve launch (0 or
     -1: two per CU; values are capped at what fits on the device at once);
   "solve_persist": 1 runs plain solves below 16 right-hand sides as one
     cooperative launch with a grid-wide barrier between levels (bit for bit
     the level passes' result); 0 (default, also -1) uses the level passes
     (a captured graph from the second solve on), measured faster;
   "gemm_queue": 1 (default, also -1) runs the FP64 products of a batch's
     merges at one depth (several problems) as one persistent launch of the
     128 x 128 tile over a tile queue, largest problems first; 0 launches the
     tuned tile over the largest problem's grid;
   "merge_small": 1 (default, also -1) builds every merge level whose
     interfaces have at most 20 nodes in one launch (one workgroup per merge:
     gather, elimination of [M | I], S and T); 0 uses the level-wise kernels
     there too;
   "bgj_lookahead": 1 (default, also -1) updates the next diagonal block's
     columns first and the other columns on a second stream (default
     priority) while the next diagonal block is inverted; 0 runs each step's
     update in one launch on the caller's stream.
   Unknown knobs or values give HPS_EINVAL. */
hps_status hps_tune_set(const char* knob, int value);

/* Number of merge levels and leaf chunks, over all builds of this process,
   whose blocked Gauss-Jordan elimination fell back to partial pivoting. */
hps_status hps_bgj_fallbacks(long long* count);

/* Autotuner.  For every problem shape in probs (only nleaf, p, q and box are
   read; coeffs may be NULL) it times every variant of the leaf kernel, of the
   FP64 MFMA GEMM (per shape bucket: log2 of M, N, K and of the batch count) and
   of the merge solver (per bucket of system rows, columns and count) on
   synthetic data of those shapes, and records the fastest in the process's
   tuning table, which later builds consult.  Buckets already in the table are
   not re-timed.  *seconds (may be NULL) receives the time spent.  Work is
   enqueued on stream (NULL = default) and waited for. */
hps_status hps_autotune(const hps_problem* probs, int nprob, void* stream, double* seconds);
/* Writes the tuning table as JSON (format "hps-tune-2") / merges such a file
   into the table (HPS_EINVAL on a malformed file or another format: the
   variant numbers of older formats meant other kernels) / empties the table. */
hps_status hps_tune_save(const char* path);
hps_status hps_tune_load(const char* path);
hps_status hps_tune_reset(void);

/* ---- launch timing (HIP events on the launch stream) --------------------- */

/* Kernel classes: 0 leaf assembly, 1 LU panel, 2 row swaps + block-row solve,
   3 LU trailing update, 4 back substitution, 5 FP64 Schur GEMM of the
   merges (T = D + Q S, eq:merge), 6 split-FP32 Schur GEMM, 7 merge gather,
   8 downward pass, 9 interface residual, 10 upward pass, 11 fused leaf
   elimination, 12 surrogate training, 13 surrogate inference, 14
   post-processing, 15 BF16 three-slice Schur GEMM, 16 body-load fluxes from
   the kept body operator, 17 leaf T = P0 - P1 Z products (section 3.2),
   18 the merges' S = M^-1 B products (eq:U_parent), 19-21 the blocked
   Gauss-Jordan steps of large merge systems (diagonal-block inverses, block
   rows, updates of the other rows), 22 whole small merges in one launch,
   23 HBS passes (a replayed apply or solve as one record; the products of
   Algorithm 3 and of the compression one record per launch).  Bit c of mask
   enables class c; every
   later launch of an enabled class records a start and stop event on its
   stream together with its algorithmic FLOPs and bytes.  Costs one event
   pair per launch while enabled. */
hps_status hps_prof_enable(unsigned mask);
/* Drops all records (waits for their events first). */
hps_status hps_prof_reset(void);
/* Totals over the recorded launches of a class: summed event time in ms,
   number of launches, algorithmic FLOPs and bytes.  Waits for the events. */
hps_status hps_prof_query(int cls, double* ms, long long* launches, double* flops, double* bytes);

/* ---- lifetime, errors --------------------------------------------------- */

/* Device memory cache.  Operators, plans and temporaries take their device
   memory from a per-device cache that keeps released blocks for reuse, so
   repeated builds of one shape do not call hipMalloc/hipFree; the
   stream-ordered scratch of solves is likewise kept in the device's default
   memory pool.  hps_mem_trim frees the parked operators (see hps_destroy),
   every cached block (blocks in use are untouched) and the pool's unused
   memory on the current device, and reports the bytes freed from the cache;
   hps_mem_stats reports the bytes cached and in use (a parked operator's
   buffers count as in use).  Either pointer may be NULL. */
hps_status hps_mem_trim(size_t* freed);
hps_status hps_mem_stats(size_t* cached, size_t* in_use);

/* Waits for the device, then releases op.  Its device buffers and level
   descriptors are parked for the next hps_build_solution_operator or
   hps_build_batch of the same leaf grid, box, p, q, mode, device_ptrs and
   kept data on the same device, which then only sets the coefficients and
   per-build options instead of planning and uploading descriptors (knob
   "parked_ops" bounds how many wait, most recent first; hps_mem_trim frees
   them).  NULL is ignored. */
void hps_destroy(hps_op* op);
const char* hps_last_error(void);
const char* hps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H */
