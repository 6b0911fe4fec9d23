// Host planner: discretization constants, the box tree and the merge index maps.
#pragma once

#include <cstdint>
#include <vector>

namespace hps {

// ---- section 2 / 3.1: nodes, differentiation, interpolation ---------------

std::vector<double> cheb_points(int p);                 // Chebyshev-Lobatto, ascending
std::vector<double> gauss_points(int q);                // Gauss-Legendre, ascending
std::vector<double> cheb_diff(int p);                   // p x p, row-major
// L[i][j] = l_j(dst_i) for the interpolant through src (barycentric form).
std::vector<double> interp_matrix(const std::vector<double>& src, const std::vector<double>& dst);

// Coefficient-independent pieces of the leaf computation (section 3.2) for
// a hx-by-hy leaf.  With n = (p-2)^2 interior Chebyshev nodes:
//   A_ii[k][k'] is formed on the device from Dx, Dy, Dxx, Dyy and the six
//   coefficient values at node k;
//   R = A_ie L1 = -c11 G11 - 2 c12 G12 - c22 G22 + c1 G1 + c2 G2 (row-wise
//   coefficients), where Gxx = (Dxx-operator E)[J_i] and E places L1 on J_e;
//   T = P0 - P1 Z with Z = A_ii^-1 R, P0 = L4 L3[:,J_e] L1, P1 = L4 L3[:,J_i].
struct LeafTables {
  int p, q, n, m;                      // m = 4q
  double hx, hy;
  std::vector<double> Dx, Dy, Dxx, Dyy;  // p x p each
  std::vector<double> G;               // 5 x n x m: G11, G12, G22, G1, G2
  std::vector<double> P0;              // m x m
  std::vector<double> P1;              // m x n
  std::vector<double> L1;              // 4(p-1) x m, rows in ascending boundary-node order
  std::vector<int> Je, Ji;
};
LeafTables make_leaf_tables(int p, int q, double hx, double hy);

// ---- section 2: tree ------------------------------------------------------

struct BoxRec {
  int i0, i1, j0, j1;
  int level, parent, ca, cb;  // ca = alpha (west/south), cb = beta; -1 for leaves
  bool vertical;              // split across x1 (alpha west) when true
};

struct Tree {
  int nx, ny, q;
  int N;                          // Gauss nodes
  int nh;                         // horizontal-edge count nx*(ny+1)
  std::vector<BoxRec> boxes;      // breadth first, root 0
  std::vector<std::vector<int>> parents_at_level;  // parent boxes per level (level = depth)
  std::vector<int> leaves;        // leaf box index per leaf id i + nx*j
  int depth;                      // max level
};
Tree build_tree(int nx, int ny, int q);

// Global Gauss ids on the boundary of a box in S,E,N,W order.
void box_boundary(const Tree& t, int i0, int i1, int j0, int j1, std::vector<int>& out);

// Merge maps of a parent box: pmap (parent order -> child position, beta encoded
// as -(pos)-1), a3/b3 (shared edge positions), Ie (parent boundary ids),
// Ii (shared edge ids).
struct MergeMaps {
  std::vector<int> pmap, a3, b3, Ie, Ii;
  int na, nb, me, m3;
};
MergeMaps merge_maps(const Tree& t, int box);

// Coordinates.
void gauss_node_xy(const Tree& t, const double box[4], std::vector<double>& xy);
void cheb_node_xy(int nx, int ny, int p, const double box[4], std::vector<double>& xy);

}  // namespace hps
