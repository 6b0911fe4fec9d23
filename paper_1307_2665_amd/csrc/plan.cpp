// Host planner: discretization constants (sections 2, 3.1, 3.2), the box tree
// (section 2) and the merge index maps (section 4, the J1/J2/J3 split).
#include "plan.h"

#include <cmath>
#include <stdexcept>

namespace hps {

std::vector<double> cheb_points(int p) {
  std::vector<double> x(p);
  for (int j = 0; j < p; ++j) x[j] = -std::cos(M_PI * j / (p - 1));
  return x;
}

// Gauss-Legendre nodes: Newton's method on P_q from the usual cosine guesses,
// with the three-term recurrence for P_q and its derivative.
std::vector<double> gauss_points(int q) {
  std::vector<double> x(q);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      // P_q(z) = pk and P_{q-1}(z) = pkm1 by the three-term recurrence.
      double pkm1 = 1.0, pk = z;
      for (int k = 2; k <= q; ++k) {
        double pkp1 = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
        pkm1 = pk;
        pk = pkp1;
      }
      double dp = q * (z * pk - pkm1) / (z * z - 1.0);
      double dz = pk / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[q - 1 - i] = z;  // guesses run from +1 down; store ascending
  }
  return x;
}

// Chebyshev differentiation matrix from the barycentric weights of the
// Chebyshev-Lobatto points, w_j = (-1)^j * (1/2 at the ends, 1 inside):
// D_ij = (w_j / w_i) / (x_i - x_j), diagonal by the negative-sum rule.
std::vector<double> cheb_diff(int p) {
  std::vector<double> x = cheb_points(p), w(p), D(p * p, 0.0);
  for (int j = 0; j < p; ++j) w[j] = ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == p - 1) ? 0.5 : 1.0);
  for (int i = 0; i < p; ++i) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      D[i * p + j] = (w[j] / w[i]) / (x[i] - x[j]);
      s += D[i * p + j];
    }
    D[i * p + i] = -s;
  }
  return D;
}

std::vector<double> interp_matrix(const std::vector<double>& src, const std::vector<double>& dst) {
  const int n = (int)src.size(), m = (int)dst.size();
  std::vector<double> w(n, 1.0), L(m * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) w[j] /= (src[j] - src[k]);
  for (int i = 0; i < m; ++i) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (dst[i] == src[j]) hit = j;
    if (hit >= 0) {
      L[i * n + hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += w[j] / (dst[i] - src[j]);
    for (int j = 0; j < n; ++j) L[i * n + j] = (w[j] / (dst[i] - src[j])) / den;
  }
  return L;
}

static std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int M,
                                  int K, int N) {
  std::vector<double> C((size_t)M * N, 0.0);
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < K; ++k) {
      double a = A[(size_t)i * K + k];
      if (a == 0.0) continue;
      for (int j = 0; j < N; ++j) C[(size_t)i * N + j] += a * B[(size_t)k * N + j];
    }
  return C;
}

LeafTables make_leaf_tables(int p, int q, double hx, double hy) {
  LeafTables t;
  t.p = p;
  t.q = q;
  t.n = (p - 2) * (p - 2);
  t.m = 4 * q;
  t.hx = hx;
  t.hy = hy;
  const int pp = p * p, m = t.m, n = t.n;
  std::vector<double> D = cheb_diff(p);
  t.Dx.resize(p * p);
  t.Dy.resize(p * p);
  for (int i = 0; i < p * p; ++i) {
    t.Dx[i] = D[i] * (2.0 / hx);
    t.Dy[i] = D[i] * (2.0 / hy);
  }
  t.Dxx = matmul(t.Dx, t.Dx, p, p, p);
  t.Dyy = matmul(t.Dy, t.Dy, p, p, p);

  for (int k = 0; k < pp; ++k) {
    int a = k % p, b = k / p;
    bool bd = (a == 0 || a == p - 1 || b == 0 || b == p - 1);
    (bd ? t.Je : t.Ji).push_back(k);
  }
  std::vector<double> xc = cheb_points(p), xg = gauss_points(q);
  std::vector<double> G2C = interp_matrix(xg, xc);  // p x q
  std::vector<double> C2G = interp_matrix(xc, xg);  // q x p

  // Step 1 of section 3.2 (L1), with corner nodes averaged over both sides.
  const int ne = (int)t.Je.size();
  t.L1.assign((size_t)ne * m, 0.0);
  for (int r = 0; r < ne; ++r) {
    int k = t.Je[r], a = k % p, b = k / p;
    int side[2], pos[2], c = 0;
    if (b == 0) { side[c] = 0; pos[c++] = a; }
    if (a == p - 1) { side[c] = 1; pos[c++] = b; }
    if (b == p - 1) { side[c] = 2; pos[c++] = a; }
    if (a == 0) { side[c] = 3; pos[c++] = b; }
    for (int s = 0; s < c; ++s)
      for (int g = 0; g < q; ++g) t.L1[(size_t)r * m + side[s] * q + g] += G2C[pos[s] * q + g] / c;
  }

  // Full-grid operators on p*p nodes: D1 = I (x) Dx, D2 = Dy (x) I.
  auto D1 = [&](int k, int kk) {
    return (k / p == kk / p) ? t.Dx[(k % p) * p + (kk % p)] : 0.0;
  };
  auto D2 = [&](int k, int kk) {
    return (k % p == kk % p) ? t.Dy[(k / p) * p + (kk / p)] : 0.0;
  };
  // E: p*p x m, L1 placed on J_e.
  std::vector<double> E((size_t)pp * m, 0.0);
  for (int r = 0; r < ne; ++r)
    for (int c = 0; c < m; ++c) E[(size_t)t.Je[r] * m + c] = t.L1[(size_t)r * m + c];
  std::vector<double> D1m((size_t)pp * pp), D2m((size_t)pp * pp);
  for (int k = 0; k < pp; ++k)
    for (int kk = 0; kk < pp; ++kk) {
      D1m[(size_t)k * pp + kk] = D1(k, kk);
      D2m[(size_t)k * pp + kk] = D2(k, kk);
    }
  std::vector<double> D1E = matmul(D1m, E, pp, pp, m);
  std::vector<double> D2E = matmul(D2m, E, pp, pp, m);
  std::vector<double> D11E = matmul(D1m, D1E, pp, pp, m);
  std::vector<double> D12E = matmul(D1m, D2E, pp, pp, m);
  std::vector<double> D22E = matmul(D2m, D2E, pp, pp, m);
  t.G.assign((size_t)5 * n * m, 0.0);
  const std::vector<double>* src[5] = {&D11E, &D12E, &D22E, &D1E, &D2E};
  for (int s = 0; s < 5; ++s)
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < m; ++c)
        t.G[((size_t)s * n + i) * m + c] = (*src[s])[(size_t)t.Ji[i] * m + c];

  // Steps 3 and 4: F = L4 L3 (m x p*p); flux rows du/dx2 on S, N and du/dx1 on E, W.
  std::vector<double> F((size_t)m * pp, 0.0);
  for (int s = 0; s < 4; ++s) {
    for (int g = 0; g < q; ++g) {
      double* row = &F[(size_t)(s * q + g) * pp];
      for (int c = 0; c < p; ++c) {
        double w = C2G[g * p + c];
        int node;
        bool dy;
        switch (s) {
          case 0: node = c; dy = true; break;                    // S: (a=c, b=0)
          case 1: node = (p - 1) + p * c; dy = false; break;     // E: (a=p-1, b=c)
          case 2: node = c + p * (p - 1); dy = true; break;      // N: (a=c, b=p-1)
          default: node = p * c; dy = false; break;              // W: (a=0, b=c)
        }
        for (int kk = 0; kk < pp; ++kk) row[kk] += w * (dy ? D2(node, kk) : D1(node, kk));
      }
    }
  }
  std::vector<double> Fe((size_t)m * ne);
  t.P1.assign((size_t)m * n, 0.0);
  for (int r = 0; r < m; ++r) {
    for (int e = 0; e < ne; ++e) Fe[(size_t)r * ne + e] = F[(size_t)r * pp + t.Je[e]];
    for (int i = 0; i < n; ++i) t.P1[(size_t)r * n + i] = F[(size_t)r * pp + t.Ji[i]];
  }
  t.P0 = matmul(Fe, t.L1, m, ne, m);
  return t;
}

Tree build_tree(int nx, int ny, int q) {
  Tree t;
  t.nx = nx;
  t.ny = ny;
  t.q = q;
  t.nh = nx * (ny + 1);
  t.N = q * (nx * (ny + 1) + (nx + 1) * ny);
  t.boxes.push_back(BoxRec{0, nx, 0, ny, 0, -1, -1, -1, false});
  for (size_t k = 0; k < t.boxes.size(); ++k) {
    BoxRec b = t.boxes[k];
    int w = b.i1 - b.i0, h = b.j1 - b.j0;
    if (w == 1 && h == 1) continue;
    bool vert = (w > h) || (w == h);
    BoxRec ca = b, cb = b;
    ca.level = cb.level = b.level + 1;
    ca.parent = cb.parent = (int)k;
    ca.ca = ca.cb = cb.ca = cb.cb = -1;
    ca.vertical = cb.vertical = false;
    if (vert) {
      int m = b.i0 + w / 2;
      ca.i1 = m;
      cb.i0 = m;
    } else {
      int m = b.j0 + h / 2;
      ca.j1 = m;
      cb.j0 = m;
    }
    t.boxes[k].vertical = vert;
    t.boxes[k].ca = (int)t.boxes.size();
    t.boxes[k].cb = (int)t.boxes.size() + 1;
    t.boxes.push_back(ca);
    t.boxes.push_back(cb);
  }
  t.depth = 0;
  for (auto& b : t.boxes) t.depth = std::max(t.depth, b.level);
  t.parents_at_level.assign(t.depth + 1, {});
  t.leaves.assign((size_t)nx * ny, -1);
  for (size_t k = 0; k < t.boxes.size(); ++k) {
    const BoxRec& b = t.boxes[k];
    if (b.ca >= 0)
      t.parents_at_level[b.level].push_back((int)k);
    else
      t.leaves[b.i0 + nx * b.j0] = (int)k;
  }
  return t;
}

static inline int hedge_id(const Tree& t, int i, int j) { return j * t.nx + i; }
static inline int vedge_id(const Tree& t, int i, int j) { return t.nh + j * (t.nx + 1) + i; }

void box_boundary(const Tree& t, int i0, int i1, int j0, int j1, std::vector<int>& out) {
  out.clear();
  const int q = t.q;
  for (int i = i0; i < i1; ++i)
    for (int k = 0; k < q; ++k) out.push_back(hedge_id(t, i, j0) * q + k);
  for (int j = j0; j < j1; ++j)
    for (int k = 0; k < q; ++k) out.push_back(vedge_id(t, i1, j) * q + k);
  for (int i = i0; i < i1; ++i)
    for (int k = 0; k < q; ++k) out.push_back(hedge_id(t, i, j1) * q + k);
  for (int j = j0; j < j1; ++j)
    for (int k = 0; k < q; ++k) out.push_back(vedge_id(t, i0, j) * q + k);
}

// Position of a node (given by edge and index along it) in a box's S,E,N,W list.
// Returns -1 when the node is not on the box boundary.
static int pos_in_box(const BoxRec& b, int q, bool horiz, int ei, int ej, int k) {
  int w = b.i1 - b.i0, h = b.j1 - b.j0;
  if (horiz) {
    if (ei < b.i0 || ei >= b.i1) return -1;
    if (ej == b.j0) return (ei - b.i0) * q + k;
    if (ej == b.j1) return (w + h + (ei - b.i0)) * q + k;
    return -1;
  }
  if (ej < b.j0 || ej >= b.j1) return -1;
  if (ei == b.i1) return (w + (ej - b.j0)) * q + k;
  if (ei == b.i0) return (2 * w + h + (ej - b.j0)) * q + k;
  return -1;
}

MergeMaps merge_maps(const Tree& t, int box) {
  const BoxRec& P = t.boxes[box];
  const BoxRec& A = t.boxes[P.ca];
  const BoxRec& B = t.boxes[P.cb];
  const int q = t.q;
  MergeMaps mm;
  mm.na = 2 * q * ((A.i1 - A.i0) + (A.j1 - A.j0));
  mm.nb = 2 * q * ((B.i1 - B.i0) + (B.j1 - B.j0));
  mm.me = 2 * q * ((P.i1 - P.i0) + (P.j1 - P.j0));
  box_boundary(t, P.i0, P.i1, P.j0, P.j1, mm.Ie);
  // Walk the parent's boundary edge by edge, in S,E,N,W order.
  auto add = [&](bool horiz, int ei, int ej) {
    for (int k = 0; k < q; ++k) {
      int pa = pos_in_box(A, q, horiz, ei, ej, k);
      if (pa >= 0) {
        mm.pmap.push_back(pa);
      } else {
        int pb = pos_in_box(B, q, horiz, ei, ej, k);
        if (pb < 0) throw std::logic_error("merge map: node on neither child");
        mm.pmap.push_back(-pb - 1);
      }
    }
  };
  for (int i = P.i0; i < P.i1; ++i) add(true, i, P.j0);
  for (int j = P.j0; j < P.j1; ++j) add(false, P.i1, j);
  for (int i = P.i0; i < P.i1; ++i) add(true, i, P.j1);
  for (int j = P.j0; j < P.j1; ++j) add(false, P.i0, j);
  // Shared edge J3, ascending along the edge.
  if (P.vertical) {
    int m = A.i1;
    for (int j = P.j0; j < P.j1; ++j)
      for (int k = 0; k < q; ++k) {
        mm.a3.push_back(pos_in_box(A, q, false, m, j, k));
        mm.b3.push_back(pos_in_box(B, q, false, m, j, k));
        mm.Ii.push_back(vedge_id(t, m, j) * q + k);
      }
  } else {
    int m = A.j1;
    for (int i = P.i0; i < P.i1; ++i)
      for (int k = 0; k < q; ++k) {
        mm.a3.push_back(pos_in_box(A, q, true, i, m, k));
        mm.b3.push_back(pos_in_box(B, q, true, i, m, k));
        mm.Ii.push_back(hedge_id(t, i, m) * q + k);
      }
  }
  mm.m3 = (int)mm.a3.size();
  return mm;
}

void gauss_node_xy(const Tree& t, const double box[4], std::vector<double>& xy) {
  std::vector<double> g = gauss_points(t.q);
  const double hx = (box[1] - box[0]) / t.nx, hy = (box[3] - box[2]) / t.ny;
  xy.assign((size_t)2 * t.N, 0.0);
  for (int j = 0; j <= t.ny; ++j)
    for (int i = 0; i < t.nx; ++i)
      for (int k = 0; k < t.q; ++k) {
        size_t id = (size_t)hedge_id(t, i, j) * t.q + k;
        xy[2 * id] = box[0] + (i + 0.5 * (g[k] + 1.0)) * hx;
        xy[2 * id + 1] = box[2] + j * hy;
      }
  for (int j = 0; j < t.ny; ++j)
    for (int i = 0; i <= t.nx; ++i)
      for (int k = 0; k < t.q; ++k) {
        size_t id = (size_t)vedge_id(t, i, j) * t.q + k;
        xy[2 * id] = box[0] + i * hx;
        xy[2 * id + 1] = box[2] + (j + 0.5 * (g[k] + 1.0)) * hy;
      }
}

void cheb_node_xy(int nx, int ny, int p, const double box[4], std::vector<double>& xy) {
  std::vector<double> c = cheb_points(p);
  const double hx = (box[1] - box[0]) / nx, hy = (box[3] - box[2]) / ny;
  xy.assign((size_t)nx * ny * p * p * 2, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t lf = (size_t)i + (size_t)nx * j;
      double x0 = box[0] + i * hx, y0 = box[2] + j * hy;
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) {
          size_t k = lf * p * p + a + (size_t)p * b;
          xy[2 * k] = x0 + 0.5 * (c[a] + 1.0) * hx;
          xy[2 * k + 1] = y0 + 0.5 * (c[b] + 1.0) * hy;
        }
    }
}

}  // namespace hps
