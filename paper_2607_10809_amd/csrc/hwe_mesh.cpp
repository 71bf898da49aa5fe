// Host precompute of the hwe library: geometry, stencils, edge Gauss points and
// the per-cell least-squares maps of the HWENO reconstruction, all in FP64,
// with cells renumbered along a Morton curve.
//
// Reconstruction basis.  About the centroid (x0, y0) of the target cell K0,
// with X = x - x0, Y = y - y0 and the central second moments
// Mxx = avg_K0 X^2, Mxy = avg_K0 XY, Myy = avg_K0 Y^2, every candidate
// polynomial is written as
//     p = Wbar_0 + c1 X + c2 Y + c3 (X^2 - Mxx) + c4 (XY - Mxy) + c5 (Y^2 - Myy),
// which has the cell average Wbar_0 on K0 by construction (the conservation
// requirement of Steps 1 and 2, Sec. 2.2).
//
// Step 1 (quadratic p1 on {K0, K1, K2, K3}): the three neighbour averages are
// equality constraints, the six union derivative integrals
//   int_{Kl + K0} p_x = |Kl| Vbar_l + |K0| Vbar_0,  int_{Kl + K0} p_y = |Kl| Ybar_l + |K0| Ybar_0
// are matched in the least-squares sense.  The solution is linear in the data:
// a 5 x 11 matrix maps
//   (dW1, dW2, dW3, V0, V1, V2, V3, Y0, Y1, Y2, Y3),  dWl = Wbar_l - Wbar_0,
// to (c1..c5).  It is computed by the null-space method: Householder QR of the
// constraint matrix, then a 2 x 2 least-squares problem on its null space.  The
// device tables keep it factored: the dW columns (5 x 3), the null-space basis
// Z (2 x 5) and the reduced solution Q (2 x 8) with the V, Y columns = Z^T Q.
//
// Step 2 (linear p_{l+1} on {K0, Kl}): with p = Wbar_0 + b X + c Y the K0 average
// holds exactly, and the rows  [dx dy] (b, c) = dWl,  b = Vbar_l,  c = Ybar_l
// (each the printed condition divided by |Kl|) are matched in least squares,
// giving (b, c) = v + d (dWl - d.v) / (1 + d.d),  v = (Vbar_l, Ybar_l),
// d = centroid offset.  Each cell stores (dx, dy, 1/(1 + d.d)) per face.
//
// Boundaries: periodic meshes are tori (neighbour geometry translated across the
// seams); on transmissive boundaries the stencil uses the target cell mirrored
// across the boundary face.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <sstream>
#include <utility>

#include "hwe_internal.h"

namespace hwe {
namespace {

struct Tri {
  double x[3], y[3];
};

double signed_area(const Tri& t) {
  return 0.5 * ((t.x[1] - t.x[0]) * (t.y[2] - t.y[0]) - (t.y[1] - t.y[0]) * (t.x[2] - t.x[0]));
}

// Geometry of a triangle: area, centroid and central second moments.  The
// moments use avg(X^2) = (dx0^2 + dx1^2 + dx2^2) / 12 over the vertex offsets
// from the centroid (exact: the edge-midpoint rule integrates quadratics).
struct CellGeo {
  double A, cx, cy, mxx, mxy, myy;
};
CellGeo cell_geo(const Tri& t) {
  CellGeo g;
  g.A = signed_area(t);
  g.cx = (t.x[0] + t.x[1] + t.x[2]) / 3.0;
  g.cy = (t.y[0] + t.y[1] + t.y[2]) / 3.0;
  double sxx = 0, sxy = 0, syy = 0;
  for (int i = 0; i < 3; ++i) {
    double dx = t.x[i] - g.cx, dy = t.y[i] - g.cy;
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
  }
  g.mxx = sxx / 12.0;
  g.mxy = sxy / 12.0;
  g.myy = syy / 12.0;
  return g;
}

// Householder QR of a column-major matrix a (rows x cols, rows >= cols):
// on return a holds R in its upper triangle and the reflectors below it;
// tau the reflector scalars.  Q is applied with apply_q / apply_qt.
void householder_qr(double* a, int rows, int cols, double* tau) {
  for (int k = 0; k < cols; ++k) {
    double* col = a + k * rows;
    double nrm = 0.0;
    for (int i = k; i < rows; ++i) nrm += col[i] * col[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) {
      tau[k] = 0.0;
      continue;
    }
    double alpha = col[k] > 0 ? -nrm : nrm;
    double v0 = col[k] - alpha;
    // v = (1, col[k+1..]/v0), tau = -v0 / alpha
    for (int i = k + 1; i < rows; ++i) col[i] /= v0;
    tau[k] = -v0 / alpha;
    col[k] = alpha;
    for (int j = k + 1; j < cols; ++j) {
      double* cj = a + j * rows;
      double s = cj[k];
      for (int i = k + 1; i < rows; ++i) s += col[i] * cj[i];
      s *= tau[k];
      cj[k] -= s;
      for (int i = k + 1; i < rows; ++i) cj[i] -= s * col[i];
    }
  }
}
// y <- Q y for the factor stored by householder_qr (Q = H0 H1 ... H_{cols-1}).
void apply_q(const double* a, int rows, int cols, const double* tau, double* y) {
  for (int k = cols - 1; k >= 0; --k) {
    const double* col = a + k * rows;
    double s = y[k];
    for (int i = k + 1; i < rows; ++i) s += col[i] * y[i];
    s *= tau[k];
    y[k] -= s;
    for (int i = k + 1; i < rows; ++i) y[i] -= s * col[i];
  }
}
// y <- Q^T y.
void apply_qt(const double* a, int rows, int cols, const double* tau, double* y) {
  for (int k = 0; k < cols; ++k) {
    const double* col = a + k * rows;
    double s = y[k];
    for (int i = k + 1; i < rows; ++i) s += col[i] * y[i];
    s *= tau[k];
    y[k] -= s;
    for (int i = k + 1; i < rows; ++i) y[i] -= s * col[i];
  }
}

// Step-1 map for one cell.  Inputs are in K0's frame, lengths scaled by
// h = sqrt(|K0|) and areas by |K0|:  d[l] (neighbour centroid offsets),
// dm[l] (neighbour moments minus K0's moments), ar[l] = |Kl| / |K0|.
// Output: M (5 x 11, row-major) in the scaled variables, and its factored form
// for the device tables: the derivative-average columns of M are Z^T Q with Z
// (2 x 5) the null-space basis of the constraints and Q (2 x 8) the reduced
// least-squares solution applied to (V0..V3, Y0..Y3); false if singular.
bool step1_map(const double d[3][2], const double dm[3][3], const double ar[3], double M[5][11], double Zo[2][5],
               double Qo[2][8]) {
  // constraint matrix C (3 x 5), stored transposed column-major: Ct is 5 x 3
  double Ct[5 * 3];
  for (int l = 0; l < 3; ++l) {
    double dx = d[l][0], dy = d[l][1];
    double row[5] = {dx, dy, dx * dx + dm[l][0], dx * dy + dm[l][1], dy * dy + dm[l][2]};
    for (int j = 0; j < 5; ++j) Ct[l * 5 + j] = row[j];
  }
  double tau[3];
  householder_qr(Ct, 5, 3, tau);
  double rdiag = 0;
  for (int k = 0; k < 3; ++k) rdiag = std::max(rdiag, std::fabs(Ct[k * 5 + k]));
  for (int k = 0; k < 3; ++k)
    if (!(std::fabs(Ct[k * 5 + k]) > 1e-12 * rdiag)) return false;
  // least-squares rows A (6 x 5): x rows then y rows
  double A[6][5];
  for (int l = 0; l < 3; ++l) {
    double dx = d[l][0], dy = d[l][1], a = ar[l];
    double rx[5] = {a + 1.0, 0.0, 2.0 * a * dx, a * dy, 0.0};
    double ry[5] = {0.0, a + 1.0, 0.0, a * dx, 2.0 * a * dy};
    for (int j = 0; j < 5; ++j) {
      A[l][j] = rx[j];
      A[3 + l][j] = ry[j];
    }
  }
  // Null-space basis Z = Q[:, 3:5] and particular map P = Q[:, 0:3] R^{-T}.
  double Z[2][5], P[3][5];
  for (int c = 0; c < 2; ++c) {
    double y[5] = {0, 0, 0, 0, 0};
    y[3 + c] = 1.0;
    apply_q(Ct, 5, 3, tau, y);
    for (int j = 0; j < 5; ++j) Z[c][j] = y[j];
  }
  for (int c = 0; c < 3; ++c) {
    // solve R^T w = e_c (R upper 3x3 in Ct), then y = Q [w; 0]
    double w[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= Ct[i * 5 + k] * w[k];  // R^T(i,k) = R(k,i) = Ct[i*5+k]
      w[i] = s / Ct[i * 5 + i];
    }
    double y[5] = {w[0], w[1], w[2], 0, 0};
    apply_q(Ct, 5, 3, tau, y);
    for (int j = 0; j < 5; ++j) P[c][j] = y[j];
  }
  // B = A Z (6 x 2), QR of B
  double B[2 * 6];
  for (int c = 0; c < 2; ++c)
    for (int r = 0; r < 6; ++r) {
      double s = 0;
      for (int j = 0; j < 5; ++j) s += A[r][j] * Z[c][j];
      B[c * 6 + r] = s;
    }
  double tb[2];
  householder_qr(B, 6, 2, tb);
  double bmax = std::max(std::fabs(B[0]), std::fabs(B[6 + 1]));
  if (!(std::fabs(B[0]) > 1e-12 * bmax) || !(std::fabs(B[6 + 1]) > 1e-12 * bmax)) return false;
  // pseudo-inverse rows: Bp (2 x 6) = R_B^{-1} Q_B^T
  double Bp[2][6];
  for (int r = 0; r < 6; ++r) {
    double y[6] = {0, 0, 0, 0, 0, 0};
    y[r] = 1.0;
    apply_qt(B, 6, 2, tb, y);
    double z1 = y[1] / B[6 + 1];
    double z0 = (y[0] - B[6 + 0] * z1) / B[0];
    Bp[0][r] = z0;
    Bp[1][r] = z1;
  }
  // c = P dW + Z Bp (b - A P dW):  columns for dW (3) and for the 6 LS right-hand sides
  double Mb[5][6], Md[5][3];
  for (int j = 0; j < 5; ++j)
    for (int r = 0; r < 6; ++r) Mb[j][r] = Z[0][j] * Bp[0][r] + Z[1][j] * Bp[1][r];
  for (int c = 0; c < 3; ++c) {
    double AP[6];
    for (int r = 0; r < 6; ++r) {
      double s = 0;
      for (int j = 0; j < 5; ++j) s += A[r][j] * P[c][j];
      AP[r] = s;
    }
    for (int j = 0; j < 5; ++j) {
      double s = P[c][j];
      for (int r = 0; r < 6; ++r) s -= Mb[j][r] * AP[r];
      Md[j][c] = s;
    }
  }
  for (int k = 0; k < 2; ++k) {
    for (int j = 0; j < 5; ++j) Zo[k][j] = Z[k][j];
    double v0 = 0, y0 = 0;
    for (int l = 0; l < 3; ++l) {
      Qo[k][1 + l] = Bp[k][l] * ar[l];
      Qo[k][5 + l] = Bp[k][3 + l] * ar[l];
      v0 += Bp[k][l];
      y0 += Bp[k][3 + l];
    }
    Qo[k][0] = v0;
    Qo[k][4] = y0;
  }
  // assemble the 11 input columns: dW1..3, V0, V1..3, Y0, Y1..3 where the
  // scaled right-hand sides are b_x,l = ar_l V_l + V0 (times h, applied by the caller)
  for (int j = 0; j < 5; ++j) {
    for (int c = 0; c < 3; ++c) M[j][c] = Md[j][c];
    double v0 = 0, y0 = 0;
    for (int l = 0; l < 3; ++l) {
      M[j][4 + l] = Mb[j][l] * ar[l];
      M[j][8 + l] = Mb[j][3 + l] * ar[l];
      v0 += Mb[j][l];
      y0 += Mb[j][3 + l];
    }
    M[j][3] = v0;
    M[j][7] = y0;
  }
  return true;
}

uint64_t spread_bits(uint32_t v) {
  uint64_t x = v & 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffULL;
  x = (x | (x << 4)) & 0x0f0f0f0fULL;
  x = (x | (x << 2)) & 0x33333333ULL;
  x = (x | (x << 1)) & 0x55555555ULL;
  return x;
}

hwe_status fail(hwe_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

}  // namespace

// Kind of a boundary face (hwe_bnd_kind): the first region of o.regions that
// holds its midpoint, else a reflective wall when it lies on a side of the box
// (s = 0: x = x0, 1: x = x1, 2: y = y0, 3: y = y1) whose bit is set in o.walls,
// else transmissive.
static int boundary_kind(const hwe_opts& o, const Tri& t, int f) {
  const int f1 = (f + 1) % 3;
  const double ex = t.x[f1] - t.x[f], ey = t.y[f1] - t.y[f];
  const double mx = 0.5 * (t.x[f] + t.x[f1]), my = 0.5 * (t.y[f] + t.y[f1]);
  const double tol = 1e-9 * std::max(o.box[1] - o.box[0], o.box[3] - o.box[2]);
  for (int r = 0; r < o.n_regions; ++r) {
    const double* b = o.regions[r].box;
    if (mx >= b[0] - tol && mx <= b[1] + tol && my >= b[2] - tol && my <= b[3] + tol) return o.regions[r].kind;
  }
  if (!o.walls) return HWE_BND_TRANSMISSIVE;
  const bool on[4] = {std::fabs(mx - o.box[0]) < tol && std::fabs(ex) < tol,
                      std::fabs(mx - o.box[1]) < tol && std::fabs(ex) < tol,
                      std::fabs(my - o.box[2]) < tol && std::fabs(ey) < tol,
                      std::fabs(my - o.box[3]) < tol && std::fabs(ey) < tol};
  for (int s = 0; s < 4; ++s)
    if (on[s] && ((o.walls >> s) & 1)) return HWE_BND_WALL;
  return HWE_BND_TRANSMISSIVE;
}

hwe_status build_host_mesh(const double* nodes, int64_t n_nodes, const int32_t* tris, int64_t n_tris,
                           const hwe_opts& o, HostMesh& h) {
  const double w2 = o.deriv_weight * o.deriv_weight;
  const bool periodic = o.bc == HWE_BC_PERIODIC;
  const double Lx = o.box[1] - o.box[0], Ly = o.box[3] - o.box[2];
  if (n_tris <= 0 || n_nodes <= 0) return fail(HWE_EINVAL, "empty mesh");
  if (n_tris > (int64_t(1) << 29)) return fail(HWE_EINVAL, "too many triangles (max 2^29)");
  if (!(Lx > 0) || !(Ly > 0)) return fail(HWE_EINVAL, "box must have x1 > x0 and y1 > y0");
  const int64_t N = n_tris;
  h.N = N;
  h.m = o.eq == HWE_EULER ? 4 : 1;

  // ---- 1. cells in caller order: unwrap, orient counter-clockwise, validate
  std::vector<Tri> T(N);
  std::vector<int32_t> tv(3 * N);
  for (int64_t k = 0; k < N; ++k) {
    int32_t v[3] = {tris[3 * k], tris[3 * k + 1], tris[3 * k + 2]};
    for (int j = 0; j < 3; ++j)
      if (v[j] < 0 || v[j] >= n_nodes) return fail(HWE_EMESH, "triangle references a missing node");
    Tri t;
    for (int j = 0; j < 3; ++j) {
      t.x[j] = nodes[2 * v[j]];
      t.y[j] = nodes[2 * v[j] + 1];
    }
    if (periodic)
      for (int j = 1; j < 3; ++j) {
        double dx = t.x[j] - t.x[0], dy = t.y[j] - t.y[0];
        t.x[j] = t.x[0] + dx - Lx * std::nearbyint(dx / Lx);
        t.y[j] = t.y[0] + dy - Ly * std::nearbyint(dy / Ly);
      }
    if (signed_area(t) < 0) {
      std::swap(t.x[1], t.x[2]);
      std::swap(t.y[1], t.y[2]);
      std::swap(v[1], v[2]);
    }
    double lmax = 0;
    for (int j = 0; j < 3; ++j) {
      int j1 = (j + 1) % 3;
      lmax = std::max(lmax, std::hypot(t.x[j1] - t.x[j], t.y[j1] - t.y[j]));
    }
    if (!(signed_area(t) > 1e-14 * lmax * lmax)) {
      std::ostringstream s;
      s << "degenerate triangle " << k;
      return fail(HWE_EMESH, s.str());
    }
    T[k] = t;
    for (int j = 0; j < 3; ++j) tv[3 * k + j] = v[j];
  }

  // ---- 2. faces -> edges by sorting the vertex-pair keys
  std::vector<std::pair<uint64_t, int64_t>> keys(3 * N);
  for (int64_t k = 0; k < N; ++k)
    for (int f = 0; f < 3; ++f) {
      uint32_t a = tv[3 * k + f], b = tv[3 * k + (f + 1) % 3];
      uint64_t key = (uint64_t(std::min(a, b)) << 32) | std::max(a, b);
      keys[3 * k + f] = {key, 3 * k + f};
    }
  std::sort(keys.begin(), keys.end());
  std::vector<int64_t> mate(3 * N, -1);  // face slot 3k+f -> partner face slot
  int64_t nb_faces = 0, n_edges = 0;
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j].first == keys[i].first) ++j;
    if (j - i > 2) return fail(HWE_EMESH, "non-manifold edge (shared by more than two triangles)");
    if (j - i == 2) {
      mate[keys[i].second] = keys[i + 1].second;
      mate[keys[i + 1].second] = keys[i].second;
    } else {
      if (periodic) return fail(HWE_EMESH, "boundary edge in a periodic mesh");
      ++nb_faces;
    }
    ++n_edges;
    i = j;
  }
  h.E = n_edges;
  h.NB = nb_faces;

  // translation from the neighbour's frame into this cell's frame, per face slot
  std::vector<double> shift(6 * N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    for (int f = 0; f < 3; ++f) {
      int64_t s = mate[3 * k + f];
      if (s < 0) continue;
      int64_t kn = s / 3;
      int g = int(s % 3), g1 = (g + 1) % 3, f1 = (f + 1) % 3;
      if (tv[3 * kn + g] != tv[3 * k + f1] || tv[3 * kn + g1] != tv[3 * k + f])
        return fail(HWE_EMESH, "inconsistent orientation across an edge");
      double sxa = T[k].x[f] - T[kn].x[g1], sya = T[k].y[f] - T[kn].y[g1];
      double sxb = T[k].x[f1] - T[kn].x[g], syb = T[k].y[f1] - T[kn].y[g];
      double tol = 1e-9 * (Lx + Ly);
      if (std::fabs(sxa - sxb) > tol || std::fabs(sya - syb) > tol)
        return fail(HWE_EMESH, "periodic seam mismatch");
      if (!periodic && (std::fabs(sxa) > tol || std::fabs(sya) > tol))
        return fail(HWE_EMESH, "non-periodic mesh with translated neighbours");
      shift[6 * k + 2 * f] = sxa;
      shift[6 * k + 2 * f + 1] = sya;
    }

  std::vector<CellGeo> G(N);
  for (int64_t k = 0; k < N; ++k) G[k] = cell_geo(T[k]);

  // ---- 3. Morton order of the centroids (wrapped into the box)
  std::vector<uint64_t> code(N);
  for (int64_t k = 0; k < N; ++k) {
    double u = (G[k].cx - o.box[0]) / Lx, v = (G[k].cy - o.box[2]) / Ly;
    if (periodic) {
      u -= std::floor(u);
      v -= std::floor(v);
    }
    u = std::min(std::max(u, 0.0), 1.0 - 1e-12);
    v = std::min(std::max(v, 0.0), 1.0 - 1e-12);
    uint32_t iu = uint32_t(u * 65536.0), iv = uint32_t(v * 65536.0);
    code[k] = spread_bits(iu) | (spread_bits(iv) << 1);
  }
  h.perm.resize(N);
  std::iota(h.perm.begin(), h.perm.end(), 0);
  std::stable_sort(h.perm.begin(), h.perm.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
  std::vector<int64_t> inv(N);
  for (int64_t i = 0; i < N; ++i) inv[h.perm[i]] = i;

  // ---- 4. edges: first cell = lower caller index; ordered by first internal cell
  struct Ed {
    int64_t key;
    int64_t c0, c1;  // caller indices; c1 = -1 on the boundary
    int f0, f1;
  };
  std::vector<Ed> ed;
  ed.reserve(n_edges);
  for (int64_t k = 0; k < N; ++k)
    for (int f = 0; f < 3; ++f) {
      int64_t s = mate[3 * k + f];
      if (s >= 0 && s / 3 < k) continue;  // recorded from the lower caller index
      Ed e;
      e.c0 = k;
      e.f0 = f;
      e.c1 = s >= 0 ? s / 3 : -1;
      e.f1 = s >= 0 ? int(s % 3) : -1;
      int64_t i0 = inv[k], i1 = e.c1 >= 0 ? inv[e.c1] : i0;
      e.key = std::min(i0, i1);
      ed.push_back(e);
    }
  std::stable_sort(ed.begin(), ed.end(), [](const Ed& a, const Ed& b) { return a.key < b.key; });
  const int64_t E = n_edges;
  h.ecell.assign(2 * E, -1);
  h.egeo.assign(size_t(kEG) * E, 0.0);
  const bool rule3 = o.edge_rule == 3;
  if (rule3) h.egp3.assign(12 * size_t(E), 0.0);
  const double gs3[3] = {0.5 - std::sqrt(15.0) / 10.0, 0.5, 0.5 + std::sqrt(15.0) / 10.0};
  std::vector<int32_t> face_edge(3 * N, -1);  // caller face slot -> edge index << 1 | second
  const double gs[2] = {0.5 - std::sqrt(3.0) / 6.0, 0.5 + std::sqrt(3.0) / 6.0};
  for (int64_t e = 0; e < E; ++e) {
    const Ed& r = ed[e];
    const Tri& t = T[r.c0];
    int f = r.f0, f1 = (f + 1) % 3;
    double ex = t.x[f1] - t.x[f], ey = t.y[f1] - t.y[f];
    double len = std::hypot(ex, ey);
    h.ecell[e] = int32_t(inv[r.c0]);
    // boundary edges: -1 transmissive, -2 wall; prescribed edges get -3 - b
    // below, once the boundary faces are numbered
    h.ecell[E + e] = r.c1 >= 0 ? int32_t(inv[r.c1]) : (boundary_kind(o, t, f) == HWE_BND_WALL ? -2 : -1);
    h.egeo[0 * E + e] = ey / len;
    h.egeo[1 * E + e] = -ex / len;
    h.egeo[2 * E + e] = len;
    for (int g = 0; g < 2; ++g) {
      double px = t.x[f] + gs[g] * ex, py = t.y[f] + gs[g] * ey;
      h.egeo[(3 + 2 * g) * E + e] = px - G[r.c0].cx;
      h.egeo[(4 + 2 * g) * E + e] = py - G[r.c0].cy;
      if (r.c1 >= 0) {
        // same physical point in the second cell's frame
        double sx = shift[6 * r.c1 + 2 * r.f1], sy = shift[6 * r.c1 + 2 * r.f1 + 1];
        h.egeo[(7 + 2 * g) * E + e] = px + sx - G[r.c1].cx;
        h.egeo[(8 + 2 * g) * E + e] = py + sy - G[r.c1].cy;
      }
    }
    if (rule3)
      for (int g = 0; g < 3; ++g) {
        double px = t.x[f] + gs3[g] * ex, py = t.y[f] + gs3[g] * ey;
        h.egp3[(2 * g) * E + e] = px - G[r.c0].cx;
        h.egp3[(2 * g + 1) * E + e] = py - G[r.c0].cy;
        if (r.c1 >= 0) {
          double sx = shift[6 * r.c1 + 2 * r.f1], sy = shift[6 * r.c1 + 2 * r.f1 + 1];
          h.egp3[(6 + 2 * g) * E + e] = px + sx - G[r.c1].cx;
          h.egp3[(7 + 2 * g) * E + e] = py + sy - G[r.c1].cy;
        }
      }
    face_edge[3 * r.c0 + r.f0] = int32_t(e << 1);
    if (r.c1 >= 0) face_edge[3 * r.c1 + r.f1] = int32_t((e << 1) | 1);
  }

  // ---- 5. per-cell arrays in internal order
  h.cen.assign(2 * N, 0);
  h.area.assign(N, 0);
  h.mom.assign(3 * N, 0);
  h.nbr.assign(3 * N, 0);
  h.nbr_back.assign(3 * N, -1);
  h.bnd_n.assign(4 * std::max<int64_t>(h.NB, 1), 0);
  h.p1.assign(size_t(kP1) * N, 0);
  h.p1f.assign(size_t(kP1F) * N, 0);
  h.p2.assign(size_t(kP2) * N, 0);
  h.cell_edge.assign(3 * N, 0);
  h.nl.assign(6 * N, 0);
  h.inv_area.assign(N, 0);
  const int gpf = o.edge_rule == 3 ? 3 : 2;  // limiter points per face
  h.gpc.assign(size_t(6 * gpf) * N, 0);
  double rmin = 1e300;
  int64_t bcount = 0;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t k = h.perm[i];
    const Tri& t = T[k];
    const CellGeo& g0 = G[k];
    h.cen[i] = g0.cx;
    h.cen[N + i] = g0.cy;
    h.area[i] = g0.A;
    h.inv_area[i] = 1.0 / g0.A;
    h.mom[i] = g0.mxx;
    h.mom[N + i] = g0.mxy;
    h.mom[2 * N + i] = g0.myy;
    double per = 0;
    // stencil geometry in K0's frame, scaled by hs = sqrt(|K0|)
    const double hs = std::sqrt(g0.A);
    double d[3][2], dm[3][3], ar[3], draw[3][2];
    for (int f = 0; f < 3; ++f) {
      int f1 = (f + 1) % 3;
      double ex = t.x[f1] - t.x[f], ey = t.y[f1] - t.y[f];
      double len = std::hypot(ex, ey);
      per += len;
      double nx = ey / len, ny = -ex / len;
      h.nl[f * N + i] = nx * len;
      h.nl[(3 + f) * N + i] = ny * len;
      for (int g = 0; g < gpf; ++g) {
        const double sg = gpf == 3 ? gs3[g] : (g == 0 ? 0.5 - std::sqrt(3.0) / 6.0 : 0.5 + std::sqrt(3.0) / 6.0);
        h.gpc[(2 * (gpf * f + g)) * N + i] = t.x[f] + sg * ex - g0.cx;
        h.gpc[(2 * (gpf * f + g) + 1) * N + i] = t.y[f] + sg * ey - g0.cy;
      }
      h.cell_edge[f * N + i] = face_edge[3 * k + f];
      int64_t s = mate[3 * k + f];
      CellGeo gn;
      double cx, cy;
      if (s >= 0) {
        int64_t kn = s / 3;
        h.nbr[f * N + i] = int32_t(inv[kn]);
        h.nbr_back[f * N + i] = int32_t(s % 3);
        gn = G[kn];
        cx = gn.cx + shift[6 * k + 2 * f];
        cy = gn.cy + shift[6 * k + 2 * f + 1];
      } else {
        // ghost: K0 mirrored across the face line
        h.nbr[f * N + i] = int32_t(-(bcount + 1));
        const int kind = boundary_kind(o, t, f);
        h.bnd_n[bcount] = nx;
        h.bnd_n[h.NB + bcount] = ny;
        h.bnd_n[2 * h.NB + bcount] = double(kind);
        h.bnd_n[3 * h.NB + bcount] = t.x[f] + 0.5 * ex;
        if (kind >= HWE_BND_STATE_A) h.ecell[E + (face_edge[3 * k + f] >> 1)] = int32_t(-3 - bcount);
        if (kind != HWE_BND_TRANSMISSIVE) {
          h.special_bnd = true;
          if (h.sb_cells.empty() || h.sb_cells.back() != int32_t(i)) h.sb_cells.push_back(int32_t(i));
        }
        ++bcount;
        Tri gt;
        for (int v = 0; v < 3; ++v) {
          double rx = t.x[v] - t.x[f], ry = t.y[v] - t.y[f];
          double dn = rx * nx + ry * ny;
          gt.x[v] = t.x[v] - 2.0 * dn * nx;
          gt.y[v] = t.y[v] - 2.0 * dn * ny;
        }
        std::swap(gt.x[1], gt.x[2]);
        std::swap(gt.y[1], gt.y[2]);
        gn = cell_geo(gt);
        cx = gn.cx;
        cy = gn.cy;
      }
      draw[f][0] = cx - g0.cx;
      draw[f][1] = cy - g0.cy;
      d[f][0] = draw[f][0] / hs;
      d[f][1] = draw[f][1] / hs;
      dm[f][0] = (gn.mxx - g0.mxx) / g0.A;
      dm[f][1] = (gn.mxy - g0.mxy) / g0.A;
      dm[f][2] = (gn.myy - g0.myy) / g0.A;
      ar[f] = gn.A / g0.A;
      // Step 2 data (unscaled: the printed rows mix units, so no rescaling).
      // With the derivative rows weighted by w the normal equations are
      // (d d^T + w^2 I)(b, c) = d dW + w^2 (V, Y), solved as
      // (b, c) = (V, Y) + d (dW - d.(V, Y)) / (w^2 + d.d).
      double dd = draw[f][0] * draw[f][0] + draw[f][1] * draw[f][1];
      h.p2[(3 * f + 0) * N + i] = draw[f][0];
      h.p2[(3 * f + 1) * N + i] = draw[f][1];
      h.p2[(3 * f + 2) * N + i] = 1.0 / (w2 + dd);
    }
    rmin = std::min(rmin, 2.0 * g0.A / per);
    double Ms[5][11];
    double Zs[2][5], Qs[2][8];
    if (!step1_map(d, dm, ar, Ms, Zs, Qs)) {
      std::ostringstream s;
      s << "rank-deficient Step-1 least squares at triangle " << k;
      return fail(HWE_ESINGULAR, s.str());
    }
    // undo the scaling: c1,c2 = c'/hs, c3..c5 = c'/hs^2; the LS right-hand
    // sides were divided by |K0| and multiplied by hs
    for (int j = 0; j < 5; ++j) {
      double sj = j < 2 ? 1.0 / hs : 1.0 / (hs * hs);
      for (int c = 0; c < 11; ++c) {
        double v = Ms[j][c] * sj;
        if (c >= 3) v *= hs;
        h.p1[size_t(j * 11 + c) * N + i] = v;
      }
      for (int c = 0; c < 3; ++c) h.p1f[size_t(kP1Md + 3 * j + c) * N + i] = Ms[j][c] * sj;
      for (int k = 0; k < 2; ++k) h.p1f[size_t(kP1Z + 5 * k + j) * N + i] = Zs[k][j] * sj;
    }
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < 8; ++c) h.p1f[size_t(kP1Q + 8 * k + c) * N + i] = Qs[k][c] * hs;
  }
  h.rmin = rmin;
  return HWE_OK;
}

}  // namespace hwe
