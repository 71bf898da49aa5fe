// Oracle for the compact ADER-HWENO step on triangles.
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow FP64 CPU implementation
// of what one explicit time step of the scheme computes.  It is used by the
// tests, by the smoke check and by the CPU-baseline leg of the benchmark, and
// never by the product library (which shares no code with it).
//
// It follows the paper's Section 2 step by step, cell by cell:
//   * finite-volume update, eq. (flx), with the space-time flux quadrature of
//     eqs. (fx) and (flux) and the local Lax-Friedrichs flux of Sec. 2.1;
//   * Taylor extrapolation in time, eqs. (tay)/(tayext), with time derivatives
//     from the Lax-Wendroff formulas of Sec. 2.1 (f' and f'' taken with
//     hyper-dual numbers applied to the flux functions themselves);
//   * the HWENO reconstruction of Sec. 2.2, Steps 1-6: constrained least
//     squares solved through their KKT systems in the monomial basis, the
//     simplified smoothness indicators of eq. (smoo1), the nonlinear weights of
//     eq. (nonlinearweight) and the combination of eq. (recon);
//   * the derivative averages of Sec. 2.3 by Green-Gauss, eq. (derave2d2),
//     with the interface value of eq. (timeflux) at tau = dt (eq. (taylor2dtime)).
//
// Readings where the paper is silent (both sides of the parity test use them):
//   time rule: 3-point Gauss-Lobatto, nodes {0, 1/2, 1} dt, weights {1,4,1}/6
//   (a 2-point Gauss-Legendre rule is an option; the interface value is the
//   Taylor polynomial at dt either way);
//   edge rule: 2-point Gauss-Legendre (a 3-point rule is an option; the
//   limiter then checks the 9 points); alpha from the two cell averages;
//   systems: component-wise reconstruction of the conservative variables;
//   periodic boundaries by exact translation across seams; transmissive
//   boundaries by a mirrored ghost cell for the stencil and W_ext := W_int
//   at boundary Gauss points; reflective walls (Euler) likewise with the
//   momentum reflected in the ghost and in W_ext; prescribed (inflow) states
//   by a mirrored ghost cell holding that state with zero derivative averages
//   and W_ext := the state at every time node; a prescribed state that
//   switches across a moving line x = x_s(t) (a shock meeting the boundary)
//   takes the side of the face midpoint at the middle of the step,
//   t_n + dt/2, for the ghost and for W_ext alike; kappa/D := 0 when kappa == 0.
//   Non-smooth points for derivatives: d|x| = sign(x) dx with sign(0) = 0;
//   max(a, b) takes a (the edge's first cell, the one with the lower caller
//   index) on ties.
//
// Everything is templated on the scalar type: double for the forward map,
// Dual (value + one tangent) for exact Jacobian-vector products, Rev (a node
// on a local tape) for the reverse mode, i.e. vector-Jacobian products, and
// for counting the floating-point operations of a step by stage.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
inline double sgn0(double x) { return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0); }
inline double absval(double a) { return std::fabs(a); }
inline Dual absval(Dual a) { return Dual(std::fabs(a.v), sgn0(a.v) * a.d); }
inline double sqrtv(double a) { return std::sqrt(a); }
inline Dual sqrtv(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
template <class T> inline T maxfirst(T a, T b) { return val(a) >= val(b) ? a : b; }

// Reverse mode.  A Rev number is a value and the index of its node on the
// calling thread's tape (-1: a constant).  Every operation records its
// operands' nodes and the partial derivatives with respect to them; a reverse
// sweep over the tape then carries adjoints from outputs to leaves.  The
// tapes are local: one cell's update (eq. (flx) and the Green-Gauss averages)
// or one cell's reconstruction (Sec. 2.2) is recorded, reversed and cleared,
// and the adjoints of its inputs are added to the cells they belong to.
// Constants equal to zero are structural zeros: x * 0, 0 / x and x + 0 record
// nothing (exact, and so are their derivatives).
//
// The same tapes count the step's floating-point operations: each node
// records whether it is an arithmetic operation (+, -, *, / or a square root;
// a sign change or |x| is not) and the stage of the step it belongs to, and
// the operations from which an output of the step can be reached are counted.
enum { kStRecon = 0, kStLimiter, kStAlpha, kStEval, kStLW, kStFlux, kStUpdate, kNStages };
thread_local int g_stage = kStRecon;
inline void stage(int s) { g_stage = s; }

struct Tape {
  std::vector<int32_t> pa, pb;
  std::vector<double> da, db;
  std::vector<uint8_t> st;  // stage * 2 + (1 if an arithmetic operation)
  void clear() {
    pa.clear();
    pb.clear();
    da.clear();
    db.clear();
    st.clear();
  }
  size_t size() const { return pa.size(); }
  int32_t push(int32_t a, double ga, int32_t b, double gb, bool flop) {
    pa.push_back(a);
    da.push_back(ga);
    pb.push_back(b);
    db.push_back(gb);
    st.push_back(uint8_t(g_stage * 2 + (flop ? 1 : 0)));
    return int32_t(pa.size() - 1);
  }
  // adj: seeded adjoints of the nodes (size() entries); on return the
  // adjoint of every node, leaves included.
  void reverse(std::vector<double>& adj) const {
    for (size_t k = pa.size(); k-- > 0;) {
      const double g = adj[k];
      if (g == 0.0) continue;
      if (pa[k] >= 0) adj[pa[k]] += da[k] * g;
      if (pb[k] >= 0) adj[pb[k]] += db[k] * g;
    }
  }
  // live: the nodes marked on entry (the outputs); on return every node an
  // output depends on.  Adds the arithmetic operations among them to count.
  void count_live(std::vector<char>& live, uint64_t count[kNStages]) const {
    for (size_t k = pa.size(); k-- > 0;) {
      if (!live[k]) continue;
      if (pa[k] >= 0) live[pa[k]] = 1;
      if (pb[k] >= 0) live[pb[k]] = 1;
      if (st[k] & 1) ++count[st[k] >> 1];
    }
  }
};
thread_local Tape* g_tape = nullptr;

struct Rev {
  double v;
  int32_t i;
  Rev() : v(0), i(-1) {}
  Rev(double a) : v(a), i(-1) {}
  Rev(double a, int32_t k) : v(a), i(k) {}
};
inline bool szero(Rev a) { return a.i < 0 && a.v == 0.0; }
inline Rev rev_node(double v, int32_t a, double ga, int32_t b, double gb, bool flop = true) {
  if (a < 0 && b < 0) return Rev(v);
  return Rev(v, g_tape->push(a, ga, b, gb, flop));
}
inline Rev rev_leaf(double v) { return Rev(v, g_tape->push(-1, 0.0, -1, 0.0, false)); }
inline Rev operator-(Rev a) { return rev_node(-a.v, a.i, -1.0, -1, 0.0, false); }
inline Rev operator+(Rev a, Rev b) {
  if (szero(a)) return b;
  if (szero(b)) return a;
  return rev_node(a.v + b.v, a.i, 1.0, b.i, 1.0);
}
inline Rev operator-(Rev a, Rev b) {
  if (szero(b)) return a;
  if (szero(a)) return -b;
  return rev_node(a.v - b.v, a.i, 1.0, b.i, -1.0);
}
inline Rev operator*(Rev a, Rev b) {
  if (szero(a) || szero(b)) return Rev(0.0);
  return rev_node(a.v * b.v, a.i, b.v, b.i, a.v);
}
inline Rev operator/(Rev a, Rev b) {
  if (szero(a)) return Rev(0.0);
  const double q = a.v / b.v;
  return rev_node(q, a.i, 1.0 / b.v, b.i, -q / b.v);
}
inline Rev& operator+=(Rev& a, Rev b) { a = a + b; return a; }
inline Rev& operator-=(Rev& a, Rev b) { a = a - b; return a; }
inline Rev& operator*=(Rev& a, Rev b) { a = a * b; return a; }
inline double val(Rev a) { return a.v; }
inline Rev absval(Rev a) { return rev_node(std::fabs(a.v), a.i, sgn0(a.v), -1, 0.0, false); }
inline Rev sqrtv(Rev a) {
  const double r = std::sqrt(a.v);
  return rev_node(r, a.i, 0.5 / r, -1, 0.0);
}

// Hyper-dual number a + e1 b1 + e2 b2 + e1 e2 b12 over scalar T
// (e1^2 = e2^2 = 0).  f(w + e1 x + e2 y + e1e2 z) has e1 part f'x and e1e2
// part f''[x, y] + f'z.
template <class T> struct HD {
  T a, e1, e2, e12;
};
template <class T> HD<T> hd(T a) { return HD<T>{a, T(0.0), T(0.0), T(0.0)}; }
template <class T> HD<T> operator+(const HD<T>& x, const HD<T>& y) {
  return HD<T>{x.a + y.a, x.e1 + y.e1, x.e2 + y.e2, x.e12 + y.e12};
}
template <class T> HD<T> operator-(const HD<T>& x, const HD<T>& y) {
  return HD<T>{x.a - y.a, x.e1 - y.e1, x.e2 - y.e2, x.e12 - y.e12};
}
template <class T> HD<T> operator*(const HD<T>& x, const HD<T>& y) {
  return HD<T>{x.a * y.a, x.a * y.e1 + x.e1 * y.a, x.a * y.e2 + x.e2 * y.a,
               x.a * y.e12 + x.e1 * y.e2 + x.e2 * y.e1 + x.e12 * y.a};
}
template <class T> HD<T> operator*(double c, const HD<T>& y) {
  return HD<T>{T(c) * y.a, T(c) * y.e1, T(c) * y.e2, T(c) * y.e12};
}
template <class T> HD<T> recip(const HD<T>& x) {
  T r = T(1.0) / x.a;
  T r2 = r * r;
  return HD<T>{r, T(0.0) - x.e1 * r2, T(0.0) - x.e2 * r2,
               T(2.0) * x.e1 * x.e2 * r2 * r - x.e12 * r2};
}
template <class T> HD<T> operator/(const HD<T>& x, const HD<T>& y) { return x * recip(y); }

// ---------------------------------------------------------------- rules
// 2-point Gauss-Legendre on each edge.  In time (the rule of eq. (flux) on
// [0, dt], nodes as fractions of dt): 3-point Gauss-Lobatto {0, 1/2, 1} with
// weights {1, 4, 1}/6 (default), or 2-point Gauss-Legendre 1/2 -+ sqrt(3)/6
// with weights 1/2.
// Gauss-Legendre rules on an edge, as fractions s of the way along it with
// weights summing to one: 2 points (1/2 -+ sqrt(3)/6, weights 1/2) and 3 points
// (1/2 -+ sqrt(15)/10 with weights 5/18, and 1/2 with weight 8/18).
struct EdgeRule {
  int n;
  double s[3], w[3];
};
const EdgeRule kEdgeRules[2] = {
    {2, {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225, 0.0}, {0.5, 0.5, 0.0}},
    {3, {0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852}, {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0}}};
struct TimeRule {
  int n;
  double node[3], w[3];
};
const TimeRule kTimeRules[2] = {{3, {0.0, 0.5, 1.0}, {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0}},
                                {2, {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225, 0.0},
                                 {0.5, 0.5, 0.0}}};

// ---------------------------------------------------------------- options
struct Opts {
  int eq;           // 0 advection, 1 Burgers, 2 Euler
  int bc;           // 0 periodic, 1 transmissive
  double box[4];    // x0 x1 y0 y1
  double adv[2];    // advection velocity
  double gas_gamma; // ratio of specific heats
  double lin_w[4];  // linear weights gamma_1..gamma_4
  double eps;       // epsilon of the nonlinear weights
  int linear_only;  // 1: use the linear weights (omega = gamma), for exactness pins
  int positivity;   // 1: scaling limiter on the reconstruction (Euler)
  int time_rule;    // 0: 3-point Gauss-Lobatto, 1: 2-point Gauss-Legendre
  double deriv_weight;  // weight of the derivative rows in the Step-2 least squares (1: as printed)
  int walls;        // Euler, non-periodic: bit s set = boundary faces on box side s (x0, x1, y0, y1) are
                    // reflective walls; the others are transmissive
  // boundary regions (non-periodic): a boundary face whose midpoint lies in
  // region r's closed rectangle takes region r's kind (first match wins); the
  // faces no region holds follow `walls`.  Kinds: 0 transmissive, 1 wall,
  // 2 prescribed state A, 3 prescribed state B, 4 A where the face midpoint
  // has x < shock_x0 + shock_speed * t, else B.
  int nreg;
  int reg_kind[8];
  double reg_box[8][4];
  double bstate[2][4];  // states A and B (conservative variables)
  double shock_x0, shock_speed;
  int edge_rule;  // Gauss-Legendre points per edge: 2 (default) or 3
};

inline const EdgeRule& edge_rule_of(const Opts& o) { return kEdgeRules[o.edge_rule == 3 ? 1 : 0]; }

enum { kBndTrans = 0, kBndWall = 1, kBndStateA = 2, kBndStateB = 3, kBndMoving = 4 };

inline int ncomp(int eq) { return eq == 2 ? 4 : 1; }

// Physical flux F(W) = (f(W), g(W)) of the three equations, templated so the
// same code is evaluated on doubles, duals and hyper-duals.
template <class N>
void flux_fg(const Opts& o, const N* W, N* f, N* g) {
  if (o.eq == 0) {
    f[0] = o.adv[0] * W[0];
    g[0] = o.adv[1] * W[0];
  } else if (o.eq == 1) {
    f[0] = 0.5 * (W[0] * W[0]);
    g[0] = f[0];
  } else {
    const N& rho = W[0];
    const N& mx = W[1];
    const N& my = W[2];
    const N& E = W[3];
    N u = mx / rho;
    N v = my / rho;
    N p = (o.gas_gamma - 1.0) * (E - 0.5 * (mx * u + my * v));
    f[0] = mx;
    f[1] = mx * u + p;
    f[2] = mx * v;
    f[3] = u * (E + p);
    g[0] = my;
    g[1] = my * u;
    g[2] = my * v + p;
    g[3] = v * (E + p);
  }
}
// Largest eigenvalue magnitude of d(F.n)/dW at a state (Sec. 2.1).
template <class T>
T spectral_radius(const Opts& o, const T* W, double nx, double ny) {
  if (o.eq == 0) return T(std::fabs(o.adv[0] * nx + o.adv[1] * ny));
  if (o.eq == 1) return absval(W[0] * T(nx + ny));
  T u = W[1] / W[0], v = W[2] / W[0];
  T p = T(o.gas_gamma - 1.0) * (W[3] - T(0.5) * (W[1] * u + W[2] * v));
  T c = sqrtv(T(o.gas_gamma) * p / W[0]);
  return absval(u * T(nx) + v * T(ny)) + c;
}

// ---------------------------------------------------------------- mesh
struct Tri {
  double x[3], y[3];  // counter-clockwise, unwrapped
};
inline double tri_area(const Tri& t) {
  return 0.5 * ((t.x[1] - t.x[0]) * (t.y[2] - t.y[0]) - (t.y[1] - t.y[0]) * (t.x[2] - t.x[0]));
}

struct Face {
  int nb;         // neighbour cell, or -1 on a boundary
  int kind;       // boundary kind (kBnd*) when nb == -1
  double mx;      // x of the face midpoint
  int nb_face;    // neighbour's face index
  double sx, sy;  // translation mapping the neighbour's frame into this cell's frame
  double nx, ny;  // outward unit normal of this cell
  double len;
  Tri ghost;      // mirrored cell when nb == -1
};

// Reflection of the momentum components (Euler, components 1 and 2) across a
// line with unit normal n: m -> m - 2 (m.n) n, applied to the averages W and,
// row by row, to the derivative averages (V, Y) (the rows mix, the columns are
// reflected by the caller).
template <class T> void reflect_momentum(double nx, double ny, T* W, T* V, T* Y) {
  T mn = W[1] * T(nx) + W[2] * T(ny);
  W[1] = W[1] - T(2.0 * nx) * mn;
  W[2] = W[2] - T(2.0 * ny) * mn;
  T vn = V[1] * T(nx) + V[2] * T(ny);
  V[1] = V[1] - T(2.0 * nx) * vn;
  V[2] = V[2] - T(2.0 * ny) * vn;
  T yn = Y[1] * T(nx) + Y[2] * T(ny);
  Y[1] = Y[1] - T(2.0 * nx) * yn;
  Y[2] = Y[2] - T(2.0 * ny) * yn;
}
template <class T> void reflect_momentum(double nx, double ny, T* W) {
  T mn = W[1] * T(nx) + W[2] * T(ny);
  W[1] = W[1] - T(2.0 * nx) * mn;
  W[2] = W[2] - T(2.0 * ny) * mn;
}

struct Mesh {
  Opts o;
  double time = 0.0;   // t_n of the next step (moving boundary states)
  double t_bnd = 0.0;  // time at which the current step evaluates them (t_n + dt/2)
  int64_t N = 0, E = 0;
  int m = 1;
  std::vector<Tri> tri;
  std::vector<double> area, cx, cy;
  std::vector<std::array<Face, 3>> face;
};

// The prescribed state of a boundary face of kind A, B or moving.
template <class T>
void boundary_state(const Mesh& M, const Face& F, T* W) {
  int which = F.kind == kBndStateB ? 1 : 0;
  if (F.kind == kBndMoving) which = F.mx < M.o.shock_x0 + M.o.shock_speed * M.t_bnd ? 0 : 1;
  for (int q = 0; q < M.m; ++q) W[q] = T(M.o.bstate[which][q]);
}
inline bool prescribed(const Face& F) { return F.kind >= kBndStateA; }

// Cell average over a triangle of a polynomial given through a callback:
// the three edge midpoints with weights 1/3 integrate quadratics exactly.
template <class Fn>
double tri_avg_quadratic(const Tri& t, Fn fn) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    int k1 = (k + 1) % 3;
    s += fn(0.5 * (t.x[k] + t.x[k1]), 0.5 * (t.y[k] + t.y[k1]));
  }
  return s / 3.0;
}

// ---------------------------------------------------------------- dense solve
// Solve M x = b for several right-hand sides (partial pivoting elimination).
// M is n x n row-major double; rhs has nr columns of scalar type T.
template <class T>
bool solve_dense(int n, std::vector<double> M, std::vector<T>& rhs, int nr) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (M[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(M[c * n + k], M[piv * n + k]);
      for (int k = 0; k < nr; ++k) std::swap(rhs[c * nr + k], rhs[piv * nr + k]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = M[r * n + c] / M[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) M[r * n + k] -= f * M[c * n + k];
      for (int k = 0; k < nr; ++k) rhs[r * nr + k] -= T(f) * rhs[c * nr + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int k = 0; k < nr; ++k) {
      T s = rhs[c * nr + k];
      for (int j = c + 1; j < n; ++j) s -= T(M[c * n + j]) * rhs[j * nr + k];
      rhs[c * nr + k] = s / T(M[c * n + c]);
    }
  }
  return true;
}

// Equality-constrained least squares: minimise |A x - b|^2 subject to C x = d
// through the KKT system [A^T A, C^T; C, 0] [x; mu] = [A^T b; d].
// A: na x n, C: nc x n (row-major), b: na x nr, d: nc x nr.  Returns x: n x nr.
template <class T>
bool constrained_lsq(int n, int na, int nc, const double* A, const double* C,
                     const std::vector<T>& b, const std::vector<T>& d, int nr,
                     std::vector<T>& x) {
  int K = n + nc;
  std::vector<double> M(K * K, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int r = 0; r < na; ++r) s += A[r * n + i] * A[r * n + j];
      M[i * K + j] = s;
    }
  for (int r = 0; r < nc; ++r)
    for (int j = 0; j < n; ++j) {
      M[(n + r) * K + j] = C[r * n + j];
      M[j * K + (n + r)] = C[r * n + j];
    }
  std::vector<T> rhs(K * nr, T(0.0));
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < nr; ++k) {
      T s = T(0.0);
      for (int r = 0; r < na; ++r) s += T(A[r * n + i]) * b[r * nr + k];
      rhs[i * nr + k] = s;
    }
  for (int r = 0; r < nc; ++r)
    for (int k = 0; k < nr; ++k) rhs[(n + r) * nr + k] = d[r * nr + k];
  if (!solve_dense(K, M, rhs, nr)) return false;
  x.assign(n * nr, T(0.0));
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < nr; ++k) x[i * nr + k] = rhs[i * nr + k];
  return true;
}

// ---------------------------------------------------------------- recon
// Polynomials are kept in the monomial basis about the target cell's
// centroid: p(x, y) = a0 + a1 X + a2 Y + a3 X^2 + a4 X Y + a5 Y^2,
// X = x - x_K0, Y = y - y_K0 (the linear ones have a3 = a4 = a5 = 0).
template <class T>
struct Recon {
  T p[4][4][6];     // [candidate l=1..4][component][coefficient]
  T beta[4][4];     // [component][l]
  T omega[4][4];    // [component][l]
  T wbar[4];        // cell averages of K0
  T theta[4];       // scaling of the reconstruction about the average (1 = none)
  double cx, cy;    // expansion point (centroid of K0)
};

// Stencil cell l of K0 (l = 0 is K0 itself), in K0's frame, and its state.
template <class T>
struct StencilCell {
  Tri t;
  double area;
  T W[4], V[4], Y[4];
};

template <class T>
void stencil_of(const Mesh& M, const T* s, int64_t k, StencilCell<T> st[4]) {
  const int m = M.m;
  const int64_t N = M.N;
  st[0].t = M.tri[k];
  st[0].area = M.area[k];
  for (int c = 0; c < m; ++c) {
    st[0].W[c] = s[(0 * m + c) * N + k];
    st[0].V[c] = s[(1 * m + c) * N + k];
    st[0].Y[c] = s[(2 * m + c) * N + k];
  }
  for (int f = 0; f < 3; ++f) {
    const Face& F = M.face[k][f];
    StencilCell<T>& c = st[f + 1];
    if (F.nb >= 0) {
      c.t = M.tri[F.nb];
      for (int v = 0; v < 3; ++v) {
        c.t.x[v] += F.sx;
        c.t.y[v] += F.sy;
      }
      c.area = M.area[F.nb];
      for (int q = 0; q < m; ++q) {
        c.W[q] = s[(0 * m + q) * N + F.nb];
        c.V[q] = s[(1 * m + q) * N + F.nb];
        c.Y[q] = s[(2 * m + q) * N + F.nb];
      }
    } else {
      // boundary: K0 mirrored across the face, state mirrored too.  The ghost
      // field is W_g(x) = S W(Mx) with M the reflection across the face line
      // (so its gradient is S grad W M); S = I on a transmissive boundary, and
      // on a wall S reflects the momentum vector by M as well.
      // A prescribed state is a ghost holding that state, flat (zero
      // derivative averages).
      c.t = F.ghost;
      c.area = M.area[k];
      for (int q = 0; q < m; ++q) {
        T vn = st[0].V[q] * T(F.nx) + st[0].Y[q] * T(F.ny);
        c.W[q] = st[0].W[q];
        c.V[q] = st[0].V[q] - T(2.0 * F.nx) * vn;
        c.Y[q] = st[0].Y[q] - T(2.0 * F.ny) * vn;
      }
      if (F.kind == kBndWall) reflect_momentum(F.nx, F.ny, c.W, c.V, c.Y);
      if (prescribed(F)) {
        boundary_state(M, F, c.W);
        for (int q = 0; q < m; ++q) c.V[q] = c.Y[q] = T(0.0);
      }
    }
  }
}

template <class T>
bool reconstruct(const Mesh& M, const T* s, int64_t k, Recon<T>& R) {
  const Opts& o = M.o;
  const int m = M.m;
  stage(kStRecon);
  StencilCell<T> st[4];
  stencil_of(M, s, k, st);
  const double x0 = M.cx[k], y0 = M.cy[k];
  R.cx = x0;
  R.cy = y0;
  for (int q = 0; q < m; ++q) {
    R.wbar[q] = st[0].W[q];
    R.theta[q] = T(1.0);
  }
  const double A0 = M.area[k];
  // scaled monomials xi = X / h, eta = Y / h keep the KKT matrices O(1)
  const double h = std::sqrt(A0);
  auto mono_avg = [&](const Tri& t, int j) {
    return tri_avg_quadratic(t, [&](double x, double y) {
      double a = (x - x0) / h, b = (y - y0) / h;
      switch (j) {
        case 0: return 1.0;
        case 1: return a;
        case 2: return b;
        case 3: return a * a;
        case 4: return a * b;
        default: return b * b;
      }
    });
  };

  // Step 1: quadratic p1 on T1 = {K0..K3}; the four cell averages exactly,
  // the six union derivative integrals in the least-squares sense.
  {
    double C[4 * 6], A[6 * 6];
    for (int l = 0; l < 4; ++l)
      for (int j = 0; j < 6; ++j) C[l * 6 + j] = mono_avg(st[l].t, j);
    // d/dx of (a0 + a1 xi + a2 eta + a3 xi^2 + a4 xi eta + a5 eta^2) = (a1 + 2 a3 xi + a4 eta)/h;
    // integral over K = |K| * average.  Every row is multiplied by h/|K0|,
    // which leaves the least-squares solution unchanged.
    for (int l = 1; l <= 3; ++l) {
      double* rx = &A[(l - 1) * 6];
      double* ry = &A[(l + 2) * 6];
      for (int j = 0; j < 6; ++j) rx[j] = ry[j] = 0.0;
      for (int u = 0; u < 2; ++u) {
        const StencilCell<T>& c = u == 0 ? st[0] : st[l];
        double w = c.area / A0;
        double mxi = mono_avg(c.t, 1), meta = mono_avg(c.t, 2);
        rx[1] += w;
        rx[3] += w * 2.0 * mxi;
        rx[4] += w * meta;
        ry[2] += w;
        ry[4] += w * mxi;
        ry[5] += w * 2.0 * meta;
      }
    }
    std::vector<T> b(6 * m), d(4 * m), x;
    for (int q = 0; q < m; ++q) {
      for (int l = 0; l < 4; ++l) d[l * m + q] = st[l].W[q];
      for (int l = 1; l <= 3; ++l) {
        b[(l - 1) * m + q] = (T(st[l].area) * st[l].V[q] + T(A0) * st[0].V[q]) * T(h / A0);
        b[(l + 2) * m + q] = (T(st[l].area) * st[l].Y[q] + T(A0) * st[0].Y[q]) * T(h / A0);
      }
    }
    if (!constrained_lsq<T>(6, 6, 4, A, C, b, d, m, x)) return false;
    for (int q = 0; q < m; ++q) {
      R.p[0][q][0] = x[0 * m + q];
      R.p[0][q][1] = x[1 * m + q] / T(h);
      R.p[0][q][2] = x[2 * m + q] / T(h);
      R.p[0][q][3] = x[3 * m + q] / T(h * h);
      R.p[0][q][4] = x[4 * m + q] / T(h * h);
      R.p[0][q][5] = x[5 * m + q] / T(h * h);
    }
  }
  // Step 2: linear p2, p3, p4 on {K0, K_l}: the K0 average exactly, the K_l
  // average and K_l derivative averages in the least-squares sense, with the
  // rows as written (each divided by the common factor |K_l|); the two
  // derivative rows are multiplied by o.deriv_weight (1 by default).
  const double wd = o.deriv_weight;
  for (int l = 1; l <= 3; ++l) {
    auto avg_x = [&](const Tri& t) { return tri_avg_quadratic(t, [&](double x, double) { return x - x0; }); };
    auto avg_y = [&](const Tri& t) { return tri_avg_quadratic(t, [&](double, double y) { return y - y0; }); };
    double C[3] = {1.0, avg_x(st[0].t), avg_y(st[0].t)};
    double A[9] = {1.0, avg_x(st[l].t), avg_y(st[l].t), 0.0, wd, 0.0, 0.0, 0.0, wd};
    std::vector<T> b(3 * m), d(m), x;
    for (int q = 0; q < m; ++q) {
      d[q] = st[0].W[q];
      b[0 * m + q] = st[l].W[q];
      b[1 * m + q] = T(wd) * st[l].V[q];
      b[2 * m + q] = T(wd) * st[l].Y[q];
    }
    if (!constrained_lsq<T>(3, 3, 1, A, C, b, d, m, x)) return false;
    for (int q = 0; q < m; ++q) {
      R.p[l][q][0] = x[0 * m + q];
      R.p[l][q][1] = x[1 * m + q];
      R.p[l][q][2] = x[2 * m + q];
      R.p[l][q][3] = R.p[l][q][4] = R.p[l][q][5] = T(0.0);
    }
  }
  // Step 4: smoothness indicators at the barycentre of K0 (X = Y = 0), eq. (smoo1).
  for (int q = 0; q < m; ++q) {
    for (int l = 0; l < 4; ++l) {
      const T* a = R.p[l][q];
      T dx = a[1], dy = a[2];
      T b = T(A0) * (dx * dx + dy * dy);
      if (l == 0) {
        T dxx = T(2.0) * a[3], dxy = a[4], dyy = T(2.0) * a[5];
        b += T(A0 * A0) * (dxx * dxx + dxy * dxy + dyy * dyy);
      }
      R.beta[q][l] = b;
    }
    // Step 5: nonlinear weights, eq. (nonlinearweight).
    T wave = (st[0].W[q] + st[1].W[q] + st[2].W[q] + st[3].W[q]) / T(4.0) + T(1e-30);
    T* beta = R.beta[q];
    T tsum = absval(beta[0] - beta[1]) + absval(beta[0] - beta[2]) + absval(beta[0] - beta[3]);
    T kappa = tsum * tsum / T(9.0);
    T wb[4];
    T ssum = T(0.0);
    for (int l = 0; l < 4; ++l) {
      if (o.linear_only) {
        wb[l] = T(o.lin_w[l]);
      } else {
        T w2 = wave * wave;
        T D = w2 * w2 * T(o.eps) + w2 * beta[l];
        T frac = val(kappa) == 0.0 ? T(0.0) : kappa / D;
        wb[l] = T(o.lin_w[l]) * (T(1.0) + frac);
      }
      ssum += wb[l];
    }
    for (int l = 0; l < 4; ++l) R.omega[q][l] = wb[l] / ssum;
  }
  if (o.positivity && o.eq == 2) {
    stage(kStLimiter);
    positivity_scaling(M, k, R);
  }
  return true;
}

// Step 6, eq. (recon): value and derivatives of the final reconstruction at
// (x, y) in K0's frame.  D[0..5] = W, W_x, W_y, W_xx, W_xy, W_yy.
template <class T>
void eval_recon(const Opts& o, const Recon<T>& R, int q, double x, double y, T D[6]) {
  const double X = x - R.cx, Y = y - R.cy;
  T pv[4][6];
  for (int l = 0; l < 4; ++l) {
    const T* a = R.p[l][q];
    pv[l][0] = a[0] + a[1] * T(X) + a[2] * T(Y) + a[3] * T(X * X) + a[4] * T(X * Y) + a[5] * T(Y * Y);
    pv[l][1] = a[1] + T(2.0 * X) * a[3] + T(Y) * a[4];
    pv[l][2] = a[2] + T(X) * a[4] + T(2.0 * Y) * a[5];
    pv[l][3] = T(2.0) * a[3];
    pv[l][4] = a[4];
    pv[l][5] = T(2.0) * a[5];
  }
  const T* w = R.omega[q];
  const double g1 = o.lin_w[0];
  for (int j = 0; j < 6; ++j) {
    T inner = pv[0][j] / T(g1);
    for (int l = 1; l < 4; ++l) inner -= T(o.lin_w[l] / g1) * pv[l][j];
    T r = w[0] * inner;
    for (int l = 1; l < 4; ++l) r += w[l] * pv[l][j];
    D[j] = r;
  }
  // scaling limiter: R -> Wbar + theta (R - Wbar)
  D[0] = R.wbar[q] + R.theta[q] * (D[0] - R.wbar[q]);
  for (int j = 1; j < 6; ++j) D[j] = R.theta[q] * D[j];
}

// Positivity-preserving scaling of the reconstruction (the scale limiter of
// Zhang and Shu cited in Sec. 3): with eps = min(1e-13, rho_bar, p_bar),
// first the density part is scaled about its average so that density >= eps at
// the six edge Gauss points of the cell, then the whole state is scaled by the
// smallest t in [0, 1] with p(Wbar + t (W - Wbar)) = eps over the points where
// the pressure would fall below eps.
template <class T>
void positivity_scaling(const Mesh& M, int64_t k, Recon<T>& R) {
  const Opts& o = M.o;
  const Tri& t = M.tri[k];
  const double gm1 = o.gas_gamma - 1.0;
  const EdgeRule& er = edge_rule_of(o);
  const int np = 3 * er.n;
  double xs[9], ys[9];
  for (int f = 0; f < 3; ++f) {
    int f1 = (f + 1) % 3;
    for (int G = 0; G < er.n; ++G) {
      xs[er.n * f + G] = t.x[f] + er.s[G] * (t.x[f1] - t.x[f]);
      ys[er.n * f + G] = t.y[f] + er.s[G] * (t.y[f1] - t.y[f]);
    }
  }
  auto pressure = [&](const T* W) { return T(gm1) * (W[3] - T(0.5) * (W[1] * W[1] + W[2] * W[2]) / W[0]); };
  const T* Wb = R.wbar;
  const double pbar = val(pressure(Wb));
  const double eps = std::min(1e-13, std::min(val(Wb[0]), pbar));
  // density
  T rmin = T(1e300);
  for (int i = 0; i < np; ++i) {
    T D[6];
    eval_recon(o, R, 0, xs[i], ys[i], D);
    if (val(D[0]) < val(rmin)) rmin = D[0];
  }
  if (val(rmin) < eps) R.theta[0] = (Wb[0] - T(eps)) / (Wb[0] - rmin);
  // pressure
  T th = T(1.0);
  for (int i = 0; i < np; ++i) {
    T W[4];
    for (int q = 0; q < 4; ++q) {
      T D[6];
      eval_recon(o, R, q, xs[i], ys[i], D);
      W[q] = D[0];
    }
    if (!(val(pressure(W)) < eps)) continue;
    // g(t) = 2 rho(t) (E(t) - eps/(gamma-1)) - |m(t)|^2, g(0) > 0 > g(1)
    T dr = W[0] - Wb[0], d1 = W[1] - Wb[1], d2 = W[2] - Wb[2], dE = W[3] - Wb[3];
    T Ep = Wb[3] - T(eps / gm1);
    T a = T(2.0) * dr * dE - (d1 * d1 + d2 * d2);
    T b = T(2.0) * (Ep * dr + Wb[0] * dE) - T(2.0) * (Wb[1] * d1 + Wb[2] * d2);
    T c = T(2.0) * Wb[0] * Ep - (Wb[1] * Wb[1] + Wb[2] * Wb[2]);
    T root;
    if (val(a) == 0.0) {
      root = T(0.0) - c / b;
    } else {
      T disc = b * b - T(4.0) * a * c;
      if (val(disc) < 0.0) disc = T(0.0);
      T sq = sqrtv(disc);
      T qq = val(b) >= 0.0 ? T(-0.5) * (b + sq) : T(-0.5) * (b - sq);
      T r1 = qq / a, r2 = c / qq;
      double v1 = val(r1), v2 = val(r2);
      bool ok1 = v1 >= 0.0 && v1 <= 1.0, ok2 = v2 >= 0.0 && v2 <= 1.0;
      root = ok1 && ok2 ? (v1 <= v2 ? r1 : r2) : (ok1 ? r1 : r2);
    }
    if (val(root) < val(th)) th = root;
  }
  if (val(th) < 1.0)
    for (int q = 0; q < 4; ++q) R.theta[q] = R.theta[q] * th;
}

// ---------------------------------------------------------------- Lax-Wendroff
// Sec. 2.1: time derivatives from spatial ones.  D[j][q]: j = W, Wx, Wy, Wxx,
// Wxy, Wyy.  Out: Wt, Wtx, Wty, Wtt per component.
template <class T>
void lax_wendroff(const Opts& o, int m, const T D[6][4], T Wt[4], T Wtx[4], T Wty[4], T Wtt[4]) {
  HD<T> Wh[4]{}, f[4]{}, g[4]{};
  auto eval = [&](int which, const T* a, const T* b, const T* c, T* out_e1, T* out_e12) {
    for (int q = 0; q < m; ++q) Wh[q] = HD<T>{D[0][q], a[q], b[q], c[q]};
    flux_fg(o, Wh, f, g);
    for (int q = 0; q < m; ++q) {
      const HD<T>& r = which == 0 ? f[q] : g[q];
      if (out_e1) out_e1[q] = r.e1;
      if (out_e12) out_e12[q] = r.e12;
    }
  };
  T zero[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  T fWx[4], gWy[4], a1[4], a2[4];
  // W_t = -f' W_x - g' W_y
  eval(0, D[1], zero, zero, fWx, nullptr);
  eval(1, D[2], zero, zero, gWy, nullptr);
  for (int q = 0; q < m; ++q) Wt[q] = T(0.0) - fWx[q] - gWy[q];
  // W_tx = -(f''[Wx,Wx] + f' Wxx) - (g''[Wx,Wy] + g' Wxy)
  eval(0, D[1], D[1], D[3], nullptr, a1);
  eval(1, D[1], D[2], D[4], nullptr, a2);
  for (int q = 0; q < m; ++q) Wtx[q] = T(0.0) - a1[q] - a2[q];
  // W_ty = -(f''[Wy,Wx] + f' Wxy) - (g''[Wy,Wy] + g' Wyy)
  eval(0, D[2], D[1], D[4], nullptr, a1);
  eval(1, D[2], D[2], D[5], nullptr, a2);
  for (int q = 0; q < m; ++q) Wty[q] = T(0.0) - a1[q] - a2[q];
  // W_tt = -(f''[Wt,Wx] + f' Wtx) - (g''[Wt,Wy] + g' Wty)
  eval(0, Wt, D[1], Wtx, nullptr, a1);
  eval(1, Wt, D[2], Wty, nullptr, a2);
  for (int q = 0; q < m; ++q) Wtt[q] = T(0.0) - a1[q] - a2[q];
}

// ---------------------------------------------------------------- the step

// One cell's new state from the reconstructions (eqs. (flx), (fx), (flux),
// (tay), (tayext), (derave2d2), (timeflux), (taylor2dtime)).
template <class T>
void update_cell(const Mesh& M, const T* s, const std::vector<Recon<T>>& R, int64_t k, double dt,
                 T Wn[4], T Vn[4], T Yn[4]) {
  const Opts& o = M.o;
  const int m = M.m;
  const int64_t N = M.N;
  T Fsum[4], Vs[4], Ys[4], Wbar[4];
  for (int q = 0; q < m; ++q) {
    Fsum[q] = Vs[q] = Ys[q] = T(0.0);
    Wbar[q] = s[q * N + k];
  }
  const Tri& t = M.tri[k];
  for (int f = 0; f < 3; ++f) {
    const Face& F = M.face[k][f];
    int f1 = (f + 1) % 3;
    T Wbn[4];
    if (F.nb >= 0)
      for (int q = 0; q < m; ++q) Wbn[q] = s[q * N + F.nb];
    // alpha: spectral radii at the two cell averages, the first argument
    // belonging to the cell with the lower index
    stage(kStAlpha);
    T alpha = T(0.0);
    if (F.nb >= 0) {
      T aK = spectral_radius(o, Wbar, F.nx, F.ny);
      T aN = spectral_radius(o, Wbn, F.nx, F.ny);
      alpha = k < F.nb ? maxfirst(aK, aN) : maxfirst(aN, aK);
    } else if (prescribed(F)) {
      T Wg[4];
      boundary_state(M, F, Wg);
      alpha = maxfirst(spectral_radius(o, Wbar, F.nx, F.ny), spectral_radius(o, Wg, F.nx, F.ny));
    } else if (F.kind == kBndWall) {
      // the ghost average is the reflected cell average: the same spectral radius
      T Wg[4];
      for (int q = 0; q < m; ++q) Wg[q] = Wbar[q];
      reflect_momentum(F.nx, F.ny, Wg);
      T aK = spectral_radius(o, Wbar, F.nx, F.ny);
      T aG = spectral_radius(o, Wg, F.nx, F.ny);
      alpha = maxfirst(aK, aG);
    }
    const EdgeRule& er = edge_rule_of(o);
    for (int G = 0; G < er.n; ++G) {
      double xg = t.x[f] + er.s[G] * (t.x[f1] - t.x[f]);
      double yg = t.y[f] + er.s[G] * (t.y[f1] - t.y[f]);
      T Di[6][4], De[6][4], tmp[6];
      stage(kStEval);
      for (int q = 0; q < m; ++q) {
        eval_recon(o, R[k], q, xg, yg, tmp);
        for (int j = 0; j < 6; ++j) Di[j][q] = tmp[j];
      }
      if (F.nb >= 0) {
        for (int q = 0; q < m; ++q) {
          eval_recon(o, R[F.nb], q, xg - F.sx, yg - F.sy, tmp);
          for (int j = 0; j < 6; ++j) De[j][q] = tmp[j];
        }
      }
      T it[4], itx[4], ity[4], itt[4], et[4], etx[4], ety[4], ett[4];
      stage(kStLW);
      lax_wendroff(o, m, Di, it, itx, ity, itt);
      if (F.nb >= 0) lax_wendroff(o, m, De, et, etx, ety, ett);
      stage(kStFlux);
      // Taylor polynomials in time, eq. (tay), of the interior and exterior values
      // (boundary: W_ext = W_int on a transmissive face, the reflected W_int on a wall)
      auto taylor = [&](double tau, T Wi[4], T We[4]) {
        for (int q = 0; q < m; ++q) {
          Wi[q] = Di[0][q] + T(tau) * it[q] + T(0.5 * tau * tau) * itt[q];
          We[q] = F.nb >= 0 ? De[0][q] + T(tau) * et[q] + T(0.5 * tau * tau) * ett[q] : Wi[q];
        }
        if (F.nb < 0 && F.kind == kBndWall) reflect_momentum(F.nx, F.ny, We);
        if (F.nb < 0 && prescribed(F)) boundary_state(M, F, We);
      };
      const TimeRule& rule = kTimeRules[o.time_rule == 1 ? 1 : 0];
      for (int sN = 0; sN < rule.n; ++sN) {
        T Wi[4], We[4], fi[4], gi[4], fe[4], ge[4];
        taylor(rule.node[sN] * dt, Wi, We);
        flux_fg(o, Wi, fi, gi);
        flux_fg(o, We, fe, ge);
        for (int q = 0; q < m; ++q) {
          T Hi = fi[q] * T(F.nx) + gi[q] * T(F.ny);
          T He = fe[q] * T(F.nx) + ge[q] * T(F.ny);
          T Hhat = T(0.5) * (He + Hi - alpha * (We[q] - Wi[q]));
          Fsum[q] += Hhat * T(rule.w[sN] * er.w[G] * F.len);
        }
      }
      {  // tau = dt: interface value of eq. (timeflux) for the derivative averages
        T Wi[4], We[4];
        taylor(dt, Wi, We);
        for (int q = 0; q < m; ++q) {
          T What = T(0.5) * (Wi[q] + We[q]);
          Vs[q] += What * T(F.nx * er.w[G] * F.len);
          Ys[q] += What * T(F.ny * er.w[G] * F.len);
        }
      }
    }
  }
  const double A = M.area[k];
  stage(kStUpdate);
  for (int q = 0; q < m; ++q) {
    Wn[q] = Wbar[q] - T(dt / A) * Fsum[q];
    Vn[q] = Vs[q] / T(A);
    Yn[q] = Ys[q] / T(A);
  }
}

int nthreads_or_default(int nt) {
#ifdef _OPENMP
  return nt > 0 ? nt : omp_get_max_threads();
#else
  (void)nt;
  return 1;
#endif
}

// Step restricted to a list of cells: reconstruct every cell whose
// reconstruction is needed (the listed cells and their face neighbours), then
// update the listed cells.  out is [3][m][nc].
template <class T>
int step_cells(const Mesh& M, const T* s, const int64_t* cells, int64_t nc, T* out, double dt, int nthr) {
  const int m = M.m;
  std::vector<char> need(M.N, 0);
  for (int64_t i = 0; i < nc; ++i) {
    int64_t k = cells[i];
    if (k < 0 || k >= M.N) return -1;
    need[k] = 1;
    for (int f = 0; f < 3; ++f)
      if (M.face[k][f].nb >= 0) need[M.face[k][f].nb] = 1;
  }
  std::vector<Recon<T>> R(M.N);
  int bad = 0;
  nthr = nthreads_or_default(nthr);
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthr) reduction(+ : bad)
  for (int64_t k = 0; k < M.N; ++k)
    if (need[k] && !reconstruct(M, s, k, R[k])) bad += 1;
  if (bad) return -3;
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthr)
  for (int64_t i = 0; i < nc; ++i) {
    T Wn[4], Vn[4], Yn[4];
    update_cell(M, s, R, cells[i], dt, Wn, Vn, Yn);
    for (int q = 0; q < m; ++q) {
      out[(0 * m + q) * nc + i] = Wn[q];
      out[(1 * m + q) * nc + i] = Vn[q];
      out[(2 * m + q) * nc + i] = Yn[q];
    }
  }
  return 0;
}

template <class T>
int step_all(const Mesh& M, const T* s, T* out, double dt, int nthr) {
  std::vector<int64_t> cells(M.N);
  for (int64_t k = 0; k < M.N; ++k) cells[k] = k;
  return step_cells(M, s, cells.data(), M.N, out, dt, nthr);
}

// ---------------------------------------------------------------- reverse mode
// The fields of a reconstruction that the update reads: the candidates'
// coefficients, the nonlinear weights, the limiter's scaling and the cell
// averages (Sec. 2.2, Steps 1-6).
template <class T, class Fn>
void recon_fields(Recon<T>& R, int m, Fn fn) {
  for (int l = 0; l < 4; ++l)
    for (int q = 0; q < m; ++q)
      for (int j = 0; j < 6; ++j) fn(R.p[l][q][j]);
  for (int q = 0; q < m; ++q)
    for (int l = 0; l < 4; ++l) fn(R.omega[q][l]);
  for (int q = 0; q < m; ++q) {
    fn(R.theta[q]);
    fn(R.wbar[q]);
  }
}

// The cell and its face neighbours, each once.
inline int stencil_cells(const Mesh& M, int64_t k, int64_t out[4]) {
  int n = 0;
  out[n++] = k;
  for (int f = 0; f < 3; ++f) {
    const int64_t c = M.face[k][f].nb;
    bool seen = c < 0;
    for (int j = 0; j < n && !seen; ++j) seen = out[j] == c;
    if (!seen) out[n++] = c;
  }
  return n;
}

// Vector-Jacobian product of one step at the state s (double [3][m][N]):
// lam_in = J^T lam_out.  Reverse of the updates first (each cell's update
// reads the averages of the cell and its face neighbours and their
// reconstructions), then of the reconstructions (each reads the state of the
// cell and its face neighbours).  The same non-smooth conventions as the
// dual numbers: d|x| = sign(x) dx with sign(0) = 0, max takes its first
// argument on ties, the limiter's branches are the forward's.
int vjp_step(const Mesh& M, const double* s, const double* lam_out, double* lam_in, double dt, int nthr) {
  const int m = M.m;
  const int64_t N = M.N;
  const size_t n3 = size_t(3 * m) * N;
  std::vector<Recon<double>> R(N);
  int bad = 0;
  nthr = nthreads_or_default(nthr);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthr) reduction(+ : bad)
  for (int64_t k = 0; k < N; ++k)
    if (!reconstruct(M, s, k, R[k])) bad += 1;
  if (bad) return -3;
  std::vector<Recon<double>> lamR(N);
  for (auto& r : lamR) recon_fields(r, m, [](double& x) { x = 0.0; });
  std::vector<double> lam_s(n3, 0.0);
  // reverse of the updates
#pragma omp parallel num_threads(nthr)
  {
    Tape tape;
    g_tape = &tape;
    std::vector<double> adj;
    std::vector<Rev> srev(n3);
    for (size_t i = 0; i < n3; ++i) srev[i] = Rev(s[i]);
    std::vector<Recon<Rev>> Rrev(N);
    std::vector<Recon<double>> lamR_t(N);
    for (auto& r : lamR_t) recon_fields(r, m, [](double& x) { x = 0.0; });
    std::vector<double> lam_t(n3, 0.0);
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < N; ++k) {
      tape.clear();
      int64_t cells[4];
      const int nc = stencil_cells(M, k, cells);
      for (int j = 0; j < nc; ++j) {
        const int64_t c = cells[j];
        for (int q = 0; q < m; ++q) srev[size_t(q) * N + c] = rev_leaf(s[size_t(q) * N + c]);
        Recon<Rev>& rr = Rrev[c];
        Recon<double>& rd = R[c];
        rr.cx = rd.cx;
        rr.cy = rd.cy;
        // copy the values, then make every field a leaf
        for (int l = 0; l < 4; ++l)
          for (int q = 0; q < m; ++q)
            for (int i = 0; i < 6; ++i) rr.p[l][q][i] = Rev(rd.p[l][q][i]);
        for (int q = 0; q < m; ++q) {
          for (int l = 0; l < 4; ++l) rr.omega[q][l] = Rev(rd.omega[q][l]);
          rr.theta[q] = Rev(rd.theta[q]);
          rr.wbar[q] = Rev(rd.wbar[q]);
        }
        recon_fields(rr, m, [](Rev& x) { x = rev_leaf(x.v); });
      }
      Rev Wn[4], Vn[4], Yn[4];
      update_cell(M, srev.data(), Rrev, k, dt, Wn, Vn, Yn);
      adj.assign(tape.size(), 0.0);
      for (int q = 0; q < m; ++q) {
        if (Wn[q].i >= 0) adj[Wn[q].i] += lam_out[size_t(q) * N + k];
        if (Vn[q].i >= 0) adj[Vn[q].i] += lam_out[size_t(m + q) * N + k];
        if (Yn[q].i >= 0) adj[Yn[q].i] += lam_out[size_t(2 * m + q) * N + k];
      }
      tape.reverse(adj);
      for (int j = 0; j < nc; ++j) {
        const int64_t c = cells[j];
        for (int q = 0; q < m; ++q) {
          Rev& x = srev[size_t(q) * N + c];
          lam_t[size_t(q) * N + c] += adj[x.i];
          x = Rev(x.v);
        }
        // the adjoints of cell c's reconstruction fields, in field order
        std::vector<double> g;
        recon_fields(Rrev[c], m, [&](Rev& x) { g.push_back(adj[x.i]); });
        size_t u = 0;
        recon_fields(lamR_t[c], m, [&](double& x) { x += g[u++]; });
      }
    }
#pragma omp critical
    {
      for (size_t i = 0; i < n3; ++i) lam_s[i] += lam_t[i];
      for (int64_t c = 0; c < N; ++c) {
        std::vector<double> g;
        recon_fields(lamR_t[c], m, [&](double& x) { g.push_back(x); });
        size_t u = 0;
        recon_fields(lamR[c], m, [&](double& x) { x += g[u++]; });
      }
    }
    g_tape = nullptr;
  }
  // reverse of the reconstructions
#pragma omp parallel num_threads(nthr)
  {
    Tape tape;
    g_tape = &tape;
    std::vector<double> adj;
    std::vector<Rev> srev(n3);
    for (size_t i = 0; i < n3; ++i) srev[i] = Rev(s[i]);
    std::vector<double> lam_t(n3, 0.0);
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < N; ++k) {
      tape.clear();
      int64_t cells[4];
      const int nc = stencil_cells(M, k, cells);
      for (int j = 0; j < nc; ++j)
        for (int b = 0; b < 3 * m; ++b) {
          const size_t ix = size_t(b) * N + cells[j];
          srev[ix] = rev_leaf(s[ix]);
        }
      Recon<Rev> Rk;
      reconstruct(M, srev.data(), k, Rk);
      adj.assign(tape.size(), 0.0);
      std::vector<double> g;
      recon_fields(lamR[k], m, [&](double& x) { g.push_back(x); });
      size_t u = 0;
      recon_fields(Rk, m, [&](Rev& x) {
        if (x.i >= 0) adj[x.i] += g[u];
        ++u;
      });
      tape.reverse(adj);
      for (int j = 0; j < nc; ++j)
        for (int b = 0; b < 3 * m; ++b) {
          const size_t ix = size_t(b) * N + cells[j];
          lam_t[ix] += adj[srev[ix].i];
          srev[ix] = Rev(s[ix]);
        }
    }
#pragma omp critical
    for (size_t i = 0; i < n3; ++i) lam_s[i] += lam_t[i];
    g_tape = nullptr;
  }
  std::memcpy(lam_in, lam_s.data(), n3 * sizeof(double));
  return 0;
}

// Operation counts of one step at the state s, per stage (kSt*), summed over
// the cells: the live arithmetic operations of every cell's reconstruction
// (those its reconstruction fields depend on) and of every cell's update (those
// its new state depends on; each cell evaluates the flux through its three
// faces, so every interior edge is evaluated twice, once from each side).
int count_step(const Mesh& M, const double* s, double dt, uint64_t out[kNStages]) {
  const int m = M.m;
  const int64_t N = M.N;
  const size_t n3 = size_t(3 * m) * N;
  for (int k = 0; k < kNStages; ++k) out[k] = 0;
  std::vector<Recon<double>> R(N);
  for (int64_t k = 0; k < N; ++k)
    if (!reconstruct(M, s, k, R[k])) return -3;
  Tape tape;
  g_tape = &tape;
  std::vector<Rev> srev(n3);
  std::vector<char> live;
  for (size_t i = 0; i < n3; ++i) srev[i] = Rev(s[i]);
  std::vector<Recon<Rev>> Rrev(N);
  for (int64_t k = 0; k < N; ++k) {
    // the reconstruction of cell k
    tape.clear();
    int64_t cells[4];
    const int nc = stencil_cells(M, k, cells);
    for (int j = 0; j < nc; ++j)
      for (int b = 0; b < 3 * m; ++b) {
        const size_t ix = size_t(b) * N + cells[j];
        srev[ix] = rev_leaf(s[ix]);
      }
    Recon<Rev> Rk;
    reconstruct(M, srev.data(), k, Rk);
    live.assign(tape.size(), 0);
    recon_fields(Rk, m, [&](Rev& x) {
      if (x.i >= 0) live[x.i] = 1;
    });
    tape.count_live(live, out);
    for (int j = 0; j < nc; ++j)
      for (int b = 0; b < 3 * m; ++b) {
        const size_t ix = size_t(b) * N + cells[j];
        srev[ix] = Rev(s[ix]);
      }
    // the update of cell k from the reconstructions of its stencil
    tape.clear();
    for (int j = 0; j < nc; ++j) {
      const int64_t c = cells[j];
      for (int q = 0; q < m; ++q) srev[size_t(q) * N + c] = rev_leaf(s[size_t(q) * N + c]);
      Recon<Rev>& rr = Rrev[c];
      const Recon<double>& rd = R[c];
      rr.cx = rd.cx;
      rr.cy = rd.cy;
      for (int l = 0; l < 4; ++l)
        for (int q = 0; q < m; ++q)
          for (int i = 0; i < 6; ++i) rr.p[l][q][i] = rd.p[l][q][i] == 0.0 && l > 0 && i > 2
                                                          ? Rev(0.0)
                                                          : rev_leaf(rd.p[l][q][i]);
      for (int q = 0; q < m; ++q) {
        for (int l = 0; l < 4; ++l) rr.omega[q][l] = rev_leaf(rd.omega[q][l]);
        rr.theta[q] = rev_leaf(rd.theta[q]);
        rr.wbar[q] = rev_leaf(rd.wbar[q]);
      }
    }
    Rev Wn[4], Vn[4], Yn[4];
    update_cell(M, srev.data(), Rrev, k, dt, Wn, Vn, Yn);
    live.assign(tape.size(), 0);
    for (int q = 0; q < m; ++q)
      for (const Rev& x : {Wn[q], Vn[q], Yn[q]})
        if (x.i >= 0) live[x.i] = 1;
    tape.count_live(live, out);
    for (int j = 0; j < nc; ++j)
      for (int q = 0; q < m; ++q) srev[size_t(q) * N + cells[j]] = Rev(s[size_t(q) * N + cells[j]]);
  }
  g_tape = nullptr;
  return 0;
}

// ---------------------------------------------------------------- mesh build
int build_mesh(Mesh& M, const double* nodes, int64_t nn, const int32_t* tris, int64_t nt) {
  const Opts& o = M.o;
  const bool periodic = o.bc == 0;
  const double Lx = o.box[1] - o.box[0], Ly = o.box[3] - o.box[2];
  M.N = nt;
  M.m = ncomp(o.eq);
  M.tri.resize(nt);
  M.area.resize(nt);
  M.cx.resize(nt);
  M.cy.resize(nt);
  M.face.resize(nt);
  std::vector<std::array<int32_t, 3>> tv(nt);
  for (int64_t k = 0; k < nt; ++k) {
    int32_t v[3] = {tris[3 * k], tris[3 * k + 1], tris[3 * k + 2]};
    for (int j = 0; j < 3; ++j)
      if (v[j] < 0 || v[j] >= nn) return -2;
    Tri t;
    for (int j = 0; j < 3; ++j) {
      t.x[j] = nodes[2 * v[j]];
      t.y[j] = nodes[2 * v[j] + 1];
      if (periodic && j > 0) {  // unwrap about the first vertex (minimal image)
        double dx = t.x[j] - t.x[0], dy = t.y[j] - t.y[0];
        t.x[j] = t.x[0] + dx - Lx * std::nearbyint(dx / Lx);
        t.y[j] = t.y[0] + dy - Ly * std::nearbyint(dy / Ly);
      }
    }
    if (tri_area(t) < 0) {  // counter-clockwise orientation
      std::swap(t.x[1], t.x[2]);
      std::swap(t.y[1], t.y[2]);
      std::swap(v[1], v[2]);
    }
    double a = tri_area(t);
    double lmax = 0.0;
    for (int j = 0; j < 3; ++j) {
      int j1 = (j + 1) % 3;
      lmax = std::max(lmax, std::hypot(t.x[j1] - t.x[j], t.y[j1] - t.y[j]));
    }
    if (!(a > 1e-14 * lmax * lmax)) return -2;
    M.tri[k] = t;
    M.area[k] = a;
    M.cx[k] = (t.x[0] + t.x[1] + t.x[2]) / 3.0;
    M.cy[k] = (t.y[0] + t.y[1] + t.y[2]) / 3.0;
    for (int j = 0; j < 3; ++j) tv[k][j] = v[j];
  }
  // faces: face f joins vertices f and f+1; match by sorted node pair
  std::map<std::pair<int32_t, int32_t>, std::vector<std::pair<int64_t, int>>> emap;
  for (int64_t k = 0; k < nt; ++k)
    for (int f = 0; f < 3; ++f) {
      int32_t a = tv[k][f], b = tv[k][(f + 1) % 3];
      emap[{std::min(a, b), std::max(a, b)}].push_back({k, f});
    }
  int64_t nedge = 0;
  for (auto& kv : emap) {
    auto& lst = kv.second;
    if (lst.size() > 2) return -2;
    if (lst.size() == 1 && periodic) return -2;
    ++nedge;
  }
  M.E = nedge;
  for (int64_t k = 0; k < nt; ++k) {
    const Tri& t = M.tri[k];
    for (int f = 0; f < 3; ++f) {
      int f1 = (f + 1) % 3;
      Face& F = M.face[k][f];
      double ex = t.x[f1] - t.x[f], ey = t.y[f1] - t.y[f];
      F.len = std::hypot(ex, ey);
      F.nx = ey / F.len;
      F.ny = -ex / F.len;
      int32_t a = tv[k][f], b = tv[k][f1];
      auto& lst = emap[{std::min(a, b), std::max(a, b)}];
      if (lst.size() == 1) {
        F.nb = -1;
        F.nb_face = -1;
        F.sx = F.sy = 0.0;
        // kind: the first region holding the face midpoint, else a wall
        // when the face lies on a box side whose bit is set in o.walls
        {
          const double mx = 0.5 * (t.x[f] + t.x[f1]), my = 0.5 * (t.y[f] + t.y[f1]);
          const double tol = 1e-9 * std::max(Lx, Ly);
          F.mx = mx;
          F.kind = -1;
          for (int r = 0; r < o.nreg && F.kind < 0; ++r)
            if (mx >= o.reg_box[r][0] - tol && mx <= o.reg_box[r][1] + tol && my >= o.reg_box[r][2] - tol &&
                my <= o.reg_box[r][3] + tol)
              F.kind = o.reg_kind[r];
          if (F.kind < 0) {
            const bool on[4] = {std::fabs(mx - o.box[0]) < tol && std::fabs(ex) < tol,
                                std::fabs(mx - o.box[1]) < tol && std::fabs(ex) < tol,
                                std::fabs(my - o.box[2]) < tol && std::fabs(ey) < tol,
                                std::fabs(my - o.box[3]) < tol && std::fabs(ey) < tol};
            F.kind = kBndTrans;
            for (int sd = 0; sd < 4; ++sd)
              if (on[sd] && ((o.walls >> sd) & 1)) F.kind = kBndWall;
          }
        }
        // mirror image of K across the face line
        for (int v = 0; v < 3; ++v) {
          double rx = t.x[v] - t.x[f], ry = t.y[v] - t.y[f];
          double dn = rx * F.nx + ry * F.ny;
          F.ghost.x[v] = t.x[v] - 2.0 * dn * F.nx;
          F.ghost.y[v] = t.y[v] - 2.0 * dn * F.ny;
        }
        // keep the ghost counter-clockwise
        std::swap(F.ghost.x[1], F.ghost.x[2]);
        std::swap(F.ghost.y[1], F.ghost.y[2]);
        continue;
      }
      auto other = lst[0].first == k && lst[0].second == f ? lst[1] : lst[0];
      F.kind = kBndTrans;
      F.mx = 0.5 * (t.x[f] + t.x[f1]);
      F.nb = static_cast<int>(other.first);
      F.nb_face = other.second;
      // translation from the neighbour's frame: compare the shared vertices
      const Tri& tn = M.tri[other.first];
      int g = other.second, g1 = (g + 1) % 3;
      // neighbour's face runs b -> a
      double sxa = t.x[f] - tn.x[g1], sya = t.y[f] - tn.y[g1];
      double sxb = t.x[f1] - tn.x[g], syb = t.y[f1] - tn.y[g];
      if (tv[other.first][g1] != a || tv[other.first][g] != b) return -2;
      double tol = 1e-9 * (std::fabs(Lx) + std::fabs(Ly) + F.len);
      if (std::fabs(sxa - sxb) > tol || std::fabs(sya - syb) > tol) return -2;
      F.sx = sxa;
      F.sy = sya;
      if (!periodic && (std::fabs(F.sx) > tol || std::fabs(F.sy) > tol)) return -2;
    }
  }
  return 0;
}

}  // namespace

// ====================================================================== C API
extern "C" {

struct or_opts {
  int eq;
  int bc;
  double box[4];
  double adv[2];
  double gas_gamma;
  double lin_w[4];
  double eps;
  int linear_only;
  int positivity;
  int time_rule;
  double deriv_weight;
  int walls;
  int nreg;
  int reg_kind[8];
  double reg_box[8][4];
  double bstate[2][4];
  double shock_x0, shock_speed;
  int edge_rule;
};

void* or_mesh_new(const double* nodes, int64_t nn, const int32_t* tris, int64_t nt, const or_opts* o,
                  int* status) {
  Mesh* M = new Mesh();
  M->o.eq = o->eq;
  M->o.bc = o->bc;
  for (int i = 0; i < 4; ++i) M->o.box[i] = o->box[i];
  M->o.adv[0] = o->adv[0];
  M->o.adv[1] = o->adv[1];
  M->o.gas_gamma = o->gas_gamma;
  for (int i = 0; i < 4; ++i) M->o.lin_w[i] = o->lin_w[i];
  M->o.eps = o->eps;
  M->o.linear_only = o->linear_only;
  M->o.positivity = o->positivity;
  M->o.time_rule = o->time_rule;
  M->o.deriv_weight = o->deriv_weight;
  M->o.walls = (o->eq == 2 && o->bc != 0) ? o->walls : 0;
  M->o.nreg = o->bc != 0 ? std::max(0, std::min(8, o->nreg)) : 0;
  for (int r = 0; r < 8; ++r) {
    M->o.reg_kind[r] = o->reg_kind[r];
    // walls exist for the Euler equations only
    if (o->eq != 2 && M->o.reg_kind[r] == kBndWall) M->o.reg_kind[r] = kBndTrans;
    for (int i = 0; i < 4; ++i) M->o.reg_box[r][i] = o->reg_box[r][i];
  }
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < 4; ++i) M->o.bstate[a][i] = o->bstate[a][i];
  M->o.edge_rule = o->edge_rule == 3 ? 3 : 2;
  M->o.shock_x0 = o->shock_x0;
  M->o.shock_speed = o->shock_speed;
  int st = build_mesh(*M, nodes, nn, tris, nt);
  if (status) *status = st;
  if (st != 0) {
    delete M;
    return nullptr;
  }
  return M;
}

void or_mesh_free(void* h) { delete static_cast<Mesh*>(h); }

int or_mesh_sizes(void* h, int64_t* N, int64_t* E, int32_t* m) {
  Mesh* M = static_cast<Mesh*>(h);
  *N = M->N;
  *E = M->E;
  *m = M->m;
  return 0;
}

// Per-cell geometry: area, centroid, and for each face the outward normal,
// length, neighbour index (-1 = boundary) and translation.  face_out is
// [N][3][6] = (nx, ny, len, nb, sx, sy).
int or_geometry(void* h, double* area, double* cx, double* cy, double* face_out) {
  Mesh* M = static_cast<Mesh*>(h);
  for (int64_t k = 0; k < M->N; ++k) {
    area[k] = M->area[k];
    cx[k] = M->cx[k];
    cy[k] = M->cy[k];
    for (int f = 0; f < 3; ++f) {
      const Face& F = M->face[k][f];
      double* o = face_out + (k * 3 + f) * 6;
      o[0] = F.nx;
      o[1] = F.ny;
      o[2] = F.len;
      o[3] = F.nb;
      o[4] = F.sx;
      o[5] = F.sy;
    }
  }
  return 0;
}

// Boundary kind of every face, [N][3] (kBnd*: 0 transmissive, 1 wall,
// 2 state A, 3 state B, 4 moving switch), -1 for interior faces.
int or_face_kinds(void* h, int32_t* out) {
  Mesh* M = static_cast<Mesh*>(h);
  for (int64_t k = 0; k < M->N; ++k)
    for (int f = 0; f < 3; ++f) out[k * 3 + f] = M->face[k][f].nb >= 0 ? -1 : M->face[k][f].kind;
  return 0;
}

// Triangle vertices in the cell's own (unwrapped, counter-clockwise) frame, [N][3][2].
int or_cell_vertices(void* h, double* out) {
  Mesh* M = static_cast<Mesh*>(h);
  for (int64_t k = 0; k < M->N; ++k)
    for (int v = 0; v < 3; ++v) {
      out[(k * 3 + v) * 2] = M->tri[k].x[v];
      out[(k * 3 + v) * 2 + 1] = M->tri[k].y[v];
    }
  return 0;
}

// Time t_n of the state given to the next or_step / or_step_cells (and the
// start time of or_run / or_jvp); only moving boundary states depend on it.
int or_set_time(void* h, double t) {
  Mesh* M = static_cast<Mesh*>(h);
  M->time = t;
  M->t_bnd = t;
  return 0;
}

// One step: s_in, s_out are [3][m][N] (averages of W, W_x, W_y).
int or_step(void* h, const double* s_in, double* s_out, double dt, int nthr) {
  Mesh* M = static_cast<Mesh*>(h);
  M->t_bnd = M->time + 0.5 * dt;
  return step_all(*M, s_in, s_out, dt, nthr);
}

int or_step_cells(void* h, const double* s_in, const int64_t* cells, int64_t nc, double* out, double dt,
                  int nthr) {
  Mesh* M = static_cast<Mesh*>(h);
  M->t_bnd = M->time + 0.5 * dt;
  return step_cells(*M, s_in, cells, nc, out, dt, nthr);
}

// nsteps steps in place with a fixed dt, from t_n = the mesh's time (which
// is left unchanged).
int or_run(void* h, double* s, double dt, int64_t nsteps, int nthr) {
  Mesh* M = static_cast<Mesh*>(h);
  std::vector<double> tmp(3 * M->m * M->N);
  for (int64_t n = 0; n < nsteps; ++n) {
    M->t_bnd = M->time + (double(n) + 0.5) * dt;
    int st = step_all(*M, s, tmp.data(), dt, nthr);
    if (st) return st;
    std::memcpy(s, tmp.data(), tmp.size() * sizeof(double));
  }
  return 0;
}

// Exact Jacobian-vector product of nsteps steps: (s, ds) -> (s_n, ds_n), in place.
int or_jvp(void* h, double* s, double* ds, double dt, int64_t nsteps, int nthr) {
  Mesh* M = static_cast<Mesh*>(h);
  size_t n = 3 * M->m * M->N;
  std::vector<Dual> a(n), b(n);
  for (size_t i = 0; i < n; ++i) a[i] = Dual(s[i], ds[i]);
  for (int64_t k = 0; k < nsteps; ++k) {
    M->t_bnd = M->time + (double(k) + 0.5) * dt;
    int st = step_all(*M, a.data(), b.data(), dt, nthr);
    if (st) return st;
    std::swap(a, b);
  }
  for (size_t i = 0; i < n; ++i) {
    s[i] = a[i].v;
    ds[i] = a[i].d;
  }
  return 0;
}

// Vector-Jacobian product of nsteps steps from the state s at the mesh's
// time: on entry lam is the adjoint of the final state, on return that of s
// (both [3][m][N]).  The forward states are kept; the steps are reversed in
// the opposite order.
int or_vjp(void* h, const double* s, double* lam, double dt, int64_t nsteps, int nthr) {
  Mesh* M = static_cast<Mesh*>(h);
  const size_t n = 3 * M->m * M->N;
  std::vector<std::vector<double>> states(nsteps);
  std::vector<double> cur(s, s + n), nxt(n);
  for (int64_t k = 0; k < nsteps; ++k) {
    states[k] = cur;
    M->t_bnd = M->time + (double(k) + 0.5) * dt;
    int st = step_all(*M, cur.data(), nxt.data(), dt, nthr);
    if (st) return st;
    std::swap(cur, nxt);
  }
  std::vector<double> lin(n);
  for (int64_t k = nsteps; k-- > 0;) {
    M->t_bnd = M->time + (double(k) + 0.5) * dt;
    int st = vjp_step(*M, states[k].data(), lam, lin.data(), dt, nthr);
    if (st) return st;
    std::memcpy(lam, lin.data(), n * sizeof(double));
  }
  return 0;
}

// Floating-point operations of one step at the state s, by stage (the live
// operations: those a result of the step depends on): out[0] reconstructions
// (Steps 1-5 with the oracle's per-step least-squares solves), out[1] the
// scaling limiter, out[2] the flux viscosities, out[3] the evaluation of the
// final reconstruction at the edge Gauss points (eq. (recon), candidate by
// candidate), out[4] the Lax-Wendroff procedure, out[5] the Taylor values,
// fluxes and quadratures of eqs. (fx), (flux), (timeflux), out[6] the update
// of eqs. (flx) and (derave2d2).  Stages 2-5 are counted from both sides of
// every edge (each cell evaluates its own faces).
int or_count_flops(void* h, const double* s, double dt, double* out) {
  Mesh* M = static_cast<Mesh*>(h);
  M->t_bnd = M->time + 0.5 * dt;
  uint64_t c[kNStages];
  int st = count_step(*M, s, dt, c);
  for (int k = 0; k < kNStages; ++k) out[k] = double(c[k]);
  return st;
}

// Reconstruction details of one cell: p[4][m][6] monomial coefficients about
// the centroid, beta[m][4], omega[m][4], centroid[2].
int or_recon_cell(void* h, const double* s, int64_t k, double* p, double* beta, double* omega,
                  double* centroid) {
  Mesh* M = static_cast<Mesh*>(h);
  Recon<double> R;
  if (!reconstruct(*M, s, k, R)) return -3;
  for (int l = 0; l < 4; ++l)
    for (int q = 0; q < M->m; ++q)
      for (int j = 0; j < 6; ++j) p[(l * M->m + q) * 6 + j] = R.p[l][q][j];
  for (int q = 0; q < M->m; ++q)
    for (int l = 0; l < 4; ++l) {
      beta[q * 4 + l] = R.beta[q][l];
      omega[q * 4 + l] = R.omega[q][l];
    }
  centroid[0] = R.cx;
  centroid[1] = R.cy;
  return 0;
}

// Scaling factors theta[m] of the limiter for cell k (1 where inactive).
int or_recon_theta(void* h, const double* s, int64_t k, double* theta) {
  Mesh* M = static_cast<Mesh*>(h);
  Recon<double> R;
  if (!reconstruct(*M, s, k, R)) return -3;
  for (int q = 0; q < M->m; ++q) theta[q] = R.theta[q];
  return 0;
}

// Final reconstruction (eq. (recon)) of cell k at points (x, y) given in the
// cell's own frame: out[np][m][6] = W, Wx, Wy, Wxx, Wxy, Wyy.
int or_eval_recon(void* h, const double* s, int64_t k, const double* xy, int64_t np, double* out) {
  Mesh* M = static_cast<Mesh*>(h);
  Recon<double> R;
  if (!reconstruct(*M, s, k, R)) return -3;
  for (int64_t i = 0; i < np; ++i)
    for (int q = 0; q < M->m; ++q) {
      double D[6];
      eval_recon(M->o, R, q, xy[2 * i], xy[2 * i + 1], D);
      for (int j = 0; j < 6; ++j) out[(i * M->m + q) * 6 + j] = D[j];
    }
  return 0;
}

// Lax-Wendroff time derivatives at np points.  D is [np][6][m]; out is [np][4][m]
// with rows W_t, W_tx, W_ty, W_tt.
int or_lax_wendroff(const or_opts* oo, const double* D, int64_t np, double* out) {
  Opts o{};
  o.eq = oo->eq;
  o.adv[0] = oo->adv[0];
  o.adv[1] = oo->adv[1];
  o.gas_gamma = oo->gas_gamma;
  int m = ncomp(o.eq);
  for (int64_t i = 0; i < np; ++i) {
    double Dl[6][4], a[4], b[4], c[4], d[4];
    for (int j = 0; j < 6; ++j)
      for (int q = 0; q < m; ++q) Dl[j][q] = D[(i * 6 + j) * m + q];
    lax_wendroff(o, m, Dl, a, b, c, d);
    for (int q = 0; q < m; ++q) {
      out[(i * 4 + 0) * m + q] = a[q];
      out[(i * 4 + 1) * m + q] = b[q];
      out[(i * 4 + 2) * m + q] = c[q];
      out[(i * 4 + 3) * m + q] = d[q];
    }
  }
  return 0;
}

// Local Lax-Friedrichs flux of Sec. 2.1 for one interface value pair:
// Hhat = 1/2 (H(We) + H(Wi) - alpha (We - Wi)), H = F.n, alpha given.
int or_llf(const or_opts* oo, const double* Wi, const double* We, double nx, double ny, double alpha,
           double* out) {
  Opts o{};
  o.eq = oo->eq;
  o.adv[0] = oo->adv[0];
  o.adv[1] = oo->adv[1];
  o.gas_gamma = oo->gas_gamma;
  int m = ncomp(o.eq);
  double fi[4], gi[4], fe[4], ge[4];
  flux_fg(o, Wi, fi, gi);
  flux_fg(o, We, fe, ge);
  for (int q = 0; q < m; ++q)
    out[q] = 0.5 * (fe[q] * nx + ge[q] * ny + fi[q] * nx + gi[q] * ny - alpha * (We[q] - Wi[q]));
  return 0;
}

// Time step of the time loop: cfl * min_K r_K / max_K lambda_K, with r_K the
// inradius and lambda_K the largest signal speed over all directions at the
// cell average.
double or_max_dt(void* h, const double* s, double cfl) {
  Mesh* M = static_cast<Mesh*>(h);
  const Opts& o = M->o;
  double rmin = 1e300, lmax = 0.0;
  for (int64_t k = 0; k < M->N; ++k) {
    double per = M->face[k][0].len + M->face[k][1].len + M->face[k][2].len;
    rmin = std::min(rmin, 2.0 * M->area[k] / per);
    double lam;
    if (o.eq == 0) {
      lam = std::hypot(o.adv[0], o.adv[1]);
    } else if (o.eq == 1) {
      lam = std::sqrt(2.0) * std::fabs(s[k]);
    } else {
      const int64_t N = M->N;
      double r = s[k], u = s[N + k] / r, v = s[2 * N + k] / r;
      double p = (o.gas_gamma - 1.0) * (s[3 * N + k] - 0.5 * r * (u * u + v * v));
      lam = std::sqrt(u * u + v * v) + std::sqrt(o.gas_gamma * p / r);
    }
    lmax = std::max(lmax, lam);
  }
  return cfl * rmin / lmax;
}

double or_spectral_radius(const or_opts* oo, const double* W, double nx, double ny) {
  Opts o{};
  o.eq = oo->eq;
  o.adv[0] = oo->adv[0];
  o.adv[1] = oo->adv[1];
  o.gas_gamma = oo->gas_gamma;
  return spectral_radius(o, W, nx, ny);
}

}  // extern "C"
