// Point-wise math of the step shared by the forward and adjoint kernels:
// flux functions, spectral radii and the Lax-Wendroff procedure.
//
// Lax-Wendroff (Sec. 2.1).  The time derivatives at a Gauss point follow from
// the conservation law W_t = -(f(W))_x - (g(W))_y applied to the quadratic
// reconstruction.  Instead of forming f' and f'' explicitly, the fluxes are
// evaluated on truncated Taylor polynomials ("jets") of the reconstruction about
// the point:
//  * a spatial jet holds the coefficients (c, x, y, xx, xy, yy) of
//    c + x X + y Y + xx X^2 + xy XY + yy Y^2; pushing it through f and g gives
//    W_t = -(f.x + g.y), W_tx = -(2 f.xx + g.xy), W_ty = -(f.xy + 2 g.yy),
//    which are the paper's first three Lax-Wendroff formulas;
//  * a time extension (t, xt, yt) with W.t = W_t, W.xt = W_tx, W.yt = W_ty gives
//    W_tt = -(f.xt + g.yt) = -(f''[W_t, W_x] + f' W_tx + g''[W_t, W_y] + g' W_ty).
#pragma once

#include <hip/hip_runtime.h>

namespace hwe {

enum { EQ_ADV = 0, EQ_BUR = 1, EQ_EUL = 2 };

// Workgroups of a launch are dispatched round-robin over the eight XCDs of an
// MI355X, each with its own L2.  Renumber them so that XCD x runs a contiguous
// range of logical blocks: cells and edges that are close in the Morton order
// (and share neighbours, tables and reconstructions) then meet in one L2.
__device__ __forceinline__ int xcd_block_id() {
  const int nb = int(gridDim.x), b = int(blockIdx.x);
  const int x = b & 7, k = b >> 3;
  const int base = nb >> 3, rem = nb & 7;
  return x * base + (x < rem ? x : rem) + k;
}

// Exchange within aligned groups of four lanes through DPP quad permutations
// (a VALU move, no LDS round trip).  CTRL is the quad_perm selector:
// kQuadXor1 swaps lanes 0<->1 and 2<->3, kQuadXor2 swaps 0<->2 and 1<->3.
constexpr int kQuadXor1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
constexpr int kQuadXor2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
template <int CTRL> __device__ __forceinline__ int quad_perm(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(quad_perm<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double quad_perm(double v) {
  const int lo = quad_perm<CTRL>(__double2loint(v)), hi = quad_perm<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// Whole-wave shift by one lane (DPP wave_shl:1, a VALU move): lane l receives
// lane l + 1's value; the last lane's result is undefined.
__device__ __forceinline__ int wave_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ float wave_next(float v) { return __int_as_float(wave_next(__float_as_int(v))); }
__device__ __forceinline__ double wave_next(double v) {
  const int lo = wave_next(__double2loint(v)), hi = wave_next(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// A 4x4 transpose across each aligned quad: lane q holds column q of the
// block in t[0..3] on entry and row q on exit (two DPP rounds: the
// off-diagonal 2x2 blocks swap, then the entries within them).
template <class T> __device__ __forceinline__ void quad_transpose4(T (&t)[4], int q) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const T got = quad_perm<kQuadXor2>((q & 2) ? t[j] : t[j + 2]);
    if (q & 2)
      t[j] = got;
    else
      t[j + 2] = got;
  }
#pragma unroll
  for (int j = 0; j < 4; j += 2) {
    const T got = quad_perm<kQuadXor1>((q & 1) ? t[j] : t[j + 1]);
    if (q & 1)
      t[j] = got;
    else
      t[j + 1] = got;
  }
}
// The value of lane c (0..3) of each aligned quad, in every lane of the quad.
template <class T> __device__ __forceinline__ T quad_bcast(T v, int c) {
  switch (c) {
    case 0: return quad_perm<0x00>(v);
    case 1: return quad_perm<0x55>(v);
    case 2: return quad_perm<0xAA>(v);
    default: return quad_perm<0xFF>(v);
  }
}

// Per-cell reconstruction tables, tiled: cells are grouped in tiles of kTile
// consecutive cells; a tile stores kTblRows rows of kTile values (row-major),
// so the tables of one tile are one contiguous block.  The table of cell i
// starts at (i / kTile) * kTblRows * kTile + i % kTile.
constexpr int kTile = 64;
// Rows: the Step-1 map in factored form, c = Md dW + Z^T (Q v) with v = (V0..V3,
// Y0..Y3) (kTblMd: Md, 5 x 3; kTblZ: Z, 2 x 5, the null-space basis of the
// three average constraints; kTblQ: Q, 2 x 8, the reduced least-squares
// solution) -- 41 numbers in place of the 55 of the 5 x 11 map -- then the
// Step-2 data (dx, dy, 1/(w^2 + d.d)) per face and the central second moments
// (Mxx, Mxy, Myy).
constexpr int kTblMd = 0, kTblZ = 15, kTblQ = 25, kTblP2 = 41, kTblMom = 50, kTblRows = 53;
__host__ __device__ __forceinline__ size_t tbl_col(int i) {
  return size_t(i / kTile) * (kTblRows * kTile) + size_t(i % kTile);
}

template <int EQ> struct NComp {
  static constexpr int m = EQ == EQ_EUL ? 4 : 1;
};

// 2-point Gauss-Legendre nodes on [0, 1]: 1/2 -+ sqrt(3)/6
constexpr double kGaussLegendre2[2] = {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225};

struct Params {
  double ax, ay;   // advection velocity
  double gam;      // ratio of specific heats
  double lw[4];    // linear weights gamma_1..4
  double eps;      // epsilon of the nonlinear weights
  int linear;      // 1: omega = gamma
  int positivity;  // 1: scaling limiter on the Euler reconstruction
  int time_rule;   // 0: 3-point Gauss-Lobatto in time, 1: 2-point Gauss-Legendre
  // prescribed boundary states: A (kind 2), B (kind 3), or A where the face
  // midpoint has x < sx0 + sv * tb, else B (kind 4); tb = the middle of the step
  double bst[2][4];
  double sx0, sv, tb;
};

// The prescribed state of a boundary face of kind 2, 3 or 4 (kind and midpoint
// x as stored per boundary face), component by component with compile-time
// indices so that the parameter block is never indexed at run time.
template <int M>
__host__ __device__ __forceinline__ void prescribed_state(const Params& P, double kind, double xm, double (&W)[M]) {
  const bool a = kind == 2.0 || (kind == 4.0 && xm < P.sx0 + P.sv * P.tb);
#pragma unroll
  for (int q = 0; q < M; ++q) W[q] = a ? P.bst[0][q] : P.bst[1][q];
}
__host__ __device__ __forceinline__ double prescribed_component(const Params& P, double kind, double xm, int q) {
  double W[4];
  prescribed_state<4>(P, kind, xm, W);
  return q == 0 ? W[0] : (q == 1 ? W[1] : (q == 2 ? W[2] : W[3]));
}

// Nothing is scheduled across this point: every load issued above it is in
// flight before the arithmetic below waits for any of them.  A kernel whose
// waves cannot hide each other's latency (one or two per SIMD) gathers its
// inputs this way in as few rounds as their index dependences allow, where the
// compiler would otherwise issue many loads next to their first use.
__host__ __device__ __forceinline__ void issue_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// The value of x is needed here (it is an operand of an empty asm statement):
// its load is issued above this point and waited for at it.  Used where the
// compiler would otherwise move a gather below a barrier, next to its use.
template <class T> __device__ __forceinline__ void arrived(const T& x) { asm volatile("" ::"v"(x)); }
__device__ __forceinline__ void arrived(const uint4& x) { asm volatile("" ::"v"(x.x), "v"(x.y), "v"(x.z), "v"(x.w)); }

// 1/x for the FP32 bulk of the mixed path: the hardware reciprocal (within an
// ulp of the quotient); FP64 keeps the correctly rounded division.
__host__ __device__ __forceinline__ float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <class T> struct SJ {  // spatial jet
  T c, x, y, xx, xy, yy;
};
template <class T> struct TJ {  // time extension of a spatial jet
  T t, xt, yt;
};

template <class T> __host__ __device__ __forceinline__ SJ<T> sj_mul(const SJ<T>& a, const SJ<T>& b) {
  SJ<T> r;
  r.c = a.c * b.c;
  r.x = a.c * b.x + a.x * b.c;
  r.y = a.c * b.y + a.y * b.c;
  r.xx = a.c * b.xx + a.x * b.x + a.xx * b.c;
  r.xy = a.c * b.xy + a.x * b.y + a.y * b.x + a.xy * b.c;
  r.yy = a.c * b.yy + a.y * b.y + a.yy * b.c;
  return r;
}
template <class T> __host__ __device__ __forceinline__ SJ<T> sj_recip(const SJ<T>& a) {
  SJ<T> r;
  T r1 = recip(a.c), r2 = r1 * r1, r3 = r2 * r1;
  r.c = r1;
  r.x = -a.x * r2;
  r.y = -a.y * r2;
  r.xx = a.x * a.x * r3 - a.xx * r2;
  r.xy = T(2) * a.x * a.y * r3 - a.xy * r2;
  r.yy = a.y * a.y * r3 - a.yy * r2;
  return r;
}
template <class T> __host__ __device__ __forceinline__ SJ<T> sj_add(const SJ<T>& a, const SJ<T>& b) {
  return SJ<T>{a.c + b.c, a.x + b.x, a.y + b.y, a.xx + b.xx, a.xy + b.xy, a.yy + b.yy};
}
template <class T> __host__ __device__ __forceinline__ SJ<T> sj_sub(const SJ<T>& a, const SJ<T>& b) {
  return SJ<T>{a.c - b.c, a.x - b.x, a.y - b.y, a.xx - b.xx, a.xy - b.xy, a.yy - b.yy};
}
template <class T> __host__ __device__ __forceinline__ SJ<T> sj_scale(T s, const SJ<T>& a) {
  return SJ<T>{s * a.c, s * a.x, s * a.y, s * a.xx, s * a.xy, s * a.yy};
}
// time extension of a product / reciprocal (a, b spatial parts, at, bt time parts)
template <class T>
__host__ __device__ __forceinline__ TJ<T> tj_mul(const SJ<T>& a, const TJ<T>& at, const SJ<T>& b, const TJ<T>& bt) {
  TJ<T> r;
  r.t = a.c * bt.t + at.t * b.c;
  r.xt = a.c * bt.xt + a.x * bt.t + at.t * b.x + at.xt * b.c;
  r.yt = a.c * bt.yt + a.y * bt.t + at.t * b.y + at.yt * b.c;
  return r;
}
template <class T>
__host__ __device__ __forceinline__ TJ<T> tj_recip(const SJ<T>& a, const TJ<T>& at, const SJ<T>& r) {
  T r2 = r.c * r.c, r3 = r2 * r.c;
  TJ<T> o;
  o.t = -at.t * r2;
  o.xt = T(2) * a.x * at.t * r3 - at.xt * r2;
  o.yt = T(2) * a.y * at.t * r3 - at.yt * r2;
  return o;
}
template <class T> __host__ __device__ __forceinline__ TJ<T> tj_add(const TJ<T>& a, const TJ<T>& b) {
  return TJ<T>{a.t + b.t, a.xt + b.xt, a.yt + b.yt};
}
template <class T> __host__ __device__ __forceinline__ TJ<T> tj_sub(const TJ<T>& a, const TJ<T>& b) {
  return TJ<T>{a.t - b.t, a.xt - b.xt, a.yt - b.yt};
}
template <class T> __host__ __device__ __forceinline__ TJ<T> tj_scale(T s, const TJ<T>& a) {
  return TJ<T>{s * a.t, s * a.xt, s * a.yt};
}

// Lax-Wendroff at one point.  D[j][q], j = W, Wx, Wy, Wxx, Wxy, Wyy.
// Outputs W_t and W_tt per component.
template <int EQ, class T>
__host__ __device__ __forceinline__ void lax_wendroff(const Params& P, const T (&D)[6][NComp<EQ>::m],
                                                     T (&Wt)[NComp<EQ>::m], T (&Wtt)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    const T ax = T(P.ax), ay = T(P.ay);
    T wt = -(ax * D[1][0] + ay * D[2][0]);
    T wtx = -(ax * D[3][0] + ay * D[4][0]);
    T wty = -(ax * D[4][0] + ay * D[5][0]);
    Wt[0] = wt;
    Wtt[0] = -(ax * wtx + ay * wty);
  } else if constexpr (EQ == EQ_BUR) {
    SJ<T> J{D[0][0], D[1][0], D[2][0], T(0.5) * D[3][0], D[4][0], T(0.5) * D[5][0]};
    SJ<T> s = sj_scale(T(0.5), sj_mul(J, J));
    TJ<T> Jt;
    Jt.t = -(s.x + s.y);
    Jt.xt = -(T(2) * s.xx + s.xy);
    Jt.yt = -(s.xy + T(2) * s.yy);
    TJ<T> st = tj_scale(T(0.5), tj_mul(J, Jt, J, Jt));
    Wt[0] = Jt.t;
    Wtt[0] = -(st.xt + st.yt);
  } else {
    const T gm1 = T(P.gam - 1.0);
    SJ<T> J[4];
    for (int q = 0; q < 4; ++q) J[q] = SJ<T>{D[0][q], D[1][q], D[2][q], T(0.5) * D[3][q], D[4][q], T(0.5) * D[5][q]};
    const SJ<T>& rho = J[0];
    const SJ<T>& mx = J[1];
    const SJ<T>& my = J[2];
    const SJ<T>& En = J[3];
    SJ<T> r = sj_recip(rho);
    SJ<T> u = sj_mul(mx, r), v = sj_mul(my, r);
    SJ<T> mxu = sj_mul(mx, u), myv = sj_mul(my, v), muv = sj_mul(mx, v);
    SJ<T> ke = sj_scale(T(0.5), sj_add(mxu, myv));
    SJ<T> p = sj_scale(gm1, sj_sub(En, ke));
    SJ<T> H = sj_add(En, p);
    SJ<T> uH = sj_mul(u, H), vH = sj_mul(v, H);
    SJ<T> f1 = sj_add(mxu, p), g2 = sj_add(myv, p);
    // f = (mx, f1, muv, uH), g = (my, muv, g2, vH)
    TJ<T> Jt[4];
    Jt[0] = TJ<T>{-(mx.x + my.y), -(T(2) * mx.xx + my.xy), -(mx.xy + T(2) * my.yy)};
    Jt[1] = TJ<T>{-(f1.x + muv.y), -(T(2) * f1.xx + muv.xy), -(f1.xy + T(2) * muv.yy)};
    Jt[2] = TJ<T>{-(muv.x + g2.y), -(T(2) * muv.xx + g2.xy), -(muv.xy + T(2) * g2.yy)};
    Jt[3] = TJ<T>{-(uH.x + vH.y), -(T(2) * uH.xx + vH.xy), -(uH.xy + T(2) * vH.yy)};
    TJ<T> rt = tj_recip(rho, Jt[0], r);
    TJ<T> ut = tj_mul(mx, Jt[1], r, rt), vt = tj_mul(my, Jt[2], r, rt);
    TJ<T> mxut = tj_mul(mx, Jt[1], u, ut), myvt = tj_mul(my, Jt[2], v, vt), muvt = tj_mul(mx, Jt[1], v, vt);
    TJ<T> ket = tj_scale(T(0.5), tj_add(mxut, myvt));
    TJ<T> pt = tj_scale(gm1, tj_sub(Jt[3], ket));
    TJ<T> Ht = tj_add(Jt[3], pt);
    TJ<T> uHt = tj_mul(u, ut, H, Ht), vHt = tj_mul(v, vt, H, Ht);
    for (int q = 0; q < 4; ++q) Wt[q] = Jt[q].t;
    Wtt[0] = -(Jt[1].xt + Jt[2].yt);
    Wtt[1] = -((mxut.xt + pt.xt) + muvt.yt);
    Wtt[2] = -(muvt.xt + (myvt.yt + pt.yt));
    Wtt[3] = -(uHt.xt + vHt.yt);
  }
}

// Normal flux H(W) = f(W) nx + g(W) ny.
template <int EQ, class T>
__host__ __device__ __forceinline__ void normal_flux(const Params& P, const T (&W)[NComp<EQ>::m], T nx, T ny,
                                                    T (&H)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    H[0] = (T(P.ax) * nx + T(P.ay) * ny) * W[0];
  } else if constexpr (EQ == EQ_BUR) {
    H[0] = T(0.5) * W[0] * W[0] * (nx + ny);
  } else {
    T r = T(1) / W[0];
    T u = W[1] * r, v = W[2] * r;
    T un = u * nx + v * ny;
    T p = T(P.gam - 1.0) * (W[3] - T(0.5) * (W[1] * u + W[2] * v));
    H[0] = W[0] * un;
    H[1] = W[1] * un + p * nx;
    H[2] = W[2] * un + p * ny;
    H[3] = (W[3] + p) * un;
  }
}

// Offset form of the normal flux: dH = H(Wb + d) - H(Wb), written so that it
// is formed from the offset d without cancellation (exactly 0 for d = 0).
// For Euler with u = mx/rho etc. at Wb and primes at Wb + d:
//   du = (dmx - u drho)/rho',  dke = (dmx u + mx' du + dmy v + my' dv)/2,
//   dp = (gamma-1)(dE - dke),  dun = du nx + dv ny,
//   dH = (drho un + rho' dun, dmx un + mx' dun + dp nx, dmy un + my' dun + dp ny,
//         (dE + dp) un + (E' + p') dun).
template <int EQ, class T> struct FluxBase {
  T w[NComp<EQ>::m];
  T u, v, p;
};
template <int EQ, class T>
__host__ __device__ __forceinline__ FluxBase<EQ, T> flux_base(const Params& P, const double (&W)[NComp<EQ>::m]) {
  FluxBase<EQ, T> b;
  for (int q = 0; q < NComp<EQ>::m; ++q) b.w[q] = T(W[q]);
  b.u = b.v = b.p = T(0);
  if constexpr (EQ == EQ_EUL) {
    const double r = 1.0 / W[0];
    const double u = W[1] * r, v = W[2] * r;
    b.u = T(u);
    b.v = T(v);
    b.p = T((P.gam - 1.0) * (W[3] - 0.5 * (W[1] * u + W[2] * v)));
  }
  return b;
}
template <int EQ, class T>
__host__ __device__ __forceinline__ void normal_flux_delta(const Params& P, const FluxBase<EQ, T>& b,
                                                          const T (&d)[NComp<EQ>::m], T nx, T ny,
                                                          T (&dH)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    dH[0] = (T(P.ax) * nx + T(P.ay) * ny) * d[0];
  } else if constexpr (EQ == EQ_BUR) {
    dH[0] = T(0.5) * (T(2) * b.w[0] + d[0]) * d[0] * (nx + ny);
  } else {
    const T rho1 = b.w[0] + d[0];
    const T mx1 = b.w[1] + d[1], my1 = b.w[2] + d[2];
    const T ir = recip(rho1);
    const T du = (d[1] - b.u * d[0]) * ir;
    const T dv = (d[2] - b.v * d[0]) * ir;
    const T dke = T(0.5) * (d[1] * b.u + mx1 * du + d[2] * b.v + my1 * dv);
    const T dp = T(P.gam - 1.0) * (d[3] - dke);
    const T un = b.u * nx + b.v * ny;
    const T dun = du * nx + dv * ny;
    dH[0] = d[0] * un + rho1 * dun;
    dH[1] = d[1] * un + mx1 * dun + dp * nx;
    dH[2] = d[2] * un + my1 * dun + dp * ny;
    dH[3] = (d[3] + dp) * un + ((b.w[3] + d[3]) + (b.p + dp)) * dun;
  }
}

// Largest |eigenvalue| of d(F.n)/dW at a cell average (flux viscosity alpha).
template <int EQ>
__host__ __device__ __forceinline__ double spectral_radius(const Params& P, const double (&W)[NComp<EQ>::m], double nx,
                                                          double ny) {
  if constexpr (EQ == EQ_ADV) {
    return fabs(P.ax * nx + P.ay * ny);
  } else if constexpr (EQ == EQ_BUR) {
    return fabs(W[0] * (nx + ny));
  } else {
    double r = 1.0 / W[0];
    double u = W[1] * r, v = W[2] * r;
    double p = (P.gam - 1.0) * (W[3] - 0.5 * (W[1] * u + W[2] * v));
    return fabs(u * nx + v * ny) + sqrt(P.gam * p * r);
  }
}

// Largest signal speed over all directions at a cell average (time-step rule).
template <int EQ>
__host__ __device__ __forceinline__ double max_speed(const Params& P, const double (&W)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    return sqrt(P.ax * P.ax + P.ay * P.ay);
  } else if constexpr (EQ == EQ_BUR) {
    return 1.4142135623730951 * fabs(W[0]);
  } else {
    double r = 1.0 / W[0];
    double u = W[1] * r, v = W[2] * r;
    double p = (P.gam - 1.0) * (W[3] - 0.5 * (W[1] * u + W[2] * v));
    return sqrt(u * u + v * v) + sqrt(P.gam * p * r);
  }
}

}  // namespace hwe
