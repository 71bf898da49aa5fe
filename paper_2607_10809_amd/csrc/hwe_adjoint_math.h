// Reverse-mode (vector-Jacobian) counterparts of the step's point-wise math,
// written by hand operation by operation from hwe_math.h / hwe_step_math.h.
// Every *_rev function recomputes the forward values it needs and accumulates
// (+=) the adjoints of its inputs.
//
// Non-smooth points follow the forward's branches: d|x| = sign(x) dx with
// sign(0) = 0, max(a, b) passes the adjoint to the branch the forward took,
// kappa/D := 0 when kappa == 0 carries no derivative.
#pragma once

#include "hwe_step_math.h"

namespace hwe {

// ------------------------------------------------------------------ jets
template <class T> __host__ __device__ __forceinline__ SJ<T> sj_zero() { return SJ<T>{T(0), T(0), T(0), T(0), T(0), T(0)}; }
template <class T> __host__ __device__ __forceinline__ TJ<T> tj_zero() { return TJ<T>{T(0), T(0), T(0)}; }
template <class T> __host__ __device__ __forceinline__ void sj_acc(SJ<T>& a, const SJ<T>& b, T s = T(1)) {
  a.c += s * b.c; a.x += s * b.x; a.y += s * b.y; a.xx += s * b.xx; a.xy += s * b.xy; a.yy += s * b.yy;
}
template <class T> __host__ __device__ __forceinline__ void tj_acc(TJ<T>& a, const TJ<T>& b, T s = T(1)) {
  a.t += s * b.t; a.xt += s * b.xt; a.yt += s * b.yt;
}

// r = a * b (spatial jets)
template <class T>
__host__ __device__ __forceinline__ void sj_mul_rev(const SJ<T>& a, const SJ<T>& b, const SJ<T>& lr, SJ<T>& la, SJ<T>& lb) {
  la.c += lr.c * b.c + lr.x * b.x + lr.y * b.y + lr.xx * b.xx + lr.xy * b.xy + lr.yy * b.yy;
  la.x += lr.x * b.c + lr.xx * b.x + lr.xy * b.y;
  la.y += lr.y * b.c + lr.xy * b.x + lr.yy * b.y;
  la.xx += lr.xx * b.c;
  la.xy += lr.xy * b.c;
  la.yy += lr.yy * b.c;
  lb.c += lr.c * a.c + lr.x * a.x + lr.y * a.y + lr.xx * a.xx + lr.xy * a.xy + lr.yy * a.yy;
  lb.x += lr.x * a.c + lr.xx * a.x + lr.xy * a.y;
  lb.y += lr.y * a.c + lr.xy * a.x + lr.yy * a.y;
  lb.xx += lr.xx * a.c;
  lb.xy += lr.xy * a.c;
  lb.yy += lr.yy * a.c;
}
// r = 1 / a
template <class T> __host__ __device__ __forceinline__ void sj_recip_rev(const SJ<T>& a, const SJ<T>& lr, SJ<T>& la) {
  const T r1 = T(1) / a.c, r2 = r1 * r1, r3 = r2 * r1;
  la.x += -lr.x * r2 + lr.xx * T(2) * a.x * r3 + lr.xy * T(2) * a.y * r3;
  la.y += -lr.y * r2 + lr.xy * T(2) * a.x * r3 + lr.yy * T(2) * a.y * r3;
  la.xx += -lr.xx * r2;
  la.xy += -lr.xy * r2;
  la.yy += -lr.yy * r2;
  const T l2 = -(lr.x * a.x + lr.y * a.y + lr.xx * a.xx + lr.xy * a.xy + lr.yy * a.yy);
  const T l3 = lr.xx * a.x * a.x + lr.xy * T(2) * a.x * a.y + lr.yy * a.y * a.y;
  const T l1 = lr.c + l2 * T(2) * r1 + l3 * T(3) * r2;
  la.c += -l1 * r2;
}
// o = tj_mul(a, at, b, bt)
template <class T>
__host__ __device__ __forceinline__ void tj_mul_rev(const SJ<T>& a, const TJ<T>& at, const SJ<T>& b, const TJ<T>& bt,
                                                   const TJ<T>& lo, SJ<T>& la, TJ<T>& lat, SJ<T>& lb, TJ<T>& lbt) {
  la.c += lo.t * bt.t + lo.xt * bt.xt + lo.yt * bt.yt;
  la.x += lo.xt * bt.t;
  la.y += lo.yt * bt.t;
  lat.t += lo.t * b.c + lo.xt * b.x + lo.yt * b.y;
  lat.xt += lo.xt * b.c;
  lat.yt += lo.yt * b.c;
  lb.c += lo.t * at.t + lo.xt * at.xt + lo.yt * at.yt;
  lb.x += lo.xt * at.t;
  lb.y += lo.yt * at.t;
  lbt.t += lo.t * a.c + lo.xt * a.x + lo.yt * a.y;
  lbt.xt += lo.xt * a.c;
  lbt.yt += lo.yt * a.c;
}
// o = tj_recip(a, at, r) with r = 1/a (spatial)
template <class T>
__host__ __device__ __forceinline__ void tj_recip_rev(const SJ<T>& a, const TJ<T>& at, const SJ<T>& r, const TJ<T>& lo,
                                                     SJ<T>& la, TJ<T>& lat, SJ<T>& lr) {
  const T r2 = r.c * r.c, r3 = r2 * r.c;
  lat.t += -lo.t * r2 + lo.xt * T(2) * a.x * r3 + lo.yt * T(2) * a.y * r3;
  lat.xt += -lo.xt * r2;
  lat.yt += -lo.yt * r2;
  la.x += lo.xt * T(2) * at.t * r3;
  la.y += lo.yt * T(2) * at.t * r3;
  const T l2 = -(lo.t * at.t + lo.xt * at.xt + lo.yt * at.yt);
  const T l3 = lo.xt * T(2) * a.x * at.t + lo.yt * T(2) * a.y * at.t;
  lr.c += l2 * T(2) * r.c + l3 * T(3) * r2;
}

// ------------------------------------------------------------------ Lax-Wendroff
// Given D and the adjoints of W_t, W_tt, accumulate the adjoints of D.
template <int EQ, class T>
__host__ __device__ __forceinline__ void lax_wendroff_rev(const Params& P, const T (&D)[6][NComp<EQ>::m],
                                                         const T (&lWt)[NComp<EQ>::m], const T (&lWtt)[NComp<EQ>::m],
                                                         T (&lD)[6][NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    const T ax = T(P.ax), ay = T(P.ay);
    // Wt = -(ax Wx + ay Wy); Wtt = -(ax wtx + ay wty), wtx = -(ax Wxx + ay Wxy), wty = -(ax Wxy + ay Wyy)
    const T lwtx = -ax * lWtt[0], lwty = -ay * lWtt[0];
    lD[1][0] += -ax * lWt[0];
    lD[2][0] += -ay * lWt[0];
    lD[3][0] += -ax * lwtx;
    lD[4][0] += -ay * lwtx - ax * lwty;
    lD[5][0] += -ay * lwty;
  } else if constexpr (EQ == EQ_BUR) {
    const SJ<T> J{D[0][0], D[1][0], D[2][0], T(0.5) * D[3][0], D[4][0], T(0.5) * D[5][0]};
    const SJ<T> s = sj_scale(T(0.5), sj_mul(J, J));
    TJ<T> Jt;
    Jt.t = -(s.x + s.y);
    Jt.xt = -(T(2) * s.xx + s.xy);
    Jt.yt = -(s.xy + T(2) * s.yy);
    // st = 1/2 tj_mul(J, Jt, J, Jt); Wtt = -(st.xt + st.yt); Wt = Jt.t
    TJ<T> lst{T(0), -lWtt[0], -lWtt[0]};
    lst = tj_scale(T(0.5), lst);
    SJ<T> lJ = sj_zero<T>();
    TJ<T> lJt{lWt[0], T(0), T(0)};
    tj_mul_rev(J, Jt, J, Jt, lst, lJ, lJt, lJ, lJt);
    SJ<T> ls = sj_zero<T>();
    ls.x += -lJt.t;
    ls.y += -lJt.t;
    ls.xx += -T(2) * lJt.xt;
    ls.xy += -lJt.xt - lJt.yt;
    ls.yy += -T(2) * lJt.yt;
    ls = sj_scale(T(0.5), ls);
    sj_mul_rev(J, J, ls, lJ, lJ);
    lD[0][0] += lJ.c;
    lD[1][0] += lJ.x;
    lD[2][0] += lJ.y;
    lD[3][0] += T(0.5) * lJ.xx;
    lD[4][0] += lJ.xy;
    lD[5][0] += T(0.5) * lJ.yy;
  } else {
    const T gm1 = T(P.gam - 1.0);
    SJ<T> J[4];
    for (int q = 0; q < 4; ++q) J[q] = SJ<T>{D[0][q], D[1][q], D[2][q], T(0.5) * D[3][q], D[4][q], T(0.5) * D[5][q]};
    const SJ<T>& rho = J[0];
    const SJ<T>& mx = J[1];
    const SJ<T>& my = J[2];
    const SJ<T>& En = J[3];
    // forward (as in lax_wendroff)
    const SJ<T> r = sj_recip(rho);
    const SJ<T> u = sj_mul(mx, r), v = sj_mul(my, r);
    const SJ<T> mxu = sj_mul(mx, u), myv = sj_mul(my, v), muv = sj_mul(mx, v);
    const SJ<T> ke = sj_scale(T(0.5), sj_add(mxu, myv));
    const SJ<T> p = sj_scale(gm1, sj_sub(En, ke));
    const SJ<T> H = sj_add(En, p);
    const SJ<T> uH = sj_mul(u, H), vH = sj_mul(v, H);
    const SJ<T> f1 = sj_add(mxu, p), g2 = sj_add(myv, p);
    TJ<T> Jt[4];
    Jt[0] = TJ<T>{-(mx.x + my.y), -(T(2) * mx.xx + my.xy), -(mx.xy + T(2) * my.yy)};
    Jt[1] = TJ<T>{-(f1.x + muv.y), -(T(2) * f1.xx + muv.xy), -(f1.xy + T(2) * muv.yy)};
    Jt[2] = TJ<T>{-(muv.x + g2.y), -(T(2) * muv.xx + g2.xy), -(muv.xy + T(2) * g2.yy)};
    Jt[3] = TJ<T>{-(uH.x + vH.y), -(T(2) * uH.xx + vH.xy), -(uH.xy + T(2) * vH.yy)};
    const TJ<T> rt = tj_recip(rho, Jt[0], r);
    const TJ<T> ut = tj_mul(mx, Jt[1], r, rt), vt = tj_mul(my, Jt[2], r, rt);
    const TJ<T> pt = tj_scale(gm1, tj_sub(Jt[3], tj_scale(T(0.5), tj_add(tj_mul(mx, Jt[1], u, ut), tj_mul(my, Jt[2], v, vt)))));
    const TJ<T> Ht = tj_add(Jt[3], pt);
    // reverse
    TJ<T> lJt[4] = {tj_zero<T>(), tj_zero<T>(), tj_zero<T>(), tj_zero<T>()};
    for (int q = 0; q < 4; ++q) lJt[q].t += lWt[q];
    TJ<T> lmxut = tj_zero<T>(), lmyvt = tj_zero<T>(), lmuvt = tj_zero<T>(), lpt = tj_zero<T>();
    TJ<T> luHt = tj_zero<T>(), lvHt = tj_zero<T>();
    lJt[1].xt += -lWtt[0];
    lJt[2].yt += -lWtt[0];
    lmxut.xt += -lWtt[1];
    lpt.xt += -lWtt[1];
    lmuvt.yt += -lWtt[1];
    lmuvt.xt += -lWtt[2];
    lmyvt.yt += -lWtt[2];
    lpt.yt += -lWtt[2];
    luHt.xt += -lWtt[3];
    lvHt.yt += -lWtt[3];
    SJ<T> lr = sj_zero<T>(), lu = sj_zero<T>(), lv = sj_zero<T>(), lH = sj_zero<T>();
    SJ<T> lJ[4] = {sj_zero<T>(), sj_zero<T>(), sj_zero<T>(), sj_zero<T>()};
    TJ<T> lut = tj_zero<T>(), lvt = tj_zero<T>(), lHt = tj_zero<T>(), lrt = tj_zero<T>();
    tj_mul_rev(v, vt, H, Ht, lvHt, lv, lvt, lH, lHt);
    tj_mul_rev(u, ut, H, Ht, luHt, lu, lut, lH, lHt);
    tj_acc(lJt[3], lHt);
    tj_acc(lpt, lHt);
    tj_acc(lJt[3], lpt, gm1);
    TJ<T> lket = tj_scale(-gm1, lpt);
    tj_acc(lmxut, lket, T(0.5));
    tj_acc(lmyvt, lket, T(0.5));
    tj_mul_rev(mx, Jt[1], v, vt, lmuvt, lJ[1], lJt[1], lv, lvt);
    tj_mul_rev(my, Jt[2], v, vt, lmyvt, lJ[2], lJt[2], lv, lvt);
    tj_mul_rev(mx, Jt[1], u, ut, lmxut, lJ[1], lJt[1], lu, lut);
    tj_mul_rev(my, Jt[2], r, rt, lvt, lJ[2], lJt[2], lr, lrt);
    tj_mul_rev(mx, Jt[1], r, rt, lut, lJ[1], lJt[1], lr, lrt);
    tj_recip_rev(rho, Jt[0], r, lrt, lJ[0], lJt[0], lr);
    // spatial definitions of the time derivatives: Jt = (-(F.x + G.y), -(2F.xx + G.xy), -(F.xy + 2G.yy))
    SJ<T> lf1 = sj_zero<T>(), lg2 = sj_zero<T>(), lmuv = sj_zero<T>(), luH = sj_zero<T>(), lvH = sj_zero<T>();
    auto back = [](const TJ<T>& l, SJ<T>& lF, SJ<T>& lG) {
      lF.x += -l.t;
      lG.y += -l.t;
      lF.xx += -T(2) * l.xt;
      lG.xy += -l.xt;
      lF.xy += -l.yt;
      lG.yy += -T(2) * l.yt;
    };
    back(lJt[0], lJ[1], lJ[2]);
    back(lJt[1], lf1, lmuv);
    back(lJt[2], lmuv, lg2);
    back(lJt[3], luH, lvH);
    SJ<T> lmxu = lf1, lmyv = lg2, lp = sj_zero<T>();
    sj_acc(lp, lf1);
    sj_acc(lp, lg2);
    sj_mul_rev(v, H, lvH, lv, lH);
    sj_mul_rev(u, H, luH, lu, lH);
    sj_acc(lJ[3], lH);
    sj_acc(lp, lH);
    sj_acc(lJ[3], lp, gm1);
    const SJ<T> lke = sj_scale(-gm1, lp);
    sj_acc(lmxu, lke, T(0.5));
    sj_acc(lmyv, lke, T(0.5));
    sj_mul_rev(mx, v, lmuv, lJ[1], lv);
    sj_mul_rev(my, v, lmyv, lJ[2], lv);
    sj_mul_rev(mx, u, lmxu, lJ[1], lu);
    sj_mul_rev(my, r, lv, lJ[2], lr);
    sj_mul_rev(mx, r, lu, lJ[1], lr);
    sj_recip_rev(rho, lr, lJ[0]);
    for (int q = 0; q < 4; ++q) {
      lD[0][q] += lJ[q].c;
      lD[1][q] += lJ[q].x;
      lD[2][q] += lJ[q].y;
      lD[3][q] += T(0.5) * lJ[q].xx;
      lD[4][q] += lJ[q].xy;
      lD[5][q] += T(0.5) * lJ[q].yy;
    }
  }
}

// ------------------------------------------------------------------ fluxes
// Reverse of normal_flux_delta: adjoints of the offset d and of the base
// (w, u, v, p) given the adjoint of dH.
template <int EQ, class T> struct FluxBaseAdj {
  T w[NComp<EQ>::m];
  T u, v, p;
};
template <int EQ, class T>
__host__ __device__ __forceinline__ void normal_flux_delta_rev(const Params& P, const FluxBase<EQ, T>& b,
                                                              const T (&d)[NComp<EQ>::m], T nx, T ny,
                                                              const T (&L)[NComp<EQ>::m], T (&ld)[NComp<EQ>::m],
                                                              FluxBaseAdj<EQ, T>& lb) {
  if constexpr (EQ == EQ_ADV) {
    ld[0] += (T(P.ax) * nx + T(P.ay) * ny) * L[0];
  } else if constexpr (EQ == EQ_BUR) {
    const T s = nx + ny;
    ld[0] += (b.w[0] + d[0]) * s * L[0];
    lb.w[0] += d[0] * s * L[0];
  } else {
    const T g = T(P.gam - 1.0);
    const T rho1 = b.w[0] + d[0];
    const T mx1 = b.w[1] + d[1], my1 = b.w[2] + d[2];
    const T ir = T(1) / rho1;
    const T nu = d[1] - b.u * d[0], nv = d[2] - b.v * d[0];
    const T du = nu * ir, dv = nv * ir;
    const T dke = T(0.5) * (d[1] * b.u + mx1 * du + d[2] * b.v + my1 * dv);
    const T dp = g * (d[3] - dke);
    const T un = b.u * nx + b.v * ny;
    const T dun = du * nx + dv * ny;
    const T E1p = (b.w[3] + d[3]) + (b.p + dp);
    // dH3 = (d3 + dp) un + E1p dun
    T ld3 = L[3] * un, ldp = L[3] * un, lun = L[3] * (d[3] + dp), lE1p = L[3] * dun, ldun = L[3] * E1p;
    lb.w[3] += lE1p;
    ld3 += lE1p;
    lb.p += lE1p;
    ldp += lE1p;
    // dH2 = d2 un + my1 dun + dp ny
    T ld2 = L[2] * un;
    lun += L[2] * d[2];
    T lmy1 = L[2] * dun;
    ldun += L[2] * my1;
    ldp += L[2] * ny;
    // dH1 = d1 un + mx1 dun + dp nx
    T ld1 = L[1] * un;
    lun += L[1] * d[1];
    T lmx1 = L[1] * dun;
    ldun += L[1] * mx1;
    ldp += L[1] * nx;
    // dH0 = d0 un + rho1 dun
    T ld0 = L[0] * un;
    lun += L[0] * d[0];
    T lrho1 = L[0] * dun;
    ldun += L[0] * rho1;
    T ldu = ldun * nx, ldv = ldun * ny;
    T lu = lun * nx, lv = lun * ny;
    ld3 += g * ldp;
    const T ldke = -g * ldp;
    const T hk = T(0.5) * ldke;
    ld1 += hk * b.u;
    lu += hk * d[1];
    lmx1 += hk * du;
    ldu += hk * mx1;
    ld2 += hk * b.v;
    lv += hk * d[2];
    lmy1 += hk * dv;
    ldv += hk * my1;
    // dv = (d2 - v d0) ir, du = (d1 - u d0) ir
    T lir = nv * ldv + nu * ldu;
    ld2 += ir * ldv;
    lv += -d[0] * ir * ldv;
    ld0 += -b.v * ir * ldv;
    ld1 += ir * ldu;
    lu += -d[0] * ir * ldu;
    ld0 += -b.u * ir * ldu;
    lrho1 += -ir * ir * lir;
    lb.w[2] += lmy1;
    ld2 += lmy1;
    lb.w[1] += lmx1;
    ld1 += lmx1;
    lb.w[0] += lrho1;
    ld0 += lrho1;
    lb.u += lu;
    lb.v += lv;
    ld[0] += ld0;
    ld[1] += ld1;
    ld[2] += ld2;
    ld[3] += ld3;
  }
}

// Reverse of flux_base (FP64): adjoint of the cell average from the adjoint
// of (w, u, v, p).
template <int EQ, class T>
__host__ __device__ __forceinline__ void flux_base_rev(const Params& P, const double (&W)[NComp<EQ>::m],
                                                      const FluxBaseAdj<EQ, T>& lb, double (&lW)[NComp<EQ>::m]) {
  for (int q = 0; q < NComp<EQ>::m; ++q) lW[q] += double(lb.w[q]);
  if constexpr (EQ == EQ_EUL) {
    const double r = 1.0 / W[0];
    const double u = W[1] * r, v = W[2] * r;
    const double gm1 = P.gam - 1.0;
    const double lp = double(lb.p);
    double lu = double(lb.u), lv = double(lb.v);
    lW[3] += gm1 * lp;
    const double hq = -0.5 * gm1 * lp;
    lW[1] += u * hq;
    lu += W[1] * hq;
    lW[2] += v * hq;
    lv += W[2] * hq;
    lW[1] += r * lu;
    lW[2] += r * lv;
    const double lr = W[1] * lu + W[2] * lv;
    lW[0] += -r * r * lr;
  }
}

// J_H(W)^T L for the normal flux H(W) = f nx + g ny at a cell average (FP64).
template <int EQ>
__host__ __device__ __forceinline__ void normal_flux_jt(const Params& P, const double (&W)[NComp<EQ>::m], double nx,
                                                       double ny, const double (&L)[NComp<EQ>::m], double s,
                                                       double (&lW)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    lW[0] += s * (P.ax * nx + P.ay * ny) * L[0];
  } else if constexpr (EQ == EQ_BUR) {
    lW[0] += s * W[0] * (nx + ny) * L[0];
  } else {
    const double g = P.gam - 1.0;
    const double r = 1.0 / W[0];
    const double u = W[1] * r, v = W[2] * r;
    const double un = u * nx + v * ny;
    const double p = g * (W[3] - 0.5 * (W[1] * u + W[2] * v));
    const double lun = L[0] * W[0] + L[1] * W[1] + L[2] * W[2] + L[3] * (W[3] + p);
    double lrho = L[0] * un, lmx = L[1] * un, lmy = L[2] * un, lE = L[3] * un;
    const double lp = L[1] * nx + L[2] * ny + L[3] * un;
    lE += g * lp;
    const double hq = -0.5 * g * lp;
    lmx += u * hq;
    double lu = W[1] * hq + lun * nx;
    lmy += v * hq;
    double lv = W[2] * hq + lun * ny;
    lmx += r * lu;
    lmy += r * lv;
    const double lr = W[1] * lu + W[2] * lv;
    lrho += -r * r * lr;
    lW[0] += s * lrho;
    lW[1] += s * lmx;
    lW[2] += s * lmy;
    lW[3] += s * lE;
  }
}

// s * gradient of spectral_radius at W (sign(0) = 0), accumulated into lW.
template <int EQ>
__host__ __device__ __forceinline__ void spectral_radius_grad(const Params& P, const double (&W)[NComp<EQ>::m],
                                                             double nx, double ny, double s,
                                                             double (&lW)[NComp<EQ>::m]) {
  if constexpr (EQ == EQ_ADV) {
    (void)P;
  } else if constexpr (EQ == EQ_BUR) {
    const double a = W[0] * (nx + ny);
    const double sg = a > 0 ? 1.0 : (a < 0 ? -1.0 : 0.0);
    lW[0] += s * sg * (nx + ny);
  } else {
    const double gm1 = P.gam - 1.0;
    const double r = 1.0 / W[0];
    const double u = W[1] * r, v = W[2] * r;
    const double p = gm1 * (W[3] - 0.5 * (W[1] * u + W[2] * v));
    const double un = u * nx + v * ny;
    const double sg = un > 0 ? 1.0 : (un < 0 ? -1.0 : 0.0);
    const double c = sqrt(P.gam * p * r);
    double lu = s * sg * nx, lv = s * sg * ny;
    double lp = 0.0, lr = 0.0;
    if (c > 0.0) {
      const double lc = s * P.gam / (2.0 * c);  // d sqrt(g p r) = g/(2c) (r dp + p dr)
      lp = lc * r;
      lr = lc * p;
    }
    lW[3] += gm1 * lp;
    const double hq = -0.5 * gm1 * lp;
    lW[1] += u * hq;
    lu += W[1] * hq;
    lW[2] += v * hq;
    lv += W[2] * hq;
    lW[1] += r * lu;
    lW[2] += r * lv;
    lr += W[1] * lu + W[2] * lv;
    lW[0] += -r * r * lr;
  }
}

// ------------------------------------------------------------------ edge lane
// Reverse of edge_lane for one side at one Gauss point (X, Y): given the
// adjoints of AH, AD, AT of this lane, accumulate the adjoints of the cell's
// coefficients a[6][M] and of its cell average.  Returns (in ADout) the
// forward AD of the lane, used by the flux viscosity's adjoint.
// WALL (Euler): the face is a reflective wall, whose exterior flux term is
// the normal flux at the mirror image, base WT = T Wbar and offsets T d(tau)
// (T reflects the momentum about the face); lAHw seeds that term's time
// integral, and lWT receives the adjoint of WT (the caller maps it back
// through T).
template <int EQ, class Real, int TR, bool WALL = false>
__host__ __device__ __forceinline__ void edge_lane_rev(const Params& P, double dt, const Real (&a)[6][NComp<EQ>::m],
                                                      const double (&Wbd)[NComp<EQ>::m], Real X, Real Y, Real nx,
                                                      Real ny, const Real (&lAH)[NComp<EQ>::m],
                                                      const Real (&lAD)[NComp<EQ>::m],
                                                      const Real (&lAT)[NComp<EQ>::m], Real (&la)[6][NComp<EQ>::m],
                                                      double (&lW)[NComp<EQ>::m], Real (&ADout)[NComp<EQ>::m],
                                                      const double* WT = nullptr, const Real* lAHw = nullptr,
                                                      double* lWT = nullptr) {
  constexpr int M = NComp<EQ>::m;
  static_assert(!WALL || EQ == EQ_EUL, "walls reflect a momentum");
  Real D[6][M], dl[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    dl[q] = a[0][q] + a[1][q] * X + a[2][q] * Y + a[3][q] * X * X + a[4][q] * X * Y + a[5][q] * Y * Y;
    D[0][q] = Real(Wbd[q]) + dl[q];
    D[1][q] = a[1][q] + Real(2) * a[3][q] * X + a[4][q] * Y;
    D[2][q] = a[2][q] + a[4][q] * X + Real(2) * a[5][q] * Y;
    D[3][q] = Real(2) * a[3][q];
    D[4][q] = a[4][q];
    D[5][q] = Real(2) * a[5][q];
  }
  Real Wt[M], Wtt[M];
  lax_wendroff<EQ, Real>(P, D, Wt, Wtt);
  const FluxBase<EQ, Real> base = flux_base<EQ, Real>(P, Wbd);
  FluxBaseAdj<EQ, Real> lb;
#pragma unroll
  for (int q = 0; q < M; ++q) lb.w[q] = Real(0);
  lb.u = lb.v = lb.p = Real(0);
  FluxBase<EQ, Real> baseT;
  FluxBaseAdj<EQ, Real> lbT;
  if constexpr (WALL) {
    double W[M];
#pragma unroll
    for (int q = 0; q < M; ++q) W[q] = WT[q];
    baseT = flux_base<EQ, Real>(P, W);
#pragma unroll
    for (int q = 0; q < M; ++q) lbT.w[q] = Real(0);
    lbT.u = lbT.v = lbT.p = Real(0);
  }
  Real ldl[M], lWt[M], lWtt[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    ldl[q] = lWt[q] = lWtt[q] = Real(0);
    ADout[q] = Real(0);
  }
  // one node of the time rule, reversed: d(tau) = dl + tau W_t + tau^2/2 W_tt
  // feeds w dH(d) into AH and w d into AD
  auto node_rev = [&](Real tau, Real w) {
    const Real h2 = Real(0.5) * tau * tau;
    Real dls[M], L[M], lds[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      dls[q] = dl[q] + tau * Wt[q] + h2 * Wtt[q];
      ADout[q] += w * dls[q];
      L[q] = w * lAH[q];
      lds[q] = w * lAD[q];
    }
    normal_flux_delta_rev<EQ, Real>(P, base, dls, nx, ny, L, lds, lb);
    if constexpr (WALL) {
      // the mirror side's flux offset at T d(tau), reversed and mapped back through T
      Real dT[M], LT[M], ldT[M];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        dT[q] = dls[q];
        LT[q] = w * lAHw[q];
        ldT[q] = Real(0);
      }
      reflect_momentum(nx, ny, dT);
      normal_flux_delta_rev<EQ, Real>(P, baseT, dT, nx, ny, LT, ldT, lbT);
      reflect_momentum(nx, ny, ldT);
#pragma unroll
      for (int q = 0; q < M; ++q) lds[q] += ldT[q];
    }
#pragma unroll
    for (int q = 0; q < M; ++q) {
      ldl[q] += lds[q];
      lWt[q] += tau * lds[q];
      lWtt[q] += h2 * lds[q];
    }
  };
  if constexpr (TR == 1) {
    node_rev(Real(kGaussLegendre2[0] * dt), Real(0.5));
    node_rev(Real(kGaussLegendre2[1] * dt), Real(0.5));
  } else {
    node_rev(Real(0), Real(1.0 / 6.0));
    node_rev(Real(0.5 * dt), Real(4.0 / 6.0));
    node_rev(Real(dt), Real(1.0 / 6.0));
  }
  // the interface value AT = d(dt)
  {
    const Real T1 = Real(dt), h2 = Real(0.5 * dt * dt);
#pragma unroll
    for (int q = 0; q < M; ++q) {
      ldl[q] += lAT[q];
      lWt[q] += T1 * lAT[q];
      lWtt[q] += h2 * lAT[q];
    }
  }
  Real lD[6][M];
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int q = 0; q < M; ++q) lD[j][q] = Real(0);
  lax_wendroff_rev<EQ, Real>(P, D, lWt, lWtt, lD);
  flux_base_rev<EQ, Real>(P, Wbd, lb, lW);
  if constexpr (WALL) {
    double W[M], l[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      W[q] = WT[q];
      l[q] = 0.0;
    }
    flux_base_rev<EQ, Real>(P, W, lbT, l);
#pragma unroll
    for (int q = 0; q < M; ++q) lWT[q] += l[q];
  }
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const Real l0 = ldl[q] + lD[0][q];
    lW[q] += double(lD[0][q]);
    la[0][q] += l0;
    la[1][q] += X * l0 + lD[1][q];
    la[2][q] += Y * l0 + lD[2][q];
    la[3][q] += X * X * l0 + Real(2) * X * lD[1][q] + Real(2) * lD[3][q];
    la[4][q] += X * Y * l0 + Y * lD[1][q] + X * lD[2][q] + lD[4][q];
    la[5][q] += Y * Y * l0 + Real(2) * Y * lD[2][q] + Real(2) * lD[5][q];
  }
}

// ------------------------------------------------------------------ limiter
// Reverse of positivity_theta (FP64), on the branches the forward takes: the
// density scale through the point of least density, the pressure scale t
// through the point whose root was taken (the quadratic's root formula
// reversed).  The threshold eps = min(1e-13, rho_bar, p_bar) is a constant of
// the derivative.  lth: adjoints of theta[0..3]; accumulates the adjoints of
// the unlimited coefficients a[4][6] (la) and of the cell average Wb (lWb).
template <class Real, int NP>
__host__ __device__ __forceinline__ void positivity_theta_rev(double gam, const double (&Wb)[4],
                                                             const Real (&a)[4][6], const double (&px)[NP],
                                                             const double (&py)[NP], const double (&lth)[4],
                                                             double (&la)[4][6], double (&lWb)[4]) {
  // ---- forward, recording the branches
  const double gm1 = gam - 1.0;
  const double pbar = gm1 * (Wb[3] - 0.5 * (Wb[1] * Wb[1] + Wb[2] * Wb[2]) / Wb[0]);
  const double eps = fmin(1e-13, fmin(Wb[0], pbar));
  double d[NP][4];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double X = px[k], Y = py[k];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      d[k][q] = double(a[q][0]) + double(a[q][1]) * X + double(a[q][2]) * Y + double(a[q][3]) * X * X +
                double(a[q][4]) * X * Y + double(a[q][5]) * Y * Y;
  }
  double rmin = 1e300;
  int kmin = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double r = Wb[0] + d[k][0];
    if (r < rmin) {
      rmin = r;
      kmin = k;
    }
  }
  const bool rho_on = rmin < eps;
  const double th_rho = rho_on ? (Wb[0] - eps) / (Wb[0] - rmin) : 1.0;
  const double Ep = Wb[3] - eps / gm1;
  const double C = 2.0 * Wb[0] * Ep - (Wb[1] * Wb[1] + Wb[2] * Wb[2]);
  double t = 1.0;
  int kt = -1;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double dr = th_rho * d[k][0], d1 = d[k][1], d2 = d[k][2], dE = d[k][3];
    const double r = Wb[0] + dr, m1 = Wb[1] + d1, m2 = Wb[2] + d2, En = Wb[3] + dE;
    const double p = gm1 * (En - 0.5 * (m1 * m1 + m2 * m2) / r);
    if (!(p < eps)) continue;
    const double A = 2.0 * dr * dE - (d1 * d1 + d2 * d2);
    const double B = 2.0 * (Ep * dr + Wb[0] * dE) - 2.0 * (Wb[1] * d1 + Wb[2] * d2);
    double root;
    if (A == 0.0) {
      root = -C / B;
    } else {
      const double disc = fmax(B * B - 4.0 * A * C, 0.0);
      const double sq = sqrt(disc);
      const double qq = B >= 0.0 ? -0.5 * (B + sq) : -0.5 * (B - sq);
      const double r1 = qq / A, r2 = C / qq;
      const bool ok1 = r1 >= 0.0 && r1 <= 1.0, ok2 = r2 >= 0.0 && r2 <= 1.0;
      root = (ok1 && ok2) ? (r1 <= r2 ? r1 : r2) : (ok1 ? r1 : r2);
    }
    if (root < t) {
      t = root;
      kt = k;
    }
  }
  // ---- reverse: theta[0] = th_rho t, theta[1..3] = t
  const double lt = lth[0] * th_rho + lth[1] + lth[2] + lth[3];
  double lthr = lth[0] * t;
  double ld[NP][4];
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) ld[k][q] = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (k != kt) continue;
    const double d0 = d[k][0], dr = th_rho * d0, d1 = d[k][1], d2 = d[k][2], dE = d[k][3];
    const double A = 2.0 * dr * dE - (d1 * d1 + d2 * d2);
    const double B = 2.0 * (Ep * dr + Wb[0] * dE) - 2.0 * (Wb[1] * d1 + Wb[2] * d2);
    double lA = 0.0, lB = 0.0, lC = 0.0;
    if (A == 0.0) {
      lC = -lt / B;
      lB = C / (B * B) * lt;
    } else {
      const double disc0 = B * B - 4.0 * A * C;
      const double disc = fmax(disc0, 0.0);
      const double sq = sqrt(disc);
      const double qq = B >= 0.0 ? -0.5 * (B + sq) : -0.5 * (B - sq);
      const double r1 = qq / A, r2 = C / qq;
      const bool ok1 = r1 >= 0.0 && r1 <= 1.0, ok2 = r2 >= 0.0 && r2 <= 1.0;
      const bool first = (ok1 && ok2) ? (r1 <= r2) : ok1;
      double lqq;
      if (first) {
        lqq = lt / A;
        lA = -qq / (A * A) * lt;
      } else {
        lC = lt / qq;
        lqq = -C / (qq * qq) * lt;
      }
      lB += -0.5 * lqq;
      const double lsq = (B >= 0.0 ? -0.5 : 0.5) * lqq;
      const double ldisc = (disc0 > 0.0 && sq > 0.0) ? lsq / (2.0 * sq) : 0.0;
      lB += 2.0 * B * ldisc;
      lA += -4.0 * C * ldisc;
      lC += -4.0 * A * ldisc;
    }
    const double ldr = 2.0 * dE * lA + 2.0 * Ep * lB;
    ld[k][3] += 2.0 * dr * lA + 2.0 * Wb[0] * lB;
    ld[k][1] += -2.0 * d1 * lA - 2.0 * Wb[1] * lB;
    ld[k][2] += -2.0 * d2 * lA - 2.0 * Wb[2] * lB;
    const double lEp = 2.0 * dr * lB + 2.0 * Wb[0] * lC;
    lWb[0] += 2.0 * dE * lB + 2.0 * Ep * lC;
    lWb[1] += -2.0 * d1 * lB - 2.0 * Wb[1] * lC;
    lWb[2] += -2.0 * d2 * lB - 2.0 * Wb[2] * lC;
    lthr += d0 * ldr;
    ld[k][0] += th_rho * ldr;
    lWb[3] += lEp;
  }
  if (rho_on) {
    const double den = Wb[0] - rmin;
    const double lrmin = lthr * (Wb[0] - eps) / (den * den);
    lWb[0] += lthr / den - lrmin;
    lWb[0] += lrmin;
#pragma unroll
    for (int k = 0; k < NP; ++k)
      if (k == kmin) ld[k][0] += lrmin;
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double X = px[k], Y = py[k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      la[q][0] += ld[k][q];
      la[q][1] += ld[k][q] * X;
      la[q][2] += ld[k][q] * Y;
      la[q][3] += ld[k][q] * X * X;
      la[q][4] += ld[k][q] * X * Y;
      la[q][5] += ld[k][q] * Y * Y;
    }
  }
}

// The reconstruction reverse without a limiter: the coefficients' adjoint
// passes through unchanged.
struct NoLimiter {
  template <class Real>
  __host__ __device__ __forceinline__ void operator()(const Real (&)[6], const Real (&la)[6], Real (&lae)[6],
                                                      double& lW0) const {
#pragma unroll
    for (int j = 0; j < 6; ++j) lae[j] = la[j];
    lW0 = 0.0;
  }
};

// ------------------------------------------------------------------ recon
// Reverse of recon_coeffs for component q of cell i: given the adjoint la[6]
// of the coefficients, write the adjoints of the stencil inputs into
// slot[s][field] (s = 0: the cell itself, s = f+1: its neighbour across face
// f; field 0 = Wbar, 1 = V, 2 = Y).  Ghost (mirror) neighbours are folded back
// into slot 0.
// SB: the mesh has walls or prescribed boundary states.  A prescribed ghost
// is a flat cell holding the prescribed state (only -W0 in its difference
// depends on the cell); a wall ghost of an Euler momentum component mixes the
// cell's two momentum components, and cross[c][field] (c = 0, 1: momentum
// components 1, 2) receives those terms of slot 0 for the kernel to exchange
// between the component lanes.  wbar, grad, N: the cell's other components.
template <int EQ, class Real, bool SB = false, class Lim = NoLimiter>
__host__ __device__ __forceinline__ void recon_rev(int i, int NB, const Params& P, const Stencil<Real>& S,
                                                  const double* __restrict__ bnd_n, const Real* __restrict__ tb,
                                                  const Real (&la_in)[6],
                                                  double (&slot)[4][3], int q = 0, int N = 0,
                                                  const double* __restrict__ wbar = nullptr,
                                                  const Real* __restrict__ grad = nullptr,
                                                  double (*cross)[3] = nullptr, const Lim& lim = Lim()) {
  // ---- forward recomputation from the gathered stencil (gather_stencil)
  const double W0 = S.W0;
  double Wsum = W0, dW[3];
  Real V[4], Y[4];
  int nb[3];
  Real gnx[3], gny[3];
  double Wn[3];
  // ghost kinds (SB): 0 mirror, 1 wall (momentum component), 2 prescribed
  int gk[3] = {0, 0, 0};
  double wna[3] = {0, 0, 0}, wnx[3] = {0, 0, 0}, wny[3] = {0, 0, 0};
  Real gV1 = Real(0), gY1 = Real(0), gV2 = Real(0), gY2 = Real(0);
  double gm1 = 0.0, gm2 = 0.0;
  if constexpr (SB && EQ == EQ_EUL) {
    if (q == 1 || q == 2) {
      constexpr int M = NComp<EQ>::m;
      gm1 = wbar[1 * size_t(N) + i];
      gm2 = wbar[2 * size_t(N) + i];
      gV1 = grad[1 * size_t(N) + i];
      gY1 = grad[(M + 1) * size_t(N) + i];
      gV2 = grad[2 * size_t(N) + i];
      gY2 = grad[(M + 2) * size_t(N) + i];
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    V[f] = S.V[f];
    Y[f] = S.Y[f];
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    nb[f] = S.nbi[f];
    Wn[f] = S.Wn[f];
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    gnx[f] = gny[f] = Real(0);
    if (nb[f] >= 0) {
      dW[f] = Wn[f] - W0;
      Wsum += Wn[f];
    } else {
      const int b = -nb[f] - 1;
      gnx[f] = Real(bnd_n[b]);
      gny[f] = Real(bnd_n[NB + b]);
      const double kind = SB ? bnd_n[2 * NB + b] : 0.0;
      if (SB && kind >= 2.0) {
        gk[f] = 2;
        const double Wd = prescribed_component(P, kind, bnd_n[3 * NB + b], q);
        dW[f] = Wd - W0;
        Wsum += Wd;
        V[f + 1] = Real(0);
        Y[f + 1] = Real(0);
      } else {
        dW[f] = 0.0;
        Wsum += W0;
        const Real vn = V[0] * gnx[f] + Y[0] * gny[f];
        V[f + 1] = V[0] - Real(2) * gnx[f] * vn;
        Y[f + 1] = Y[0] - Real(2) * gny[f] * vn;
        if constexpr (SB && EQ == EQ_EUL) {
          if ((q == 1 || q == 2) && kind == 1.0) {
            // as the forward: m -> m - 2 (m.n) n in the average, the momentum
            // rows of the gradient mixed the same way
            gk[f] = 1;
            const double dnx = bnd_n[b], dny = bnd_n[NB + b], na = q == 1 ? dnx : dny;
            wnx[f] = dnx;
            wny[f] = dny;
            wna[f] = na;
            dW[f] = -2.0 * na * (gm1 * dnx + gm2 * dny);
            Wsum += dW[f];
            const Real nx = gnx[f], ny = gny[f];
            const Real v1 = gV1 * nx + gY1 * ny, v2 = gV2 * nx + gY2 * ny;
            const Real R1x = gV1 - Real(2) * nx * v1, R1y = gY1 - Real(2) * ny * v1;
            const Real R2x = gV2 - Real(2) * nx * v2, R2y = gY2 - Real(2) * ny * v2;
            const Real rn = Real(2) * Real(na);
            V[f + 1] = V[f + 1] - rn * (nx * R1x + ny * R2x);
            Y[f + 1] = Y[f + 1] - rn * (nx * R1y + ny * R2y);
          }
        }
      }
    }
  }
  Real c[5];
  step1_apply<Real>(tb, Real(dW[0]), Real(dW[1]), Real(dW[2]), V, Y, c);
  Real bl[3], cl[3], pdx[3], pdy[3], piv[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    pdx[f] = tb[(kTblP2 + 3 * f) * kTile];
    pdy[f] = tb[(kTblP2 + 3 * f + 1) * kTile];
    piv[f] = tb[(kTblP2 + 3 * f + 2) * kTile];
    const Real t = (Real(dW[f]) - pdx[f] * V[f + 1] - pdy[f] * Y[f + 1]) * piv[f];
    bl[f] = V[f + 1] + pdx[f] * t;
    cl[f] = Y[f + 1] + pdy[f] * t;
  }
  const double g1 = P.lw[0];
  const double A0 = S.A0;
  double w[4], beta[4], wb[4] = {0, 0, 0, 0}, Dl[4] = {0, 0, 0, 0};
  double wave = 0.0, w2 = 0.0, ts = 0.0, kappa = 0.0, ssum = 1.0;
  if (P.linear) {
    for (int l = 0; l < 4; ++l) w[l] = P.lw[l];
  } else {
    const double c1 = c[0], c2 = c[1], c3 = c[2], c4 = c[3], c5 = c[4];
    beta[0] = A0 * (c1 * c1 + c2 * c2) + A0 * A0 * (4.0 * c3 * c3 + c4 * c4 + 4.0 * c5 * c5);
    for (int f = 0; f < 3; ++f) {
      const double b = bl[f], cc = cl[f];
      beta[f + 1] = A0 * (b * b + cc * cc);
    }
    wave = Wsum * 0.25 + 1e-30;
    w2 = wave * wave;
    ts = fabs(beta[0] - beta[1]) + fabs(beta[0] - beta[2]) + fabs(beta[0] - beta[3]);
    kappa = ts * ts / 9.0;
    ssum = 0.0;
    for (int l = 0; l < 4; ++l) {
      Dl[l] = w2 * w2 * P.eps + w2 * beta[l];
      const double frac = kappa == 0.0 ? 0.0 : kappa / Dl[l];
      wb[l] = P.lw[l] * (1.0 + frac);
      ssum += wb[l];
    }
    for (int l = 0; l < 4; ++l) w[l] = wb[l] / ssum;
  }
  const Real k1 = Real(w[0] / g1);
  Real kl[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) kl[f] = Real(w[f + 1] - w[0] * P.lw[f + 1] / g1);
  const Real mxx = tb[kTblMom * kTile], mxy = tb[(kTblMom + 1) * kTile], myy = tb[(kTblMom + 2) * kTile];
  // the limiter (if any) between the coefficients and their adjoint: the
  // unlimited coefficients as the forward forms them (Step 6)
  Real la[6];
  double lW0lim;
  {
    Real R1 = k1 * c[0], R2 = k1 * c[1];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      R1 += kl[f] * bl[f];
      R2 += kl[f] * cl[f];
    }
    const Real R3 = k1 * c[2], R4 = k1 * c[3], R5 = k1 * c[4];
    const Real au[6] = {-(R3 * mxx + R4 * mxy + R5 * myy), R1, R2, R3, R4, R5};
    lim(au, la_in, la, lW0lim);
  }
  // ---- reverse
  const Real lR1 = la[1], lR2 = la[2];
  const Real lR3 = la[3] - mxx * la[0], lR4 = la[4] - mxy * la[0], lR5 = la[5] - myy * la[0];
  Real lc[5];
  lc[0] = k1 * lR1;
  lc[1] = k1 * lR2;
  lc[2] = k1 * lR3;
  lc[3] = k1 * lR4;
  lc[4] = k1 * lR5;
  const double lk1 = double(lR1 * c[0] + lR2 * c[1] + lR3 * c[2] + lR4 * c[3] + lR5 * c[4]);
  Real lbl[3], lcl[3];
  double lkl[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    lkl[f] = double(lR1 * bl[f] + lR2 * cl[f]);
    lbl[f] = kl[f] * lR1;
    lcl[f] = kl[f] * lR2;
  }
  double lWsum = 0.0;
  if (!P.linear) {
    double lw[4];
    const double ig1 = 1.0 / g1;
    lw[0] = lk1 * ig1;
    for (int f = 0; f < 3; ++f) {
      lw[0] -= lkl[f] * P.lw[f + 1] * ig1;
      lw[f + 1] = lkl[f];
    }
    // w_l = wb_l / S
    double dotw = 0.0;
    for (int l = 0; l < 4; ++l) dotw += lw[l] * w[l];
    double lwb[4];
    const double iss = 1.0 / ssum;
    for (int l = 0; l < 4; ++l) lwb[l] = (lw[l] - dotw) * iss;
    double lkappa = 0.0, lw2 = 0.0, lbeta[4] = {0, 0, 0, 0};
    if (kappa != 0.0) {
      for (int l = 0; l < 4; ++l) {
        const double iD = 1.0 / Dl[l], t = lwb[l] * P.lw[l] * iD;
        lkappa += t;
        const double lD = -t * kappa * iD;
        lw2 += lD * (2.0 * w2 * P.eps + beta[l]);
        lbeta[l] += lD * w2;
      }
    }
    const double lwave = 2.0 * wave * lw2;
    lWsum = 0.25 * lwave;
    const double lts = (2.0 / 9.0) * ts * lkappa;
    for (int l = 1; l < 4; ++l) {
      const double df = beta[0] - beta[l];
      const double sg = df > 0 ? 1.0 : (df < 0 ? -1.0 : 0.0);
      lbeta[0] += sg * lts;
      lbeta[l] -= sg * lts;
    }
    const double c1 = c[0], c2 = c[1], c3 = c[2], c4 = c[3], c5 = c[4];
    lc[0] += Real(2.0 * A0 * c1 * lbeta[0]);
    lc[1] += Real(2.0 * A0 * c2 * lbeta[0]);
    lc[2] += Real(8.0 * A0 * A0 * c3 * lbeta[0]);
    lc[3] += Real(2.0 * A0 * A0 * c4 * lbeta[0]);
    lc[4] += Real(8.0 * A0 * A0 * c5 * lbeta[0]);
    for (int f = 0; f < 3; ++f) {
      lbl[f] += Real(2.0 * A0 * double(bl[f]) * lbeta[f + 1]);
      lcl[f] += Real(2.0 * A0 * double(cl[f]) * lbeta[f + 1]);
    }
  }
  // Step 2 reverse
  Real lV[4] = {Real(0), Real(0), Real(0), Real(0)}, lY[4] = {Real(0), Real(0), Real(0), Real(0)};
  double ldW[3] = {0, 0, 0};
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const Real lt = pdx[f] * lbl[f] + pdy[f] * lcl[f];
    lV[f + 1] += lbl[f] - pdx[f] * piv[f] * lt;
    lY[f + 1] += lcl[f] - pdy[f] * piv[f] * lt;
    ldW[f] += double(piv[f] * lt);
  }
  // Step 1 reverse: c = Md dW + Z^T u, u = Q v
  Real lu[2] = {Real(0), Real(0)};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const Real* t = tb + (kTblMd + 3 * j) * kTile;
    ldW[0] += double(t[0] * lc[j]);
    ldW[1] += double(t[kTile] * lc[j]);
    ldW[2] += double(t[2 * kTile] * lc[j]);
    lu[0] += tb[(kTblZ + j) * kTile] * lc[j];
    lu[1] += tb[(kTblZ + 5 + j) * kTile] * lc[j];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const Real* t = tb + (kTblQ + 8 * k) * kTile;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      lV[l] += t[l * kTile] * lu[k];
      lY[l] += t[(4 + l) * kTile] * lu[k];
    }
  }
  // stencil inputs -> slots
  for (int s = 0; s < 4; ++s) slot[s][0] = slot[s][1] = slot[s][2] = 0.0;
  slot[0][0] += lWsum + lW0lim;
  slot[0][1] += double(lV[0]);
  slot[0][2] += double(lY[0]);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (nb[f] >= 0) {
      slot[f + 1][0] += ldW[f] + lWsum;
      slot[0][0] -= ldW[f];
      slot[f + 1][1] += double(lV[f + 1]);
      slot[f + 1][2] += double(lY[f + 1]);
    } else if (SB && gk[f] == 2) {
      // prescribed ghost: dW = Wd - W0, no derivative averages
      slot[0][0] -= ldW[f];
    } else {
      // ghost: W = W0 (dW = 0 identically), gradient reflected by I - 2 n n^T
      slot[0][0] += lWsum;
      const Real lvn = gnx[f] * lV[f + 1] + gny[f] * lY[f + 1];
      slot[0][1] += double(lV[f + 1] - Real(2) * gnx[f] * lvn);
      slot[0][2] += double(lY[f + 1] - Real(2) * gny[f] * lvn);
      if constexpr (SB && EQ == EQ_EUL) {
        if (gk[f] == 1) {
          // wall: dW = -2 n_q (m.n), also summed into W_ave; the mixed rows
          // -2 n_q (n_x R_1 + n_y R_2) with R_c the mirrored gradient of m_c
          const double lmn = -2.0 * wna[f] * (ldW[f] + lWsum);
          cross[0][0] += lmn * wnx[f];
          cross[1][0] += lmn * wny[f];
          const Real nx = gnx[f], ny = gny[f], rn = Real(2) * Real(wna[f]);
          const Real a = lV[f + 1], b = lY[f + 1];
          const Real l1x = -rn * nx * a, l2x = -rn * ny * a, l1y = -rn * nx * b, l2y = -rn * ny * b;
          const Real lv1 = -Real(2) * (nx * l1x + ny * l1y), lv2 = -Real(2) * (nx * l2x + ny * l2y);
          cross[0][1] += double(l1x + nx * lv1);
          cross[0][2] += double(l1y + ny * lv1);
          cross[1][1] += double(l2x + nx * lv2);
          cross[1][2] += double(l2y + ny * lv2);
        }
      }
    }
  }
}

}  // namespace hwe
