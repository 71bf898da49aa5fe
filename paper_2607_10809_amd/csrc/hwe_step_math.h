// Per-item arithmetic of the three step kernels (one cell-component, one
// edge lane, one cell), written as functions of plain pointers so that the
// kernels in hwe_kernels.hip are thin index maps.
//
// Layouts (internal cell order, N cells, E edges, M components):
//   wbar [M][N] double, grad [2][M][N] Real (W_x then W_y averages),
//   R [N][6][M] Real: R - Wbar_K = a0 + a1 X + a2 Y + a3 X^2 + a4 XY + a5 Y^2
//     about the centroid of K (one contiguous record per cell),
//   F [E][M] double, G [E][M] Real (one record per edge).
#pragma once

#include <type_traits>

#include "hwe_math.h"

namespace hwe {

// Contiguous records (a cell's R, an edge's F or G) moved with 16-byte
// accesses; records start 16-byte aligned (M = 4: 96 or 192 bytes per R,
// 32 per F, 16 or 32 per G).  Scalar equations fall back to element access.
template <int K, class T>
__host__ __device__ __forceinline__ void load_record(const T* __restrict__ src, T* dst) {
  if constexpr ((K * sizeof(T)) % 16 == 0) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    constexpr int W = 16 / sizeof(T);
    const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
    for (int k = 0; k < K / W; ++k) {
      const V v = s[k];
      if constexpr (W == 2) {
        dst[2 * k] = v.x;
        dst[2 * k + 1] = v.y;
      } else {
        dst[4 * k] = v.x;
        dst[4 * k + 1] = v.y;
        dst[4 * k + 2] = v.z;
        dst[4 * k + 3] = v.w;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = src[k];
  }
}
template <int K, class T>
__host__ __device__ __forceinline__ void store_record(T* __restrict__ dst, const T* src) {
  if constexpr ((K * sizeof(T)) % 16 == 0) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    constexpr int W = 16 / sizeof(T);
    V* d = reinterpret_cast<V*>(dst);
#pragma unroll
    for (int k = 0; k < K / W; ++k) {
      V v;
      if constexpr (W == 2) {
        v.x = src[2 * k];
        v.y = src[2 * k + 1];
      } else {
        v.x = src[4 * k];
        v.y = src[4 * k + 1];
        v.z = src[4 * k + 2];
        v.w = src[4 * k + 3];
      }
      d[k] = v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = src[k];
  }
}

// ------------------------------------------------------------------ table tiles
// A block of kThreads work-items copies one tile of the tiled reconstruction
// table (kTblRows rows of kTile values) into LDS with 16-byte loads.  load()
// only issues the global loads, so independent gathers can be issued before
// store() waits for them.  The stage holds (kFull + 1) * kThreads chunks; the
// lanes past the tile's end reload an earlier chunk (in bounds) into the
// padding.  Tables are allocated in whole tiles.
template <class Real, int kThreads> struct TileCopy {
  static constexpr int kChunks = kTblRows * kTile * int(sizeof(Real)) / 16;
  static constexpr int kFull = kChunks / kThreads, kRest = kChunks - kFull * kThreads;
  static constexpr int kStage = (kFull + 1) * kThreads;
  static_assert(kTblRows * kTile * sizeof(Real) % 16 == 0, "a tile is a whole number of 16-byte chunks");
  uint4 buf[kFull];
  uint4 rest;
  __device__ __forceinline__ void load(const Real* __restrict__ tbl, int tile, int t) {
    const uint4* src = reinterpret_cast<const uint4*>(tbl + size_t(tile) * (kTblRows * kTile));
#pragma unroll
    for (int r = 0; r < kFull; ++r) buf[r] = src[t + r * kThreads];
    rest = src[t + kFull * kThreads - (t < kRest ? 0 : kThreads)];
  }
  __device__ __forceinline__ void arrived_all() const {
#pragma unroll
    for (int r = 0; r < kFull; ++r) arrived(buf[r]);
    arrived(rest);
  }
  __device__ __forceinline__ void store(uint4* stage, int t) const {
#pragma unroll
    for (int r = 0; r < kFull; ++r) stage[t + r * kThreads] = buf[r];
    stage[t + kFull * kThreads] = rest;
  }
};

// ------------------------------------------------------------------ Steps 1-6
// The stencil of component q of cell i: its own average and derivative
// averages and its three face neighbours'.  All loads are issued before any
// is used: a ghost face (nbi < 0) reads the cell itself; recon_from_stencil
// replaces those values.
template <class Real> struct Stencil {
  int nbi[3];
  double W0, Wn[3], A0;  // A0: the cell's area
  Real V[4], Y[4];
};
// Every gathered value of S has arrived (arrived() in hwe_math.h).
template <class Real> __device__ __forceinline__ void stencil_arrived(const Stencil<Real>& S) {
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    arrived(S.Wn[f]);
    arrived(S.V[f + 1]);
    arrived(S.Y[f + 1]);
  }
  arrived(S.W0);
  arrived(S.A0);
  arrived(S.V[0]);
  arrived(S.Y[0]);
}
template <int EQ, class Real>
__host__ __device__ __forceinline__ Stencil<Real> gather_stencil(int i, int q, int N,
                                                                const double* __restrict__ wbar,
                                                                const Real* __restrict__ grad,
                                                                const int32_t* __restrict__ nbr,
                                                                const double* __restrict__ area) {
  constexpr int M = NComp<EQ>::m;
  Stencil<Real> S;
#pragma unroll
  for (int f = 0; f < 3; ++f) S.nbi[f] = nbr[f * N + i];
  S.A0 = area[i];
  S.W0 = wbar[q * N + i];
  S.V[0] = grad[q * N + i];
  S.Y[0] = grad[(M + q) * N + i];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int c = S.nbi[f] >= 0 ? S.nbi[f] : i;
    S.Wn[f] = wbar[q * N + c];
    S.V[f + 1] = grad[q * N + c];
    S.Y[f + 1] = grad[(M + q) * N + c];
  }
  return S;
}

// Step 1 from the factored table (tb: the cell's column, row k at
// tb[k * kTile]): u = Q (V0..V3, Y0..Y3), then c = Md (dW1..dW3) + Z^T u.
template <class Real>
__host__ __device__ __forceinline__ void step1_apply(const Real* __restrict__ tb, Real d0, Real d1, Real d2,
                                                    const Real (&V)[4], const Real (&Y)[4], Real (&c)[5]) {
  Real u[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const Real* t = tb + (kTblQ + 8 * k) * kTile;
    Real s = Real(0);
#pragma unroll
    for (int l = 0; l < 4; ++l) s += t[l * kTile] * V[l] + t[(4 + l) * kTile] * Y[l];
    u[k] = s;
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const Real* t = tb + (kTblMd + 3 * j) * kTile;
    c[j] = t[0] * d0 + t[kTile] * d1 + t[2 * kTile] * d2 + tb[(kTblZ + j) * kTile] * u[0] +
           tb[(kTblZ + 5 + j) * kTile] * u[1];
  }
}

// Reconstruction of component q of cell i (Sec. 2.2) from its stencil.
// Writes the six coefficients a0..a5 of R - Wbar (monomials about the centroid).
// tb: the cell's column of the tiled geometry table (row k at tb[k * kTile]).
// On a reflective wall (Euler) the momentum components of the ghost are
// reflected too, which mixes the two momentum rows: wbar and grad are read for
// the cell's other momentum component there.
template <int EQ, class Real>
__host__ __device__ __forceinline__ void recon_from_stencil(int i, int q, int N, int NB, const Params& P,
                                                           const Stencil<Real>& S,
                                                           const double* __restrict__ bnd_n,
                                                           const Real* __restrict__ tb,
                                                           const double* __restrict__ wbar,
                                                           const Real* __restrict__ grad, Real (&a)[6]) {
  const double W0 = S.W0;
  Real V[4], Y[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    V[l] = S.V[l];
    Y[l] = S.Y[l];
  }
  double Wsum = W0, dW[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (S.nbi[f] >= 0) {
      dW[f] = S.Wn[f] - W0;
      Wsum += S.Wn[f];
    } else {
      // ghost: K0 mirrored across the face, gradient columns reflected; a
      // prescribed face's ghost holds the prescribed state, flat
      const int b = -S.nbi[f] - 1;
      const Real nx = Real(bnd_n[b]), ny = Real(bnd_n[NB + b]);
      const double kind = bnd_n[2 * NB + b];
      const Real vn = V[0] * nx + Y[0] * ny;
      if (kind >= 2.0) {
        const double Wd = prescribed_component(P, kind, bnd_n[3 * NB + b], q);
        dW[f] = Wd - W0;
        Wsum += Wd;
        V[f + 1] = Real(0);
        Y[f + 1] = Real(0);
      } else {
        dW[f] = 0.0;
        Wsum += W0;
        V[f + 1] = V[0] - Real(2) * nx * vn;
        Y[f + 1] = Y[0] - Real(2) * ny * vn;
      }
      if constexpr (EQ == EQ_EUL) {
        if ((q == 1 || q == 2) && kind == 1.0) {
          // wall: m -> m - 2 (m.n) n in the average, and the rows of the two
          // momentum components mixed the same way
          constexpr int M = NComp<EQ>::m;
          const double dnx = bnd_n[b], dny = bnd_n[NB + b], na = q == 1 ? dnx : dny;
          const double mn = wbar[1 * size_t(N) + i] * dnx + wbar[2 * size_t(N) + i] * dny;
          dW[f] = -2.0 * na * mn;
          Wsum += dW[f];
          const Real V1 = grad[1 * size_t(N) + i], Y1 = grad[(M + 1) * size_t(N) + i];
          const Real V2 = grad[2 * size_t(N) + i], Y2 = grad[(M + 2) * size_t(N) + i];
          const Real v1 = V1 * nx + Y1 * ny, v2 = V2 * nx + Y2 * ny;
          const Real R1x = V1 - Real(2) * nx * v1, R1y = Y1 - Real(2) * ny * v1;
          const Real R2x = V2 - Real(2) * nx * v2, R2y = Y2 - Real(2) * ny * v2;
          const Real rn = Real(2) * Real(na);
          V[f + 1] = V[f + 1] - rn * (nx * R1x + ny * R2x);
          Y[f + 1] = Y[f + 1] - rn * (nx * R1y + ny * R2y);
        }
      }
    }
  }
  // Step 1: c = Md dW + Z^T (Q v); W differences formed in FP64
  Real c[5];
  step1_apply<Real>(tb, Real(dW[0]), Real(dW[1]), Real(dW[2]), V, Y, c);
  // Step 2: linear candidates on {K0, K_l}
  Real bl[3], cl[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const Real* t2 = tb + (kTblP2 + 3 * f) * kTile;
    const Real dx = t2[0], dy = t2[kTile], iv = t2[2 * kTile];
    const Real t = (Real(dW[f]) - dx * V[f + 1] - dy * Y[f + 1]) * iv;
    bl[f] = V[f + 1] + dx * t;
    cl[f] = Y[f + 1] + dy * t;
  }
  // Steps 4-5 in FP64: smoothness indicators at the centroid, nonlinear weights
  const double g1 = P.lw[0];
  double w[4];
  if (P.linear) {
#pragma unroll
    for (int l = 0; l < 4; ++l) w[l] = P.lw[l];
  } else {
    const double A0 = S.A0;
    const double c1 = c[0], c2 = c[1], c3 = c[2], c4 = c[3], c5 = c[4];
    double beta[4];
    beta[0] = A0 * (c1 * c1 + c2 * c2) + A0 * A0 * (4.0 * c3 * c3 + c4 * c4 + 4.0 * c5 * c5);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const double b = bl[f], cc = cl[f];
      beta[f + 1] = A0 * (b * b + cc * cc);
    }
    const double wave = Wsum * 0.25 + 1e-30;
    const double w2 = wave * wave;
    const double ts = fabs(beta[0] - beta[1]) + fabs(beta[0] - beta[2]) + fabs(beta[0] - beta[3]);
    const double kappa = ts * ts / 9.0;
    double ssum = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const double D = w2 * w2 * P.eps + w2 * beta[l];
      const double frac = kappa == 0.0 ? 0.0 : kappa / D;
      w[l] = P.lw[l] * (1.0 + frac);
      ssum += w[l];
    }
    const double inv = 1.0 / ssum;
#pragma unroll
    for (int l = 0; l < 4; ++l) w[l] *= inv;
  }
  // Step 6: R = (w1/g1) p1 + sum_l (w_l - w1 g_l/g1) p_l, minus Wbar_0
  const Real k1 = Real(w[0] / g1);
  Real R1 = k1 * c[0], R2 = k1 * c[1];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const Real kl = Real(w[f + 1] - w[0] * P.lw[f + 1] / g1);
    R1 += kl * bl[f];
    R2 += kl * cl[f];
  }
  const Real R3 = k1 * c[2], R4 = k1 * c[3], R5 = k1 * c[4];
  const Real* mo = tb + kTblMom * kTile;
  a[0] = -(R3 * mo[0] + R4 * mo[kTile] + R5 * mo[2 * kTile]);
  a[1] = R1;
  a[2] = R2;
  a[3] = R3;
  a[4] = R4;
  a[5] = R5;
}

// Gather and reconstruct in one call (tb as in recon_from_stencil).
template <int EQ, class Real>
__host__ __device__ __forceinline__ void recon_coeffs(int i, int q, int N, int NB, const Params& P,
                                                     const double* __restrict__ wbar, const Real* __restrict__ grad,
                                                     const int32_t* __restrict__ nbr, const double* __restrict__ bnd_n,
                                                     const Real* __restrict__ tb, const double* __restrict__ area,
                                                     Real (&a)[6]) {
  const Stencil<Real> S = gather_stencil<EQ, Real>(i, q, N, wbar, grad, nbr, area);
  recon_from_stencil<EQ, Real>(i, q, N, NB, P, S, bnd_n, tb, wbar, grad, a);
}

template <int EQ, class Real>
__host__ __device__ __forceinline__ void store_coeffs(int i, int q, int N, const Real (&a)[6], Real* __restrict__ R) {
  constexpr int M = NComp<EQ>::m;
  (void)N;
#pragma unroll
  for (int j = 0; j < 6; ++j) R[(size_t(i) * 6 + j) * M + q] = a[j];
}

// Positivity-preserving scaling of the Euler reconstruction of one cell (the
// scale limiter of Zhang and Shu cited in Sec. 3), in FP64.  a[q][0..5]: the
// coefficients of R - Wbar per component, px/py: the NP edge Gauss points of
// the cell (3 faces x 2, or x 3 with the 3-point edge rule) relative to its
// centroid.  With eps = min(1e-13, rho_bar, p_bar):
// theta_rho scales the density part so that rho >= eps at the points; then t
// is the smallest root in [0, 1] of p(Wbar + t (W - Wbar)) = eps over the
// points where p < eps, solved through
//   g(t) = 2 rho(t) (E(t) - eps/(gamma-1)) - |m(t)|^2 = A t^2 + B t + C.
// Results: theta[0] = theta_rho t, theta[1..3] = t (1 where inactive).
template <class Real, int NP>
__host__ __device__ __forceinline__ void positivity_theta(double gam, const double (&Wb)[4], const Real (&a)[4][6],
                                                         const double (&px)[NP], const double (&py)[NP],
                                                         double (&theta)[4]) {
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
#pragma unroll
  for (int k = 0; k < NP; ++k) rmin = fmin(rmin, Wb[0] + d[k][0]);
  const double th_rho = rmin < eps ? (Wb[0] - eps) / (Wb[0] - rmin) : 1.0;
  double t = 1.0;
  const double Ep = Wb[3] - eps / gm1;
  const double C = 2.0 * Wb[0] * Ep - (Wb[1] * Wb[1] + Wb[2] * Wb[2]);
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
    t = root < t ? root : t;
  }
  theta[0] = th_rho * t;
  theta[1] = theta[2] = theta[3] = t;
}

// ------------------------------------------------------------------ edge lane
// One side (0: the edge's first cell, 1: its second) at one Gauss point, in two
// parts.  edge_point_at: the reconstruction's offset d = W - Wbar at the point
// (X, Y) from the cell's centroid and its time derivatives W_t, W_tt by the
// Lax-Wendroff procedure.  edge_point: the same at Gauss point g of the
// 2-point rule (zeros when cell < 0), egp: [8][E] Gauss-point offsets from the
// centroids (side 0 points 0, 1; side 1 points 0, 1).
template <int EQ, class Real>
__host__ __device__ __forceinline__ void edge_point_at(int cell, const Params& P,
                                                      const double (&Wbd)[NComp<EQ>::m], const Real* __restrict__ R,
                                                      Real X, Real Y, Real (&dl)[NComp<EQ>::m],
                                                      Real (&Wt)[NComp<EQ>::m], Real (&Wtt)[NComp<EQ>::m]) {
  constexpr int M = NComp<EQ>::m;
  Real ac[6][M];
  load_record<6 * M>(R + size_t(cell) * (6 * M), &ac[0][0]);
  Real D[6][M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const Real a0 = ac[0][q], a1 = ac[1][q], a2 = ac[2][q], a3 = ac[3][q], a4 = ac[4][q], a5 = ac[5][q];
    dl[q] = a0 + a1 * X + a2 * Y + a3 * X * X + a4 * X * Y + a5 * Y * Y;  // W - Wbar at the point
    D[0][q] = Real(Wbd[q]) + dl[q];
    D[1][q] = a1 + Real(2) * a3 * X + a4 * Y;
    D[2][q] = a2 + a4 * X + Real(2) * a5 * Y;
    D[3][q] = Real(2) * a3;
    D[4][q] = a4;
    D[5][q] = Real(2) * a5;
  }
  lax_wendroff<EQ, Real>(P, D, Wt, Wtt);
}

template <int EQ, class Real>
__host__ __device__ __forceinline__ void edge_point(int e, int cell, int side, int g, int E, const Params& P,
                                                   const double (&Wbd)[NComp<EQ>::m], const Real* __restrict__ R,
                                                   const Real* __restrict__ egp, Real (&dl)[NComp<EQ>::m],
                                                   Real (&Wt)[NComp<EQ>::m], Real (&Wtt)[NComp<EQ>::m]) {
  constexpr int M = NComp<EQ>::m;
#pragma unroll
  for (int q = 0; q < M; ++q) dl[q] = Wt[q] = Wtt[q] = Real(0);
  if (cell < 0) return;
  const Real X = egp[(4 * side + 2 * g) * E + e];
  const Real Y = egp[(4 * side + 2 * g + 1) * E + e];
  edge_point_at<EQ, Real>(cell, P, Wbd, R, X, Y, dl, Wt, Wtt);
}

// edge_nodes: the time integrals, over the nodes of the time rule TR (0:
// 3-point Gauss-Lobatto, 1: 2-point Gauss-Legendre), of the normal-flux offset
// dH = H(Wbar + d) - H(Wbar) (AH) and of d (AD), and d at t_n + dt (AT), with
// d(tau) = dl + tau W_t + tau^2/2 W_tt.  (nx, ny): the edge's unit normal.
template <int EQ, class Real, int TR>
__host__ __device__ __forceinline__ void edge_nodes(const Params& P, double dt, const double (&Wbd)[NComp<EQ>::m],
                                                   Real nx, Real ny, const Real (&dl)[NComp<EQ>::m],
                                                   const Real (&Wt)[NComp<EQ>::m], const Real (&Wtt)[NComp<EQ>::m],
                                                   Real (&AH)[NComp<EQ>::m], Real (&AD)[NComp<EQ>::m],
                                                   Real (&AT)[NComp<EQ>::m]) {
  constexpr int M = NComp<EQ>::m;
#pragma unroll
  for (int q = 0; q < M; ++q) AH[q] = AD[q] = Real(0);
  const FluxBase<EQ, Real> base = flux_base<EQ, Real>(P, Wbd);
  // one node of the time rule: Taylor value d(tau) and the weighted sums
  auto node = [&](Real tau, Real w, Real (&dls)[M]) {
    const Real h2 = Real(0.5) * tau * tau;
    Real dH[M];
#pragma unroll
    for (int q = 0; q < M; ++q) dls[q] = dl[q] + tau * Wt[q] + h2 * Wtt[q];
    normal_flux_delta<EQ, Real>(P, base, dls, nx, ny, dH);
#pragma unroll
    for (int q = 0; q < M; ++q) {
      AH[q] += w * dH[q];
      AD[q] += w * dls[q];
    }
  };
  Real d[M];
  if constexpr (TR == 1) {
    // 2-point Gauss-Legendre, nodes (1/2 -+ sqrt(3)/6) dt, weights 1/2; the
    // interface value at dt is the Taylor polynomial there
    node(Real(kGaussLegendre2[0] * dt), Real(0.5), d);
    node(Real(kGaussLegendre2[1] * dt), Real(0.5), d);
    const Real T1 = Real(dt), h2 = Real(0.5 * dt * dt);
#pragma unroll
    for (int q = 0; q < M; ++q) AT[q] = dl[q] + T1 * Wt[q] + h2 * Wtt[q];
  } else {
    // Gauss-Lobatto nodes 0, dt/2, dt with weights 1/6, 4/6, 1/6; the node at
    // dt also gives the interface value
    node(Real(0), Real(1.0 / 6.0), d);
    node(Real(0.5 * dt), Real(4.0 / 6.0), d);
    node(Real(dt), Real(1.0 / 6.0), d);
#pragma unroll
    for (int q = 0; q < M; ++q) AT[q] = d[q];
  }
}

// Reflection of the momentum components (Euler: 1 and 2) across a line with
// unit normal n: m -> m - 2 (m.n) n.
template <class T>
__host__ __device__ __forceinline__ void reflect_momentum(T nx, T ny, T (&W)[4]) {
  const T mn = W[1] * nx + W[2] * ny;
  W[1] = W[1] - T(2) * nx * mn;
  W[2] = W[2] - T(2) * ny * mn;
}

// FP64 terms of one side at its cell average: the normal flux H(Wbar) and the
// spectral radius of d(F.n)/dW there.
template <int EQ>
__host__ __device__ __forceinline__ double side_terms(const Params& P, const double (&W)[NComp<EQ>::m], double nx,
                                                     double ny, double (&H)[NComp<EQ>::m]) {
  normal_flux<EQ, double>(P, W, nx, ny, H);
  return spectral_radius<EQ>(P, W, nx, ny);
}

// Local Lax-Friedrichs edge flux in FP64 from the Gauss-averaged side sums
// (A: first cell, O: second cell):
//   F_e = |e| (1/2)(H(W_int) + H(W_ext) - alpha (W_ext - W_int))
//       = |e| (1/2)(H(Wbar_0) + H(Wbar_1) + AH + OH - alpha (Wbar_1 - Wbar_0 + OD - AD)),
// alpha = max of the spectral radii at the two cell averages (first cell on ties).
// Boundary edges (no second cell): W_ext = W_int, F_e = |e| (H(Wbar_0) + AH).
template <int EQ, class Real>
__host__ __device__ __forceinline__ void edge_flux(int e, int E, double len, bool second, const double (&Wl)[NComp<EQ>::m],
                                                  const double (&Hl)[NComp<EQ>::m], double la,
                                                  const double (&Wr)[NComp<EQ>::m], const double (&Hr)[NComp<EQ>::m],
                                                  double lb, const Real (&AH)[NComp<EQ>::m],
                                                  const Real (&AD)[NComp<EQ>::m], const Real (&OH)[NComp<EQ>::m],
                                                  const Real (&OD)[NComp<EQ>::m], double* __restrict__ F) {
  constexpr int M = NComp<EQ>::m;
  double f[M];
  const double alpha = la >= lb ? la : lb;
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const double jump = (Wr[q] - Wl[q]) + double(OD[q] - AD[q]);
    f[q] = second ? len * 0.5 * ((Hl[q] + Hr[q]) + double(AH[q] + OH[q]) - alpha * jump)
                  : len * (Hl[q] + double(AH[q]));
  }
  store_record<M>(F + size_t(e) * M, f);
}

// Gauss average of the interface value of eq. (timeflux) at t_n + dt, as an
// offset from the mean of the two cell averages (boundary: from the one cell).
template <int EQ, class Real>
__host__ __device__ __forceinline__ void edge_value(int e, int E, bool second, const Real (&AT)[NComp<EQ>::m],
                                                   const Real (&OT)[NComp<EQ>::m], Real* __restrict__ G) {
  constexpr int M = NComp<EQ>::m;
  Real v[M];
#pragma unroll
  for (int q = 0; q < M; ++q) v[q] = second ? Real(0.5) * (AT[q] + OT[q]) : AT[q];
  store_record<M>(G + size_t(e) * M, v);
}

// ------------------------------------------------------------------ update
// eq. (flx) with FP64 accumulation (walls: the ghost average reflected), and eq. (derave2d2):  using sum_e n_e|e| = 0
// over the closed cell, |K| Vbar = sum_e n_e|e| (Wface_e - Wbar_K + G_e) where
// Wface_e = mean of the two cell averages, so a constant state gives exactly 0.
template <int EQ, class Real>
__host__ __device__ __forceinline__ void update_point(int i, int N, int E, int NB, const Params& P, double dt,
                                                     const double* __restrict__ wbar,
                                                     const double* __restrict__ bnd_n,
                                                     const int32_t* __restrict__ nbr,
                                                     const int32_t* __restrict__ cell_edge,
                                                     const Real* __restrict__ nl, const double* __restrict__ inv_area,
                                                     const double* __restrict__ F, const Real* __restrict__ G,
                                                     double* __restrict__ wout, Real* __restrict__ gout) {
  constexpr int M = NComp<EQ>::m;
  const size_t sN = size_t(N);
  double W0[M], fs[M], vs[M], ys[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    W0[q] = wbar[q * sN + i];
    fs[q] = vs[q] = ys[q] = 0.0;
  }
  // indices first, then every gather at once (a boundary face reads the cell
  // itself in place of the absent neighbour and contributes no difference)
  int ce[3], nb[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    ce[f] = cell_edge[f * sN + i];
    nb[f] = nbr[f * sN + i];
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int e = ce[f] >> 1;
    const bool second = (ce[f] & 1) != 0;
    const int c = nb[f] >= 0 ? nb[f] : i;
    const double nlx = nl[f * sN + i], nly = nl[(3 + f) * sN + i];
    double Fe[M];
    Real Ge[M];
    load_record<M>(F + size_t(e) * M, Fe);
    load_record<M>(G + size_t(e) * M, Ge);
    double d[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const double Wn = wbar[q * sN + c];
      fs[q] += second ? -Fe[q] : Fe[q];
      d[q] = 0.5 * (Wn - W0[q]);  // exactly 0 on a boundary face (Wn is the cell's own)
    }
    if (nb[f] < 0) {
      const int b = -nb[f] - 1;
      const double kind = bnd_n[2 * NB + b];
      if (kind >= 2.0) {
        // prescribed state: half the difference of the ghost average
        double Wd[M];
        prescribed_state<M>(P, kind, bnd_n[3 * NB + b], Wd);
#pragma unroll
        for (int q = 0; q < M; ++q) d[q] = 0.5 * (Wd[q] - W0[q]);
      }
      if constexpr (EQ == EQ_EUL) {
        // wall: the ghost average is the reflected one, half the difference is
        // -(m.n) n in the momentum components
        if (kind == 1.0) {
          const double bx = bnd_n[b], by = bnd_n[NB + b];
          const double mn = W0[1] * bx + W0[2] * by;
          d[1] = -mn * bx;
          d[2] = -mn * by;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const double gq = double(Ge[q]) + d[q];
      vs[q] += nlx * gq;
      ys[q] += nly * gq;
    }
  }
  const double ia = inv_area[i];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    wout[q * sN + i] = W0[q] - dt * ia * fs[q];
    gout[q * sN + i] = Real(ia * vs[q]);
    gout[(M + q) * sN + i] = Real(ia * ys[q]);
  }
}

}  // namespace hwe
