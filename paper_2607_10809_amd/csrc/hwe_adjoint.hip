// Adjoint (vector-Jacobian product) of one explicit step, for gfx950.
//
//   hwe_step_adjoint(state_n, lam_{n+1}) = J(state_n)^T lam_{n+1}
//
// Four launches on the caller's stream, none with atomics:
//   1. the forward reconstruction kernel (R of every cell at state_n), skipped
//      when the caller hands in the R that a step kept for this state;
//   2. adj_face_kernel, three work-items per cell (21 cells per wave), one per
//      face: from the cell's and the neighbour's lam_{n+1} it forms the
//      adjoints of the edge flux F_e and of the interface-value integral G_e,
//      then reverses the cell's own side of the edge (Lax-Wendroff, Taylor
//      extrapolation, offset-form normal flux at the Gauss points) and the
//      flux base terms; the three sum their results with cross-lane shuffles
//      and the first writes the cell's coefficient adjoints;
//   3. adj_recon_kernel, one work-item per (cell, component q): the reverse of
//      the reconstruction of component q (Steps 1-6, including the
//      nonlinear-weight derivatives) into four stencil "slots" (the cell
//      itself and its three neighbours); for Euler each block stages its
//      table tile through LDS, as the forward reconstruction does;
//   4. adj_gather_kernel, one work-item per (cell, component): its own slot, the slots its
//      neighbours wrote for it, the Green-Gauss terms of the derivative
//      averages and the derivative of the flux viscosity alpha (only on the
//      cell whose spectral radius the max selected).
// Meshes with reflective walls or prescribed boundary states run the
// reconstruction reverse instantiated with SB = true, and the face reverse
// twice: SB = false over every cell, and beside it, on a second stream, SB =
// true over the cells with such a face (a boundary face's flux, interface
// value, alpha and Green-Gauss terms, all local to its cell, are reversed
// there), whose outputs then replace those cells' records; the scaling
// limiter is reversed inside the reconstruction reverse (template NPT = its
// points per cell).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hwe_adjoint_math.h"
#include "hwe_internal.h"

namespace hwe {

hwe_status hip_fail(hipError_t err, const char* what);

namespace {

constexpr int kBlock = 256;


// Stencil-slot adjoints, cell-major: cell i's record holds 4 slots (itself,
// then its neighbours across faces 0-2) x 3 fields (Wbar, V, Y) x M
// components.  The Wbar field is FP64 (it adds into the cell-average adjoint,
// FP64 in both precisions): a [N][4][M] double block; the V and Y fields are
// Real, like the derivative-average adjoints they add into: a [N][4][2][M]
// block after it (FP32 in the mixed path, which halves their traffic).  A
// neighbour's slot for this cell is one M-run of each block.
template <int M> __device__ __forceinline__ size_t slot_w(int i, int sl, int q) {
  return (size_t(i) * 4 + sl) * M + q;
}
template <int M> __device__ __forceinline__ size_t slot_vy(int i, int sl, int fl, int q) {
  return ((size_t(i) * 4 + sl) * 2 + (fl - 1)) * M + q;
}
template <int M, class Real, class P> __device__ __forceinline__ auto slot_vy_block(P* slots, int N) {
  using R = std::conditional_t<std::is_const_v<P>, const Real, Real>;
  return reinterpret_cast<R*>(slots + size_t(N) * 4 * M);
}

// GP: Gauss points per edge (2, or 3 for the 3-point rule; egp holds 2 GP rows
// per side).
constexpr int kFaceCells = 21;  // cells per wave in adj_face_kernel (63 of 64 lanes)
// Blocks of the face kernel: one wave each in FP64, where a wave fills its
// SIMD's registers (finer blocks place the waves more evenly: adjoint step
// about 2% shorter), four in the mixed path.
template <class Real> constexpr int kFaceBlock = sizeof(Real) == 8 ? 64 : 256;

template <int EQ, class Real, int TR, int GP, bool SB>
__global__ __launch_bounds__(kFaceBlock<Real>, sizeof(Real) == 4 ? 2 : 1) void adj_face_kernel(
    int N, int E, int NB, Params P, double dt, const double* __restrict__ wbar, const double* __restrict__ lw,
    const Real* __restrict__ lg, const Real* __restrict__ R, const int32_t* __restrict__ nbr,
    const int32_t* __restrict__ cell_edge, const double* __restrict__ enl, const Real* __restrict__ egp,
    const double* __restrict__ inv_area, const Real* __restrict__ nl, const double* __restrict__ bnd_n,
    Real* __restrict__ lacell, double* __restrict__ lwcell, double* __restrict__ sface,
    const int32_t* __restrict__ cells, int ncells) {
  constexpr int M = NComp<EQ>::m;
  constexpr bool kWall = SB && EQ == EQ_EUL;
  const int gid = xcd_block_id() * kFaceBlock<Real> + threadIdx.x;
  const int wv = gid >> 6, wl = gid & 63;
  const int c = wl / 3, lane = wl - 3 * c;                 // lane = the face
  // SB: only the cells with a wall or prescribed face (cells[0..ncells)),
  // their outputs written compactly by list position (sface then [3][ncells])
  const int k = wv * kFaceCells + c;
  const bool valid = wl < 3 * kFaceCells && (SB ? k < ncells : k < N);
  const int i = SB ? (valid ? cells[k] : 0) : k;
  const int ic = valid ? i : N - 1;
  const size_t sN = size_t(N), sE = size_t(E), sO = SB ? size_t(ncells) : sN;
  Real la[6][M];
  double lWf[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    lWf[q] = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) la[j][q] = Real(0);
  }
  {
    const int f = lane;
    // Every load of the lane is issued before any arithmetic, in two rounds:
    // what the cell index fixes, then what the face's edge and neighbour fix
    // (nbr < 0: boundary face, no neighbour; the neighbour's loads then read
    // the cell itself and are not used).  With one wave per SIMD nothing else
    // hides a load's latency, so the waits are kept to these two.
    const int ce = cell_edge[f * sN + ic];
    const int nbv = nbr[f * sN + ic];
    double WK[M], lwK[M], lgxK[M], lgyK[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      WK[q] = wbar[q * sN + ic];
      lwK[q] = lw[q * sN + ic];
      lgxK[q] = double(lg[q * sN + ic]);
      lgyK[q] = double(lg[(M + q) * sN + ic]);
    }
    const double iaK = inv_area[ic];
    const double nlx = double(nl[f * sN + ic]), nly = double(nl[(3 + f) * sN + ic]);
    Real a[6][M];
    load_record<6 * M>(R + size_t(ic) * (6 * M), &a[0][0]);
    const int e = ce >> 1, side = ce & 1;
    const bool has = nbv >= 0;
    const int nb = has ? nbv : -1, nc = has ? nbv : ic;
    const double nx = enl[e], ny = enl[sE + e], len = enl[2 * sE + e];
    const double ianc = inv_area[nc];
    double Wc[M], lwn[M], lgxn[M], lgyn[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      Wc[q] = wbar[q * sN + nc];
      lwn[q] = lw[q * sN + nc];
      lgxn[q] = double(lg[q * sN + nc]);
      lgyn[q] = double(lg[(M + q) * sN + nc]);
    }
    Real Xg[GP], Yg[GP];
#pragma unroll
    for (int g = 0; g < GP; ++g) {
      Xg[g] = egp[(2 * GP * side + 2 * g) * sE + e];
      Yg[g] = egp[(2 * GP * side + 2 * g + 1) * sE + e];
    }
    issue_fence();
    const double sigma = side ? -1.0 : 1.0;
    double Wn[M], lF[M], lG[M];
    const double ian = has ? ianc : 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      Wn[q] = has ? Wc[q] : WK[q];
      lF[q] = has ? -dt * sigma * (iaK * lwK[q] - ian * lwn[q]) : -dt * iaK * lwK[q];
      lG[q] = has ? nlx * (iaK * lgxK[q] - ian * lgxn[q]) + nly * (iaK * lgyK[q] - ian * lgyn[q])
                  : iaK * (nlx * lgxK[q] + nly * lgyK[q]);
    }
    // SB: a boundary face may be a reflective wall (exterior: the mirror image
    // T Wbar_K, T reflecting the momentum about the face) or hold a prescribed
    // state Wx; both give the two-sided flux with the cell as side 0
    bool presc = false, wall = false;
    double Wx[M], bx = 0.0, by = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) Wx[q] = WK[q];
    if constexpr (SB) {
      if (!has) {
        const int b = -nbv - 1;
        const double kind = bnd_n[2 * size_t(NB) + b];
        presc = kind >= 2.0;
        if (presc) prescribed_state<M>(P, kind, bnd_n[3 * size_t(NB) + b], Wx);
        if constexpr (kWall) {
          wall = kind == 1.0;
          bx = bnd_n[b];
          by = bnd_n[NB + b];
          if (wall) reflect_momentum(nx, ny, Wx);
        }
      }
    }
    double alpha = 0.0, la0 = 0.0, la1 = 0.0;
    if (nb >= 0) {
      la0 = side ? spectral_radius<EQ>(P, Wn, nx, ny) : spectral_radius<EQ>(P, WK, nx, ny);
      la1 = side ? spectral_radius<EQ>(P, WK, nx, ny) : spectral_radius<EQ>(P, Wn, nx, ny);
      alpha = la0 >= la1 ? la0 : la1;
    } else if (SB && (presc || wall)) {
      la0 = spectral_radius<EQ>(P, WK, nx, ny);
      la1 = spectral_radius<EQ>(P, Wx, nx, ny);
      alpha = la0 >= la1 ? la0 : la1;
    }
    // flux base terms:  d/dWbar_K of |e| 1/2 (H(Wbar_K) + sigma alpha Wbar_K) . lF
    if (nb >= 0 || (SB && (presc || wall))) {
      normal_flux_jt<EQ>(P, WK, nx, ny, lF, 0.5 * len, lWf);
#pragma unroll
      for (int q = 0; q < M; ++q) lWf[q] += 0.5 * len * sigma * alpha * lF[q];
      if constexpr (kWall) {
        if (wall) {
          // |e| 1/2 (H(T Wbar_K) - alpha T Wbar_K), mapped back through T
          double t[M];
#pragma unroll
          for (int q = 0; q < M; ++q) t[q] = 0.0;
          normal_flux_jt<EQ>(P, Wx, nx, ny, lF, 0.5 * len, t);
#pragma unroll
          for (int q = 0; q < M; ++q) t[q] -= 0.5 * len * alpha * lF[q];
          reflect_momentum(nx, ny, t);
#pragma unroll
          for (int q = 0; q < M; ++q) lWf[q] += t[q];
        }
      }
    } else {
      normal_flux_jt<EQ>(P, WK, nx, ny, lF, len, lWf);
    }
    // the wall's mirror terms take T lF and T lG
    double TlF[M], TlG[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
      TlF[q] = lF[q];
      TlG[q] = lG[q];
    }
    if constexpr (kWall) {
      reflect_momentum(nx, ny, TlF);
      reflect_momentum(nx, ny, TlG);
    }
    double lWT[M];
#pragma unroll
    for (int q = 0; q < M; ++q) lWT[q] = 0.0;
    double sT = 0.0;
    double s = 0.0;
    auto point = [&](int g) {
      // seeds of Gauss point g (weight wg; 1/2 each with 2 points)
      const double wg = GP == 2 ? 0.5 : (g == 1 ? 8.0 / 18.0 : 5.0 / 18.0);
      Real sAH[M], sAD[M], sAT[M], sAHw[M];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        if (nb >= 0 || (SB && presc)) {
          sAH[q] = Real(wg * (0.5 * len * lF[q]));
          sAD[q] = Real(wg * (0.5 * len * sigma * alpha * lF[q]));
          sAT[q] = Real(wg * (0.5 * lG[q]));
        } else if (kWall && wall) {
          // the exterior offsets are T d: its AD and AT terms come back through T
          sAH[q] = Real(wg * (0.5 * len * lF[q]));
          sAD[q] = Real(wg * (0.5 * len * alpha * (lF[q] - TlF[q])));
          sAT[q] = Real(wg * (0.5 * (lG[q] + TlG[q])));
        } else {
          sAH[q] = Real(wg * (len * lF[q]));
          sAD[q] = Real(0);
          sAT[q] = Real(wg * lG[q]);
        }
        sAHw[q] = wall ? sAH[q] : Real(0);
      }
      const Real X = Xg[g], Y = Yg[g];
      Real ADg[M];
      edge_lane_rev<EQ, Real, TR, kWall>(P, dt, a, WK, X, Y, Real(nx), Real(ny), sAH, sAD, sAT, la, lWf, ADg, Wx,
                                         sAHw, lWT);
#pragma unroll
      for (int q = 0; q < M; ++q) {
        s += wg * lF[q] * double(ADg[q]);
        sT += wg * TlF[q] * double(ADg[q]);
      }
    };
    if constexpr (GP == 2) {
#pragma unroll
      for (int g = 0; g < 2; ++g) point(g);
    } else {
      // kept rolled: unrolling three point reversals spills
#pragma unroll 1
      for (int g = 0; g < GP; ++g) point(g);
    }
    if constexpr (SB) {
      if (presc || wall) {
        // the flux viscosity on the branch the max took (a prescribed state is
        // constant): d alpha . (-|e|/2) lF . ((W_ext - Wbar_K) + (AD_ext - AD_K))
        double jb = (wall ? sT : 0.0) - s;
#pragma unroll
        for (int q = 0; q < M; ++q) jb += lF[q] * (Wx[q] - WK[q]);
        const double sc = -0.5 * len * jb;
        if (la0 >= la1) {
          spectral_radius_grad<EQ>(P, WK, nx, ny, sc, lWf);
        } else if (kWall && wall) {
          double t[M];
#pragma unroll
          for (int q = 0; q < M; ++q) t[q] = 0.0;
          spectral_radius_grad<EQ>(P, Wx, nx, ny, sc, t);
          if constexpr (kWall) reflect_momentum(nx, ny, t);
#pragma unroll
          for (int q = 0; q < M; ++q) lWf[q] += t[q];
        }
        // Green-Gauss: half the difference of the ghost average to the cell's
        if (presc) {
#pragma unroll
          for (int q = 0; q < M; ++q) lWf[q] -= 0.5 * lG[q];
        }
        if constexpr (kWall) {
          if (wall) {
            // -(m.n) n in the momentum components; the mirror's offset base
            const double lmn = -(bx * lG[1] + by * lG[2]);
            lWf[1] += lmn * bx;
            lWf[2] += lmn * by;
            reflect_momentum(nx, ny, lWT);
#pragma unroll
            for (int q = 0; q < M; ++q) lWf[q] += lWT[q];
          }
        }
      }
    }
    if (valid) sface[f * sO + (SB ? k : ic)] = s;
  }
  // sum over the cell's three lanes into its first (lanes 3c + 1 and 3c + 2
  // reached by whole-wave DPP shifts, no LDS round trip)
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const double a1 = wave_next(lWf[q]), a2 = wave_next(a1);
    lWf[q] = (lWf[q] + a1) + a2;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const Real b1 = wave_next(la[j][q]), b2 = wave_next(b1);
      la[j][q] = (la[j][q] + b1) + b2;
    }
  }
  if (valid && lane == 0) {
    const int o = SB ? k : i;
    store_record<6 * M>(lacell + size_t(o) * (6 * M), &la[0][0]);
#pragma unroll
    for (int q = 0; q < M; ++q) lwcell[size_t(o) * M + q] = lWf[q];
  }
}

// The listed cells' face-reverse outputs (compact, by list position) copied
// over their records: one work-item per (listed cell, value), the 6M
// coefficient adjoints, then the M flux-base adjoints, then the 3 face scalars.
template <int M, class Real>
__global__ __launch_bounds__(256) void adj_face_patch_kernel(int N, int n, const int32_t* __restrict__ cells,
                                                             const Real* __restrict__ la_c,
                                                             const double* __restrict__ lw_c,
                                                             const double* __restrict__ sf_c,
                                                             Real* __restrict__ lacell, double* __restrict__ lwcell,
                                                             double* __restrict__ sface) {
  constexpr int W = 7 * M + 3;
  const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= int64_t(n) * W) return;
  const int k = int(g / W), j = int(g - int64_t(k) * W);
  const size_t i = size_t(cells[k]);
  if (j < 6 * M)
    lacell[i * (6 * M) + j] = la_c[size_t(k) * (6 * M) + j];
  else if (j < 7 * M)
    lwcell[i * M + (j - 6 * M)] = lw_c[size_t(k) * M + (j - 6 * M)];
  else
    sface[size_t(j - 7 * M) * N + i] = sf_c[size_t(j - 7 * M) * n + k];
}

// One work-item per (cell, component q): the reverse of the reconstruction of
// component q (Steps 1-6, with the nonlinear-weight derivatives) from the
// coefficient adjoints the face kernel summed, into the cell's stencil slots.
// The scaling limiter between the reconstruction and its adjoint (Euler): the
// four component lanes of a cell (an aligned quad) share the unlimited
// coefficients, the cell average and the adjoints of the scales, and each
// lane keeps its component of the limiter's reverse.  The limited
// coefficients are theta_q a_q; so la_q <- theta_q la_q + (dtheta/da)^T lth.
template <class Real, int NPT> struct ScalingLimiterRev {
  int q, N, i;
  double gam, W0;
  const double* gpc;
  __device__ __forceinline__ void operator()(const Real (&au)[6], const Real (&la)[6], Real (&lae)[6],
                                             double& lW0) const {
    Real all[4][6];
    double Wb[4], lth[4];
    double lthq = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) lthq += double(au[j]) * double(la[j]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int j = 0; j < 6; ++j) all[c][j] = quad_bcast(au[j], c);
      Wb[c] = quad_bcast(W0, c);
      lth[c] = quad_bcast(lthq, c);
    }
    double px[NPT], py[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      px[k] = gpc[(2 * k) * size_t(N) + i];
      py[k] = gpc[(2 * k + 1) * size_t(N) + i];
    }
    double th[4];
    positivity_theta<Real, NPT>(gam, Wb, all, px, py, th);
    double lall[4][6], lWb[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 6; ++j) lall[c][j] = 0.0;
    positivity_theta_rev<Real, NPT>(gam, Wb, all, px, py, lth, lall, lWb);
    const Real tq = Real(q == 0 ? th[0] : (q == 1 ? th[1] : (q == 2 ? th[2] : th[3])));
    double lq[6] = {lall[0][0], lall[0][1], lall[0][2], lall[0][3], lall[0][4], lall[0][5]};
    double lw = lWb[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
#pragma unroll
      for (int j = 0; j < 6; ++j) lq[j] = q == c ? lall[c][j] : lq[j];
      lw = q == c ? lWb[c] : lw;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) lae[j] = tq * la[j] + Real(lq[j]);
    lW0 = lw;
  }
};

// NPT: the limiter's points per cell (0: no limiter, 6, or 9 with the
// 3-point edge rule).
template <int EQ, class Real, bool SB, int NPT>
__global__ __launch_bounds__(kBlock) void adj_recon_kernel(
    int N, int NB, Params P, const double* __restrict__ wbar, const Real* __restrict__ grad,
    const int32_t* __restrict__ nbr, const double* __restrict__ bnd_n, const Real* __restrict__ tbl,
    const double* __restrict__ area, const double* __restrict__ gpc, const Real* __restrict__ lacell,
    const double* __restrict__ lwcell, double* __restrict__ slots) {
  constexpr int M = NComp<EQ>::m;
  const int blk = xcd_block_id();
  const int gid = blk * kBlock + threadIdx.x;
  const int i = gid / M, q = gid - (gid / M) * M;
  Real laq[6];
  double slot[4][3], lw0;  // lw0: the face kernel's direct adjoint of the cell average
  if constexpr (EQ == EQ_EUL) {
    // one block per table tile, staged through LDS as in the forward reconstruction
    static_assert(kBlock == kTile * 4, "one Euler block per table tile");
    using Copy = TileCopy<Real, kBlock>;
    __shared__ uint4 stage[Copy::kStage];
    Copy tile;
    tile.load(tbl, blk, threadIdx.x);
    const int ic = i < N ? i : N - 1;
    const Stencil<Real> S = gather_stencil<EQ, Real>(ic, q, N, wbar, grad, nbr, area);
#pragma unroll
    for (int j = 0; j < 6; ++j) laq[j] = lacell[(size_t(ic) * 6 + j) * M + q];
    lw0 = lwcell[size_t(ic) * M + q];
    // the gathers arrive with the table tile, before its LDS store and the
    // barrier (left to itself the compiler issues them after the barrier: a
    // third round of latency)
    tile.arrived_all();
    stencil_arrived(S);
    arrived(lw0);
#pragma unroll
    for (int j = 0; j < 6; ++j) arrived(laq[j]);
    tile.store(stage, threadIdx.x);
    __syncthreads();
    if (i >= N) return;  // whole cells: the four lanes of a quad leave together
    double cross[2][3] = {{0, 0, 0}, {0, 0, 0}};
    const Real* tb = reinterpret_cast<const Real*>(stage) + (i % kTile);
    if constexpr (NPT > 0) {
      const ScalingLimiterRev<Real, NPT> lim{q, N, i, P.gam, S.W0, gpc};
      recon_rev<EQ, Real, SB>(i, NB, P, S, bnd_n, tb, laq, slot, q, N, wbar, grad, cross, lim);
    } else {
      recon_rev<EQ, Real, SB>(i, NB, P, S, bnd_n, tb, laq, slot, q, N, wbar, grad, cross);
    }
    if constexpr (SB) {
      // wall ghosts: the momentum lanes (q = 1, 2 of the quad) exchange the
      // terms each produced for the other's component
      static_assert(kBlock % 64 == 0 && M == 4, "a cell's four lanes form an aligned quad");
      constexpr int kSwap12 = 3 | (2 << 2) | (1 << 4) | (0 << 6);  // lanes 0<->3, 1<->2
#pragma unroll
      for (int fl = 0; fl < 3; ++fl) {
        const double own = q == 1 ? cross[0][fl] : (q == 2 ? cross[1][fl] : 0.0);
        const double give = q == 1 ? cross[1][fl] : (q == 2 ? cross[0][fl] : 0.0);
        slot[0][fl] += own + quad_perm<kSwap12>(give);
      }
    }
  } else {
    if (i >= N) return;
    const Stencil<Real> S = gather_stencil<EQ, Real>(i, q, N, wbar, grad, nbr, area);
#pragma unroll
    for (int j = 0; j < 6; ++j) laq[j] = lacell[(size_t(i) * 6 + j) * M + q];
    lw0 = lwcell[size_t(i) * M + q];
    recon_rev<EQ, Real, SB>(i, NB, P, S, bnd_n, tbl + tbl_col(i), laq, slot, q, N, wbar, grad, nullptr);
  }
  slot[0][0] += lw0;
  Real* vy = slot_vy_block<M, Real>(slots, N);
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    slots[slot_w<M>(i, sl, q)] = slot[sl][0];
    vy[slot_vy<M>(i, sl, 1, q)] = Real(slot[sl][1]);
    vy[slot_vy<M>(i, sl, 2, q)] = Real(slot[sl][2]);
  }
}

// One work-item per (cell, component q).  Every load is issued before the
// arithmetic that uses it, with boundary faces (no neighbour) reading the cell
// itself and contributing nothing: the faces' index loads, then one round of
// data gathers.  The flux-viscosity term needs the whole state vectors of both
// cells; each component's work-item forms it and keeps its own component.
template <int EQ, class Real>
__global__ __launch_bounds__(kBlock) void adj_gather_kernel(
    int N, int E, Params P, double dt, const double* __restrict__ wbar, const double* __restrict__ lw,
    const Real* __restrict__ lg, const int32_t* __restrict__ nbr, const int32_t* __restrict__ nbr_back,
    const int32_t* __restrict__ cell_edge, const double* __restrict__ enl, const double* __restrict__ inv_area,
    const Real* __restrict__ nl, const double* __restrict__ slots, const double* __restrict__ sface,
    double* __restrict__ lw_out, Real* __restrict__ lg_out) {
  constexpr int M = NComp<EQ>::m;
  const int gid = xcd_block_id() * kBlock + threadIdx.x;
  const int i = gid / M, q = gid - (gid / M) * M;
  if (i >= N) return;
  const size_t sN = size_t(N), sE = size_t(E);
  const Real* vy = slot_vy_block<M, Real>(slots, N);
  // per face: neighbour, back-slot, edge and side, n|e| of the cell's face,
  // the edge normal and length, and the two sides' point sums of the face
  // kernel; per component: the cell's average and its adjoint
  int nbf[3], bkf[3], cef[3];
  double nlxf[3], nlyf[3], nxf[3], nyf[3], lenf[3], sownf[3], sothf[3];
  double WK[M], lwK[M];
  // the neighbours' values for every face, issued as soon as the neighbour
  // indices are known (Euler: each component lane loads its own component,
  // broadcast by DPP later)
  constexpr int MC = M == 4 ? 1 : M;
  double sWf[3], sVf[3], sYf[3], lgxnf[3], lgynf[3], ianf[3], Wcf[3][MC], lwcf[3][MC];
  auto load_neighbours = [&]() {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const bool has = nbf[f] >= 0;
      const int nb = has ? nbf[f] : i;
      const int bk = has ? bkf[f] : 0;
      sWf[f] = slots[slot_w<M>(nb, 1 + bk, q)];
      sVf[f] = double(vy[slot_vy<M>(nb, 1 + bk, 1, q)]);
      sYf[f] = double(vy[slot_vy<M>(nb, 1 + bk, 2, q)]);
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const int cq = M == 4 ? q : c;
        Wcf[f][c] = wbar[cq * sN + nb];
        lwcf[f][c] = lw[cq * sN + nb];
      }
      lgxnf[f] = double(lg[q * sN + nb]);
      lgynf[f] = double(lg[(M + q) * sN + nb]);
      ianf[f] = inv_area[nb];
    }
  };
  // the cell's own values
  const double iaK = inv_area[i];
  const double lgxK = double(lg[q * sN + i]), lgyK = double(lg[(M + q) * sN + i]);
  double aW = slots[slot_w<M>(i, 0, q)];
  double aV = double(vy[slot_vy<M>(i, 0, 1, q)]);
  double aY = double(vy[slot_vy<M>(i, 0, 2, q)]);
  if constexpr (M == 4) {
    // the quad's four lanes are the cell's components: a value the whole quad
    // needs is loaded once (lane f for face f) and broadcast by DPP
    const int fq = q < 3 ? q : 0;
    const int nb_l = nbr[fq * sN + i], bk_l = nbr_back[fq * sN + i], ce_l = cell_edge[fq * sN + i];
    const bool has_l = nb_l >= 0;
    const int e_l = ce_l >> 1;
    const double nlx_l = double(nl[fq * sN + i]), nly_l = double(nl[(3 + fq) * sN + i]);
    const double nx_l = enl[e_l], ny_l = enl[sE + e_l], len_l = enl[2 * sE + e_l];
    const double so_l = sface[fq * sN + i];
    const double st_l = sface[(has_l ? bk_l : 0) * sN + (has_l ? nb_l : i)];
    const double WKq = wbar[q * sN + i], lwKq = lw[q * sN + i];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      nbf[f] = quad_bcast(nb_l, f);
      bkf[f] = quad_bcast(bk_l, f);
      cef[f] = quad_bcast(ce_l, f);
    }
    load_neighbours();
    issue_fence();
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      nlxf[f] = quad_bcast(nlx_l, f);
      nlyf[f] = quad_bcast(nly_l, f);
      nxf[f] = quad_bcast(nx_l, f);
      nyf[f] = quad_bcast(ny_l, f);
      lenf[f] = quad_bcast(len_l, f);
      sownf[f] = quad_bcast(so_l, f);
      sothf[f] = quad_bcast(st_l, f);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
      WK[c] = quad_bcast(WKq, c);
      lwK[c] = quad_bcast(lwKq, c);
    }
  } else {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      nbf[f] = nbr[f * sN + i];
      bkf[f] = nbr_back[f * sN + i];
      cef[f] = cell_edge[f * sN + i];
      const bool has = nbf[f] >= 0;
      const int e = cef[f] >> 1;
      nlxf[f] = double(nl[f * sN + i]);
      nlyf[f] = double(nl[(3 + f) * sN + i]);
      nxf[f] = enl[e];
      nyf[f] = enl[sE + e];
      lenf[f] = enl[2 * sE + e];
      sownf[f] = sface[f * sN + i];
      sothf[f] = sface[(has ? bkf[f] : 0) * sN + (has ? nbf[f] : i)];
    }
    load_neighbours();
#pragma unroll
    for (int c = 0; c < M; ++c) {
      WK[c] = wbar[c * sN + i];
      lwK[c] = lw[c * sN + i];
    }
    issue_fence();
  }
  double aWall[M];  // flux-viscosity adjoint, all components
#pragma unroll
  for (int c = 0; c < M; ++c) aWall[c] = 0.0;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const bool has = nbf[f] >= 0;
    const int side = cef[f] & 1;
    const double sW = sWf[f], sV = sVf[f], sY = sYf[f];
    double Wn[M], lwn[M];
    if constexpr (M == 4) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        Wn[c] = quad_bcast(Wcf[f][0], c);
        lwn[c] = quad_bcast(lwcf[f][0], c);
      }
    } else {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        Wn[c] = Wcf[f][c];
        lwn[c] = lwcf[f][c];
      }
    }
    const double lgxn = lgxnf[f], lgyn = lgynf[f];
    const double ian = ianf[f];
    const double nlx = nlxf[f], nly = nlyf[f];
    const double nx = nxf[f], ny = nyf[f], len = lenf[f];
    const double sown = sownf[f], soth = sothf[f];
    // every value feeds a select, so no load waits behind a branch
    // Green-Gauss: |K| Vbar_K includes n|e| (Wbar_nb - Wbar_K)/2 (and the neighbour the mirror term)
    const double gg = -0.5 * (nlx * (iaK * lgxK + ian * lgxn) + nly * (iaK * lgyK + ian * lgyn));
    aW += has ? sW + gg : 0.0;
    aV += has ? sV : 0.0;
    aY += has ? sY : 0.0;
    // flux viscosity: alpha = max(lambda(Wbar_0), lambda(Wbar_1)), first cell on ties;
    // its derivative goes to the cell whose spectral radius the max selected
    const double lK = spectral_radius<EQ>(P, WK, nx, ny), ln = spectral_radius<EQ>(P, Wn, nx, ny);
    const double l0 = side == 0 ? lK : ln, l1 = side == 0 ? ln : lK;
    const bool mine = has && ((l0 >= l1) ? (side == 0) : (side == 1));
    const double ia0 = side == 0 ? iaK : ian, ia1 = side == 0 ? ian : iaK;
    double jb = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const double lw0 = side == 0 ? lwK[c] : lwn[c], lw1 = side == 0 ? lwn[c] : lwK[c];
      const double W0 = side == 0 ? WK[c] : Wn[c], W1 = side == 0 ? Wn[c] : WK[c];
      const double lFq = -dt * (ia0 * lw0 - ia1 * lw1);
      jb += lFq * (W1 - W0);
    }
    const double s0 = side == 0 ? sown : soth, s1 = side == 0 ? soth : sown;
    jb += s1 - s0;
    spectral_radius_grad<EQ>(P, WK, nx, ny, mine ? -0.5 * len * jb : 0.0, aWall);
  }
  double av = aWall[0], lq = lwK[0];
#pragma unroll
  for (int c = 1; c < M; ++c) {
    av = q == c ? aWall[c] : av;
    lq = q == c ? lwK[c] : lq;
  }
  lw_out[q * sN + i] = lq + aW + av;
  lg_out[q * sN + i] = Real(aV);
  lg_out[(M + q) * sN + i] = Real(aY);
}

unsigned grid_for(int64_t items) { return unsigned((items + kBlock - 1) / kBlock); }

template <int EQ, class Real>
hwe_status adjoint_impl(hwe_mesh_s* M, const Params& P, const double* wbar, const Real* grad, const double* lw,
                        const Real* lg, double* lw_out, Real* lg_out, double dt, hipStream_t st, const Real* tbl,
                        const Real* nl, const Real* egp, const Real* R) {
  const HostMesh& h = M->h;
  const DevMesh& d = M->d;
  const int N = int(h.N), E = int(h.E), NB = int(h.NB);
  auto face_grid = [](int64_t cells) {
    const int64_t waves = (cells + kFaceCells - 1) / kFaceCells;
    return dim3{unsigned((waves * 64 + kFaceBlock<Real> - 1) / kFaceBlock<Real>)};
  };
  const dim3 grid = face_grid(N), sb_grid = face_grid(d.n_sb);
  Real* lacell = static_cast<Real*>(d.lacell);
  const bool sb = h.special_bnd;
  // Every cell by the kernel without special boundaries (its registers fit);
  // beside it, on the handle's second stream, the cells with a wall or
  // prescribed face by the kernel that treats them (it spills and runs few
  // waves, on the double Mach mesh 1% of the cells: alone it would leave the
  // chip idle for its latency), into compact buffers that are copied over
  // those cells' records once both are done.
  const bool split = sb && d.n_sb > 0;
  hipStream_t sst = static_cast<hipStream_t>(d.sb_stream);
  if (split) {
    hipError_t e1 = hipEventRecord(static_cast<hipEvent_t>(d.sb_fork), st);
    if (e1 != hipSuccess) return hip_fail(e1, "hipEventRecord");
    e1 = hipStreamWaitEvent(sst, static_cast<hipEvent_t>(d.sb_fork), 0);
    if (e1 != hipSuccess) return hip_fail(e1, "hipStreamWaitEvent");
  }
#define HWE_ADJ_CELL(TRV, GPV)                                                                                        \
  do {                                                                                                                \
    if (split)                                                                                                        \
      hipLaunchKernelGGL((adj_face_kernel<EQ, Real, TRV, GPV, true>), sb_grid, dim3(kFaceBlock<Real>), 0, sst, N, E,    \
                         NB, P, dt, wbar, lw, lg, R, d.nbr, d.cell_edge, d.enl, egp, d.inv_area, nl, d.bnd_n,         \
                         static_cast<Real*>(d.sb_la), d.sb_lw, d.sb_sface, d.sb_cells, d.n_sb);                      \
    hipLaunchKernelGGL((adj_face_kernel<EQ, Real, TRV, GPV, false>), grid, dim3(kFaceBlock<Real>), 0, st, N, E, NB, P,  \
                       dt, wbar, lw, lg, R, d.nbr, d.cell_edge, d.enl, egp, d.inv_area, nl, d.bnd_n, lacell, d.lwcell, \
                       d.sface, nullptr, 0);                                                                        \
  } while (0)
  if (M->opts.edge_rule == 3) {
    if (P.time_rule == 1)
      HWE_ADJ_CELL(1, 3);
    else
      HWE_ADJ_CELL(0, 3);
  } else if (P.time_rule == 1) {
    HWE_ADJ_CELL(1, 2);
  } else {
    HWE_ADJ_CELL(0, 2);
  }
#undef HWE_ADJ_CELL
  if (split) {
    hipError_t e1 = hipEventRecord(static_cast<hipEvent_t>(d.sb_join), sst);
    if (e1 != hipSuccess) return hip_fail(e1, "hipEventRecord");
    e1 = hipStreamWaitEvent(st, static_cast<hipEvent_t>(d.sb_join), 0);
    if (e1 != hipSuccess) return hip_fail(e1, "hipStreamWaitEvent");
    constexpr int W = 7 * NComp<EQ>::m + 3;
    hipLaunchKernelGGL((adj_face_patch_kernel<NComp<EQ>::m, Real>), dim3(grid_for(int64_t(d.n_sb) * W)), dim3(kBlock),
                       0, st, N, d.n_sb, d.sb_cells, static_cast<const Real*>(d.sb_la), d.sb_lw, d.sb_sface, lacell,
                       d.lwcell, d.sface);
  }
  const dim3 rgrid(grid_for(int64_t(N) * NComp<EQ>::m));
#define HWE_ADJ_RECON(SBV, NPTV)                                                                                    \
  hipLaunchKernelGGL((adj_recon_kernel<EQ, Real, SBV, NPTV>), rgrid, dim3(kBlock), 0, st, N, NB, P, wbar, grad,     \
                     d.nbr, d.bnd_n, tbl, d.area, d.gpc, lacell, d.lwcell, d.slots)
  const int npt = (EQ == EQ_EUL && P.positivity) ? (M->opts.edge_rule == 3 ? 9 : 6) : 0;
  if constexpr (EQ == EQ_EUL) {
    if (npt == 6) {
      if (sb)
        HWE_ADJ_RECON(true, 6);
      else
        HWE_ADJ_RECON(false, 6);
    } else if (npt == 9) {
      if (sb)
        HWE_ADJ_RECON(true, 9);
      else
        HWE_ADJ_RECON(false, 9);
    }
  }
  if (npt == 0) {
    if (sb)
      HWE_ADJ_RECON(true, 0);
    else
      HWE_ADJ_RECON(false, 0);
  }
#undef HWE_ADJ_RECON
  hipLaunchKernelGGL((adj_gather_kernel<EQ, Real>), dim3(grid_for(int64_t(N) * NComp<EQ>::m)), dim3(kBlock), 0, st, N, E, P, dt, wbar, lw, lg,
                     d.nbr, d.nbr_back, d.cell_edge, d.enl, d.inv_area, nl, d.slots, d.sface, lw_out, lg_out);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  return HWE_OK;
}

}  // namespace

hwe_status launch_adjoint(hwe_mesh_s* M, const double* wbar_n, const void* grad_n, const void* R_n, const double* lw,
                          const void* lg, double* lw_out, void* lg_out, double dt, void* stream) {
  if (!R_n) {
    hwe_status s = launch_recon(M, wbar_n, grad_n, M->d.R, M->time + 0.5 * dt, stream);
    if (s != HWE_OK) return s;
    R_n = M->d.R;
  }
  Params P = params_of(M->opts);
  P.tb = M->time + 0.5 * dt;  // as the step: moving boundary states at the middle of the step
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevMesh& d = M->d;
  if (M->opts.prec == HWE_FP64) {
    auto g = static_cast<const double*>(grad_n);
    auto l = static_cast<const double*>(lg);
    auto o = static_cast<double*>(lg_out);
    switch (M->opts.eq) {
      case HWE_ADVECTION:
        return adjoint_impl<EQ_ADV, double>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tbl, d.nl, d.egp, static_cast<const double*>(R_n));
      case HWE_BURGERS:
        return adjoint_impl<EQ_BUR, double>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tbl, d.nl, d.egp, static_cast<const double*>(R_n));
      default:
        return adjoint_impl<EQ_EUL, double>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tbl, d.nl, d.egp, static_cast<const double*>(R_n));
    }
  }
  auto g = static_cast<const float*>(grad_n);
  auto l = static_cast<const float*>(lg);
  auto o = static_cast<float*>(lg_out);
  switch (M->opts.eq) {
    case HWE_ADVECTION:
      return adjoint_impl<EQ_ADV, float>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tblf, d.nlf, d.egpf, static_cast<const float*>(R_n));
    case HWE_BURGERS:
      return adjoint_impl<EQ_BUR, float>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tblf, d.nlf, d.egpf, static_cast<const float*>(R_n));
    default:
      return adjoint_impl<EQ_EUL, float>(M, P, wbar_n, g, lw, l, lw_out, o, dt, st, d.tblf, d.nlf, d.egpf, static_cast<const float*>(R_n));
  }
}

}  // namespace hwe
