// HIP kernels of the explicit ADER-HWENO step for gfx950, and their launchers.
// The per-item arithmetic lives in hwe_step_math.h.
//
// One step = three kernels on the caller's stream, none of which uses atomics:
//   recon_kernel  : one work-item per cell.  Gathers the 4-cell stencil, applies
//                   the precomputed least-squares maps (Steps 1-2), smoothness
//                   indicators and nonlinear weights in FP64 (Steps 4-5) and
//                   writes the final reconstruction R - Wbar (Step 6) as six
//                   monomial coefficients per component.
//   edge_kernel   : four work-items per edge: (side, Gauss point).  Each
//                   evaluates R and its derivatives at its point, runs the
//                   Lax-Wendroff procedure, the Taylor extrapolation at the
//                   Lobatto nodes 0, dt/2, dt, and the time integral of the
//                   normal flux; lanes are then combined with cross-lane
//                   shuffles into the local Lax-Friedrichs edge flux F_e and the
//                   edge integral of the interface value at t_n + dt.
//   edge3_kernel  : the same with the 3-point edge rule, eight work-items per
//                   edge (one idle lane per side).
//   update_kernel : one work-item per cell gathers its three edges: eq. (flx)
//                   accumulated in FP64, and the Green-Gauss derivative
//                   averages, eq. (derave2d2), written in a form that is exactly
//                   zero for a constant state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <sstream>

#include "hwe_internal.h"
#include "hwe_math.h"
#include "hwe_step_math.h"

namespace hwe {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- kernels
// One work-item per (cell, component); the M lanes of a cell are adjacent.
// For Euler a block covers exactly one table tile (64 cells x 4 components):
// the tile's tables are one contiguous block, staged into LDS with 16-byte
// loads that are all in flight together, while the stencil gathers proceed.
// Euler: the four component lanes of a cell (an aligned quad) transpose
// their six coefficients with DPP exchanges so that lane q writes row q of the
// cell's [6][4] record (one 16-byte store in FP32, two in FP64) and half of
// rows 4-5, instead of six scalar stores each.  R is 16-byte aligned.
template <class Real>
__device__ __forceinline__ void store_coeffs_quad(int i, int q, const Real (&a)[6], Real* __restrict__ R,
                                                  bool valid) {
  Real t[4] = {a[0], a[1], a[2], a[3]};
  quad_transpose4(t, q);  // rows 0-3
  // rows 4-5: lane q takes entries 16 + 2q and 17 + 2q of the record, i.e.
  // row 4 + q/2, columns 2 (q mod 2) and 2 (q mod 2) + 1
  constexpr int kEven = 0 | (2 << 2) | (0 << 4) | (2 << 6), kOdd = 1 | (3 << 2) | (1 << 4) | (3 << 6);
  const Real x4 = quad_perm<kEven>(a[4]), x5 = quad_perm<kEven>(a[5]);
  const Real y4 = quad_perm<kOdd>(a[4]), y5 = quad_perm<kOdd>(a[5]);
  const Real b[2] = {(q >> 1) ? x5 : x4, (q >> 1) ? y5 : y4};
  if (!valid) return;
  Real* rec = R + size_t(i) * 24;
  store_record<4>(rec + 4 * q, t);
  if constexpr (sizeof(Real) == 8) {
    store_record<2>(rec + 16 + 2 * q, b);
  } else {
    float2 v;
    v.x = b[0];
    v.y = b[1];
    *reinterpret_cast<float2*>(rec + 16 + 2 * q) = v;
  }
}

// NPT: the limiter's points per cell (6, or 9 with the 3-point edge rule);
// 0 compiles the limiter out (fewer registers, which lets the kernel's waves
// share a SIMD with a long adjoint wave when a reverse sweep recomputes a
// segment beside the adjoints).
template <int EQ, class Real, int NPT>
__global__ __launch_bounds__(kBlock) void recon_kernel(int N, int NB, Params P, const double* __restrict__ wbar,
                                                        const Real* __restrict__ grad,
                                                        const int32_t* __restrict__ nbr,
                                                        const double* __restrict__ bnd_n,
                                                        const Real* __restrict__ tbl,
                                                        const double* __restrict__ area,
                                                        const double* __restrict__ gpc, Real* __restrict__ R) {
  constexpr int M = NComp<EQ>::m;
  const int blk = xcd_block_id();
  const int gid = blk * kBlock + threadIdx.x;
  const int i = gid / M, q = gid - (gid / M) * M;
  if constexpr (EQ == EQ_EUL) {
    static_assert(kBlock == kTile * 4, "one Euler block per table tile");
    using Copy = TileCopy<Real, kBlock>;
    __shared__ uint4 stage[Copy::kStage];
    Copy tile;
    tile.load(tbl, blk, threadIdx.x);
    // all four component lanes of a cell stay active for the limiter's shuffles
    const bool valid = i < N;
    const int ic = valid ? i : N - 1;
    const Stencil<Real> S = gather_stencil<EQ, Real>(ic, q, N, wbar, grad, nbr, area);
    // the limiter's points, loaded with the stencil rather than after the arithmetic
    constexpr int kPts = NPT > 0 ? NPT : 1;
    double px[kPts], py[kPts];
    if constexpr (NPT > 0) {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        px[k] = gpc[(2 * k) * size_t(N) + ic];
        py[k] = gpc[(2 * k + 1) * size_t(N) + ic];
      }
    }
    // the table tile and every gather arrive together, in two rounds (the
    // neighbour indices, then the rest), before the LDS store and the barrier
    tile.arrived_all();
    stencil_arrived(S);
    if constexpr (NPT > 0) {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        arrived(px[k]);
        arrived(py[k]);
      }
    }
    tile.store(stage, threadIdx.x);
    __syncthreads();
    const Real* tb = reinterpret_cast<const Real*>(stage) + (i % kTile);
    Real a[6];
    recon_from_stencil<EQ, Real>(ic, q, N, NB, P, S, bnd_n, tb, wbar, grad, a);
    if constexpr (NPT > 0) {
      // the cell's four component lanes are an aligned quad
      Real all[4][6];
      double Wb[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int j = 0; j < 6; ++j) all[c][j] = quad_bcast(a[j], c);
        Wb[c] = quad_bcast(S.W0, c);
      }
      double th[4];
      positivity_theta<Real, NPT>(P.gam, Wb, all, px, py, th);
      const Real tq = Real(th[q]);
#pragma unroll
      for (int j = 0; j < 6; ++j) a[j] *= tq;
    }
    store_coeffs_quad<Real>(i, q, a, R, valid);
  } else {
    if (i >= N) return;
    Real a[6];
    recon_coeffs<EQ, Real>(i, q, N, NB, P, wbar, grad, nbr, bnd_n, tbl + tbl_col(i), area, a);
    store_coeffs<EQ, Real>(i, q, N, a, R);
  }
}

// Four work-items per edge (side, Gauss point), adjacent in the wave: lane
// 4k + 2 side + g.  Every lane loads its side's cell, cell average and the
// edge normal; the Gauss points are combined with quad_perm exchanges, then
// the (side 0) lanes take the other side's sums and FP64 terms the same way.
// On a reflective wall the second side is the first one's mirror image.
template <int EQ, class Real, int TR>
__global__ __launch_bounds__(kBlock) void edge_kernel(int E, int N, int NB, Params P, double dt,
                                                       const double* __restrict__ wbar,
                                                       const Real* __restrict__ R,
                                                       const int32_t* __restrict__ ecell,
                                                       const double* __restrict__ bnd_n,
                                                       const double* __restrict__ enl,
                                                       const Real* __restrict__ egp, double* __restrict__ F,
                                                       Real* __restrict__ G) {
  constexpr int M = NComp<EQ>::m;
  const int gid = xcd_block_id() * kBlock + threadIdx.x;
  const int e = gid >> 2, side = (gid >> 1) & 1, g = gid & 1;
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  // second cell: -1 on a transmissive boundary, -2 on a reflective wall,
  // -3 - b on prescribed boundary face b; a lane without a cell reads the
  // edge's first cell
  const int cell = valid ? ecell[side * E + ec] : -1;
  const int cc = cell >= 0 ? cell : ecell[ec];
  const double nx = enl[ec], ny = enl[E + ec], len = enl[2 * E + ec];
  double Wb[M];
#pragma unroll
  for (int q = 0; q < M; ++q) Wb[q] = wbar[q * size_t(N) + cc];
  Real dl[M], Wt[M], Wtt[M];
  edge_point<EQ, Real>(ec, cell, side, g, E, P, Wb, R, egp, dl, Wt, Wtt);
  const bool wall = cell == -2;
  // a prescribed exterior is a flat cell holding the state (no offsets)
  const bool presc = cell <= -3;
  if (presc) {
    const int b = -cell - 3;
    prescribed_state<M>(P, bnd_n[2 * size_t(NB) + b], bnd_n[3 * size_t(NB) + b], Wb);
  }
  if constexpr (EQ == EQ_EUL) {
    // the exterior of a wall is the interior with its momentum reflected: the
    // wall lane takes the first side's point values from its quad partner
    if (__ballot(wall) != 0) {  // uniform over the wave
      Real pdl[M], pWt[M], pWtt[M];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        pdl[q] = quad_perm<kQuadXor2>(dl[q]);
        pWt[q] = quad_perm<kQuadXor2>(Wt[q]);
        pWtt[q] = quad_perm<kQuadXor2>(Wtt[q]);
      }
      if (wall) {
        const Real rx = Real(nx), ry = Real(ny);
        reflect_momentum(rx, ry, pdl);
        reflect_momentum(rx, ry, pWt);
        reflect_momentum(rx, ry, pWtt);
        reflect_momentum(nx, ny, Wb);
#pragma unroll
        for (int q = 0; q < M; ++q) {
          dl[q] = pdl[q];
          Wt[q] = pWt[q];
          Wtt[q] = pWtt[q];
        }
      }
    }
  }
  Real AH[M], AD[M], AT[M];
#pragma unroll
  for (int q = 0; q < M; ++q) AH[q] = AD[q] = AT[q] = Real(0);
  if (cell >= 0 || wall || presc) edge_nodes<EQ, Real, TR>(P, dt, Wb, Real(nx), Real(ny), dl, Wt, Wtt, AH, AD, AT);
  double Hb[M];
  const double lam = side_terms<EQ>(P, Wb, nx, ny, Hb);
  // Gauss points (weights 1/2 each): combine lanes g = 0, 1
#pragma unroll
  for (int q = 0; q < M; ++q) {
    AH[q] = Real(0.5) * (AH[q] + quad_perm<kQuadXor1>(AH[q]));
    AD[q] = Real(0.5) * (AD[q] + quad_perm<kQuadXor1>(AD[q]));
    AT[q] = Real(0.5) * (AT[q] + quad_perm<kQuadXor1>(AT[q]));
  }
  // the other side's sums and FP64 terms
  Real OH[M], OD[M], OT[M];
  double Wo[M], Ho[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    OH[q] = quad_perm<kQuadXor2>(AH[q]);
    OD[q] = quad_perm<kQuadXor2>(AD[q]);
    OT[q] = quad_perm<kQuadXor2>(AT[q]);
    Wo[q] = quad_perm<kQuadXor2>(Wb[q]);
    Ho[q] = quad_perm<kQuadXor2>(Hb[q]);
  }
  const double lo = quad_perm<kQuadXor2>(lam);
  const bool second = quad_perm<kQuadXor2>(cell) != -1;  // a cell, wall or prescribed state on the other side
  if (!valid || side != 0) return;
  if (g == 0)
    edge_flux<EQ, Real>(e, E, len, second, Wb, Hb, lam, Wo, Ho, lo, AH, AD, OH, OD, F);
  else
    edge_value<EQ, Real>(e, E, second, AT, OT, G);
}

// The 3-point edge rule: eight work-items per edge, (side, Gauss point g =
// 0..2) plus one idle lane per side (g = 3), so that the sums over the points
// stay within a quad (DPP) and the two sides meet across a 4-lane shuffle.
// Weights 5/18, 8/18, 5/18 at 1/2 -+ sqrt(15)/10 and 1/2 along the edge.
template <int EQ, class Real, int TR>
__global__ __launch_bounds__(kBlock) void edge3_kernel(int E, int N, int NB, Params P, double dt,
                                                        const double* __restrict__ wbar,
                                                        const Real* __restrict__ R,
                                                        const int32_t* __restrict__ ecell,
                                                        const double* __restrict__ bnd_n,
                                                        const double* __restrict__ enl,
                                                        const Real* __restrict__ egp, double* __restrict__ F,
                                                        Real* __restrict__ G) {
  constexpr int M = NComp<EQ>::m;
  const int gid = xcd_block_id() * kBlock + threadIdx.x;
  const int e = gid >> 3, side = (gid >> 2) & 1, g = gid & 3;
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const int cell = valid ? ecell[side * E + ec] : -1;
  const int cc = cell >= 0 ? cell : ecell[ec];
  const double nx = enl[ec], ny = enl[E + ec], len = enl[2 * E + ec];
  const bool point = g < 3;
  double Wb[M];
#pragma unroll
  for (int q = 0; q < M; ++q) Wb[q] = wbar[q * size_t(N) + cc];
  Real dl[M], Wt[M], Wtt[M];
#pragma unroll
  for (int q = 0; q < M; ++q) dl[q] = Wt[q] = Wtt[q] = Real(0);
  if (cell >= 0 && point) {
    const Real X = egp[(6 * side + 2 * g) * size_t(E) + ec];
    const Real Y = egp[(6 * side + 2 * g + 1) * size_t(E) + ec];
    edge_point_at<EQ, Real>(cell, P, Wb, R, X, Y, dl, Wt, Wtt);
  }
  const bool wall = cell == -2;
  const bool presc = cell <= -3;
  if (presc) {
    const int b = -cell - 3;
    prescribed_state<M>(P, bnd_n[2 * size_t(NB) + b], bnd_n[3 * size_t(NB) + b], Wb);
  }
  if constexpr (EQ == EQ_EUL) {
    // a wall lane takes the first side's values at its point, momentum reflected
    if (__ballot(wall) != 0) {
      Real pdl[M], pWt[M], pWtt[M];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        pdl[q] = __shfl_xor(dl[q], 4);
        pWt[q] = __shfl_xor(Wt[q], 4);
        pWtt[q] = __shfl_xor(Wtt[q], 4);
      }
      if (wall) {
        const Real rx = Real(nx), ry = Real(ny);
        reflect_momentum(rx, ry, pdl);
        reflect_momentum(rx, ry, pWt);
        reflect_momentum(rx, ry, pWtt);
        reflect_momentum(nx, ny, Wb);
#pragma unroll
        for (int q = 0; q < M; ++q) {
          dl[q] = pdl[q];
          Wt[q] = pWt[q];
          Wtt[q] = pWtt[q];
        }
      }
    }
  }
  Real AH[M], AD[M], AT[M];
#pragma unroll
  for (int q = 0; q < M; ++q) AH[q] = AD[q] = AT[q] = Real(0);
  if (point && (cell >= 0 || wall || presc))
    edge_nodes<EQ, Real, TR>(P, dt, Wb, Real(nx), Real(ny), dl, Wt, Wtt, AH, AD, AT);
  const Real wg = g == 1 ? Real(8.0 / 18.0) : (point ? Real(5.0 / 18.0) : Real(0));
  double Hb[M];
  const double lam = side_terms<EQ>(P, Wb, nx, ny, Hb);
#pragma unroll
  for (int q = 0; q < M; ++q) {
    AH[q] *= wg;
    AD[q] *= wg;
    AT[q] *= wg;
    AH[q] += quad_perm<kQuadXor1>(AH[q]);
    AD[q] += quad_perm<kQuadXor1>(AD[q]);
    AT[q] += quad_perm<kQuadXor1>(AT[q]);
    AH[q] += quad_perm<kQuadXor2>(AH[q]);
    AD[q] += quad_perm<kQuadXor2>(AD[q]);
    AT[q] += quad_perm<kQuadXor2>(AT[q]);
  }
  Real OH[M], OD[M], OT[M];
  double Wo[M], Ho[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    OH[q] = __shfl_xor(AH[q], 4);
    OD[q] = __shfl_xor(AD[q], 4);
    OT[q] = __shfl_xor(AT[q], 4);
    Wo[q] = __shfl_xor(Wb[q], 4);
    Ho[q] = __shfl_xor(Hb[q], 4);
  }
  const double lo = __shfl_xor(lam, 4);
  const bool second = __shfl_xor(cell, 4) != -1;
  if (!valid || side != 0) return;
  if (g == 0)
    edge_flux<EQ, Real>(e, E, len, second, Wb, Hb, lam, Wo, Ho, lo, AH, AD, OH, OD, F);
  else if (g == 1)
    edge_value<EQ, Real>(e, E, second, AT, OT, G);
}

// The update is one round of latency-bound gathers (every cell's work-item is
// resident at once): 64-work-item blocks spread it more evenly over the CUs
// and XCDs than 256 (FP64 update 16.2 -> 15.0 us on C3, the same bits).
constexpr int kUpdateBlock = 64;
template <int EQ, class Real>
__global__ __launch_bounds__(kUpdateBlock) void update_kernel(int N, int E, int NB, Params P, double dt,
                                                         const double* __restrict__ wbar,
                                                         const double* __restrict__ bnd_n,
                                                         const int32_t* __restrict__ nbr,
                                                         const int32_t* __restrict__ cell_edge,
                                                         const Real* __restrict__ nl,
                                                         const double* __restrict__ inv_area,
                                                         const double* __restrict__ F, const Real* __restrict__ G,
                                                         double* __restrict__ wout, Real* __restrict__ gout) {
  const int i = xcd_block_id() * kUpdateBlock + threadIdx.x;
  if (i >= N) return;
  update_point<EQ, Real>(i, N, E, NB, P, dt, wbar, bnd_n, nbr, cell_edge, nl, inv_area, F, G, wout, gout);
}

// ---------------------------------------------------------------- reductions
// Step size of the time loop (Sec. 3 states the CFL number): the largest
// signal speed over the cells, reduced per block and then over the blocks;
// dt = cfl * (smallest inradius, a mesh constant) / that speed.
template <int EQ>
__global__ __launch_bounds__(kBlock) void max_speed_kernel(int N, Params P, const double* __restrict__ wbar,
                                                            double* __restrict__ part) {
  constexpr int M = NComp<EQ>::m;
  __shared__ double sh[kBlock];
  double mx = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    double W[M];
    for (int q = 0; q < M; ++q) W[q] = wbar[q * N + i];
    double s = max_speed<EQ>(P, W);
    mx = s > mx ? s : mx;
    if (s != s) mx = s;  // propagate NaN
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      double o = sh[threadIdx.x + w];
      double a = sh[threadIdx.x];
      sh[threadIdx.x] = (o > a || o != o) ? o : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void finish_dt_kernel(int nparts, const double* __restrict__ part, double num,
                                                            double* __restrict__ dt) {
  __shared__ double sh[kBlock];
  double mx = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    double o = part[i];
    mx = (o > mx || o != o) ? o : mx;
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      double o = sh[threadIdx.x + w];
      double a = sh[threadIdx.x];
      sh[threadIdx.x] = (o > a || o != o) ? o : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) dt[0] = num / sh[0];
}

template <int EQ>
__global__ __launch_bounds__(kBlock) void check_kernel(int N, Params P, const double* __restrict__ wbar,
                                                        int32_t* __restrict__ part) {
  constexpr int M = NComp<EQ>::m;
  __shared__ int32_t sh[kBlock];
  int32_t fl = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    double W[M];
    for (int q = 0; q < M; ++q) {
      W[q] = wbar[q * N + i];
      if (!isfinite(W[q])) fl |= 1;
    }
    if constexpr (EQ == EQ_EUL) {
      if (!(W[0] > 0.0)) fl |= 2;
      double p = (P.gam - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
      if (!(p > 0.0)) fl |= 4;
    }
  }
  sh[threadIdx.x] = fl;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] |= sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void finish_or_kernel(int nparts, const int32_t* __restrict__ part,
                                                            int32_t* __restrict__ out) {
  __shared__ int32_t sh[kBlock];
  int32_t fl = 0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) fl |= part[i];
  sh[threadIdx.x] = fl;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] |= sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ---------------------------------------------------------------- helpers
}  // namespace

hwe_status hip_fail(hipError_t err, const char* what) {
  std::ostringstream s;
  s << what << ": " << hipGetErrorString(err);
  set_error(s.str());
  return HWE_EHIP;
}

namespace {

template <class T>
hwe_status dev_copy(T** dst, const T* src, size_t n) {
  hipError_t err = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T));
  if (err != hipSuccess) return hip_fail(err, "hipMalloc");
  if (n) {
    err = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err, "hipMemcpy");
  }
  return HWE_OK;
}
template <class T>
hwe_status dev_copy_f32(float** dst, const std::vector<T>& src) {
  std::vector<float> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = float(src[i]);
  return dev_copy(dst, tmp.data(), tmp.size());
}
hwe_status dev_alloc(void** dst, size_t bytes) {
  hipError_t err = hipMalloc(dst, std::max<size_t>(bytes, 16));
  if (err != hipSuccess) return hip_fail(err, "hipMalloc");
  return HWE_OK;
}

unsigned grid_for(int64_t items) { return unsigned((items + kBlock - 1) / kBlock); }

// The reconstruction launch: the limiter checks the edge rule's points.
template <int EQ, class Real>
void recon_launch(hwe_mesh_s* M, const Params& P, const double* wbar, const Real* grad, const Real* tbl, Real* R,
                  hipStream_t st) {
  const DevMesh& d = M->d;
  const int N = int(M->h.N), NB = int(M->h.NB);
  const dim3 grid(grid_for(int64_t(N) * NComp<EQ>::m));
  if (!P.positivity)
    hipLaunchKernelGGL((recon_kernel<EQ, Real, 0>), grid, dim3(kBlock), 0, st, N, NB, P, wbar, grad, d.nbr, d.bnd_n,
                       tbl, d.area, d.gpc, R);
  else if (M->opts.edge_rule == 3)
    hipLaunchKernelGGL((recon_kernel<EQ, Real, 9>), grid, dim3(kBlock), 0, st, N, NB, P, wbar, grad, d.nbr, d.bnd_n,
                       tbl, d.area, d.gpc, R);
  else
    hipLaunchKernelGGL((recon_kernel<EQ, Real, 6>), grid, dim3(kBlock), 0, st, N, NB, P, wbar, grad, d.nbr, d.bnd_n,
                       tbl, d.area, d.gpc, R);
}

// The edge stage: the kernel for the mesh's edge rule and the time rule.
template <int EQ, class Real>
void edge_impl(hwe_mesh_s* M, const Params& P, double dt, const double* wbar, const Real* R, const Real* egp,
               double* F, Real* G, hipStream_t st) {
  const DevMesh& d = M->d;
  const int N = int(M->h.N), E = int(M->h.E), NB = int(M->h.NB);
  if (M->opts.edge_rule == 3) {
    if (P.time_rule == 1)
      hipLaunchKernelGGL((edge3_kernel<EQ, Real, 1>), dim3(grid_for(8 * int64_t(E))), dim3(kBlock), 0, st, E, N, NB,
                         P, dt, wbar, R, d.ecell, d.bnd_n, d.enl, egp, F, G);
    else
      hipLaunchKernelGGL((edge3_kernel<EQ, Real, 0>), dim3(grid_for(8 * int64_t(E))), dim3(kBlock), 0, st, E, N, NB,
                         P, dt, wbar, R, d.ecell, d.bnd_n, d.enl, egp, F, G);
  } else if (P.time_rule == 1) {
    hipLaunchKernelGGL((edge_kernel<EQ, Real, 1>), dim3(grid_for(4 * int64_t(E))), dim3(kBlock), 0, st, E, N, NB, P,
                       dt, wbar, R, d.ecell, d.bnd_n, d.enl, egp, F, G);
  } else {
    hipLaunchKernelGGL((edge_kernel<EQ, Real, 0>), dim3(grid_for(4 * int64_t(E))), dim3(kBlock), 0, st, E, N, NB, P,
                       dt, wbar, R, d.ecell, d.bnd_n, d.enl, egp, F, G);
  }
}

template <int EQ, class Real>
hwe_status step_impl(hwe_mesh_s* M, const Params& P, const double* wbar_in, const Real* grad_in, double* wbar_out,
                     Real* grad_out, double dt, hipStream_t st, const Real* tbl, const Real* nl,
                     const Real* egp, Real* R, double* F, Real* G) {
  const HostMesh& h = M->h;
  const DevMesh& d = M->d;
  const int N = int(h.N), E = int(h.E), NB = int(h.NB);
  constexpr int Mc = NComp<EQ>::m;
  // optional per-kernel events (profiling mode only)
  hipEvent_t* ev = nullptr;
  if (d.prof_n < d.prof_cap) ev = reinterpret_cast<hipEvent_t*>(&M->d.prof_ev[4 * size_t(d.prof_n)]);
  hipError_t ev_err = hipSuccess;
  auto record = [&](int j) {
    if (!ev) return;
    const hipError_t e = hipEventRecord(ev[j], st);
    if (e != hipSuccess && ev_err == hipSuccess) ev_err = e;
  };
  record(0);
  recon_launch<EQ, Real>(M, P, wbar_in, grad_in, tbl, R, st);
  record(1);
  edge_impl<EQ, Real>(M, P, dt, wbar_in, R, egp, F, G, st);
  record(2);
  hipLaunchKernelGGL((update_kernel<EQ, Real>), dim3((N + kUpdateBlock - 1) / kUpdateBlock), dim3(kUpdateBlock), 0, st, N, E, NB, P, dt, wbar_in,
                     d.bnd_n, d.nbr, d.cell_edge, nl, d.inv_area, F, G, wbar_out, grad_out);
  record(3);
  if (ev) ++M->d.prof_n;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  if (ev_err != hipSuccess) return hip_fail(ev_err, "hipEventRecord");
  return HWE_OK;
}

template <int EQ, class Real>
hwe_status recon_impl(hwe_mesh_s* M, const Params& P, const double* wbar, const Real* grad, Real* R, hipStream_t st,
                      const Real* tbl) {
  const HostMesh& h = M->h;
  const DevMesh& d = M->d;
  const int N = int(h.N), NB = int(h.NB);
  constexpr int Mc = NComp<EQ>::m;
  recon_launch<EQ, Real>(M, P, wbar, grad, tbl, R, st);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  return HWE_OK;
}

}  // namespace

Params params_of(const hwe_opts& o) {
  Params P;
  P.positivity = o.positivity ? 1 : 0;
  P.ax = o.adv[0];
  P.ay = o.adv[1];
  P.gam = o.gas_gamma;
  for (int l = 0; l < 4; ++l) P.lw[l] = o.lin_w[l];
  P.eps = o.eps;
  P.linear = o.linear_weights ? 1 : 0;
  P.time_rule = o.time_rule;
  for (int a = 0; a < 2; ++a)
    for (int q = 0; q < 4; ++q) P.bst[a][q] = o.bstate[a][q];
  P.sx0 = o.shock_x0;
  P.sv = o.shock_speed;
  P.tb = 0.0;
  return P;
}

// Host tables [k][N] -> tiled device layout (see kTile), padded to whole tiles
// with zeros.
static std::vector<double> tiled_tables(const HostMesh& h) {
  const int N = int(h.N);
  const int tiles = (N + kTile - 1) / kTile;
  std::vector<double> t(size_t(tiles) * kTblRows * kTile, 0.0);
  for (int i = 0; i < N; ++i) {
    double* col = t.data() + tbl_col(i);
    static_assert(kTblMd == kP1Md && kTblZ == kP1Z && kTblQ == kP1Q && kTblP2 == kP1F, "table rows");
    for (int k = 0; k < kP1F; ++k) col[k * kTile] = h.p1f[size_t(k) * N + i];
    for (int k = 0; k < 9; ++k) col[(kTblP2 + k) * kTile] = h.p2[size_t(k) * N + i];
    for (int k = 0; k < 3; ++k) col[(kTblMom + k) * kTile] = h.mom[size_t(k) * N + i];
  }
  return t;
}

hwe_status upload_mesh(hwe_mesh_s* M) {
  const HostMesh& h = M->h;
  DevMesh& d = M->d;
  d.device = M->opts.device;
  hipError_t err = hipSetDevice(d.device);
  if (err != hipSuccess) return hip_fail(err, "hipSetDevice");
  hwe_status s;
#define HWE_TRY(x)           \
  do {                       \
    s = (x);                 \
    if (s != HWE_OK) return s; \
  } while (0)
  HWE_TRY(dev_copy(&d.nbr, h.nbr.data(), h.nbr.size()));
  HWE_TRY(dev_copy(&d.cell_edge, h.cell_edge.data(), h.cell_edge.size()));
  HWE_TRY(dev_copy(&d.ecell, h.ecell.data(), h.ecell.size()));
  HWE_TRY(dev_copy(&d.nbr_back, h.nbr_back.data(), h.nbr_back.size()));
  HWE_TRY(dev_copy(&d.bnd_n, h.bnd_n.data(), h.bnd_n.size()));
  HWE_TRY(dev_copy(&d.area, h.area.data(), h.area.size()));
  HWE_TRY(dev_copy(&d.inv_area, h.inv_area.data(), h.inv_area.size()));
  if (M->opts.positivity) HWE_TRY(dev_copy(&d.gpc, h.gpc.data(), h.gpc.size()));
  const size_t N = size_t(h.N), E = size_t(h.E), m = size_t(h.m);
  HWE_TRY(dev_copy(&d.enl, h.egeo.data(), 3 * E));
  const std::vector<double> tiled = tiled_tables(h);
  if (M->opts.prec == HWE_FP64) {
    HWE_TRY(dev_copy(&d.tbl, tiled.data(), tiled.size()));
    HWE_TRY(dev_copy(&d.nl, h.nl.data(), h.nl.size()));
    if (M->opts.edge_rule == 3)
      HWE_TRY(dev_copy(&d.egp, h.egp3.data(), h.egp3.size()));
    else
      HWE_TRY(dev_copy(&d.egp, h.egeo.data() + 3 * E, 8 * E));
  } else {
    HWE_TRY(dev_copy_f32(&d.tblf, tiled));
    HWE_TRY(dev_copy_f32(&d.nlf, h.nl));
    if (M->opts.edge_rule == 3)
      HWE_TRY(dev_copy_f32(&d.egpf, h.egp3));
    else
      HWE_TRY(dev_copy_f32(&d.egpf, std::vector<double>(h.egeo.begin() + 3 * E, h.egeo.end())));
  }
  const size_t rs = M->opts.prec == HWE_FP64 ? sizeof(double) : sizeof(float);
  HWE_TRY(dev_alloc(&d.R, 6 * m * N * rs));
  HWE_TRY(dev_alloc(&d.F, m * E * sizeof(double)));
  HWE_TRY(dev_alloc(&d.G, m * E * rs));
  HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.slots), 12 * m * N * sizeof(double)));
  HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.sface), 3 * N * sizeof(double)));
  if (!h.sb_cells.empty()) {
    const size_t nsb = h.sb_cells.size();
    HWE_TRY(dev_copy(&d.sb_cells, h.sb_cells.data(), nsb));
    d.n_sb = int(nsb);
    HWE_TRY(dev_alloc(&d.sb_la, 6 * m * nsb * rs));
    HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.sb_lw), m * nsb * sizeof(double)));
    HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.sb_sface), 3 * nsb * sizeof(double)));
    hipStream_t sst;
    err = hipStreamCreateWithFlags(&sst, hipStreamNonBlocking);
    if (err != hipSuccess) return hip_fail(err, "hipStreamCreateWithFlags");
    d.sb_stream = sst;
    hipEvent_t ev[2];
    for (int j = 0; j < 2; ++j) {
      err = hipEventCreateWithFlags(&ev[j], hipEventDisableTiming);
      if (err != hipSuccess) return hip_fail(err, "hipEventCreateWithFlags");
      (j == 0 ? d.sb_fork : d.sb_join) = ev[j];
    }
  }
  HWE_TRY(dev_alloc(&d.lacell, 6 * m * N * rs));
  HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.lwcell), m * N * sizeof(double)));
  HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.red), kRedBlocks * sizeof(double)));
  HWE_TRY(dev_alloc(reinterpret_cast<void**>(&d.redi), kRedBlocks * sizeof(int32_t)));
#undef HWE_TRY
  return HWE_OK;
}

void free_device(hwe_mesh_s* M) {
  DevMesh& d = M->d;
  if (d.device < 0) return;
  hipSetDevice(d.device);
  hipDeviceSynchronize();
  void* ptrs[] = {d.nbr, d.cell_edge, d.ecell, d.nbr_back, d.bnd_n, d.area, d.tbl, d.nl, d.inv_area,
                  d.gpc, d.enl, d.egp, d.tblf, d.nlf, d.egpf, d.R, d.F, d.G, d.slots, d.sface, d.lacell, d.lwcell,
                  d.red, d.redi, d.sb_cells, d.sb_la, d.sb_lw, d.sb_sface};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (void* e : {d.sb_fork, d.sb_join})
    if (e) hipEventDestroy(static_cast<hipEvent_t>(e));
  if (d.sb_stream) hipStreamDestroy(static_cast<hipStream_t>(d.sb_stream));
  for (void* e : d.prof_ev) hipEventDestroy(static_cast<hipEvent_t>(e));
  d = DevMesh();
}

namespace {
// The step with its scratch (reconstruction R, edge fluxes F, interface values
// G) at the given device addresses.
hwe_status launch_step_with(hwe_mesh_s* M, const double* wbar_in, const void* grad_in, double* wbar_out,
                            void* grad_out, double dt, void* R, double* F, void* G, void* stream) {
  Params P = params_of(M->opts);
  P.tb = M->time + 0.5 * dt;  // moving boundary states: the middle of the step
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevMesh& d = M->d;
  if (M->opts.prec == HWE_FP64) {
    auto gi = static_cast<const double*>(grad_in);
    auto go = static_cast<double*>(grad_out);
    auto r = static_cast<double*>(R);
    auto g = static_cast<double*>(G);
    switch (M->opts.eq) {
      case HWE_ADVECTION:
        return step_impl<EQ_ADV, double>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tbl, d.nl, d.egp, r, F, g);
      case HWE_BURGERS:
        return step_impl<EQ_BUR, double>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tbl, d.nl, d.egp, r, F, g);
      default:
        return step_impl<EQ_EUL, double>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tbl, d.nl, d.egp, r, F, g);
    }
  }
  auto gi = static_cast<const float*>(grad_in);
  auto go = static_cast<float*>(grad_out);
  auto r = static_cast<float*>(R);
  auto g = static_cast<float*>(G);
  switch (M->opts.eq) {
    case HWE_ADVECTION:
      return step_impl<EQ_ADV, float>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tblf, d.nlf, d.egpf, r, F, g);
    case HWE_BURGERS:
      return step_impl<EQ_BUR, float>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tblf, d.nlf, d.egpf, r, F, g);
    default:
      return step_impl<EQ_EUL, float>(M, P, wbar_in, gi, wbar_out, go, dt, st, d.tblf, d.nlf, d.egpf, r, F, g);
  }
}

// Scratch of hwe_step_noalloc: one array per GPU for the whole library, held
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is a stand-in, not device memory): the device
// address is resolved once per device by scratch_setup and kept in
// g_scratch_dev.
constexpr size_t kStaticScratchBytes = size_t(HWE_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

hwe_status launch_step(hwe_mesh_s* M, const double* wbar_in, const void* grad_in, double* wbar_out, void* grad_out,
                       double dt, void* R_keep, void* stream) {
  const DevMesh& d = M->d;
  return launch_step_with(M, wbar_in, grad_in, wbar_out, grad_out, dt, R_keep ? R_keep : d.R,
                          static_cast<double*>(d.F), d.G, stream);
}

hwe_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device ordinal out of range for the static scratch");
    return HWE_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return HWE_OK;
  // the caller made `device` current
  void* ptr = nullptr;
  hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (err != hipSuccess) return hip_fail(err, "hipGetSymbolAddress(scratch)");
  if (!ptr) {
    set_error("hipGetSymbolAddress(scratch) returned a null address");
    return HWE_EHIP;
  }
  g_scratch_dev[device] = ptr;
  return HWE_OK;
}

size_t step_scratch_bytes(const hwe_mesh_s* M) {
  const size_t N = size_t(M->h.N), E = size_t(M->h.E), m = size_t(M->h.m);
  const size_t rs = M->opts.prec == HWE_FP64 ? sizeof(double) : sizeof(float);
  return align256(6 * m * N * rs) + align256(m * E * sizeof(double)) + align256(m * E * rs);
}

hwe_status launch_step_noalloc(hwe_mesh_s* M, const double* wbar_in, const void* grad_in, double* wbar_out,
                               void* grad_out, double dt, void* stream) {
  const size_t need = step_scratch_bytes(M);
  if (need > kStaticScratchBytes) {
    std::ostringstream msg;
    msg << "the mesh needs " << need << " bytes of step scratch; the static scratch holds " << kStaticScratchBytes;
    set_error(msg.str());
    return HWE_EINVAL;
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = M->d.device >= 0 && M->d.device < kMaxDevices ? g_scratch_dev[M->d.device] : nullptr;
  }
  if (!base) {
    set_error("the static scratch of this device was not set up");
    return HWE_EHIP;
  }
  const size_t N = size_t(M->h.N), E = size_t(M->h.E), m = size_t(M->h.m);
  const size_t rs = M->opts.prec == HWE_FP64 ? sizeof(double) : sizeof(float);
  unsigned char* b = static_cast<unsigned char*>(base);
  void* R = b;
  double* F = reinterpret_cast<double*>(b + align256(6 * m * N * rs));
  void* G = b + align256(6 * m * N * rs) + align256(m * E * sizeof(double));
  return launch_step_with(M, wbar_in, grad_in, wbar_out, grad_out, dt, R, F, G, stream);
}

hwe_status launch_recon(hwe_mesh_s* M, const double* wbar, const void* grad, void* R_out, double tb, void* stream) {
  Params P = params_of(M->opts);
  P.tb = tb;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevMesh& d = M->d;
  if (M->opts.prec == HWE_FP64) {
    auto g = static_cast<const double*>(grad);
    auto R = static_cast<double*>(R_out);
    switch (M->opts.eq) {
      case HWE_ADVECTION: return recon_impl<EQ_ADV, double>(M, P, wbar, g, R, st, d.tbl);
      case HWE_BURGERS: return recon_impl<EQ_BUR, double>(M, P, wbar, g, R, st, d.tbl);
      default: return recon_impl<EQ_EUL, double>(M, P, wbar, g, R, st, d.tbl);
    }
  }
  auto g = static_cast<const float*>(grad);
  auto R = static_cast<float*>(R_out);
  switch (M->opts.eq) {
    case HWE_ADVECTION: return recon_impl<EQ_ADV, float>(M, P, wbar, g, R, st, d.tblf);
    case HWE_BURGERS: return recon_impl<EQ_BUR, float>(M, P, wbar, g, R, st, d.tblf);
    default: return recon_impl<EQ_EUL, float>(M, P, wbar, g, R, st, d.tblf);
  }
}

hwe_status launch_edge(hwe_mesh_s* M, const void* R, const double* wbar, double dt, double* F_out, void* G_out,
                       void* stream) {
  Params P = params_of(M->opts);
  P.tb = M->time + 0.5 * dt;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevMesh& d = M->d;
  if (M->opts.prec == HWE_FP64) {
    auto r = static_cast<const double*>(R);
    auto g = static_cast<double*>(G_out);
    switch (M->opts.eq) {
      case HWE_ADVECTION: edge_impl<EQ_ADV, double>(M, P, dt, wbar, r, d.egp, F_out, g, st); break;
      case HWE_BURGERS: edge_impl<EQ_BUR, double>(M, P, dt, wbar, r, d.egp, F_out, g, st); break;
      default: edge_impl<EQ_EUL, double>(M, P, dt, wbar, r, d.egp, F_out, g, st);
    }
  } else {
    auto r = static_cast<const float*>(R);
    auto g = static_cast<float*>(G_out);
    switch (M->opts.eq) {
      case HWE_ADVECTION: edge_impl<EQ_ADV, float>(M, P, dt, wbar, r, d.egpf, F_out, g, st); break;
      case HWE_BURGERS: edge_impl<EQ_BUR, float>(M, P, dt, wbar, r, d.egpf, F_out, g, st); break;
      default: edge_impl<EQ_EUL, float>(M, P, dt, wbar, r, d.egpf, F_out, g, st);
    }
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  return HWE_OK;
}

hwe_status launch_max_dt(hwe_mesh_s* M, const double* wbar, double cfl, double* dt_dev, void* stream) {
  const Params P = params_of(M->opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = int(M->h.N);
  const int nb = std::min<int>(kRedBlocks, int(grid_for(N)));
  switch (M->opts.eq) {
    case HWE_ADVECTION:
      hipLaunchKernelGGL(max_speed_kernel<EQ_ADV>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.red);
      break;
    case HWE_BURGERS:
      hipLaunchKernelGGL(max_speed_kernel<EQ_BUR>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.red);
      break;
    default:
      hipLaunchKernelGGL(max_speed_kernel<EQ_EUL>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.red);
  }
  hipLaunchKernelGGL(finish_dt_kernel, dim3(1), dim3(kBlock), 0, st, nb, M->d.red, cfl * M->h.rmin, dt_dev);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  return HWE_OK;
}

hwe_status launch_check(hwe_mesh_s* M, const double* wbar, int32_t* flags, void* stream) {
  const Params P = params_of(M->opts);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = int(M->h.N);
  const int nb = std::min<int>(kRedBlocks, int(grid_for(N)));
  switch (M->opts.eq) {
    case HWE_ADVECTION:
      hipLaunchKernelGGL(check_kernel<EQ_ADV>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.redi);
      break;
    case HWE_BURGERS:
      hipLaunchKernelGGL(check_kernel<EQ_BUR>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.redi);
      break;
    default:
      hipLaunchKernelGGL(check_kernel<EQ_EUL>, dim3(nb), dim3(kBlock), 0, st, N, P, wbar, M->d.redi);
  }
  hipLaunchKernelGGL(finish_or_kernel, dim3(1), dim3(kBlock), 0, st, nb, M->d.redi, flags);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_fail(err, "kernel launch");
  return HWE_OK;
}

hwe_status profile_begin(hwe_mesh_s* M, int n_steps) {
  DevMesh& d = M->d;
  for (void* e : d.prof_ev) hipEventDestroy(static_cast<hipEvent_t>(e));
  d.prof_ev.assign(4 * size_t(n_steps), nullptr);
  for (auto& e : d.prof_ev) {
    hipEvent_t h;
    hipError_t err = hipEventCreate(&h);
    if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
    e = h;
  }
  d.prof_cap = n_steps;
  d.prof_n = 0;
  return HWE_OK;
}

hwe_status profile_end(hwe_mesh_s* M, double* ms_sum, int* n_done) {
  DevMesh& d = M->d;
  ms_sum[0] = ms_sum[1] = ms_sum[2] = 0.0;
  for (int k = 0; k < d.prof_n; ++k) {
    hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(&d.prof_ev[4 * size_t(k)]);
    hipError_t err = hipEventSynchronize(ev[3]);
    if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize");
    for (int j = 0; j < 3; ++j) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[j], ev[j + 1]);
      if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
      ms_sum[j] += ms;
    }
  }
  *n_done = d.prof_n;
  for (void* e : d.prof_ev) hipEventDestroy(static_cast<hipEvent_t>(e));
  d.prof_ev.clear();
  d.prof_cap = d.prof_n = 0;
  return HWE_OK;
}



}  // namespace hwe
