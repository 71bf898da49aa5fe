// Internal declarations of the hwe library (host precompute + device state).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hwe.h"

namespace hwe {

// Thread-local error message set by a failing C-ABI call.
void set_error(const std::string& msg);

// Number of double entries of the per-cell Step-1 map (5 coefficients x 11 inputs).
constexpr int kP1 = 55;
// The factored Step-1 map of the device tables: rows kP1Md + 3j + c (the map's
// dW columns, 5 x 3), kP1Z + 5k + j (the null-space basis, 2 x 5) and
// kP1Q + 8k + v (the reduced solution on V0..V3, Y0..Y3, 2 x 8); 41 rows.
constexpr int kP1Md = 0, kP1Z = 15, kP1Q = 25, kP1F = 41;
// Per-cell Step-2 data: (dx, dy, 1/(1 + dx^2 + dy^2)) for each of the three faces.
constexpr int kP2 = 9;
// Per-edge geometry: nx, ny, length, then the Gauss-point offsets (X, Y) from the
// centroid of the edge's first cell (points 0, 1) and of its second cell (0, 1).
constexpr int kEG = 11;

// Everything precomputed on the host, in the internal (Morton) cell order.
struct HostMesh {
  int64_t N = 0, E = 0, NB = 0;
  int m = 1;
  std::vector<int64_t> perm;       // internal cell -> caller triangle
  std::vector<double> cen;         // [2][N] centroid (cell's own frame)
  std::vector<double> area;        // [N]
  std::vector<double> mom;         // [3][N] central second moments Mxx, Mxy, Myy
  std::vector<int32_t> nbr;        // [3][N] neighbour across face f; -(b+1) for boundary face b
  std::vector<int32_t> nbr_back;   // [3][N] the neighbour's face index that points back (-1 on boundary)
  std::vector<double> bnd_n;       // [4][NB] outward unit normal of boundary face b, its kind
                                   // (hwe_bnd_kind, as a double) and the x of its midpoint
  bool special_bnd = false;        // some boundary face is a wall or prescribed
  std::vector<int32_t> sb_cells;   // the cells with a wall or prescribed face, ascending
  std::vector<double> p1;          // [55][N] Step-1 map (row-major 5 x 11 per cell; host tests)
  std::vector<double> p1f;         // [41][N] factored Step-1 map (device tables)
  std::vector<double> p2;          // [9][N] Step-2 data
  std::vector<int32_t> cell_edge;  // [3][N] (edge << 1) | (cell is the edge's second cell)
  std::vector<double> nl;          // [6][N] outward normal times length: x of faces 0..2, then y
  std::vector<double> inv_area;    // [N]
  std::vector<double> gpc;         // [6G][N] offsets (X, Y) from the centroid of the G Gauss
                                   // points (2, or 3 with the 3-point rule) of faces 0..2:
                                   // row 2(Gf+g) (X), 2(Gf+g)+1 (Y) (limiter only)
  std::vector<int32_t> ecell;      // [2][E] first cell (lower caller index), then the second cell, or
                                   // on a boundary edge -1 (transmissive), -2 (wall) or -3 - b
                                   // (prescribed state; b = the boundary face)
  std::vector<double> egeo;        // [11][E]
  std::vector<double> egp3;        // [12][E] with the 3-point edge rule: offsets (X, Y) from the
                                   // centroid of the first cell of points 0..2 (rows 2g, 2g+1),
                                   // then from the second cell's (rows 6 + 2g, 7 + 2g)
  double rmin = 0.0;               // smallest inradius
};

// Device copies (FP64 always, FP32 copies for the mixed path) and scratch.
struct DevMesh {
  int device = -1;
  // connectivity
  int32_t* nbr = nullptr;
  int32_t* cell_edge = nullptr;
  int32_t* ecell = nullptr;
  int32_t* nbr_back = nullptr;
  // FP64 geometry / tables
  double* bnd_n = nullptr;
  double* area = nullptr;
  double* tbl = nullptr;    // tiled reconstruction tables (Step-1 map, Step-2 data, moments)
  double* nl = nullptr;
  double* inv_area = nullptr;
  double* gpc = nullptr;    // [12][N] (limiter only)
  double* enl = nullptr;    // [3][E] edge normal and length (FP64 in both precisions)
  double* egp = nullptr;    // [8][E] Gauss-point offsets (FP64 path); [12][E] with the 3-point rule
  // FP32 copies for the mixed path
  float* tblf = nullptr;
  float* nlf = nullptr;
  float* egpf = nullptr;
  // scratch: reconstruction coefficients [N][6][m] (double or float by
  // precision), edge flux [E][m] (double) and interface-value offset [E][m]
  // (double or float); hipMalloc's 256-byte alignment keeps every record 16-byte aligned
  void* R = nullptr;
  void* F = nullptr;
  void* G = nullptr;
  // adjoint scratch: stencil-slot adjoints [N][4][3][m] and per-face scalars [3][N]
  double* slots = nullptr;
  double* sface = nullptr;
  int32_t* sb_cells = nullptr;  // HostMesh::sb_cells (null when there are none)
  int n_sb = 0;
  // the face reverse of the listed cells runs beside the one over every cell:
  // on its own stream (hipStream_t, default priority, created with the list),
  // joined by two events (hipEvent_t), into compact outputs that a small
  // kernel copies over the listed cells' records after the join
  void* sb_stream = nullptr;
  void* sb_fork = nullptr;
  void* sb_join = nullptr;
  void* sb_la = nullptr;       // [n_sb][6][m] Real
  double* sb_lw = nullptr;     // [n_sb][m]
  double* sb_sface = nullptr;  // [3][n_sb]
  // adjoint scratch: per-cell coefficient adjoints [N][6][m] (Real) and
  // flux-base adjoints [N][m] (double) handed from the face to the recon kernel
  void* lacell = nullptr;
  double* lwcell = nullptr;
  // reductions
  double* red = nullptr;   // [kRedBlocks]
  int32_t* redi = nullptr; // [kRedBlocks]
  // per-kernel event profiling (hwe_profile_begin / hwe_profile_end)
  std::vector<void*> prof_ev;  // hipEvent_t, 4 per profiled step
  int prof_cap = 0, prof_n = 0;
  void* prof_stream = nullptr;
};

constexpr int kRedBlocks = 1024;

}  // namespace hwe

struct hwe_mesh_s {
  hwe_opts opts;
  double time = 0.0;  // hwe_set_time: time of the next step's input state
  hwe::HostMesh h;
  hwe::DevMesh d;
};

namespace hwe {
// Host precompute (hwe_mesh.cpp).  Returns HWE_OK or an error status with the
// message set.
hwe_status build_host_mesh(const double* nodes, int64_t n_nodes, const int32_t* tris, int64_t n_tris,
                           const hwe_opts& o, HostMesh& h);
// Device upload / release (hwe_kernels.hip).
hwe_status upload_mesh(hwe_mesh_s* M);
void free_device(hwe_mesh_s* M);
// Launchers (hwe_kernels.hip).  All asynchronous on stream.
// R_keep (may be null): caller memory [N][6][m] that receives the
// reconstruction of the step and is read by its edge kernel in place of the
// handle's scratch R.
hwe_status launch_step(hwe_mesh_s* M, const double* wbar_in, const void* grad_in, double* wbar_out,
                       void* grad_out, double dt, void* R_keep, void* stream);
// hwe_step with its scratch in the library's static device array (see
// hwe_step_noalloc); HWE_EINVAL when the mesh needs more than the array holds.
hwe_status launch_step_noalloc(hwe_mesh_s* M, const double* wbar_in, const void* grad_in, double* wbar_out,
                               void* grad_out, double dt, void* stream);
// Bytes of step scratch (R, F, G, each 256-byte aligned) a handle needs.
size_t step_scratch_bytes(const hwe_mesh_s* M);
// Resolve the static scratch's device address on `device` (current) once.
hwe_status scratch_setup(int device);
// tb: the time at which moving boundary states are evaluated (a step uses
// the middle of the step)
hwe_status launch_recon(hwe_mesh_s* M, const double* wbar, const void* grad, void* R_out, double tb, void* stream);
hwe_status launch_edge(hwe_mesh_s* M, const void* R, const double* wbar, double dt, double* F_out, void* G_out,
                       void* stream);
// R_n (may be null): the reconstruction of state n kept by a step; null
// recomputes it into the handle's scratch.
hwe_status launch_adjoint(hwe_mesh_s* M, const double* wbar_n, const void* grad_n, const void* R_n, const double* lw,
                          const void* lg, double* lw_out, void* lg_out, double dt, void* stream);
hwe_status launch_max_dt(hwe_mesh_s* M, const double* wbar, double cfl, double* dt_dev, void* stream);
hwe_status launch_check(hwe_mesh_s* M, const double* wbar, int32_t* flags, void* stream);
hwe_status profile_begin(hwe_mesh_s* M, int n_steps);
// Equation parameters of a handle, as passed to the kernels.
struct Params;
Params params_of(const hwe_opts& o);
hwe_status profile_end(hwe_mesh_s* M, double* ms_sum, int* n_done);
}  // namespace hwe
