// C-ABI entry points of the hwe library: argument validation, handle lifetime
// and dispatch to the host precompute and the HIP launchers.  No C++
// exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "hwe_internal.h"

namespace hwe {
namespace {
thread_local std::string g_last_error;

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

hwe_status need_device(hwe_mesh m) {
  if (!m) {
    set_error("null mesh handle");
    return HWE_EINVAL;
  }
  if (m->d.device < 0) {
    set_error("host-only mesh handle (opts.device = -1)");
    return HWE_ENODEV;
  }
  return HWE_OK;
}

hwe_status check_dt(double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) {
    set_error("dt must be positive and finite");
    return HWE_EINVAL;
  }
  return HWE_OK;
}

size_t real_size(hwe_mesh m) { return m->opts.prec == HWE_FP64 ? sizeof(double) : sizeof(float); }

hwe_status set_dev(hwe_mesh m) {
  hipError_t e = hipSetDevice(m->d.device);
  if (e != hipSuccess) {
    set_error(std::string("hipSetDevice: ") + hipGetErrorString(e));
    return HWE_EHIP;
  }
  return HWE_OK;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace hwe

using namespace hwe;

extern "C" {

const char* hwe_last_error(void) { return g_last_error.c_str(); }

hwe_status hwe_opts_default(hwe_opts* o) {
  if (!o) {
    set_error("null opts");
    return HWE_EINVAL;
  }
  std::memset(o, 0, sizeof(*o));
  o->eq = HWE_ADVECTION;
  o->bc = HWE_BC_PERIODIC;
  o->prec = HWE_FP64;
  o->linear_weights = 0;
  o->box[0] = 0.0;
  o->box[1] = 1.0;
  o->box[2] = 0.0;
  o->box[3] = 1.0;
  o->adv[0] = 1.0;
  o->adv[1] = 1.0;
  o->gas_gamma = 1.4;
  o->lin_w[0] = 0.94;
  o->lin_w[1] = 0.02;
  o->lin_w[2] = 0.02;
  o->lin_w[3] = 0.02;
  o->eps = 1e-8;
  o->device = 0;
  o->time_rule = 0;
  o->deriv_weight = 1.0;
  o->walls = 0;
  o->n_regions = 0;
  o->edge_rule = 2;
  return HWE_OK;
}

namespace {

bool finite_value(double v) { return v == v && v < 1e300 && v > -1e300; }

// Buffers read or written as whole records (a cell's reconstruction, an edge's
// flux) are moved with 16-byte accesses.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Region list, prescribed states and the moving switch.
bool regions_ok(const hwe_opts& o) {
  if (o.n_regions < 0 || o.n_regions > HWE_MAX_REGIONS) return false;
  if (o.n_regions > 0 && o.bc != HWE_BC_TRANSMISSIVE) return false;
  for (int r = 0; r < o.n_regions; ++r) {
    const hwe_region& g = o.regions[r];
    if (g.kind < HWE_BND_TRANSMISSIVE || g.kind > HWE_BND_MOVING) return false;
    if (g.kind == HWE_BND_WALL && o.eq != HWE_EULER) return false;
    for (int k = 0; k < 4; ++k)
      if (!finite_value(g.box[k])) return false;
    if (!(g.box[0] <= g.box[1]) || !(g.box[2] <= g.box[3])) return false;
  }
  const int m = o.eq == HWE_EULER ? 4 : 1;
  for (int a = 0; a < 2; ++a)
    for (int q = 0; q < m; ++q)
      if (!finite_value(o.bstate[a][q])) return false;
  return finite_value(o.shock_x0) && finite_value(o.shock_speed);
}

}  // namespace

hwe_status hwe_mesh_init(const double* nodes, int64_t n_nodes, const int32_t* tris, int64_t n_tris,
                         const hwe_opts* opts, hwe_mesh* out) {
  if (!nodes || !tris || !opts || !out) {
    set_error("null argument");
    return HWE_EINVAL;
  }
  *out = nullptr;
  const hwe_opts& o = *opts;
  if (o.eq < HWE_ADVECTION || o.eq > HWE_EULER || o.bc < 0 || o.bc > 1 || o.prec < 0 || o.prec > 1 ||
      o.positivity < 0 || o.positivity > 1 || (o.positivity && o.eq != HWE_EULER) || o.time_rule < 0 ||
      o.time_rule > 1 || !(o.deriv_weight > 0.0) || !(o.deriv_weight < 1e300) || o.walls < 0 || o.walls > 15 ||
      (o.walls && (o.eq != HWE_EULER || o.bc != HWE_BC_TRANSMISSIVE)) || !regions_ok(o) ||
      (o.edge_rule != 2 && o.edge_rule != 3)) {
    set_error("invalid option value");
    return HWE_EINVAL;
  }
  if (!(o.lin_w[0] > 0) || !(o.eps > 0) || (o.eq == HWE_EULER && !(o.gas_gamma > 1.0))) {
    set_error("invalid weights, eps or gas_gamma");
    return HWE_EINVAL;
  }
  hwe_mesh_s* M = new (std::nothrow) hwe_mesh_s();
  if (!M) {
    set_error("out of host memory");
    return HWE_ENOMEM;
  }
  M->opts = o;
  hwe_status s;
  try {
    s = build_host_mesh(nodes, n_nodes, tris, n_tris, o, M->h);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory");
    s = HWE_ENOMEM;
  } catch (...) {
    set_error("unexpected failure in the host precompute");
    s = HWE_EMESH;
  }
  if (s == HWE_OK && o.device >= 0) {
    // the kernels index in 32 bits: the state's (2m + m) N entries per
    // component block (N < 2^28 for m = 4), and 4 (8 with the 3-point edge
    // rule) work-items per edge
    const int64_t e_max = int64_t(1) << (o.edge_rule == 3 ? 28 : 29);
    if (M->h.N >= (int64_t(1) << 28) || M->h.E >= e_max) {
      set_error("mesh too large for 32-bit device indexing (N < 2^28, E < 2^29, or 2^28 with the 3-point edge rule)");
      s = HWE_EINVAL;
    } else {
      s = upload_mesh(M);
      if (s == HWE_OK) s = scratch_setup(o.device);
    }
  }
  if (s != HWE_OK) {
    free_device(M);
    delete M;
    return s;
  }
  *out = M;
  return HWE_OK;
}

hwe_status hwe_mesh_destroy(hwe_mesh m) {
  if (!m) return HWE_OK;
  free_device(m);
  delete m;
  return HWE_OK;
}

hwe_status hwe_mesh_info(hwe_mesh m, int64_t* n_cells, int64_t* n_edges, int32_t* m_comp) {
  if (!m) {
    set_error("null mesh handle");
    return HWE_EINVAL;
  }
  if (n_cells) *n_cells = m->h.N;
  if (n_edges) *n_edges = m->h.E;
  if (m_comp) *m_comp = m->h.m;
  return HWE_OK;
}

hwe_status hwe_set_time(hwe_mesh m, double t) {
  if (!m || !finite_value(t)) {
    set_error("null mesh handle or non-finite time");
    return HWE_EINVAL;
  }
  m->time = t;
  return HWE_OK;
}

hwe_status hwe_mesh_cell_perm(hwe_mesh m, int64_t* perm_host) {
  if (!m || !perm_host) {
    set_error("null argument");
    return HWE_EINVAL;
  }
  std::memcpy(perm_host, m->h.perm.data(), sizeof(int64_t) * m->h.N);
  return HWE_OK;
}

namespace {

// Argument checks shared by hwe_step and hwe_step_keep; recon (may be null)
// is the kept-reconstruction buffer, which must not overlap the state buffers.
hwe_status check_step(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out, void* grad_out,
                      double dt, const void* recon) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if ((s = check_dt(dt)) != HWE_OK) return s;
  if (!wbar_in || !grad_in || !wbar_out || !grad_out) {
    set_error("null state pointer");
    return HWE_EINVAL;
  }
  const size_t N = size_t(m->h.N), mm = size_t(m->h.m);
  const size_t wb = mm * N * sizeof(double), gb = 2 * mm * N * real_size(m);
  if (overlaps(wbar_in, wb, wbar_out, wb) || overlaps(wbar_in, wb, grad_out, gb) ||
      overlaps(grad_in, gb, wbar_out, wb) || overlaps(grad_in, gb, grad_out, gb) ||
      overlaps(wbar_out, wb, grad_out, gb)) {
    set_error("output buffers overlap the inputs or each other");
    return HWE_EINVAL;
  }
  if (recon) {
    const size_t rb = 6 * mm * N * real_size(m);
    const void* st[4] = {wbar_in, grad_in, wbar_out, grad_out};
    const size_t sz[4] = {wb, gb, wb, gb};
    for (int k = 0; k < 4; ++k)
      if (overlaps(st[k], sz[k], recon, rb)) {
        set_error("the reconstruction buffer overlaps a state buffer");
        return HWE_EINVAL;
      }
  }
  return set_dev(m);
}

hwe_status check_adjoint(hwe_mesh m, const double* wbar_n, const void* grad_n, const void* recon_n,
                         const double* lam_wbar_np1, const void* lam_grad_np1, double* lam_wbar_n, void* lam_grad_n,
                         double dt) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if ((s = check_dt(dt)) != HWE_OK) return s;
  if (!wbar_n || !grad_n || !lam_wbar_np1 || !lam_grad_np1 || !lam_wbar_n || !lam_grad_n) {
    set_error("null state pointer");
    return HWE_EINVAL;
  }
  const size_t N = size_t(m->h.N), mm = size_t(m->h.m);
  const size_t wb = mm * N * sizeof(double), gb = 2 * mm * N * real_size(m);
  const size_t rb = 6 * mm * N * real_size(m);
  const void* ins[5] = {wbar_n, grad_n, lam_wbar_np1, lam_grad_np1, recon_n};
  const size_t insz[5] = {wb, gb, wb, gb, rb};
  for (int k = 0; k < 5; ++k)
    if (ins[k] && (overlaps(ins[k], insz[k], lam_wbar_n, wb) || overlaps(ins[k], insz[k], lam_grad_n, gb))) {
      set_error("output buffers overlap the inputs");
      return HWE_EINVAL;
    }
  if (overlaps(lam_wbar_n, wb, lam_grad_n, gb)) {
    set_error("output buffers overlap each other");
    return HWE_EINVAL;
  }
  return set_dev(m);
}

}  // namespace

hwe_status hwe_step(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out, void* grad_out,
                    double dt, void* stream) {
  hwe_status s = check_step(m, wbar_in, grad_in, wbar_out, grad_out, dt, nullptr);
  if (s != HWE_OK) return s;
  return launch_step(m, wbar_in, grad_in, wbar_out, grad_out, dt, nullptr, stream);
}

hwe_status hwe_step_noalloc(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out,
                            void* grad_out, double dt, void* stream) {
  hwe_status s = check_step(m, wbar_in, grad_in, wbar_out, grad_out, dt, nullptr);
  if (s != HWE_OK) return s;
  return launch_step_noalloc(m, wbar_in, grad_in, wbar_out, grad_out, dt, stream);
}

hwe_status hwe_step_keep(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out, void* grad_out,
                         double dt, void* recon_out, void* stream) {
  if (!recon_out || !aligned16(recon_out)) {
    set_error("null or misaligned reconstruction buffer (16-byte alignment required)");
    return HWE_EINVAL;
  }
  hwe_status s = check_step(m, wbar_in, grad_in, wbar_out, grad_out, dt, recon_out);
  if (s != HWE_OK) return s;
  return launch_step(m, wbar_in, grad_in, wbar_out, grad_out, dt, recon_out, stream);
}

hwe_status hwe_step_adjoint(hwe_mesh m, const double* wbar_n, const void* grad_n, const double* lam_wbar_np1,
                            const void* lam_grad_np1, double* lam_wbar_n, void* lam_grad_n, double dt, void* stream) {
  hwe_status s = check_adjoint(m, wbar_n, grad_n, nullptr, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt);
  if (s != HWE_OK) return s;
  return launch_adjoint(m, wbar_n, grad_n, nullptr, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt, stream);
}

hwe_status hwe_step_adjoint_kept(hwe_mesh m, const double* wbar_n, const void* grad_n, const void* recon_n,
                                 const double* lam_wbar_np1, const void* lam_grad_np1, double* lam_wbar_n,
                                 void* lam_grad_n, double dt, void* stream) {
  if (!recon_n || !aligned16(recon_n)) {
    set_error("null or misaligned reconstruction buffer (16-byte alignment required)");
    return HWE_EINVAL;
  }
  hwe_status s = check_adjoint(m, wbar_n, grad_n, recon_n, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt);
  if (s != HWE_OK) return s;
  return launch_adjoint(m, wbar_n, grad_n, recon_n, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt, stream);
}

hwe_status hwe_max_dt(hwe_mesh m, const double* wbar, double cfl, double* dt_dev, void* stream) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if (!wbar || !dt_dev || !(cfl > 0.0) || !std::isfinite(cfl)) {
    set_error("null pointer or invalid cfl");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  return launch_max_dt(m, wbar, cfl, dt_dev, stream);
}

hwe_status hwe_check_state(hwe_mesh m, const double* wbar, int32_t* flags_dev, void* stream) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if (!wbar || !flags_dev) {
    set_error("null pointer");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  return launch_check(m, wbar, flags_dev, stream);
}

hwe_status hwe_debug_recon(hwe_mesh m, const double* wbar, const void* grad, void* R_out, void* stream) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if (!wbar || !grad || !R_out) {
    set_error("null pointer");
    return HWE_EINVAL;
  }
  if (!aligned16(R_out)) {
    set_error("misaligned reconstruction buffer (16-byte alignment required)");
    return HWE_EINVAL;
  }
  const size_t N = size_t(m->h.N), mm = size_t(m->h.m);
  if (overlaps(R_out, 6 * mm * N * real_size(m), wbar, mm * N * sizeof(double)) ||
      overlaps(R_out, 6 * mm * N * real_size(m), grad, 2 * mm * N * real_size(m))) {
    set_error("the output buffer overlaps the state");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  return launch_recon(m, wbar, grad, R_out, m->time, stream);
}

hwe_status hwe_debug_edge(hwe_mesh m, const void* R, const double* wbar, double dt, double* F_out, void* G_out,
                          void* stream) {
  if ((R && !aligned16(R)) || (F_out && !aligned16(F_out)) || (G_out && !aligned16(G_out))) {
    set_error("misaligned record buffer (16-byte alignment required)");
    return HWE_EINVAL;
  }
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if ((s = check_dt(dt)) != HWE_OK) return s;
  if (!R || !wbar || !F_out || !G_out) {
    set_error("null pointer");
    return HWE_EINVAL;
  }
  const size_t N = size_t(m->h.N), E = size_t(m->h.E), mm = size_t(m->h.m);
  const size_t rb = 6 * mm * N * real_size(m), wb = mm * N * sizeof(double);
  const size_t fb = mm * E * sizeof(double), gb = mm * E * real_size(m);
  if (overlaps(F_out, fb, G_out, gb) || overlaps(F_out, fb, R, rb) || overlaps(F_out, fb, wbar, wb) ||
      overlaps(G_out, gb, R, rb) || overlaps(G_out, gb, wbar, wb)) {
    set_error("output buffers overlap the inputs or each other");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  return launch_edge(m, R, wbar, dt, F_out, G_out, stream);
}

hwe_status hwe_profile_begin(hwe_mesh m, int32_t n_steps) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if (n_steps <= 0 || n_steps > (1 << 20)) {
    set_error("n_steps out of range");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  return profile_begin(m, n_steps);
}

hwe_status hwe_profile_end(hwe_mesh m, double* ms_sum, int32_t* n_steps_done) {
  hwe_status s = need_device(m);
  if (s != HWE_OK) return s;
  if (!ms_sum || !n_steps_done) {
    set_error("null pointer");
    return HWE_EINVAL;
  }
  if ((s = set_dev(m)) != HWE_OK) return s;
  int n = 0;
  s = profile_end(m, ms_sum, &n);
  *n_steps_done = n;
  return s;
}

hwe_status hwe_debug_host_array(hwe_mesh m, int32_t which, double* out) {
  if (!m || !out) {
    set_error("null argument");
    return HWE_EINVAL;
  }
  const HostMesh& h = m->h;
  switch (which) {
    case 0:
      std::memcpy(out, h.p1.data(), h.p1.size() * sizeof(double));
      return HWE_OK;
    case 1:
      std::memcpy(out, h.cen.data(), h.cen.size() * sizeof(double));
      return HWE_OK;
    case 2:
      std::memcpy(out, h.area.data(), h.area.size() * sizeof(double));
      return HWE_OK;
    case 3:
      std::memcpy(out, h.mom.data(), h.mom.size() * sizeof(double));
      return HWE_OK;
    case 4:
      for (size_t k = 0; k < h.nbr.size(); ++k) out[k] = double(h.nbr[k]);
      return HWE_OK;
    case 6:
      std::memcpy(out, h.p1f.data(), h.p1f.size() * sizeof(double));
      return HWE_OK;
    case 7:
      for (size_t k = 0; k < h.cell_edge.size(); ++k) out[k] = double(h.cell_edge[k]);
      return HWE_OK;
    case 8:
      for (size_t k = 0; k < h.ecell.size(); ++k) out[k] = double(h.ecell[k]);
      return HWE_OK;
    case 5:
      // boundary kind of each face, -1 on interior faces
      for (size_t k = 0; k < h.nbr.size(); ++k)
        out[k] = h.nbr[k] >= 0 ? -1.0 : h.bnd_n[2 * h.NB + (-h.nbr[k] - 1)];
      return HWE_OK;
    default:
      set_error("unknown array id");
      return HWE_EINVAL;
  }
}

}  // extern "C"
