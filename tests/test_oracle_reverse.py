"""Oracle pins for its reverse mode (the vector-Jacobian product of the step,
recorded on local tapes per cell and reversed), the reference of the GPU
adjoint's element-wise comparisons.

Two pins tie it to the dual-number JVP, which is itself pinned against
central differences of the step (tests/test_oracle_step.py,
tests/test_oracle_boundaries.py, tests/test_oracle_limiter.py):
* the transpose identity <J^T lam, v> = <lam, J v> on every boundary kind, the
  limiter, the variant rules and several steps;
* element by element, J^T lam against the full Jacobian assembled column by
  column from JVPs on small meshes.
"""
import numpy as np
import pytest

from oracle import OracleMesh
from workloads import (advection_workload, burgers_workload, double_mach_workload, near_vacuum_state,
                       riemann_workload, shock_tube_workload, split_square_mesh, vortex_workload, wedge_workload)

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _case(name):
    """(oracle mesh, state, dt, start time)"""
    rng = np.random.default_rng(7)
    if name == "advection":
        wl = advection_workload(n=8)
        om = OracleMesh.from_workload(wl)
        return om, wl.state0, om.max_dt(wl.state0, 0.3), 0.0
    if name == "burgers_shocked":
        wl = burgers_workload(n=10, T=1.5 / np.pi)
        om = OracleMesh.from_workload(wl)
        dt = om.max_dt(wl.state0, 0.3)
        return om, om.run(wl.state0, dt, 40), dt, 0.0
    if name == "vortex":
        wl = vortex_workload(n=8)
        om = OracleMesh.from_workload(wl)
        return om, wl.state0, om.max_dt(wl.state0, 0.3), 0.0
    if name == "vortex_variants":
        wl = vortex_workload(n=8)
        om = OracleMesh.from_workload(wl, time_rule=1, edge_rule=3, deriv_weight=0.5)
        return om, wl.state0, om.max_dt(wl.state0, 0.3), 0.0
    if name in ("sod_walls", "double_mach_moving", "wedge_walls_inflow"):
        wl, t0 = {"sod_walls": (shock_tube_workload("sod", nx=24), 0.0),
                  "double_mach_moving": (double_mach_workload(n=4), 0.012),
                  "wedge_walls_inflow": (wedge_workload(nx=16, ny=8), 0.0)}[name]
        om = OracleMesh.from_workload(wl)
        s0 = wl.state0 * (1.0 + 1e-3 * rng.uniform(-1, 1, wl.state0.shape))
        s0[1:] = 0.1 * rng.normal(size=s0[1:].shape) * np.abs(s0[0])[None] / wl.mesh.h
        return om, s0, om.max_dt(s0, 0.3), t0
    if name in ("limiter_pressure", "limiter_density"):
        wl = riemann_workload(n=12)
        om = OracleMesh.from_workload(wl, positivity=1)
        s0 = near_vacuum_state(wl, 41, name.split("_")[1], untie=True)
        return om, s0, om.max_dt(s0, 0.2), 0.0
    raise KeyError(name)


CASES = ["advection", "burgers_shocked", "vortex", "vortex_variants", "sod_walls", "double_mach_moving",
         "wedge_walls_inflow", "limiter_pressure", "limiter_density"]


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nsteps", [1, 3])
def test_reverse_mode_is_the_transpose_of_the_jvp(name, nsteps):
    om, s0, dt, t0 = _case(name)
    rng = np.random.default_rng(11)
    lam = rng.normal(size=s0.shape)
    v = rng.normal(size=s0.shape) * (np.abs(s0) + 1e-3 * np.abs(s0).max())
    vj = om.vjp(s0, lam, dt, nsteps, t=t0)
    _, jv = om.jvp(s0, v, dt, nsteps, t=t0)
    a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
    scale = float(np.abs(vj * v).sum())
    print(name, nsteps, a, b, abs(a - b) / scale, flush=True)
    assert abs(a - b) <= 1e-12 * scale


def _jacobian(om, s0, dt, t0):
    """The full Jacobian of one step, column by column from JVPs: (n, n)."""
    n = s0.size
    J = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        _, col = om.jvp(s0, e.reshape(s0.shape), dt, 1, t=t0)
        J[:, j] = col.ravel()
    return J


@pytest.mark.parametrize("name", ["euler_periodic", "euler_walls_limiter", "burgers"])
def test_reverse_mode_equals_the_assembled_jacobian_transpose(name):
    rng = np.random.default_rng(5)
    if name == "euler_periodic":
        box = (0.0, 10.0, 0.0, 10.0)
        mesh = split_square_mesh(3, box, jitter=0.1, seed=2, periodic=True)
        om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=0, box=box)
        N = om.N
        rho, u, v, p = (rng.uniform(0.8, 1.2, N), rng.uniform(-0.5, 0.5, N), rng.uniform(-0.5, 0.5, N),
                        rng.uniform(0.8, 1.2, N))
        s0 = np.zeros((3, 4, N))
        s0[0] = [rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)]
        s0[1:] = 0.05 * rng.normal(size=(2, 4, N))
    elif name == "euler_walls_limiter":
        box = (0.0, 1.0, 0.0, 1.0)
        mesh = split_square_mesh(3, box, jitter=0.1, seed=3, periodic=False)
        om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=1, box=box, walls=5, positivity=1)
        N = om.N
        rho, u, v, p = (rng.uniform(0.5, 1.5, N), rng.uniform(-0.5, 0.5, N), rng.uniform(-0.5, 0.5, N),
                        rng.uniform(1e-3, 2e-3, N))
        s0 = np.zeros((3, 4, N))
        s0[0] = [rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)]
        s0[1:] = 2.0 * rng.normal(size=(2, 4, N))
    else:
        box = (0.0, 1.0, 0.0, 1.0)
        mesh = split_square_mesh(4, box, jitter=0.2, seed=4, periodic=True)
        om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box)
        N = om.N
        s0 = np.zeros((3, 1, N))
        s0[0, 0] = rng.uniform(-1, 1, N)
        s0[1:, 0] = rng.normal(size=(2, N))
    dt = om.max_dt(s0, 0.3)
    if name == "euler_walls_limiter":
        limited = sum(bool(om.recon_theta(s0, k).min() < 1.0) for k in range(om.N))
        assert limited >= 4, limited
    J = _jacobian(om, s0, dt, 0.0)
    for seed in range(3):
        lam = np.random.default_rng(seed).normal(size=s0.shape)
        ref = (J.T @ lam.ravel()).reshape(s0.shape)
        got = om.vjp(s0, lam, dt, 1)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(name, seed, err, flush=True)
        assert err <= 1e-13


def test_operation_counts_are_per_cell_and_per_edge_constants():
    """The live operation counts of one step (the tape's arithmetic nodes that a
    result depends on) on periodic vortex meshes of 128 and 512 cells: every
    cell and every edge does the same work up to data-dependent branches (the
    kappa = 0 case of the weights, the losing radius of the flux viscosity),
    so the counts per cell (reconstruction, update) and per edge (viscosity,
    evaluation, Lax-Wendroff, fluxes) agree within 1% between the sizes.  A
    step of linear advection, whose fluxes are linear, needs far fewer
    Lax-Wendroff operations per point than the Euler equations."""
    per = []
    for n in (8, 16):
        wl = vortex_workload(n=n)
        om = OracleMesh.from_workload(wl)
        c = om.count_flops(wl.state0, om.max_dt(wl.state0, 0.3))
        per.append(np.array([c["recon"] / om.N, c["update"] / om.N,
                             *(c[k] / (2 * om.E) for k in ("alpha", "eval", "lax_wendroff", "flux"))]))
        assert c["limiter"] == 0
    assert np.allclose(per[0], per[1], rtol=1e-2, atol=0), per
    wl = advection_workload(n=8)
    om = OracleMesh.from_workload(wl)
    c = om.count_flops(wl.state0, om.max_dt(wl.state0, 0.3))
    lw_adv = c["lax_wendroff"] / (2 * om.E) / 4       # 2 sides x 2 Gauss points per edge evaluation
    lw_eul = per[1][4] / 4
    print("vortex per cell / per edge:", per[1], "LW per point and side: advection", lw_adv, "Euler", lw_eul,
          flush=True)
    assert 0 < lw_adv < 30 and lw_eul > 500


def test_benchmark_flop_constants_are_the_oracle_counts():
    """bench.py's algorithmic operation counts (edge stage per edge, whole
    step per cell) are the oracle's live counts on the 512-cell vortex."""
    import bench
    wl = vortex_workload(n=16)
    om = OracleMesh.from_workload(wl)
    c = om.count_flops(wl.state0, om.max_dt(wl.state0, 0.3))
    pe = {k: c[k] / (2 * om.E) for k in ("alpha", "eval", "lax_wendroff", "flux")}
    edge = pe["alpha"] + pe["lax_wendroff"] + pe["flux"]
    cell_step = (c["recon"] + c["update"]) / om.N + sum(pe.values()) * om.E / om.N
    assert abs(edge - bench.EDGE_ALG_FLOP_PER_EDGE) <= 1.0, edge
    assert abs(cell_step - bench.ALG_FLOP_PER_CELL_STEP) <= 1.0, cell_step
