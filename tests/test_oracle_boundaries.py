"""Oracle pins for prescribed (inflow) boundary states and for a prescribed
state that switches across a moving shock position (Sec. 4: the double Mach
reflection problems, the forward step, the Shu-Osher problem).

A prescribed face has a ghost cell that holds the state with zero derivative
averages, and the exterior value at its Gauss points is that state at every
time node.  A moving face takes state A where its midpoint has
x < x0 + speed * (t_n + dt / 2), else B.

* face kinds follow the region rectangles (checked against the faces' own
  coordinates, first match wins);
* a uniform state with the same state prescribed all round stays uniform, and a
  supersonic inflow keeps the cells near the inlet at the inflow state exactly
  until the waves from the step arrive;
* prescribed ends equal to the end states give the transmissive result to
  round-off while no wave has reached them (the nonlinear weights of a flat
  cell sum to one only to rounding, so the interior value differs from the
  prescribed one in the last bits);
* a planar Mach 10 shock running along a strip with the moving switch on both
  long sides: the shock position from the total mass matches x0 + 10 t within
  a small fraction of a cell, and the density error converges at first order;
* the double Mach reflection far from the wall (y > 0.6) converges to the
  exactly moving oblique shock, which a frozen top boundary does not.
"""
import numpy as np
import pytest

from oracle import OracleMesh
from oracle.oracle import BND_KINDS
from workloads import (DMR_A, DMR_B, cell_average_states, double_mach_workload, forward_step_workload,
                       moving_shock_workload, piecewise_average_states, shock_tube_workload, split_square_mesh,
                       wedge_workload)
from workloads.problems import _two_state

pytestmark = pytest.mark.usefixtures("oracle_lib")

R3 = np.sqrt(3.0)


def _run(om, s, T, cfl=0.3):
    t = 0.0
    while t < T - 1e-14 * T:
        dt = min(om.max_dt(s, cfl), T - t)
        s = om.step(s, dt, t=t)
        t += dt
    return s


def test_face_kinds_follow_the_regions():
    wl = double_mach_workload(n=12)
    om = OracleMesh.from_workload(wl)
    kinds = om.face_kinds()
    V = om.cell_vertices()
    for k in range(om.N):
        for f in range(3):
            if kinds[k, f] < 0:
                continue
            a, b = V[k, f], V[k, (f + 1) % 3]
            mx, my = 0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1])
            if abs(my) < 1e-12:
                want = "A" if mx < 1.0 / 6.0 else "wall"
            elif abs(my - 1.0) < 1e-12:
                want = "moving"
            elif abs(mx) < 1e-12:
                want = "A"
            else:
                assert abs(mx - 4.0) < 1e-12
                want = "transmissive"
            assert kinds[k, f] == BND_KINDS[want], (k, f, mx, my)


def test_uniform_state_with_the_same_state_prescribed_all_round():
    W = np.array([1.2, 0.6, -0.3, 2.9])
    mesh = split_square_mesh((10, 6), (0.0, 1.0, 0.0, 0.6), jitter=0.2, seed=31, periodic=False)
    regions = (("A", (0.0, 1.0, 0.0, 0.6)),)
    om = OracleMesh(mesh.nodes, mesh.tris, 2, bc=1, box=mesh.box, regions=regions, states=(W, W))
    s = np.zeros((3, 4, mesh.n_cells))
    s[0] = W[:, None]
    out = om.run(s, 0.2 * om.max_dt(s, 1.0), 10)
    assert np.abs(out[0] - W[:, None]).max() <= 1e-13
    assert np.abs(out[1:]).max() <= 1e-12


def test_supersonic_inlet_stays_at_the_inflow_state():
    # a step moves a perturbation by at most a couple of cell layers (compact
    # stencil), so after 3 steps the cells at x < 0.2 (8 layers upstream of the
    # step face at x = 0.6) must still hold the inflow state exactly
    wl = forward_step_workload(n=20)
    om = OracleMesh.from_workload(wl)
    g = om.geometry()
    s = wl.state0
    t = 0.0
    for _ in range(3):
        dt = om.max_dt(s, 0.3)
        s = om.step(s, dt, t=t)
        t += dt
    W = np.asarray(wl.states[0])
    near = g["cx"] < 0.2
    assert near.sum() > 100
    assert np.abs(s[0][:, near] - W[:, None]).max() <= 1e-13 * np.abs(W).max()
    assert np.abs(s[1:][:, :, near]).max() <= 1e-12
    assert np.abs(s[0] - W[:, None]).max() > 1e-3      # the step did act downstream


def test_prescribed_ends_equal_transmissive_ends_before_the_waves_arrive():
    wl = shock_tube_workload("sod", nx=60)
    x0, x1, y0, y1 = wl.mesh.box
    WL, WR = wl.state0[0][:, 0], wl.state0[0][:, -1]
    a = OracleMesh.from_workload(wl)
    b = OracleMesh.from_workload(wl, regions=(("A", (x0, x0, y0, y1)), ("B", (x1, x1, y0, y1))), states=(WL, WR))
    dt = 0.5 * a.max_dt(wl.state0, 0.3)
    sa = a.run(wl.state0, dt, 20)
    sb = b.run(wl.state0, dt, 20)
    scale = np.abs(sa).max(axis=2, keepdims=True) + 1e-300
    assert (np.abs(sa - sb) / scale).max() <= 1e-12
    assert np.abs(sa - wl.state0).max() > 1e-3     # the waves did move


def _moving_shock_run(nx):
    wl = moving_shock_workload(nx=nx)
    om = OracleMesh.from_workload(wl)
    s = _run(om, wl.state0, wl.T)
    g = om.geometry()
    H = wl.mesh.box[3] - wl.mesh.box[2]
    rA, rB = wl.states[0][0], wl.states[1][0]
    xs = ((s[0, 0] * g["area"]).sum() / H - rB) / (rA - rB)
    xe = wl.extra["x_shock"](wl.T)
    ex = piecewise_average_states(wl.mesh, _two_state(wl.states[0], wl.states[1], 1.0, 0.0, xe), [(1.0, 0.0, xe)])
    l1 = float((np.abs(s[0, 0] - ex[0, 0]) * g["area"]).sum() / g["area"].sum())
    return xs, xe, l1, wl.mesh.h


def test_moving_shock_position_and_convergence():
    xs1, xe, l1a, h1 = _moving_shock_run(50)
    xs2, _, l1b, h2 = _moving_shock_run(100)
    print("moving shock: x from mass", xs1, xs2, "exact", xe, "L1", l1a, l1b, flush=True)
    assert abs(xs1 - xe) <= 0.05 * h1
    assert abs(xs2 - xe) <= 0.05 * h2
    assert l1b <= 0.05
    assert l1a / l1b >= 1.6


def test_run_and_jvp_follow_the_steps_through_the_moving_switch():
    """Every entry of the oracle that steps in time evaluates the moving
    boundary states at the middle of each step, as one step does (whose
    switch time the shock-position test above fixes): four steps of run, and
    the primal output of the JVP, equal four single steps from t0, t0 + dt,
    ... bitwise, on the double Mach mesh while the switch crosses top faces."""
    wl = double_mach_workload(n=12)
    om = OracleMesh.from_workload(wl)
    dt = om.max_dt(wl.state0, 0.3)
    t0 = 0.012 + 12 * dt          # the switch passes a top face midpoint within the next four steps
    b = wl.state0
    for k in range(4):
        b = om.step(b, dt, t=t0 + k * dt)
    a = om.run(wl.state0, dt, 4, t=t0)
    j, _ = om.jvp(wl.state0, np.zeros_like(wl.state0), dt, 4, t=t0)
    assert np.array_equal(a, b)
    assert np.array_equal(j, b)
    # the switch moves across a face within these steps: the top boundary
    # faces' states are not the same at t0 and at t0 + 4 dt
    assert np.abs(om.step(wl.state0, dt, t=t0 + 4 * dt) - om.step(wl.state0, dt, t=t0)).max() > 0.0


def test_prescribed_ghost_is_a_flat_cell_holding_the_state():
    """Reading: the ghost across a prescribed face is the cell's mirror image
    across the face, holding the prescribed state with zero derivative
    averages.  So the reconstruction of a cell with such a face (candidates,
    smoothness indicators, weights) equals, to round-off, its reconstruction on
    the mesh extended by that mirror triangle as an ordinary cell holding the
    state and zero derivative averages, the face then interior.  The cell's own
    derivative averages are far from zero, so a ghost that kept them (mirrored)
    would differ."""
    mesh = split_square_mesh((6, 6), (0.0, 1.0, 0.0, 1.0), jitter=0.2, seed=33, periodic=False)
    Wb = [1.4, 0.5, 0.1, 2.9]
    kw = dict(eq=2, bc=1, box=(0.0, 1.0, 0.0, 1.0), regions=[("A", (-0.01, 0.01, -1.0, 2.0))], states=[Wb, Wb])
    A = OracleMesh(mesh.nodes, mesh.tris, **kw)
    kinds = A.face_kinds()

    def f(x, y, t):
        b = np.exp(-8.0 * ((x - 0.1) ** 2 + (y - 0.5) ** 2))
        return np.stack([1.0 + 0.4 * b, 0.3 + 0.5 * b, -0.2 * b + 0 * x, 2.5 + 0.8 * b], -1)

    s_A = cell_average_states(mesh, f)
    checked = 0
    for k in range(A.N):
        for fc in range(3):
            if kinds[k, fc] != 2:
                continue
            a, b = mesh.tris[k, fc], mesh.tris[k, (fc + 1) % 3]
            c = mesh.tris[k, (fc + 2) % 3]
            nodes = np.concatenate([mesh.nodes, mesh.nodes[c][None] * np.array([[-1.0, 1.0]])])
            tris = np.concatenate([mesh.tris, np.array([[b, a, len(mesh.nodes)]])]).astype(np.int32)
            P = nodes[tris[-1]]
            assert (P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[1, 1] - P[0, 1]) * (P[2, 0] - P[0, 0]) > 0
            B = OracleMesh(nodes, tris, **kw)
            s_B = np.concatenate([s_A, np.zeros((3, 4, 1))], axis=2)
            s_B[0, :, -1] = Wb
            rA, rB = A.recon_cell(s_A, k), B.recon_cell(s_B, k)
            assert np.abs(s_A[1:, :, k]).max() > 0.3
            for key in ("p", "beta", "omega"):
                err = np.abs(rA[key] - rB[key]).max() / np.abs(rA[key]).max()
                assert err <= 1e-11, (k, key, err)
            checked += 1
    assert checked >= 6


def test_double_mach_far_field_converges_to_the_moving_shock():
    T = 0.02
    errs = []
    for n in (12, 24):
        wl = double_mach_workload(n=n)
        om = OracleMesh.from_workload(wl)
        s = _run(om, wl.state0, T)
        g = om.geometry()
        c = R3 / 6.0 + 20.0 * T
        ex = piecewise_average_states(wl.mesh, _two_state(DMR_A, DMR_B, R3, -1.0, c), [(R3, -1.0, c)])
        sel = g["cy"] > 0.6
        errs.append(float((np.abs(s[0, 0] - ex[0, 0]) * g["area"])[sel].sum() / g["area"][sel].sum()))
    print("double Mach far field L1", errs, flush=True)
    assert errs[1] <= 0.025
    assert errs[0] / errs[1] >= 1.6


@pytest.mark.parametrize("name", ["sod_walls", "double_mach_moving", "wedge_walls_inflow"])
def test_jvp_with_walls_and_prescribed_states_against_central_differences(name):
    """The oracle's dual-number JVP (the reference of the GPU adjoint on these
    meshes) through reflective walls, prescribed inflow states and the moving
    switch, against central differences of its step: the data are untied (no
    equal neighbours, no gas at rest, seeded derivative averages) so that no
    kink of |.| or of a max falls inside a difference stencil; every output
    agrees to 1e-7 of its block's largest."""
    wl, t0 = {"sod_walls": (shock_tube_workload("sod", nx=40), 0.0),
              "double_mach_moving": (double_mach_workload(n=12), 0.012),
              "wedge_walls_inflow": (wedge_workload(nx=32, ny=12), 0.0)}[name]
    om = OracleMesh.from_workload(wl)
    rng = np.random.default_rng(3)
    s0 = wl.state0 * (1.0 + 1e-3 * rng.uniform(-1, 1, wl.state0.shape))
    s0[0, 1:3] += 1e-2 * np.abs(s0[0, 0]) * rng.uniform(-1, 1, s0[0, 1:3].shape)
    s0[1:] = 0.1 * rng.normal(size=s0[1:].shape) * np.abs(s0[0])[None] / wl.mesh.h
    dt = om.max_dt(s0, 0.3)
    v = rng.normal(size=s0.shape) * np.abs(s0)
    _, jv = om.jvp(s0, v, dt, 1, t=t0)
    scale = np.abs(jv).max(axis=2, keepdims=True)

    def fd(e):
        return (om.step(s0 + e * v, dt, t=t0) - om.step(s0 - e * v, dt, t=t0)) / (2 * e)

    f1, f2 = fd(1e-6), fd(5e-7)
    smooth = np.abs(f1 - f2) <= 1e-5 * scale
    rel = float((np.abs(f2 - jv) / scale).max())
    print(name, "smooth outputs", smooth.mean(), "JVP vs central differences", rel, flush=True)
    assert smooth.all()
    assert rel <= 1e-7
