"""Oracle pins for the whole step: invariants, exactness, convergence orders, JVP.

* free-stream preservation and round-off mass conservation (flux form, eq. (flx));
* one step of linear advection is exact on quadratic data with the linear
  weights (Taylor, Lax-Wendroff, Simpson-in-time and 2-point Gauss are all exact
  there) and on linear data with the nonlinear weights;
* invariance under cell and vertex renumbering and under a shift of the origin;
* third-order convergence against exact solutions (Tables 1-3 report ~3);
* dual-number JVP against central finite differences of the forward map.
"""
import numpy as np
import pytest

from oracle import OracleMesh
from workloads import (advection_workload, burgers_workload, cell_average_states, density_wave_workload,
                       split_square_mesh, vortex_workload)

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _l1(a, b, area):
    return float(np.sum(np.abs(a - b) * area) / np.sum(area))


@pytest.mark.parametrize("eq,bc", [(1, 0), (2, 0), (2, 1), (0, 1)])
def test_free_stream_is_preserved(eq, bc):
    box = (0.0, 2.0, -1.0, 1.0)
    mesh = split_square_mesh(10, box, jitter=0.3, seed=21, periodic=(bc == 0))
    om = OracleMesh(mesh.nodes, mesh.tris, eq=eq, bc=bc, box=box)
    m = om.m
    s = np.zeros((3, m, om.N))
    W0 = np.array([1.3, 0.5, -0.7, 3.1])[:m] if eq == 2 else np.array([0.8])
    s[0] = W0[:, None]
    out = om.run(s, 0.01, 5)
    assert np.abs(out[0] - s[0]).max() <= 1e-14 * np.abs(W0).max()
    h = 0.2
    assert np.abs(out[1:]).max() <= 1e-12 * np.abs(W0).max() / h


@pytest.mark.parametrize("which", ["burgers_shock", "vortex"])
def test_mass_is_conserved_to_round_off(which):
    if which == "burgers_shock":
        wl = burgers_workload(n=12, T=1.5 / np.pi)
        nsteps = 200
    else:
        wl = vortex_workload(n=8)
        nsteps = 60
    om = OracleMesh.from_workload(wl)
    area = om.geometry()["area"]
    dt = om.max_dt(wl.state0, 0.3)
    s = om.run(wl.state0, dt, nsteps)
    m0 = (wl.state0[0] * area).sum(axis=1)
    m1 = (s[0] * area).sum(axis=1)
    scale = (np.abs(wl.state0[0]) * area).sum(axis=1)
    assert np.all(np.abs(m1 - m0) <= 1e-13 * scale), (m1 - m0) / scale


def _deep_interior(om, layers=2):
    nb = om.geometry()["nbr"]
    ok = (nb >= 0).all(axis=1)
    for _ in range(layers - 1):
        ok = ok & np.array([ok[nb[k]].all() if ok[k] else False for k in range(om.N)])
    return np.nonzero(ok)[0]


@pytest.mark.parametrize("time_rule,edge_rule", [(0, 2), (1, 2), (0, 3)])
def test_one_advection_step_is_exact_on_quadratics_with_linear_weights(time_rule, edge_rule):
    """Either time rule integrates the quadratic-in-time linear flux exactly,
    and either edge rule the quadratic-in-space one."""
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(8, box, jitter=0.25, seed=12, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box, adv=(0.7, -0.4), linear_only=1,
                    time_rule=time_rule, edge_rule=edge_rule)
    q = lambda x, y: 0.4 - 1.3 * x + 0.6 * y + 0.8 * x * x - 0.5 * x * y + 1.1 * y * y
    f = lambda x, y, t: q(x - 0.7 * t, y + 0.4 * t)[..., None]
    s0 = cell_average_states(mesh, f, 0.0)
    dt = 0.03
    s1 = om.step(s0, dt)
    ex = cell_average_states(mesh, f, dt)
    cells = _deep_interior(om, 2)
    assert cells.size > 20
    err = np.abs(s1[:, 0, cells] - ex[:, 0, cells]).max(axis=1)
    assert err[0] < 1e-14 and err[1] < 1e-12 and err[2] < 1e-12, err


@pytest.mark.parametrize("time_rule,wd", [(0, 1.0), (1, 0.4)])
def test_one_step_is_exact_on_linear_data_with_nonlinear_weights(time_rule, wd):
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(8, box, jitter=0.25, seed=13, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box, adv=(1.0, 1.0), time_rule=time_rule,
                    deriv_weight=wd)
    f = lambda x, y, t: (2.0 + 0.9 * (x - t) - 0.3 * (y - t))[..., None]
    s0 = cell_average_states(mesh, f, 0.0)
    dt = 0.02
    s1 = om.step(s0, dt)
    ex = cell_average_states(mesh, f, dt)
    cells = _deep_interior(om, 2)
    assert np.abs(s1[:, 0, cells] - ex[:, 0, cells]).max() < 1e-12


@pytest.mark.parametrize("eq", [1, 2])
def test_renumbering_and_origin_shift_invariance(eq):
    box = (0.0, 2.0, 0.0, 2.0)
    mesh = split_square_mesh(7, box, jitter=0.2, seed=5, periodic=True)
    m = 4 if eq == 2 else 1
    if eq == 2:
        wl = vortex_workload(n=7)
        f = None
        s0 = wl.state0
        mesh, box = wl.mesh, wl.mesh.box
    else:
        s0 = cell_average_states(mesh, lambda x, y, t: (0.5 + np.sin(np.pi * (x + 2 * y)))[..., None])
    om = OracleMesh(mesh.nodes, mesh.tris, eq=eq, bc=0, box=box)
    dt = 0.3 * om.max_dt(s0, 0.3)
    ref = om.run(s0, dt, 3)
    rng = np.random.default_rng(1)
    perm = rng.permutation(om.N)                 # new cell i is old cell perm[i]
    rot = rng.integers(0, 3, om.N)
    tris = np.stack([np.roll(t, r) for t, r in zip(mesh.tris[perm], rot)])
    om2 = OracleMesh(mesh.nodes, tris, eq=eq, bc=0, box=box)
    out = om2.run(s0[:, :, perm], dt, 3)
    assert np.allclose(out, ref[:, :, perm], rtol=0, atol=1e-12 * np.abs(ref).max())
    # shift of the origin (and of the periodic box) by a non-representable amount
    d = np.array([0.3, -0.7])
    sbox = (box[0] + d[0], box[1] + d[0], box[2] + d[1], box[3] + d[1])
    om3 = OracleMesh(mesh.nodes + d, mesh.tris, eq=eq, bc=0, box=sbox)
    out3 = om3.run(s0, dt, 3)
    assert np.allclose(out3, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def _orders(errs):
    e = np.array(errs)
    return np.log2(e[:-1] / e[1:])


def test_convergence_linear_advection():
    errs = []
    for n in (10, 20, 40):
        wl = advection_workload(n=n, jitter=0.1, T=0.25)
        om = OracleMesh.from_workload(wl)
        dt = om.max_dt(wl.state0, 0.3)
        s = om.run_to(wl.state0, wl.T, dt)
        errs.append(_l1(s[0, 0], wl.exact_state(wl.T)[0, 0], om.geometry()["area"]))
    o = _orders(errs)
    assert o[-1] > 2.6, (errs, o)


@pytest.mark.parametrize("time_rule", [0, 1])
def test_convergence_burgers_paper_example_4_1(time_rule):
    """Example 4.1: u0 = 0.5 + sin(pi(x+y)/2) on (-2,2)^2, T = 0.5/pi (smooth);
    third order with either time rule."""
    errs = []
    for n in (10, 20, 40):
        wl = burgers_workload(n=n, box=(-2.0, 2.0, -2.0, 2.0), jitter=0.1)
        om = OracleMesh.from_workload(wl, time_rule=time_rule)
        dt = om.max_dt(wl.state0, 0.3)
        s = om.run_to(wl.state0, wl.T, dt)
        errs.append(_l1(s[0, 0], wl.exact_state(wl.T)[0, 0], om.geometry()["area"]))
    o = _orders(errs)
    assert o[-1] > 2.6, (errs, o)


def test_convergence_euler_density_wave_paper_example_4_2():
    errs = []
    for n in (8, 16, 32):
        wl = density_wave_workload(n=n, T=0.25)
        om = OracleMesh.from_workload(wl)
        dt = om.max_dt(wl.state0, 0.3)
        s = om.run_to(wl.state0, wl.T, dt)
        errs.append(_l1(s[0, 0], wl.exact_state(wl.T)[0, 0], om.geometry()["area"]))
    o = _orders(errs)
    assert (o > 2.6).all(), (errs, o)


def test_time_rules_differ_only_at_fifth_order_in_dt():
    """Burgers: the flux is quartic in time along the Taylor polynomial, which
    neither 3-point Gauss-Lobatto (error dt^5/120 on tau^4) nor 2-point
    Gauss-Legendre (-dt^5/180) integrates exactly: the two one-step results
    differ, by an amount that falls as dt^5 (local error per unit time dt^4,
    times dt for one step)."""
    wl = burgers_workload(n=12, box=(-2.0, 2.0, -2.0, 2.0), jitter=0.1)
    oa = OracleMesh.from_workload(wl, time_rule=0)
    ob = OracleMesh.from_workload(wl, time_rule=1)
    d = []
    for dt in (0.02, 0.01):
        a, b = oa.step(wl.state0, dt), ob.step(wl.state0, dt)
        d.append(np.abs(a[0] - b[0]).max())
    assert d[0] > 0 and d[1] > 0
    assert 20 < d[0] / d[1] < 50, d                   # ~2^5


def test_edge_rules_agree_on_advection_and_differ_at_fourth_order_on_burgers():
    """Linear advection: the flux along an edge is a quadratic polynomial, which
    the 2- and 3-point Gauss-Legendre rules both integrate exactly, so the
    steps agree to round-off.  Burgers: the flux is quartic along the edge and
    the 2-point rule's error (the 4th derivative term) makes the one-step
    results differ by O(h^4) at a fixed CFL number."""
    wl = advection_workload(n=16, jitter=0.2)
    a, b = OracleMesh.from_workload(wl), OracleMesh.from_workload(wl, edge_rule=3)
    dt = a.max_dt(wl.state0, 0.3)
    sa, sb = a.run(wl.state0, dt, 10), b.run(wl.state0, dt, 10)
    assert np.abs(sa - sb).max() <= 1e-13 * np.abs(sa).max()
    d = []
    for n in (24, 48):
        wl = burgers_workload(n=n, box=(-2.0, 2.0, -2.0, 2.0), jitter=0.1)
        a, b = OracleMesh.from_workload(wl), OracleMesh.from_workload(wl, edge_rule=3)
        dt = 0.1 * 4.0 / n
        d.append(np.abs(a.step(wl.state0, dt)[0] - b.step(wl.state0, dt)[0]).max())
    assert d[1] > 0 and 10 < d[0] / d[1] < 24, d          # ~2^4


@pytest.mark.parametrize("eq", [0, 1, 2])
def test_dual_jvp_matches_central_differences(eq):
    if eq == 2:
        wl = vortex_workload(n=5)
    elif eq == 1:
        wl = burgers_workload(n=5, T=1.0)
    else:
        wl = advection_workload(n=5)
    om = OracleMesh.from_workload(wl)
    rng = np.random.default_rng(eq)
    # split-square cells mirrored across a diagonal can hold bit-identical
    # averages, which puts alpha = max(., .) exactly on its tie; a small seeded
    # perturbation keeps the finite differences away from that kink
    s0 = wl.state0 * (1.0 + 1e-3 * rng.uniform(-1, 1, wl.state0.shape))
    dt = om.max_dt(s0, 0.3)
    v = rng.normal(size=s0.shape)
    v *= 1e-2 * np.abs(s0).max() / np.abs(v).max()
    out, jv = om.jvp(s0, v, dt, 3)
    assert np.allclose(out, om.run(s0, dt, 3), rtol=0, atol=1e-14 * np.abs(out).max())
    # the weights make the map strongly nonlinear on coarse meshes: the central
    # difference error must fall like eps^2 towards the JVP
    errs = []
    for eps in (1e-3, 1e-4, 1e-5):
        fd = (om.run(s0 + eps * v, dt, 3) - om.run(s0 - eps * v, dt, 3)) / (2 * eps)
        errs.append(np.abs(jv - fd).max() / np.abs(jv).max())
    assert errs[-1] <= 2e-6, errs
    assert errs[1] <= max(0.05 * errs[0], 1e-9), errs
