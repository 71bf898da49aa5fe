"""GPU tests of the hand-written adjoint (hwe_step_adjoint) and the checkpointed rollout.

* dot-product test: <J^T lam, v> from the HIP adjoint against <lam, J v> from
  the oracle's dual-number JVP (FP64, several equations; periodic and
  transmissive boundaries, reflective walls, prescribed inflow states and the
  moving switch between two states, with the 2- and 3-point edge rules);
* a checkpointed rollout from t0 > 0 across the moving switch against the
  oracle's multi-step JVP;
* the full gradient on a tiny mesh against the oracle's Jacobian assembled
  column by column from its JVPs;
* the C5 misfit gradient (vortex, 204,800 triangles, 200 steps, checkpoint
  every 20) against central finite differences on 32 random directions of the
  initial density (relative error <= 1e-6 in FP64);
* checkpointing does not change the gradient (bitwise).
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import OracleMesh  # noqa: E402
from workloads import (advection_workload, burgers_workload, fd_directions, make_vortex,  # noqa: E402
                       cell_average_states, double_mach_workload, moving_shock_workload, near_vacuum_state,
                       perturbed_vortex_target_center, riemann_workload, shock_tube_workload, shu_osher_workload,
                       split_square_mesh, vortex_workload, wedge_workload)
from workloads.problems import Workload  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mesh(wl, precision="fp64", **kw):
    from paper_2607_10809_amd.hwe import Mesh
    return Mesh.from_workload(wl, precision=precision, **kw)


def _gpu_vjp(mesh, state, lam, dt):
    import torch
    w, g = mesh.to_device(state)
    lw, lg = mesh.to_device(lam)
    ow, og = mesh.adjoint(w, g, lw, lg, dt)
    torch.cuda.synchronize()
    return mesh.to_host(ow, og)


def _perturbed(wl, rng, rel=1e-3):
    return wl.state0 * (1.0 + rel * rng.uniform(-1, 1, wl.state0.shape))


@pytest.mark.parametrize("case", ["advection", "burgers", "vortex", "riemann"])
def test_dot_product_against_oracle_jvp(case):
    rng = np.random.default_rng(hash(case) % 1000)
    wl = {"advection": lambda: advection_workload(n=20), "burgers": lambda: burgers_workload(n=24, T=1.0),
          "vortex": lambda: vortex_workload(n=24), "riemann": lambda: riemann_workload(n=24)}[case]()
    om = OracleMesh.from_workload(wl)
    s0 = _perturbed(wl, rng)
    if case == "riemann":
        s0 = om.run(s0, om.max_dt(s0, 0.3), 5)       # a state with developed waves and boundary ghosts
    dt = om.max_dt(s0, 0.3)
    mesh = _mesh(wl)
    for _ in range(3):
        v = rng.normal(size=s0.shape)
        lam = rng.normal(size=s0.shape)
        _, jv = om.jvp(s0, v, dt, 1)
        vj = _gpu_vjp(mesh, s0, lam, dt)
        a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
        scale = float(np.abs(vj * v).sum())
        print(case, "<J^T l, v> =", a, "<l, J v> =", b, flush=True)
        assert abs(a - b) <= 1e-11 * scale


def _closed_box_workload():
    """Euler in the unit square with reflective walls all round (a smooth bump)."""
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(12, box, jitter=0.2, seed=22, periodic=False)

    def f(x, y, t):
        r = 1.0 + 0.3 * np.exp(-30 * ((x - 0.4) ** 2 + (y - 0.55) ** 2))
        return np.stack([r, 0.2 * r, -0.1 * r, 2.5 + 0.025 * r + 0 * x], -1)

    return Workload(name="closed box", eq=2, m=4, mesh=mesh, state0=cell_average_states(mesh, f), T=0.1, cfl=0.3,
                    walls=0b1111)


# boundary cases: (workload, start time, oracle pre-steps to develop waves, options)
BOUNDARY_CASES = {
    "sod_walls": (lambda: shock_tube_workload("sod", nx=40), 0.0, 10, {}),
    "closed_box_walls": (_closed_box_workload, 0.0, 5, {}),
    "shu_osher_inflow": (lambda: shu_osher_workload(nx=60, height=0.3), 0.0, 5, {}),
    "double_mach_moving": (lambda: double_mach_workload(n=12), 0.012, 0, {}),
    "wedge_walls_inflow": (lambda: wedge_workload(nx=32, ny=12), 0.0, 5, {}),
    "moving_shock": (lambda: moving_shock_workload(nx=40), 0.01, 0, {}),
    "double_mach_edge3_gauss": (lambda: double_mach_workload(n=12), 0.012, 0, {"edge_rule": 3, "time_rule": 1}),
    "closed_box_edge3": (_closed_box_workload, 0.0, 5, {"edge_rule": 3}),
}


@pytest.mark.parametrize("case", list(BOUNDARY_CASES))
def test_dot_product_with_walls_and_prescribed_states(case):
    """The adjoint on meshes with reflective walls, prescribed inflow states
    and the moving switch between two states, against the oracle's JVP of the
    step from the same time."""
    make, t0, pre, opts = BOUNDARY_CASES[case]
    wl = make()
    rng = np.random.default_rng(sum(map(ord, case)))
    om = OracleMesh.from_workload(wl, **opts)
    s0 = _perturbed(wl, rng)
    if pre:
        s0 = om.run(s0, om.max_dt(s0, 0.3), pre, t=t0)
    dt = om.max_dt(s0, 0.3)
    mesh = _mesh(wl, **opts)
    for _ in range(3):
        v = rng.normal(size=s0.shape)
        lam = rng.normal(size=s0.shape)
        _, jv = om.jvp(s0, v, dt, 1, t=t0)
        import torch
        w, g = mesh.to_device(s0)
        lw, lg = mesh.to_device(lam)
        ow, og = mesh.adjoint(w, g, lw, lg, dt, t=t0)
        torch.cuda.synchronize()
        vj = mesh.to_host(ow, og)
        a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
        scale = float(np.abs(vj * v).sum())
        print(case, "<J^T l, v> =", a, "<l, J v> =", b, "rel", abs(a - b) / scale, flush=True)
        assert abs(a - b) <= 1e-11 * scale


def test_mixed_adjoint_with_walls_close_to_fp64():
    import torch
    wl = double_mach_workload(n=12)
    rng = np.random.default_rng(23)
    s0 = _perturbed(wl, rng)
    dt = OracleMesh.from_workload(wl).max_dt(s0, 0.3)
    lam = rng.normal(size=s0.shape)
    out = []
    for prec in ("fp64", "mixed"):
        mesh = _mesh(wl, prec)
        w, g = mesh.to_device(s0)
        lw, lg = mesh.to_device(lam)
        ow, og = mesh.adjoint(w, g, lw, lg, dt, t=0.012)
        torch.cuda.synchronize()
        out.append(mesh.to_host(ow, og))
    err = float(np.abs(out[1][0] - out[0][0]).max() / np.abs(out[0][0]).max())
    print("double Mach: mixed vs fp64 adjoint (Wbar block) rel max", err, flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_wall_adjoint_graph_replays_equal_eager(prec):
    """On a mesh with walls and prescribed states the adjoint forks the face
    reverse of the cells with such a face onto the handle's own stream and
    joins it back by events.  A HIP graph captured from the caller's stream
    holds that branch: three replays, each after new adjoint inputs are copied
    in and with eager adjoints and synchronisations between them, equal the
    eager adjoint of the same inputs bitwise."""
    import torch
    wl = double_mach_workload(n=12)
    rng = np.random.default_rng(41)
    s0 = _perturbed(wl, rng)
    dt = OracleMesh.from_workload(wl).max_dt(s0, 0.3)
    mesh = _mesh(wl, prec)
    mesh.set_time(0.012)
    w, g = mesh.to_device(s0)
    lw, lg = mesh.to_device(rng.normal(size=s0.shape))
    ow, og = mesh.empty_state()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(device=mesh.device)
    s.wait_stream(torch.cuda.current_stream(mesh.device))
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            mesh.adjoint(w, g, lw, lg, dt, out=(ow, og), stream=s)
    torch.cuda.current_stream(mesh.device).wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        nw, ng = mesh.to_device(rng.normal(size=s0.shape))
        lw.copy_(nw)
        lg.copy_(ng)
        graph.replay()
        torch.cuda.synchronize()
        rw, rg = mesh.adjoint(w, g, lw, lg, dt)
        torch.cuda.synchronize()
        print(prec, "replay", rep, "max |diff|", float((ow - rw).abs().max()), flush=True)
        assert torch.equal(ow, rw) and torch.equal(og, rg), rep


def test_rollout_through_a_moving_boundary_against_the_oracle_jvp():
    """The checkpointed rollout from t0 > 0 sets each step's time (the moving
    switch) in the forward pass, the recomputation and the adjoints: the
    gradient of <lam, s_n> equals the oracle's n-step JVP."""
    import torch
    from paper_2607_10809_amd.autograd import rollout
    wl = double_mach_workload(n=12)
    rng = np.random.default_rng(29)
    om = OracleMesh.from_workload(wl)
    s0 = _perturbed(wl, rng)
    dt, n, t0 = om.max_dt(s0, 0.3), 6, 0.012
    mesh = _mesh(wl)
    lam = rng.normal(size=s0.shape)
    w0, g0 = mesh.to_device(s0)
    lw, lg = mesh.to_device(lam)
    w = w0.clone().requires_grad_(True)
    g = g0.clone().requires_grad_(True)
    wT, gT = rollout(mesh, w, g, dt, n, ckpt=4, t0=t0)
    ((wT * lw).sum() + (gT * lg).sum()).backward()
    torch.cuda.synchronize()
    grad = mesh.to_host(w.grad, g.grad)
    for _ in range(2):
        v = rng.normal(size=s0.shape)
        _, jv = om.jvp(s0, v, dt, n, t=t0)
        a, b = float(np.sum(grad * v)), float(np.sum(lam * jv))
        scale = float(np.abs(grad * v).sum())
        print("double Mach rollout from t0: <grad, v> =", a, "<l, J^n v> =", b, "rel", abs(a - b) / scale,
              flush=True)
        assert abs(a - b) <= 1e-10 * scale


@pytest.mark.parametrize("time_rule,wd,er", [(1, 1.0, 2), (1, 0.3, 2), (0, 1.0, 3), (1, 0.3, 3)])
def test_dot_product_variants(time_rule, wd, er):
    """The adjoint with the Gauss-Legendre time rule, weighted Step-2 rows and
    the 3-point edge rule."""
    rng = np.random.default_rng(17)
    wl = vortex_workload(n=24)
    om = OracleMesh.from_workload(wl, time_rule=time_rule, deriv_weight=wd, edge_rule=er)
    s0 = _perturbed(wl, rng)
    dt = om.max_dt(s0, 0.3)
    mesh = _mesh(wl, time_rule=time_rule, deriv_weight=wd, edge_rule=er)
    for _ in range(2):
        v = rng.normal(size=s0.shape)
        lam = rng.normal(size=s0.shape)
        _, jv = om.jvp(s0, v, dt, 1)
        vj = _gpu_vjp(mesh, s0, lam, dt)
        a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
        scale = float(np.abs(vj * v).sum())
        print(f"time rule {time_rule}, weight {wd}, edge rule {er}: <J^T l, v> = {a}, <l, J v> = {b}", flush=True)
        assert abs(a - b) <= 1e-11 * scale


def test_full_gradient_against_oracle_jacobian_tiny_mesh():
    """J^T lam of 3 steps on an 18-triangle vortex mesh, against the oracle's
    Jacobian built column by column from dual-number JVPs."""
    import torch
    rng = np.random.default_rng(5)
    wl = vortex_workload(n=3)
    om = OracleMesh.from_workload(wl)
    s0 = _perturbed(wl, rng)
    dt = om.max_dt(s0, 0.3)
    nsteps = 3
    n = s0.size
    lam = rng.normal(size=s0.shape)
    ref = np.empty(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        _, jv = om.jvp(s0, e.reshape(s0.shape), dt, nsteps)
        ref[k] = np.sum(lam * jv)
    from paper_2607_10809_amd.autograd import rollout
    mesh = _mesh(wl)
    w, g = mesh.to_device(s0)
    w.requires_grad_(True)
    g.requires_grad_(True)
    wT, gT = rollout(mesh, w, g, dt, nsteps, ckpt=2)
    lw, lg = mesh.to_device(lam)
    (torch.sum(wT * lw) + torch.sum(gT * lg)).backward()
    got = mesh.to_host(w.grad, g.grad).ravel()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print("tiny-mesh full gradient rel max err", err, flush=True)
    assert err <= 1e-11


@pytest.fixture(scope="module")
def c5():
    """Vortex (204,800 triangles), target = forward run from a perturbed centre."""
    import torch
    from paper_2607_10809_amd.autograd import rollout  # noqa: F401
    wl = vortex_workload()
    tc = perturbed_vortex_target_center()
    tgt0 = cell_average_states(wl.mesh, make_vortex(center=tc))
    mesh = _mesh(wl)
    w0, g0 = mesh.to_device(wl.state0)
    dt = mesh.max_dt(w0, wl.cfl)
    tw, tg = mesh.to_device(tgt0)
    tw, _ = mesh.run(tw, tg, dt, 200)
    torch.cuda.synchronize()
    return wl, mesh, dt, tw[0].clone()


def _misfit(mesh, w0, g0, dt, tgt, nsteps=200):
    w, _ = mesh.run(w0, g0, dt, nsteps)
    d = w[0] - tgt
    return 0.5 * float(torch_dot(d, d))


def torch_dot(a, b):
    import torch
    return torch.dot(a, b).item()


def test_c5_gradient_against_central_differences(c5):
    import torch
    from paper_2607_10809_amd.autograd import rollout
    wl, mesh, dt, tgt = c5
    w0, g0 = mesh.to_device(wl.state0)
    w = w0.clone().requires_grad_(True)
    g = g0.clone().requires_grad_(True)
    wT, gT = rollout(mesh, w, g, dt, 200, ckpt=20)
    loss = 0.5 * ((wT[0] - tgt) ** 2).sum()
    loss.backward()
    grad_rho = w.grad[0].detach()
    dirs = fd_directions(mesh.N, 32)                  # caller order, unit norm
    worst = 0.0
    for k in range(32):
        v = torch.from_numpy(dirs[k][mesh.perm]).to(w0.device)
        ad = float(torch.dot(grad_rho, v))
        best = np.inf
        for eps in (1e-2, 1e-3, 1e-4):
            wp = w0.clone()
            wp[0] += eps * v
            wm = w0.clone()
            wm[0] -= eps * v
            fd = (_misfit(mesh, wp, g0, dt, tgt) - _misfit(mesh, wm, g0, dt, tgt)) / (2 * eps)
            best = min(best, abs(fd - ad) / max(abs(ad), 1e-300))
        worst = max(worst, best)
        print(f"dir {k}: <grad, v> = {ad:.12e}, best central-difference rel err {best:.2e}", flush=True)
    assert worst <= 1e-6


def test_c5_mixed_gradient_against_fp64_and_central_differences(c5):
    """The C5 misfit gradient of the mixed path (FP32 bulk, FP64 cell averages,
    weights and accumulation), through the same 200-step checkpointed rollout,
    against the FP64 gradient: relative L2 and max errors on the density slice
    within 1e-5 (the FP32 step's relative rounding, ~1e-7 per step, over 200
    steps); and against central differences of the mixed misfit on the 32
    directions within 1e-4 (the FP32 rounding of the forward enters the
    differences as noise / eps)."""
    import torch
    from paper_2607_10809_amd.autograd import rollout
    wl, mesh64, dt, tgt = c5
    grads = {}
    meshes = {"fp64": mesh64, "mixed": _mesh(wl, "mixed")}
    for prec, mesh in meshes.items():
        w0, g0 = mesh.to_device(wl.state0)
        w = w0.clone().requires_grad_(True)
        g = g0.clone().requires_grad_(True)
        wT, gT = rollout(mesh, w, g, dt, 200, ckpt=20)
        loss = 0.5 * ((wT[0] - tgt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        grads[prec] = mesh.to_host(w.grad, g.grad.double())[0, 0]
    a, b = grads["mixed"], grads["fp64"]
    l2 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    mx = float(np.abs(a - b).max() / np.abs(b).max())
    mesh = meshes["mixed"]
    w0, g0 = mesh.to_device(wl.state0)
    dirs = fd_directions(mesh.N, 32)
    worst = 0.0
    for k in range(32):
        v = dirs[k]
        ad = float(np.dot(a, v))
        vd = torch.from_numpy(v[mesh.perm]).to(w0.device)
        best = np.inf
        for eps in (1e-2, 1e-3):
            wp = w0.clone()
            wp[0] += eps * vd
            wm = w0.clone()
            wm[0] -= eps * vd
            fd = (_misfit(mesh, wp, g0, dt, tgt) - _misfit(mesh, wm, g0, dt, tgt)) / (2 * eps)
            best = min(best, abs(fd - ad) / max(abs(ad), 1e-300))
        worst = max(worst, best)
    print(f"C5 mixed gradient vs FP64: rel L2 {l2:.2e}, rel max {mx:.2e}; vs central differences of the mixed "
          f"misfit, worst of 32 directions {worst:.2e}", flush=True)
    assert l2 <= 1e-5 and mx <= 1e-5
    assert worst <= 1e-4


def test_checkpointing_does_not_change_the_gradient():
    import torch
    from paper_2607_10809_amd.autograd import rollout
    wl = vortex_workload(n=24)
    mesh = _mesh(wl)
    w0, g0 = mesh.to_device(wl.state0)
    dt = mesh.max_dt(w0, wl.cfl)
    grads = []
    # checkpoint intervals, with and without the recomputation overlapping the
    # adjoints, with the last segment kept from the forward pass or recomputed
    # (a last segment of 5 steps with ckpt 7)
    for ck, overlap, keep in ((1, True, True), (7, True, True), (7, False, True), (7, True, False),
                              (40, True, True), (40, True, False), (1, False, False)):
        w = w0.clone().requires_grad_(True)
        g = g0.clone().requires_grad_(True)
        wT, gT = rollout(mesh, w, g, dt, 40, ckpt=ck, overlap=overlap, keep_last=keep)
        (wT[0] ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((w.grad.clone(), g.grad.clone()))
    for a in grads[1:]:
        assert torch.equal(a[0], grads[0][0]) and torch.equal(a[1], grads[0][1])


@pytest.mark.parametrize("case,precision", [("advection", "fp64"), ("burgers", "fp64"), ("vortex", "fp64"),
                                            ("vortex", "mixed"), ("burgers", "mixed")])
def test_kept_reconstruction_is_bitwise(case, precision):
    """hwe_step_keep = hwe_step and writes what hwe_debug_recon returns;
    hwe_step_adjoint_kept with that buffer = hwe_step_adjoint, all bitwise."""
    import torch
    from paper_2607_10809_amd._lib import HweError
    rng = np.random.default_rng(31)
    wl = {"advection": lambda: advection_workload(n=20), "burgers": lambda: burgers_workload(n=24, T=1.0),
          "vortex": lambda: vortex_workload(n=24)}[case]()
    mesh = _mesh(wl, precision)
    w, g = mesh.to_device(_perturbed(wl, rng))
    lw, lg = mesh.to_device(rng.normal(size=wl.state0.shape))
    dt = mesh.max_dt(w, wl.cfl)
    a = mesh.step(w, g, dt)
    R = mesh.empty_recon()
    b = mesh.step(w, g, dt, keep=R)
    ref = mesh.debug_recon(w, g).permute(2, 0, 1)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(R, ref)
    x = mesh.adjoint(w, g, lw, lg, dt)
    y = mesh.adjoint(w, g, lw, lg, dt, recon=R)
    torch.cuda.synchronize()
    assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])
    # a reconstruction buffer that overlaps an output state buffer is refused
    es = torch.finfo(mesh.gdtype).bits // 8
    raw = torch.empty(6 * mesh.m * mesh.N * es, dtype=torch.uint8, device=mesh.device)
    Rbad = raw.view(mesh.gdtype).view(mesh.N, 6, mesh.m)
    wo = raw[:8 * mesh.m * mesh.N].view(torch.float64).view(mesh.m, mesh.N)
    with pytest.raises(HweError):
        mesh.step(w, g, dt, out=(wo, torch.empty_like(g)), keep=Rbad)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kept_reconstruction_with_a_moving_switch_is_bitwise(precision):
    """The kept reconstruction of a step from t (moving boundary states at
    t + dt/2) serves the adjoint of that step bitwise."""
    import torch
    rng = np.random.default_rng(37)
    wl = double_mach_workload(n=12)
    mesh = _mesh(wl, precision)
    w, g = mesh.to_device(_perturbed(wl, rng))
    lw, lg = mesh.to_device(rng.normal(size=wl.state0.shape))
    dt, t = mesh.max_dt(w, wl.cfl), 0.012
    a = mesh.step(w, g, dt, t=t)
    R = mesh.empty_recon()
    b = mesh.step(w, g, dt, keep=R, t=t)
    x = mesh.adjoint(w, g, lw, lg, dt, t=t)
    y = mesh.adjoint(w, g, lw, lg, dt, recon=R, t=t)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])


def test_mixed_adjoint_close_to_fp64():
    import torch
    rng = np.random.default_rng(9)
    wl = vortex_workload(n=40)
    s0 = wl.state0
    lam = rng.normal(size=s0.shape)
    om = OracleMesh.from_workload(wl)
    dt = om.max_dt(s0, 0.3)
    a = _gpu_vjp(_mesh(wl), s0, lam, dt)
    b = _gpu_vjp(_mesh(wl, "mixed"), s0, lam, dt)
    err = float(np.abs(a[0] - b[0]).max() / np.abs(a[0]).max())
    print("mixed vs fp64 adjoint (Wbar block) rel max", err, flush=True)
    assert err <= 1e-4
    torch.cuda.synchronize()


EDGE_POINTS = {2: (0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0),
               3: (0.5 - np.sqrt(15.0) / 10.0, 0.5, 0.5 + np.sqrt(15.0) / 10.0)}


def _touching_cells(om, s, rule):
    """Cells scaled for their density, and for each the cell itself and the
    neighbour across the face of its least-density point: there the limited
    density is eps = 1e-13 at a flux point, and the step's sensitivities
    (through 1/rho in the Lax-Wendroff jets) reach 1e24 and more."""
    V = om.cell_vertices()
    nbr = om.geometry()["nbr"]
    limited, touch = 0, set()
    for k in range(om.N):
        th = om.recon_theta(s, k)
        if not th[0] < th[1]:
            continue
        limited += 1
        pts = np.array([V[k, f] + t * (V[k, (f + 1) % 3] - V[k, f]) for f in range(3) for t in EDGE_POINTS[rule]])
        f = int(np.argmin(om.eval_recon(s, k, pts)[:, 0, 0])) // len(EDGE_POINTS[rule])
        touch.add(k)
        if nbr[k, f] >= 0:
            touch.add(int(nbr[k, f]))
    return limited, sorted(touch)


# limiter cases: (workload, seed of the data, branch, options)
LIMITER_CASES = {
    "riemann_pressure": (lambda: riemann_workload(n=24), 41, "pressure", {}),
    "riemann_pressure_edge3": (lambda: riemann_workload(n=24), 43, "pressure", {"edge_rule": 3}),
    "closed_riemann_walls_pressure": (lambda: dataclasses.replace(riemann_workload(n=24), walls=0b1111), 47,
                                      "pressure", {}),
    "riemann_density_at_rest": (lambda: riemann_workload(n=24), 41, "density", {}),
    "riemann_density_at_rest_edge3": (lambda: riemann_workload(n=24), 41, "density", {"edge_rule": 3}),
}


@pytest.mark.parametrize("case", list(LIMITER_CASES))
def test_dot_product_with_the_scaling_limiter(case):
    """The adjoint through the positivity-preserving scaling limiter (on the
    branches the forward takes; its threshold eps a constant) against the
    oracle's JVP, on data where it acts.  With the density scaling, the
    adjoint seeds vanish on the cells next to the touching point, whose
    1e24-scale sensitivities no FP64 comparison resolves; the scaling's
    derivative still reaches the seeds through the cell's other faces."""
    import torch
    make, seed, branch, opts = LIMITER_CASES[case]
    wl = make()
    om = OracleMesh.from_workload(wl, positivity=1, **opts)
    s0 = near_vacuum_state(wl, seed, branch)
    mask = np.ones(om.N)
    if branch == "density":
        nlim, touch = _touching_cells(om, s0, opts.get("edge_rule", 2))
        mask[touch] = 0.0
    else:
        nlim = sum(bool(om.recon_theta(s0, k)[1] < 1.0) for k in range(om.N))
    dt = om.max_dt(s0, 0.2)
    mesh = _mesh(wl, positivity=True, **opts)
    rng = np.random.default_rng(seed + 1)
    for _ in range(3):
        v = rng.normal(size=s0.shape) * np.abs(s0)
        lam = rng.normal(size=s0.shape) * mask
        _, jv = om.jvp(s0, v, dt, 1)
        w, g = mesh.to_device(s0)
        lw, lg = mesh.to_device(lam)
        ow, og = mesh.adjoint(w, g, lw, lg, dt)
        torch.cuda.synchronize()
        vj = mesh.to_host(ow, og)
        a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
        scale = float(np.abs(vj * v).sum())
        print(case, nlim, "limited cells: <J^T l, v> =", a, "<l, J v> =", b, "rel", abs(a - b) / scale, flush=True)
        assert abs(a - b) <= 1e-11 * scale
    assert nlim >= (100 if branch == "pressure" else 1)


def _face_neighbours(tris):
    """(N, 3) neighbour of each cell across each face (the cell itself across a
    boundary face, as its mirrored ghost holds its average)."""
    tris = np.asarray(tris, dtype=np.int64)
    N = len(tris)
    a = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    b = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    key = np.minimum(a, b) * (int(tris.max()) + 1) + np.maximum(a, b)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.flatnonzero(ks[1:] == ks[:-1])
    fa, fb = order[same], order[same + 1]                  # face ids f * N + cell
    nb = np.repeat(np.arange(N)[:, None], 3, axis=1)
    nb[fa % N, fa // N] = fb % N
    nb[fb % N, fb // N] = fa % N
    return nb


def test_c4_adjoint_with_the_limiter_full_size():
    """The adjoint at the 980,000-triangle Riemann configuration with the
    limiter on, at a state the GPU reached after 100 steps at CFL 0.2: the dot
    product against the oracle's JVP of the same step, and every entry against
    the oracle's reverse mode (relative to its block's largest, 1e-10), except
    where the step's linearization is set by round-off.  That is where the
    gas is at rest: there a momentum component is zero up to round-off over a
    whole stencil, so its W_ave is the 1e-30 floor plus noise, the nonlinear
    weights of eq. (nonlinearweight) are ratios of noise-level smoothness
    indicators, and the derivative through W_ave (the cell-average block only)
    multiplies noise-level candidates by 1/W_ave.  Two correct FP64
    evaluations differ there at the 1e-3 level (the oracle against itself
    from a one-ulp perturbed state: 3e-3); those entries, the cell averages'
    adjoints of a component whose stencil average at the cell or a neighbour
    is below 1e-12 of the component's largest value (about 8% of the
    entries), are reported, not compared."""
    import torch
    wl = riemann_workload()
    mesh = _mesh(wl, positivity=True)
    om = OracleMesh.from_workload(wl, positivity=1)
    w, g = mesh.to_device(wl.state0)
    w, g = mesh.run(w, g, mesh.max_dt(w, 0.2), 100)
    torch.cuda.synchronize()
    s = mesh.to_host(w, g)
    dt = om.max_dt(s, 0.2)
    rng = np.random.default_rng(61)
    v = rng.normal(size=s.shape) * np.abs(s)
    lam = rng.normal(size=s.shape)
    _, jv = om.jvp(s, v, dt, 1)
    lw, lg = mesh.to_device(lam)
    ow, og = mesh.adjoint(w, g, lw, lg, dt)
    torch.cuda.synchronize()
    vj = mesh.to_host(ow, og)
    a, b = float(np.sum(vj * v)), float(np.sum(lam * jv))
    scale = float(np.abs(vj * v).sum())
    print("C4 limited adjoint: <J^T l, v> =", a, "<l, J v> =", b, "rel", abs(a - b) / scale, flush=True)
    assert abs(a - b) <= 1e-11 * scale
    ref = om.vjp(s, lam, dt, 1)
    rel = np.abs(vj - ref) / np.abs(ref).max(axis=-1, keepdims=True)
    nb = _face_neighbours(wl.mesh.tris)
    W = s[0]
    wave = (W + W[:, nb[:, 0]] + W[:, nb[:, 1]] + W[:, nb[:, 2]]) / 4.0
    tiny = np.abs(wave) < 1e-12 * np.abs(W).max(axis=1, keepdims=True)
    mask = np.zeros(rel.shape, dtype=bool)
    mask[0] = tiny | tiny[:, nb[:, 0]] | tiny[:, nb[:, 1]] | tiny[:, nb[:, 2]]
    print(f"C4 limited adjoint element by element: rel max per block {rel[~mask].max():.2e} on "
          f"{(~mask).mean():.1%} of the entries; {rel[mask].max():.2e} where the linearization is set by "
          f"round-off", flush=True)
    assert rel[~mask].max() <= 1e-10
    assert mask.mean() < 0.15


def test_mixed_adjoint_with_the_limiter_close_to_fp64():
    import torch
    wl = riemann_workload(n=24)
    om = OracleMesh.from_workload(wl, positivity=1)
    s0 = om.run(wl.state0, om.max_dt(wl.state0, 0.2), 60)      # two cells limited
    dt = om.max_dt(s0, 0.2)
    lam = np.random.default_rng(53).normal(size=s0.shape)
    out = []
    for prec in ("fp64", "mixed"):
        mesh = _mesh(wl, prec, positivity=True)
        w, g = mesh.to_device(s0)
        lw, lg = mesh.to_device(lam)
        ow, og = mesh.adjoint(w, g, lw, lg, dt)
        torch.cuda.synchronize()
        out.append(mesh.to_host(ow, og))
    err = float(np.abs(out[1][0] - out[0][0]).max() / np.abs(out[0][0]).max())
    print("limited Riemann: mixed vs fp64 adjoint (Wbar block) rel max", err, flush=True)
    assert err <= 1e-4
