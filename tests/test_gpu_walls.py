"""GPU tests of reflective walls (Euler) against the oracle.

* the Lax and Sod shock tubes (strips between walls, transmissive ends): a
  100-step prefix (FP64 within 1e-10 relative L1 of the oracle, mixed within
  2e-5), one step from the oracle's state at the final time, and full runs in
  both precisions close to the exact 1-D Riemann solution;
* a longer strip (38,400 triangles): a 40-step prefix and one late step, also
  with the limiter;
* uniform states between walls stay uniform; a closed box conserves mass;
* a wall is a mirror, at the size of the vortex workload: the step on a half
  domain with a wall equals the step on the domain doubled by the mirror image
  of its mesh, from mirror-symmetric data with momentum across the wall.
(The adjoint on wall meshes is tested in test_gpu_adjoint.py.)
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from exact_riemann import sample  # noqa: E402
from gpu_util import gpu_run, gpu_run_to  # noqa: E402
from oracle import OracleMesh  # noqa: E402
from workloads import cell_average_states, shock_tube_workload, split_square_mesh  # noqa: E402

pytestmark = pytest.mark.gpu
GAMMA = 1.4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mesh(wl, precision="fp64", **kw):
    from paper_2607_10809_amd.hwe import Mesh
    return Mesh.from_workload(wl, precision=precision, **kw)


def _rel_l1_blocks(a, b, area):
    """Area-weighted L1 distance per block (W, V, Y), summed over the components
    and relative to the block's L1 norm (the transverse momentum of a 1-D
    problem is a small, mesh-induced component: it is not normalised alone)."""
    num = (np.abs(a - b) * area).sum(axis=(-1, -2))
    den = (np.abs(b) * area).sum(axis=(-1, -2))
    return float((num / den).max())


def _exact_rho(wl):
    L, R, T = wl.extra["left"], wl.extra["right"], wl.T
    f = lambda x, y, t: sample(x / T, (L[0], L[1], L[3]), (R[0], R[1], R[3]))[0][..., None]
    return cell_average_states(wl.mesh, f, T)[0, 0]


@pytest.mark.parametrize("name,bound", [("lax", 0.013), ("sod", 0.0045)])
def test_shock_tube_full_run(name, bound):
    """Like the four-quadrant problem, the strip is sensitive to round-off: a
    difference of 1e-13 after one step stays there for ~100 steps and then
    grows by ~10x per 10 steps on the jittered mesh (measured: the one-step
    maps agree to 3e-13 all along).  Parity is therefore checked on a 100-step
    prefix and by one step from the oracle's final state; the full GPU runs are
    checked against the exact 1-D solution."""
    wl = shock_tube_workload(name, nx=100)
    om = OracleMesh.from_workload(wl)
    dt = om.max_dt(wl.state0, wl.cfl)
    area = om.geometry()["area"]
    ref = om.run(wl.state0, dt, 100)
    e64 = _rel_l1_blocks(gpu_run(_mesh(wl), wl.state0, dt, 100), ref, area)
    em = _rel_l1_blocks(gpu_run(_mesh(wl, "mixed"), wl.state0, dt, 100)[:1], ref[:1], area)
    sT = om.run_to(wl.state0, wl.T, dt)
    one_ref = om.step(sT, dt)
    one = gpu_run(_mesh(wl), sT, dt, 1)
    e1 = float(np.abs(one - one_ref).max() / np.abs(one_ref).max())
    ex = _exact_rho(wl)
    eex = {}
    for prec in ("fp64", "mixed"):
        got = gpu_run_to(_mesh(wl, prec), wl.state0, wl.T, dt)
        eex[prec] = (np.abs(got[0, 0] - ex) * area).sum() / area.sum()
    print(f"{name}: 100-step prefix L1 fp64 {e64:.2e} mixed {em:.2e}; one step at T {e1:.2e}; "
          f"density L1 vs exact {eex}", flush=True)
    assert e64 <= 1e-10 and em <= 2e-5 and e1 <= 1e-12
    assert eex["fp64"] < bound and eex["mixed"] < bound


def test_long_strip_prefix_and_limiter():
    """38,400 triangles: a 40-step prefix, and one step from the oracle's state
    after 300 steps, with and without the limiter."""
    wl = shock_tube_workload("lax", nx=400, height=0.12)      # 400 x 48 squares
    for kw in ({}, {"positivity": 1}):
        om = OracleMesh.from_workload(wl, **kw)
        dt = om.max_dt(wl.state0, wl.cfl)
        area = om.geometry()["area"]
        ref = om.run(wl.state0, dt, 40)
        err = _rel_l1_blocks(gpu_run(_mesh(wl, positivity=bool(kw)), wl.state0, dt, 40), ref, area)
        late = om.run(ref, dt, 260)
        one_ref = om.step(late, dt)
        one = gpu_run(_mesh(wl, positivity=bool(kw)), late, dt, 1)
        e1 = float(np.abs(one - one_ref).max() / np.abs(one_ref).max())
        print("long strip", kw, "40-step prefix L1", err, "one step after 300:", e1, flush=True)
        assert err <= 1e-10 and e1 <= 1e-12


def _cons(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("flow", ["rest", "along_walls"])
def test_uniform_states_between_walls(flow):
    from paper_2607_10809_amd.hwe import Mesh
    box = (0.0, 1.0, 0.0, 0.5)
    mesh = split_square_mesh((24, 12), box, jitter=0.2, seed=21, periodic=False)
    W, walls = (_cons(1.3, 0.0, 0.0, 0.8), 0b1111) if flow == "rest" else (_cons(0.9, 0.7, 0.0, 1.1), 0b1100)
    s0 = np.zeros((3, 4, mesh.n_cells))
    s0[0] = W[:, None]
    for prec in ("fp64", "mixed"):
        m = Mesh(mesh.nodes, mesh.tris, eq="euler", bc="transmissive", box=box, precision=prec, walls=walls)
        s = gpu_run(m, s0, 1e-3, 50)
        assert np.abs(s[0] - s0[0]).max() <= 1e-13 * np.abs(W).max(), prec
        assert np.abs(s[1:]).max() <= (1e-12 if prec == "fp64" else 1e-5), prec


def test_closed_box_conserves_mass_and_matches_the_oracle():
    from paper_2607_10809_amd.hwe import Mesh
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(40, box, jitter=0.2, seed=22, periodic=False)

    def f(x, y, t):
        r = 1.0 + 0.3 * np.exp(-30 * ((x - 0.4) ** 2 + (y - 0.55) ** 2))
        return np.stack([r, 0.2 * r, -0.1 * r, 1.0 / (GAMMA - 1) + 0.025 * r + 0 * x], -1)

    s0 = cell_average_states(mesh, f)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=1, box=box, walls=0b1111)
    dt = om.max_dt(s0, 0.3)
    area = om.geometry()["area"]
    m = Mesh(mesh.nodes, mesh.tris, eq="euler", bc="transmissive", box=box, walls=0b1111)
    got = gpu_run(m, s0, dt, 100)
    mass0 = (s0[0, 0] * area).sum()
    drift = abs((got[0, 0] * area).sum() - mass0) / mass0
    # the derivative averages of this problem amplify round-off (the oracle
    # itself turns a 1e-13 perturbation into 6e-9 within 20 steps with walls):
    # parity on a 5-step prefix and by one step from the oracle's step-40 state
    ref5 = om.run(s0, dt, 5)
    e5 = float(np.abs(gpu_run(m, s0, dt, 5) - ref5).max() / np.abs(ref5).max())
    late = om.run(ref5, dt, 35)
    one_ref = om.step(late, dt)
    e1 = float(np.abs(gpu_run(m, late, dt, 1) - one_ref).max() / np.abs(one_ref).max())
    print("closed box: mass drift over 100 steps", drift, "5-step rel max", e5, "one step at 40", e1, flush=True)
    assert np.isfinite(got).all()
    assert drift <= 1e-13 and e5 <= 1e-12 and e1 <= 1e-12



def _mirror_state(s):
    """The mirror image across x = 0 of a [3][4][N] state: density, y-momentum
    and energy even in x, x-momentum odd."""
    t = s.copy()
    t[0, 1] *= -1.0
    t[1, [0, 2, 3]] *= -1.0
    t[2, 1] *= -1.0
    return t


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_wall_equals_the_mirror_image_flow_full_size(prec):
    """The property the oracle's walls-as-mirrors pin checks on a small mesh,
    on the GPU at the vortex workload's size: 204,800 triangles on [0, 1]^2
    with a wall at x = 0, 20 steps from data with momentum across the wall,
    against 20 steps on the 409,600 triangles of the domain doubled by the
    mirror image of the mesh (no wall there), from the data and its mirror
    image.  Both halves of the doubled run match (the image mirrored back):
    FP64 to 1e-12 of each block's largest value, mixed to 2e-5."""
    from paper_2607_10809_amd.hwe import Mesh
    half = split_square_mesh((320, 320), (0.0, 1.0, 0.0, 1.0), jitter=0.1, seed=3, periodic=False)
    nodes, tris = half.nodes, half.tris.astype(np.int64)
    on_axis = nodes[:, 0] == 0.0
    image = np.empty(len(nodes), dtype=np.int64)
    image[on_axis] = np.flatnonzero(on_axis)
    image[~on_axis] = len(nodes) + np.arange(int((~on_axis).sum()))
    full_nodes = np.concatenate([nodes, nodes[~on_axis] * np.array([-1.0, 1.0])])
    full_tris = np.concatenate([tris, image[tris][:, [0, 2, 1]]]).astype(np.int32)

    def f(x, y, t):
        b = np.exp(-20.0 * ((x - 0.25) ** 2 + (y - 0.5) ** 2))
        r, u, v, p = 1.0 + 0.3 * b, -0.6 * b, 0.1 + 0 * x, 1.0 + 0.2 * b
        return np.stack([r, r * u, r * v, p / (GAMMA - 1) + 0.5 * r * (u * u + v * v)], -1)

    s_half = cell_average_states(half, f)
    s_full = np.concatenate([s_half, _mirror_state(s_half)], axis=2)
    wall = Mesh(nodes, half.tris, eq="euler", bc="transmissive", box=(0.0, 1.0, 0.0, 1.0), precision=prec,
                walls=0b0001)
    mirror = Mesh(full_nodes, full_tris, eq="euler", bc="transmissive", box=(-1.0, 1.0, 0.0, 1.0), precision=prec)
    dt = wall.max_dt(wall.to_device(s_half)[0], 0.3)
    a = gpu_run(wall, s_half, dt, 20)
    b = gpu_run(mirror, s_full, dt, 20)
    N = s_half.shape[2]
    bound = 1e-12 if prec == "fp64" else 2e-5
    for blk in range(3):
        scale = np.abs(a[blk]).max()
        e_in = np.abs(b[blk, :, :N] - a[blk]).max() / scale
        e_img = np.abs(b[blk, :, N:] - _mirror_state(a)[blk]).max() / scale
        print(f"{prec} block {blk}: wall vs mirror {e_in:.2e}, image {e_img:.2e}", flush=True)
        assert e_in <= bound and e_img <= bound
