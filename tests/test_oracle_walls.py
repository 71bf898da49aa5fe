"""Oracle pins for reflective walls (Euler): the ghost cell is the mirror image
of the interior cell with its momentum reflected, and the exterior value at a
wall Gauss point is the reflected interior value.

* a gas at rest, and a uniform flow along the walls, stay exactly uniform;
* a closed box conserves mass to round-off (no mass crosses a wall);
* the Lax and Sod shock tubes, run as 2-D strips between walls, converge to the
  exact 1-D Riemann solution (tests/exact_riemann.py, written from the shock and
  rarefaction relations) in L1;
* a wall is a mirror: the step on a half domain with a wall equals the step on
  the domain doubled by the mirror image of its mesh, from mirror-symmetric
  data, with momentum across the wall.
"""
import numpy as np
import pytest

from exact_riemann import sample
from oracle import OracleMesh
from workloads import cell_average_states, shock_tube_workload, split_square_mesh

pytestmark = pytest.mark.usefixtures("oracle_lib")

GAMMA = 1.4


def _cons(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


def _uniform(mesh, W):
    s = np.zeros((3, 4, mesh.n_cells))
    s[0] = W[:, None]
    return s


@pytest.mark.parametrize("flow", ["rest", "along_walls"])
def test_uniform_states_are_preserved_between_walls(flow):
    box = (0.0, 1.0, 0.0, 0.5)
    mesh = split_square_mesh((12, 6), box, jitter=0.2, seed=21, periodic=False)
    if flow == "rest":      # closed box: every side a wall
        W, walls = _cons(1.3, 0.0, 0.0, 0.8), 0b1111
    else:                   # channel: walls at y = 0, 0.5; uniform u along them
        W, walls = _cons(0.9, 0.7, 0.0, 1.1), 0b1100
    om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=1, box=box, walls=walls)
    s0 = _uniform(mesh, W)
    s = om.run(s0, om.max_dt(s0, 0.3), 20)
    assert np.abs(s[0] - s0[0]).max() <= 1e-13 * np.abs(W).max()
    assert np.abs(s[1:]).max() <= 1e-12


def test_closed_box_conserves_mass():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(10, box, jitter=0.2, seed=22, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=1, box=box, walls=0b1111)

    def f(x, y, t):
        r = 1.0 + 0.3 * np.exp(-30 * ((x - 0.4) ** 2 + (y - 0.55) ** 2))
        return np.stack([r, 0.2 * r, -0.1 * r, 1.0 / (GAMMA - 1) + 0.5 * r * 0.05 + 0 * x], -1)

    s0 = cell_average_states(mesh, f)
    area = om.geometry()["area"]
    mass0 = (s0[0, 0] * area).sum()
    s = om.run(s0, om.max_dt(s0, 0.3), 60)
    assert np.isfinite(s).all()
    assert abs((s[0, 0] * area).sum() - mass0) <= 1e-14 * mass0
    # the walls reflect the flow: the x-momentum changes (a transmissive box would not stop it)
    assert abs((s[0, 1] * area).sum() - (s0[0, 1] * area).sum()) > 1e-6


def _l1_against_exact(name, nx):
    wl = shock_tube_workload(name, nx=nx)
    L, R, T = wl.extra["left"], wl.extra["right"], wl.T
    om = OracleMesh.from_workload(wl)
    s = om.run_to(wl.state0, T, om.max_dt(wl.state0, wl.cfl))
    exact = lambda x, y, t: sample(x / T, (L[0], L[1], L[3]), (R[0], R[1], R[3]))[0][..., None]
    ex = cell_average_states(wl.mesh, exact, T)[0, 0]
    area = om.geometry()["area"]
    return (np.abs(s[0, 0] - ex) * area).sum() / area.sum(), s


@pytest.mark.parametrize("name,bound", [("lax", 0.013), ("sod", 0.0045)])
def test_shock_tubes_converge_to_the_exact_riemann_solution(name, bound):
    e50, _ = _l1_against_exact(name, 50)
    e100, s = _l1_against_exact(name, 100)
    assert np.isfinite(s).all()
    assert e100 < bound, (e50, e100)
    assert e50 / e100 > 1.4, (e50, e100)


def _mirror_state(s):
    """The state of the mirror image across x = 0: density, y-momentum and
    energy even in x, x-momentum odd; the x-derivative averages change sign
    where the field is even, the y-derivative averages where it is odd."""
    t = s.copy()
    t[0, 1] *= -1.0
    t[1, [0, 2, 3]] *= -1.0
    t[2, 1] *= -1.0
    return t


def test_wall_step_equals_the_mirror_image_flow():
    """The reading of a reflective wall (the ghost cell is the cell's mirror
    image across the face holding the reflected average and both rows of the
    derivative averages reflected; the exterior value at a wall point is the
    reflected interior value; the flux viscosity takes the reflected average)
    makes a wall equivalent to a mirror.  So five steps on [0, 1]^2 with a wall
    at x = 0 equal, cell by cell to round-off, five steps on [-1, 1] x [0, 1]
    meshed by the same triangles and their mirror images (no wall at x = 0),
    from the data and its mirror image; the flow crosses x = 0 where the wall
    stands, so the reflection of the normal momentum is exercised."""
    half = split_square_mesh((8, 8), (0.0, 1.0, 0.0, 1.0), jitter=0.2, seed=31, periodic=False)
    nodes, tris = half.nodes, half.tris.astype(np.int64)
    on_axis = nodes[:, 0] == 0.0
    image = np.empty(len(nodes), dtype=np.int64)
    image[on_axis] = np.flatnonzero(on_axis)
    image[~on_axis] = len(nodes) + np.arange(int((~on_axis).sum()))
    full_nodes = np.concatenate([nodes, nodes[~on_axis] * np.array([-1.0, 1.0])])
    full_tris = np.concatenate([tris, image[tris][:, [0, 2, 1]]]).astype(np.int32)   # counter-clockwise

    def f(x, y, t):
        b = np.exp(-20.0 * ((x - 0.25) ** 2 + (y - 0.5) ** 2))
        r, u, v, p = 1.0 + 0.3 * b, -0.6 * b, 0.1 + 0 * x, 1.0 + 0.2 * b
        return np.stack([r, r * u, r * v, p / (GAMMA - 1) + 0.5 * r * (u * u + v * v)], -1)

    s_half = cell_average_states(half, f)
    s_full = np.concatenate([s_half, _mirror_state(s_half)], axis=2)
    wall = OracleMesh(nodes, half.tris, eq=2, bc=1, box=(0.0, 1.0, 0.0, 1.0), walls=0b0001)
    mirror = OracleMesh(full_nodes, full_tris, eq=2, bc=1, box=(-1.0, 1.0, 0.0, 1.0))
    dt = wall.max_dt(s_half, 0.3)
    a = wall.run(s_half, dt, 5)
    b = mirror.run(s_full, dt, 5)
    N = s_half.shape[2]
    assert np.abs(s_half[0, 1, :]).max() > 0.05           # momentum towards the wall
    for blk in range(3):
        scale = np.abs(a[blk]).max()
        e_in = np.abs(b[blk, :, :N] - a[blk]).max() / scale
        e_img = np.abs(b[blk, :, N:] - _mirror_state(a)[blk]).max() / scale
        print(f"block {blk}: wall vs mirror {e_in:.2e}, image {e_img:.2e}", flush=True)
        assert e_in <= 1e-12 and e_img <= 1e-12
