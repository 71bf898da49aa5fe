"""Oracle pins for reflective walls (Euler): the ghost cell is the mirror image
of the interior cell with its momentum reflected, and the exterior value at a
wall Gauss point is the reflected interior value.

* a gas at rest, and a uniform flow along the walls, stay exactly uniform;
* a closed box conserves mass to round-off (no mass crosses a wall);
* the Lax and Sod shock tubes, run as 2-D strips between walls, converge to the
  exact 1-D Riemann solution (tests/exact_riemann.py, written from the shock and
  rarefaction relations) in L1.
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
