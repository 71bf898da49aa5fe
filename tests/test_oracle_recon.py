"""Oracle pins for the HWENO reconstruction (Sec. 2.2, Steps 1-6).

Pins: polynomial exactness (P3), brute-force constrained least squares on the
printed rows (P2), smoothness-indicator closed forms and weight special cases /
invariances (P4), and one exact-rational stencil checked with sympy.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import OracleMesh
from workloads import cell_average_states, split_square_mesh

pytestmark = pytest.mark.usefixtures("oracle_lib")

GAM = np.array([0.94, 0.02, 0.02, 0.02])


def _tri_quad(P, fn, n=8):
    """Brute-force average of fn over triangle P (3x2): Duffy-collapsed n x n Gauss."""
    x, w = np.polynomial.legendre.leggauss(n)
    t, w = 0.5 * (x + 1), 0.5 * w
    u, v = np.meshgrid(t, t, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    X = P[0] + u[..., None] * (P[1] - P[0]) + (u * v)[..., None] * (P[2] - P[1])
    return float(np.sum(2 * wu * wv * u * fn(X[..., 0], X[..., 1])))


def _quadratic():
    c = dict(c0=0.3, cx=-1.1, cy=0.7, cxx=0.9, cxy=-0.4, cyy=0.35)
    q = lambda x, y: (c["c0"] + c["cx"] * x + c["cy"] * y + c["cxx"] * x * x + c["cxy"] * x * y
                      + c["cyy"] * y * y)
    qx = lambda x, y: c["cx"] + 2 * c["cxx"] * x + c["cxy"] * y
    qy = lambda x, y: c["cy"] + c["cxy"] * x + 2 * c["cyy"] * y
    return c, q, qx, qy


def _interior_cells(om):
    nb = om.geometry()["nbr"]
    return np.nonzero((nb >= 0).all(axis=1))[0]


def _poly_state(mesh, q, qx, qy):
    f = lambda x, y, t: q(x, y)[..., None]
    s = cell_average_states(mesh, f)
    return s


def test_p1_reproduces_quadratics():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(7, box, jitter=0.25, seed=5, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box)
    c, q, qx, qy = _quadratic()
    s = _poly_state(mesh, q, qx, qy)
    g = om.geometry()
    for k in _interior_cells(om)[::3]:
        r = om.recon_cell(s, k)
        x0, y0 = r["centroid"]
        a = r["p"][0, 0]
        expect = [q(x0, y0), qx(x0, y0), qy(x0, y0), c["cxx"], c["cxy"], c["cyy"]]
        assert np.allclose(a, expect, rtol=0, atol=2e-12), (k, a, expect)
        assert np.isclose(r["centroid"][0], g["cx"][k]) and np.isclose(r["centroid"][1], g["cy"][k])


def test_linear_data_is_reproduced_by_every_candidate_and_the_weights_are_linear():
    box = (0.0, 2.0, 0.0, 2.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=9, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box)
    q = lambda x, y: 1.5 - 0.8 * x + 2.2 * y
    s = cell_average_states(mesh, lambda x, y, t: q(x, y)[..., None])
    for k in _interior_cells(om):
        r = om.recon_cell(s, k)
        x0, y0 = r["centroid"]
        for l in range(4):
            assert np.allclose(r["p"][l, 0, :3], [q(x0, y0), -0.8, 2.2], atol=1e-12)
            assert np.allclose(r["p"][l, 0, 3:], 0.0, atol=1e-10)
        # equal smoothness indicators: kappa ~ 0 and omega = gamma
        assert np.allclose(r["beta"][0], r["beta"][0, 0], rtol=1e-10)
        assert np.allclose(r["omega"][0], GAM, rtol=1e-12)
        # final reconstruction (nonlinear weights) is the linear function itself
        V = om.cell_vertices()[k]
        pts = np.array([V.mean(0), 0.5 * (V[0] + V[1]), 0.2 * V[0] + 0.3 * V[1] + 0.5 * V[2]])
        D = om.eval_recon(s, k, pts)[:, 0, :]
        assert np.allclose(D[:, 0], q(pts[:, 0], pts[:, 1]), atol=1e-12)
        assert np.allclose(D[:, 1], -0.8, atol=1e-11) and np.allclose(D[:, 2], 2.2, atol=1e-11)
        assert np.allclose(D[:, 3:], 0.0, atol=1e-9)


def test_linear_weight_mode_reproduces_quadratics_at_any_point():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=2, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box, linear_only=1)
    c, q, qx, qy = _quadratic()
    s = _poly_state(mesh, q, qx, qy)
    V = om.cell_vertices()
    for k in _interior_cells(om)[::2]:
        pts = np.array([V[k].mean(0), V[k][0], 0.5 * (V[k][1] + V[k][2])])
        D = om.eval_recon(s, k, pts)[:, 0, :]
        X, Y = pts[:, 0], pts[:, 1]
        assert np.allclose(D[:, 0], q(X, Y), atol=1e-12)
        assert np.allclose(D[:, 1], qx(X, Y), atol=1e-10)
        assert np.allclose(D[:, 2], qy(X, Y), atol=1e-10)
        assert np.allclose(D[:, 3:], [2 * c["cxx"], c["cxy"], 2 * c["cyy"]], atol=1e-8)


def _stencil_vertices(om, k):
    g = om.geometry()
    V = om.cell_vertices()
    cells = [V[k]]
    for f in range(3):
        j = g["nbr"][k, f]
        cells.append(V[j] + g["shift"][k, f])
    return cells, [k] + list(g["nbr"][k])


@pytest.mark.parametrize("wd", [1.0, 0.35])
def test_least_squares_against_brute_force_nullspace_solution(wd):
    """wd: weight of the Step-2 derivative rows (1 = as printed)."""
    box = (0.0, 3.0, 0.0, 3.0)
    mesh = split_square_mesh(6, box, jitter=0.3, seed=4, periodic=True)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box, deriv_weight=wd)
    rng = np.random.default_rng(0)
    s = np.empty((3, 1, om.N))
    s[0, 0] = rng.uniform(0.5, 1.5, om.N)
    s[1:, 0] = rng.uniform(-2, 2, (2, om.N))
    for k in [0, 7, 33, 50, om.N - 1]:
        cells, ids = _stencil_vertices(om, k)
        r = om.recon_cell(s, k)
        x0, y0 = r["centroid"]
        mon = [lambda x, y: np.ones_like(x), lambda x, y: x - x0, lambda x, y: y - y0,
               lambda x, y: (x - x0) ** 2, lambda x, y: (x - x0) * (y - y0), lambda x, y: (y - y0) ** 2]
        dmx = [lambda x, y: 0 * x, lambda x, y: 1 + 0 * x, lambda x, y: 0 * x,
               lambda x, y: 2 * (x - x0), lambda x, y: (y - y0), lambda x, y: 0 * x]
        dmy = [lambda x, y: 0 * x, lambda x, y: 0 * x, lambda x, y: 1 + 0 * x,
               lambda x, y: 0 * x, lambda x, y: (x - x0), lambda x, y: 2 * (y - y0)]
        area = [0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[1, 1] - P[0, 1]) * (P[2, 0] - P[0, 0]))
                for P in cells]
        # Step 1: equality rows = the four cell averages, LS rows = union derivative integrals
        Cm = np.array([[_tri_quad(P, fj) for fj in mon] for P in cells])
        d = np.array([s[0, 0, i] for i in ids])
        A, b = [], []
        for l in range(1, 4):
            for dm, blk in ((dmx, 1), (dmy, 2)):
                row = [area[0] * _tri_quad(cells[0], fj) + area[l] * _tri_quad(cells[l], fj) for fj in dm]
                A.append(row)
                b.append(area[l] * s[blk, 0, ids[l]] + area[0] * s[blk, 0, ids[0]])
        A, b = np.array(A), np.array(b)
        xp = np.linalg.lstsq(Cm, d, rcond=None)[0]
        Z = sla.null_space(Cm)
        y = np.linalg.lstsq(A @ Z, b - A @ xp, rcond=None)[0]
        p1 = xp + Z @ y
        assert np.allclose(r["p"][0, 0], p1, rtol=1e-9, atol=1e-9 * np.abs(p1).max()), (k, r["p"][0, 0], p1)
        # Step 2: the K0 average exactly; K_l average and derivative averages in LS
        for l in range(1, 4):
            C2 = np.array([[_tri_quad(cells[0], fj) for fj in mon[:3]]])
            A2 = np.array([[_tri_quad(cells[l], fj) for fj in mon[:3]], [0, wd, 0], [0, 0, wd]])
            b2 = np.array([s[0, 0, ids[l]], wd * s[1, 0, ids[l]], wd * s[2, 0, ids[l]]])
            xp = np.linalg.lstsq(C2, [s[0, 0, k]], rcond=None)[0]
            Z = sla.null_space(C2)
            y = np.linalg.lstsq(A2 @ Z, b2 - A2 @ xp, rcond=None)[0]
            pl = xp + Z @ y
            assert np.allclose(r["p"][l, 0, :3], pl, rtol=1e-10, atol=1e-12), (k, l)


def test_smoothness_indicator_closed_form_for_quadratics():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=8, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box)
    c, q, qx, qy = _quadratic()
    s = _poly_state(mesh, q, qx, qy)
    g = om.geometry()
    for k in _interior_cells(om):
        r = om.recon_cell(s, k)
        A = g["area"][k]
        x0, y0 = g["cx"][k], g["cy"][k]
        beta1 = A * (qx(x0, y0) ** 2 + qy(x0, y0) ** 2) + A * A * (
            (2 * c["cxx"]) ** 2 + c["cxy"] ** 2 + (2 * c["cyy"]) ** 2)
        assert np.isclose(r["beta"][0, 0], beta1, rtol=1e-10)
        for l in range(1, 4):
            b, cc = r["p"][l, 0, 1], r["p"][l, 0, 2]
            assert np.isclose(r["beta"][0, l], A * (b * b + cc * cc), rtol=1e-13)


def test_weight_special_cases_and_scale_invariance():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=1, periodic=True)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=0, box=box)
    N = om.N
    const = np.zeros((3, 4, N))
    const[0] = np.array([1.2, 0.3, -0.4, 2.5])[:, None]
    for k in range(0, N, 7):
        r = om.recon_cell(const, k)
        assert (r["beta"] == 0).all()
        assert np.allclose(r["omega"], GAM[None, :] / GAM.sum(), rtol=1e-15, atol=0)
    rng = np.random.default_rng(3)
    s = np.empty((3, 4, N))
    s[0] = rng.uniform(0.5, 2.0, (4, N))
    s[1:] = rng.uniform(-3, 3, (2, 4, N))
    for k in range(0, N, 11):
        r1 = om.recon_cell(s, k)
        r2 = om.recon_cell(3.7 * s, k)
        assert np.allclose(r2["omega"], r1["omega"], rtol=1e-11)
        assert np.allclose(r1["omega"].sum(axis=1), 1.0, rtol=1e-14)
        assert (r1["omega"] > 0).all()


def test_nonlinear_weights_damp_the_candidate_across_a_jump():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(8, box, jitter=0.0, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=1, box=box)
    g = om.geometry()
    cx = g["cx"]
    s = np.zeros((3, 1, om.N))
    s[0, 0] = np.where(cx < 0.5, 1.0, 2.0)
    # a cell left of the jump whose neighbour across one face is right of it
    k = next(k for k in _interior_cells(om) if cx[k] < 0.5 and (cx[g["nbr"][k]] > 0.5).any())
    r = om.recon_cell(s, k)
    jump_faces = [f for f in range(3) if cx[g["nbr"][k, f]] > 0.5]
    smooth_faces = [f for f in range(3) if cx[g["nbr"][k, f]] < 0.5]
    w = r["omega"][0]
    for f in jump_faces:
        for f2 in smooth_faces:
            assert w[1 + f] < 1e-3 * w[1 + f2]
    assert w[0] < 1e-3 * w[1 + smooth_faces[0]]


def test_exact_rational_stencil_with_sympy():
    """One stencil of right triangles with rational data, solved exactly."""
    sp = pytest.importorskip("sympy")
    # target cell (0,0),(1,0),(0,1) and its three face neighbours
    nodes = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [0, -1], [-1, 0], [1, -1], [-1, 1]], float)
    tris = np.array([[0, 1, 2], [1, 3, 2], [0, 4, 1], [0, 2, 5]], np.int32)
    om = OracleMesh(nodes, tris, eq=1, bc=1, box=(-1, 1, -1, 1))
    Wv = [sp.Rational(1), sp.Rational(3, 2), sp.Rational(1, 2), sp.Rational(5, 4)]
    Vv = [sp.Rational(1, 3), sp.Rational(-1, 2), sp.Rational(2), sp.Rational(1, 5)]
    Yv = [sp.Rational(-1, 4), sp.Rational(1, 7), sp.Rational(0), sp.Rational(3, 2)]
    s = np.zeros((3, 1, 4))
    s[0, 0], s[1, 0], s[2, 0] = [float(v) for v in Wv], [float(v) for v in Vv], [float(v) for v in Yv]
    g = om.geometry()
    order = [0] + list(g["nbr"][0])
    x, y = sp.symbols("x y")
    X0, Y0 = sp.Rational(1, 3), sp.Rational(1, 3)
    a = sp.symbols("a0:6")
    p = a[0] + a[1] * (x - X0) + a[2] * (y - Y0) + a[3] * (x - X0) ** 2 + a[4] * (x - X0) * (y - Y0) \
        + a[5] * (y - Y0) ** 2
    V = om.cell_vertices()

    def integ(expr, P):
        P = [(sp.Rational(int(round(px))), sp.Rational(int(round(py)))) for px, py in P]
        u, v = sp.symbols("u v")
        X = P[0][0] + u * (P[1][0] - P[0][0]) + v * (P[2][0] - P[0][0])
        Y = P[0][1] + u * (P[1][1] - P[0][1]) + v * (P[2][1] - P[0][1])
        J = abs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]))
        e = expr.subs({x: X, y: Y}, simultaneous=True) * J
        return sp.integrate(sp.integrate(e, (v, 0, 1 - u)), (u, 0, 1))

    P = [V[i] for i in order]
    area = [sp.Rational(1, 2)] * 4
    cons = [sp.Eq(integ(p, P[l]), area[l] * Wv[order[l]]) for l in range(4)]
    res = []
    for l in range(1, 4):
        res.append(integ(sp.diff(p, x), P[l]) + integ(sp.diff(p, x), P[0])
                   - (area[l] * Vv[order[l]] + area[0] * Vv[0]))
        res.append(integ(sp.diff(p, y), P[l]) + integ(sp.diff(p, y), P[0])
                   - (area[l] * Yv[order[l]] + area[0] * Yv[0]))
    lam = sp.symbols("l0:4")
    Lg = sum(r_ ** 2 for r_ in res) + sum(lam[i] * (c.lhs - c.rhs) for i, c in enumerate(cons))
    sol = sp.solve([sp.diff(Lg, v) for v in list(a) + list(lam)], list(a) + list(lam), dict=True)[0]
    p1 = [sol[ai] for ai in a]
    r = om.recon_cell(s, 0)
    assert np.allclose(r["p"][0, 0], [float(v) for v in p1], rtol=1e-12, atol=1e-13)
    A0 = sp.Rational(1, 2)
    beta1 = A0 * (p1[1] ** 2 + p1[2] ** 2) + A0 ** 2 * ((2 * p1[3]) ** 2 + p1[4] ** 2 + (2 * p1[5]) ** 2)
    assert np.isclose(r["beta"][0, 0], float(beta1), rtol=1e-12)
