"""Oracle pins for the parts of the step that reduce to a closed form the paper
fixes: the nonlinear weights of Sec. 2.2 Step 5 (eq. (nonlinearweight): the
average W_ave = (sum of the four stencil averages)/4 + 1e-30, the factor
kappa = (|b1-b2| + |b1-b3| + |b1-b4|)^2 / 9 and the denominators
W_ave^4 eps + W_ave^2 beta_s), the smoothness indicators of eq. (smoo1) on a
linear field, the flux viscosity of the local Lax-Friedrichs flux of Sec. 2.1
(the largest of the spectral radii at the two cell averages) and the time-step
rule of the time loop (Sec. 3 fixes the CFL number; the step is
CFL * min inradius / max signal speed).

Each expected value is derived here from the paper's formula without calling
the oracle's version of it: exact rationals (sympy) for the weights, the
closed-form Euler flux and eigenvalues for the flux viscosity, the inradius of
a right isosceles triangle for the time step.
"""
import numpy as np
import pytest

import oracle as O
from oracle import OracleMesh
from workloads import cell_average_states, split_square_mesh

pytestmark = pytest.mark.usefixtures("oracle_lib")

sp = pytest.importorskip("sympy")
GAMMA_LIN = [sp.Rational(94, 100), sp.Rational(2, 100), sp.Rational(2, 100), sp.Rational(2, 100)]
EPS = sp.Rational(1, 10 ** 8)


# ---------------------------------------------------------------- Step 5 weights
def _rational_stencil():
    """Target cell (0,0),(1,0),(0,1) and its three face neighbours (right
    triangles with integer vertices), Burgers (one component)."""
    nodes = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [0, -1], [-1, 0], [1, -1], [-1, 1]], float)
    tris = np.array([[0, 1, 2], [1, 3, 2], [0, 4, 1], [0, 2, 5]], np.int32)
    return nodes, tris


def _integ(expr, P, x, y):
    """Exact integral of a polynomial over the triangle with integer vertices P."""
    P = [(sp.Rational(int(round(px))), sp.Rational(int(round(py)))) for px, py in P]
    u, v = sp.symbols("u v")
    X = P[0][0] + u * (P[1][0] - P[0][0]) + v * (P[2][0] - P[0][0])
    Y = P[0][1] + u * (P[1][1] - P[0][1]) + v * (P[2][1] - P[0][1])
    J = abs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]))
    e = expr.subs({x: X, y: Y}, simultaneous=True) * J
    return sp.integrate(sp.integrate(e, (v, 0, 1 - u)), (u, 0, 1))


def _exact_weights(Wv, Vv, Yv, order, P):
    """Steps 1, 2, 4 and 5 of Sec. 2.2 for cell 0 in exact arithmetic.

    Step 1: the quadratic p1 with the four cell averages exactly and the six
    union derivative integrals in the least-squares sense (Lagrange
    multipliers).  Step 2: the linear p_l with the K0 average exactly and the
    K_l average and derivative averages in the least-squares sense.  Step 4:
    eq. (smoo1) at the barycentre.  Step 5: eq. (nonlinearweight)."""
    x, y = sp.symbols("x y")
    X0 = sum(sp.Rational(int(round(px))) for px, _ in P[0]) / 3
    Y0 = sum(sp.Rational(int(round(py))) for _, py in P[0]) / 3
    area = [abs(_integ(sp.Integer(1), Pl, x, y)) for Pl in P]
    a = sp.symbols("a0:6")
    p1 = a[0] + a[1] * (x - X0) + a[2] * (y - Y0) + a[3] * (x - X0) ** 2 + a[4] * (x - X0) * (y - Y0) \
        + a[5] * (y - Y0) ** 2
    cons = [_integ(p1, P[l], x, y) - area[l] * Wv[order[l]] for l in range(4)]
    res = []
    for l in range(1, 4):
        res.append(_integ(sp.diff(p1, x), P[l], x, y) + _integ(sp.diff(p1, x), P[0], x, y)
                   - (area[l] * Vv[order[l]] + area[0] * Vv[0]))
        res.append(_integ(sp.diff(p1, y), P[l], x, y) + _integ(sp.diff(p1, y), P[0], x, y)
                   - (area[l] * Yv[order[l]] + area[0] * Yv[0]))
    lam = sp.symbols("l0:4")
    Lg = sum(r_ ** 2 for r_ in res) + sum(lam[i] * c for i, c in enumerate(cons))
    sol = sp.solve([sp.diff(Lg, v) for v in list(a) + list(lam)], list(a) + list(lam), dict=True)[0]
    c1 = [sol[ai] for ai in a]
    A0 = area[0]
    betas = [A0 * (c1[1] ** 2 + c1[2] ** 2) + A0 ** 2 * ((2 * c1[3]) ** 2 + c1[4] ** 2 + (2 * c1[5]) ** 2)]
    lin = []
    for l in range(1, 4):
        b0, b1, b2 = sp.symbols("b0:3")
        pl = b0 + b1 * (x - X0) + b2 * (y - Y0)
        r = [(_integ(pl, P[l], x, y) - area[l] * Wv[order[l]]) / area[l], b1 - Vv[order[l]], b2 - Yv[order[l]]]
        mu = sp.symbols("mu")
        Lg = sum(ri ** 2 for ri in r) + mu * (_integ(pl, P[0], x, y) - area[0] * Wv[0])
        s2 = sp.solve([sp.diff(Lg, v) for v in (b0, b1, b2, mu)], [b0, b1, b2, mu], dict=True)[0]
        lin.append((s2[b0], s2[b1], s2[b2]))
        betas.append(A0 * (s2[b1] ** 2 + s2[b2] ** 2))
    W_ave = sum(Wv) / 4 + sp.Rational(1, 10 ** 30)
    kappa = (abs(betas[0] - betas[1]) + abs(betas[0] - betas[2]) + abs(betas[0] - betas[3])) ** 2 / 9
    wbar = [GAMMA_LIN[s] * (1 + kappa / (W_ave ** 4 * EPS + W_ave ** 2 * betas[s])) for s in range(4)]
    omega = [w / sum(wbar) for w in wbar]
    return c1, lin, betas, omega


@pytest.mark.parametrize("case", ["smooth", "kink"])
def test_nonlinear_weights_on_an_exact_rational_stencil(case):
    """omega of eq. (nonlinearweight) on a stencil whose smoothness indicators
    all differ (kappa > 0 and kappa / D of order one), in exact arithmetic.

    A wrong kappa normalisation (no /9), a wrong W_ave (/3), a D without its
    W_ave^2 factor or a missing normalisation of the weights moves omega by
    more than 1e-3 relative here."""
    nodes, tris = _rational_stencil()
    om = OracleMesh(nodes, tris, eq=1, bc=1, box=(-1, 1, -1, 1))
    R = sp.Rational
    if case == "smooth":
        Wv = [R(1), R(3, 2), R(1, 2), R(5, 4)]
        Vv = [R(1, 3), R(-1, 2), R(2), R(1, 5)]
        Yv = [R(-1, 4), R(1, 7), R(0), R(3, 2)]
    else:
        Wv = [R(2), R(7, 4), R(1, 10), R(19, 10)]
        Vv = [R(-1, 2), R(3, 4), R(-5, 2), R(1, 8)]
        Yv = [R(3, 5), R(-2, 3), R(1, 4), R(-1, 9)]
    s = np.zeros((3, 1, 4))
    s[0, 0], s[1, 0], s[2, 0] = [float(v) for v in Wv], [float(v) for v in Vv], [float(v) for v in Yv]
    g = om.geometry()
    order = [0] + list(g["nbr"][0])
    V = om.cell_vertices()
    P = [V[i] for i in order]
    c1, lin, betas, omega = _exact_weights(Wv, Vv, Yv, order, P)
    r = om.recon_cell(s, 0)
    # the candidates and indicators (the inputs of Step 5) ...
    assert np.allclose(r["p"][0, 0], [float(v) for v in c1], rtol=1e-12, atol=1e-13)
    for l in range(1, 4):
        assert np.allclose(r["p"][l, 0, :3], [float(v) for v in lin[l - 1]], rtol=1e-12, atol=1e-13), l
    assert np.allclose(r["beta"][0], [float(b) for b in betas], rtol=1e-12)
    # ... and the weights, far from the linear ones
    om_exact = np.array([float(w) for w in omega])
    assert np.allclose(r["omega"][0], om_exact, rtol=1e-11, atol=0), (r["omega"][0], om_exact)
    assert np.abs(om_exact - np.array([0.94, 0.02, 0.02, 0.02])).max() > 1e-2
    kappa = float((abs(betas[0] - betas[1]) + abs(betas[0] - betas[2]) + abs(betas[0] - betas[3])) ** 2 / 9)
    W_ave = float(sum(Wv) / 4)
    assert 0.05 < kappa / (W_ave ** 2 * float(max(betas))) and kappa / (W_ave ** 2 * float(min(betas))) < 1e4


def test_smoothness_indicators_of_a_linear_field():
    """On the averages of q = c + a x + b y every candidate is q itself (Steps
    1-2), so eq. (smoo1) gives beta_l = |K0| (a^2 + b^2) for every l."""
    box = (0.0, 2.0, 0.0, 2.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=9, periodic=False)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box)
    a, b = -0.8, 2.2
    s = cell_average_states(mesh, lambda x, y, t: (1.5 + a * x + b * y)[..., None])
    g = om.geometry()
    nb = g["nbr"]
    for k in np.nonzero((nb >= 0).all(axis=1))[0][::3]:
        r = om.recon_cell(s, k)
        assert np.allclose(r["beta"][0], g["area"][k] * (a * a + b * b), rtol=1e-11)


# ---------------------------------------------------------------- LLF viscosity in the step
def _euler_flux_n(W, n):
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = 0.4 * (E - 0.5 * (mx * u + my * v))
    un = u * n[0] + v * n[1]
    return np.array([rho * un, mx * un + p * n[0], my * un + p * n[1], (E + p) * un])


def _euler_radius(W, n):
    """|u.n| + c: the largest |eigenvalue| of d(F.n)/dW for a gamma-law gas."""
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = 0.4 * (E - 0.5 * (mx * u + my * v))
    return abs(u * n[0] + v * n[1]) + np.sqrt(1.4 * p / rho)


def _assembled_update(om, s, k, dt, pick):
    """New averages of cell k assembled from the oracle's point values (the
    final reconstruction at the edge Gauss points and its Lax-Wendroff time
    derivatives) with this file's own quadrature, Taylor series, flux and
    viscosity: eqs. (flx), (fx), (flux), (tay), (derave2d2), (timeflux)."""
    g = om.geometry()
    V = om.cell_vertices()
    gl = [0.5 - np.sqrt(3) / 6, 0.5 + np.sqrt(3) / 6]
    taus, wt = [0.0, 0.5, 1.0], [1 / 6, 4 / 6, 1 / 6]
    Wk = s[0, :, k]
    Fs, Vs, Ys = np.zeros(4), np.zeros(4), np.zeros(4)
    for f in range(3):
        nb = g["nbr"][k, f]
        n = g["normal"][k, f]
        ln = g["length"][k, f]
        sh = g["shift"][k, f]
        alpha = pick(_euler_radius(Wk, n), _euler_radius(s[0, :, nb], n))
        A, B = V[k][f], V[k][(f + 1) % 3]
        for sg in gl:
            xg = A + sg * (B - A)
            Di = om.eval_recon(s, k, xg)[0].T          # (6, m)
            De = om.eval_recon(s, nb, xg - sh)[0].T
            ti = O.lax_wendroff(2, Di[None])[0]        # Wt, Wtx, Wty, Wtt
            te = O.lax_wendroff(2, De[None])[0]
            for tau, w in zip(taus, wt):
                T = tau * dt
                Wi = Di[0] + T * ti[0] + 0.5 * T * T * ti[3]
                We = De[0] + T * te[0] + 0.5 * T * T * te[3]
                H = 0.5 * (_euler_flux_n(We, n) + _euler_flux_n(Wi, n) - alpha * (We - Wi))
                Fs += w * 0.5 * ln * H
            Wi = Di[0] + dt * ti[0] + 0.5 * dt * dt * ti[3]
            We = De[0] + dt * te[0] + 0.5 * dt * dt * te[3]
            Wh = 0.5 * (Wi + We)
            Vs += 0.5 * ln * n[0] * Wh
            Ys += 0.5 * ln * n[1] * Wh
    A = g["area"][k]
    return np.stack([Wk - dt / A * Fs, Vs / A, Ys / A])


def test_step_uses_the_larger_spectral_radius_of_the_two_cell_averages():
    """alpha of the local Lax-Friedrichs flux (Sec. 2.1) is the larger of the
    spectral radii of d(F.n)/dW at the two cell averages: the oracle's step
    equals the update assembled with max, and differs visibly from the one
    assembled with min (the data jumps across the cells' faces)."""
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(6, box, jitter=0.2, seed=3, periodic=True)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=2, bc=0, box=box)
    rng = np.random.default_rng(11)
    N = om.N
    rho = rng.uniform(0.5, 2.0, N)
    u, v = rng.uniform(-1.5, 1.5, N), rng.uniform(-1.5, 1.5, N)
    p = rng.uniform(0.3, 3.0, N)
    s = np.zeros((3, 4, N))
    s[0] = [rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)]
    s[1:] = 0.3 * rng.normal(size=(2, 4, N))
    dt = 2e-3
    cells = np.array([0, 17, 40, N - 1])
    got = om.step_cells(s, cells, dt)
    for i, k in enumerate(cells):
        ref = _assembled_update(om, s, k, dt, max)
        alt = _assembled_update(om, s, k, dt, min)
        scale = np.abs(ref[0]).max()
        assert np.abs(got[0, :, i] - ref[0]).max() <= 1e-13 * scale, (k, got[0, :, i], ref[0])
        assert np.abs(got[1:, :, i] - ref[1:]).max() <= 1e-12 * np.abs(ref[1:]).max()
        assert np.abs(alt[0] - ref[0]).max() > 1e-6 * scale


def test_llf_viscosity_is_the_larger_radius_for_burgers():
    """Burgers: lambda = |W (nx + ny)|; a jump from 0.2 to -1.3 across a face
    makes max and min differ by a factor 6.5 in the step's update."""
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(5, box, jitter=0.15, seed=4, periodic=True)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box)
    g = om.geometry()
    s = np.zeros((3, 1, om.N))
    s[0, 0] = np.where(g["cx"] < 0.5, 0.2, -1.3)
    dt = 1e-3
    out = om.step(s, dt)
    # a cell next to the jump: its update carries -1/2 alpha (W_ext - W_int)
    k = next(k for k in range(om.N) if g["cx"][k] < 0.5 and (g["cx"][g["nbr"][k]] > 0.5).any())
    V = om.cell_vertices()
    gl = [0.5 - np.sqrt(3) / 6, 0.5 + np.sqrt(3) / 6]
    Fs = {max: 0.0, min: 0.0}
    for f in range(3):
        nb, n, ln, sh = g["nbr"][k, f], g["normal"][k, f], g["length"][k, f], g["shift"][k, f]
        lam_k, lam_n = abs(s[0, 0, k] * (n[0] + n[1])), abs(s[0, 0, nb] * (n[0] + n[1]))
        A, B = V[k][f], V[k][(f + 1) % 3]
        for sg in gl:
            xg = A + sg * (B - A)
            Di = om.eval_recon(s, k, xg)[0, 0]
            De = om.eval_recon(s, nb, xg - sh)[0, 0]
            ti = O.lax_wendroff(1, Di[None, :, None])[0, :, 0]
            te = O.lax_wendroff(1, De[None, :, None])[0, :, 0]
            for tau, w in zip([0.0, 0.5, 1.0], [1 / 6, 4 / 6, 1 / 6]):
                T = tau * dt
                wi = Di[0] + T * ti[0] + 0.5 * T * T * ti[3]
                we = De[0] + T * te[0] + 0.5 * T * T * te[3]
                for pick in (max, min):
                    H = 0.5 * (0.5 * we * we * (n[0] + n[1]) + 0.5 * wi * wi * (n[0] + n[1])
                               - pick(lam_k, lam_n) * (we - wi))
                    Fs[pick] += w * 0.5 * ln * H
    A = g["area"][k]
    ref = s[0, 0, k] - dt / A * Fs[max]
    alt = s[0, 0, k] - dt / A * Fs[min]
    assert abs(out[0, 0, k] - ref) <= 1e-14 * abs(ref)
    assert abs(alt - ref) > 1e-4 * abs(ref)


# ---------------------------------------------------------------- time step
@pytest.mark.parametrize("eq", [0, 1, 2])
def test_time_step_rule_on_a_regular_mesh(eq):
    """dt = CFL * min_K r_K / max_K lambda_K.  On n x n split squares of side h
    every cell is a right isosceles triangle with inradius h (2 - sqrt 2)/2;
    lambda is sqrt(ax^2 + ay^2) (advection), sqrt(2)|u| (Burgers: the flux
    direction is (1, 1) u) and |(u, v)| + c (Euler)."""
    n, L = 8, 2.0
    box = (0.0, L, 0.0, L)
    mesh = split_square_mesh(n, box, jitter=0.0, periodic=True)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=eq, bc=0, box=box, adv=(0.6, -1.7))
    h = L / n
    r = h * (2.0 - np.sqrt(2.0)) / 2.0
    rng = np.random.default_rng(eq)
    m = 4 if eq == 2 else 1
    s = np.zeros((3, m, om.N))
    if eq == 0:
        s[0, 0] = rng.uniform(-1, 1, om.N)
        lam = np.hypot(0.6, -1.7)
    elif eq == 1:
        s[0, 0] = rng.uniform(-1, 1, om.N)
        s[0, 0, 5] = -2.5
        lam = np.sqrt(2.0) * 2.5
    else:
        rho = rng.uniform(0.5, 2.0, om.N)
        u, v = rng.uniform(-1, 1, om.N), rng.uniform(-1, 1, om.N)
        p = rng.uniform(0.2, 2.0, om.N)
        s[0] = [rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)]
        lam = float(np.max(np.hypot(u, v) + np.sqrt(1.4 * p / rho)))
    dt = om.max_dt(s, 0.3)
    assert np.isclose(dt, 0.3 * r / lam, rtol=1e-13), (dt, 0.3 * r / lam)
