"""Oracle pins for the Lax-Wendroff procedure and the local Lax-Friedrichs flux.

The Lax-Wendroff time derivatives are checked against exact symbolic
Cauchy-Kovalevskaya derivatives of polynomial fields (sympy): W_t = -(f_x + g_y),
W_tx and W_ty as x/y derivatives of that field, and
W_tt = -d/dx(f'(W) W_t) - d/dy(g'(W) W_t) (Sec. 2.1).
"""
import numpy as np
import pytest

import oracle as O

sp = pytest.importorskip("sympy")
GG = sp.Rational(7, 5)


def _sym_flux(eq, W):
    if eq == 0:
        return [W[0]], [W[0]]
    if eq == 1:
        return [W[0] ** 2 / 2], [W[0] ** 2 / 2]
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = (GG - 1) * (E - (mx * u + my * v) / 2)
    return [mx, mx * u + p, mx * v, u * (E + p)], [my, my * u, my * v + p, v * (E + p)]


def _fields(eq, rng):
    x, y = sp.symbols("x y")
    m = 4 if eq == 2 else 1
    base = [1.2, 0.4, -0.3, 3.0] if eq == 2 else [0.7]
    W = []
    for q in range(m):
        c = [sp.Rational(int(v), 1000) for v in rng.integers(-300, 300, size=5)]
        W.append(sp.nsimplify(base[q]) + c[0] * x + c[1] * y + c[2] * x * x + c[3] * x * y + c[4] * y * y)
    return x, y, W


@pytest.mark.parametrize("eq", [0, 1, 2])
def test_lax_wendroff_matches_symbolic_cauchy_kovalevskaya(eq):
    rng = np.random.default_rng(10 + eq)
    x, y, W = _fields(eq, rng)
    m = len(W)
    f, g = _sym_flux(eq, W)
    Wt = [-(sp.diff(f[q], x) + sp.diff(g[q], y)) for q in range(m)]
    # d/dt f(W) = sum_j df/dW_j * W_t,j ; build it with a symbolic state vector
    Ws = sp.symbols("w0:%d" % m)
    fs, gs = _sym_flux(eq, list(Ws))
    sub = dict(zip(Ws, W))
    ft = [sum(sp.diff(fs[q], Ws[j]).subs(sub) * Wt[j] for j in range(m)) for q in range(m)]
    gt = [sum(sp.diff(gs[q], Ws[j]).subs(sub) * Wt[j] for j in range(m)) for q in range(m)]
    Wtt = [-(sp.diff(ft[q], x) + sp.diff(gt[q], y)) for q in range(m)]
    pts = [(0.0, 0.0), (0.13, -0.21), (-0.3, 0.25)]
    D = np.zeros((len(pts), 6, m))
    ref = np.zeros((len(pts), 4, m))
    for i, (px, py) in enumerate(pts):
        s = {x: px, y: py}
        for q in range(m):
            D[i, :, q] = [float(e.subs(s)) for e in
                          (W[q], sp.diff(W[q], x), sp.diff(W[q], y), sp.diff(W[q], x, 2),
                           sp.diff(W[q], x, y), sp.diff(W[q], y, 2))]
            ref[i, :, q] = [float(e.subs(s)) for e in
                            (Wt[q], sp.diff(Wt[q], x), sp.diff(Wt[q], y), Wtt[q])]
    adv = (1.0, 1.0)
    out = O.lax_wendroff(eq, D, adv=adv)
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_lax_wendroff_translating_vortex():
    """Exact Euler solution translating with (1,1): W_t = -(W_x + W_y), W_tt = (d_x + d_y)^2 W."""
    x, y = sp.symbols("x y")
    gam = GG
    r2 = (x - 5) ** 2 + (y - 5) ** 2
    rho = (1 - 25 * (gam - 1) / (8 * gam * sp.pi ** 2) * sp.exp(1 - r2)) ** (1 / (gam - 1))
    g = 5 / (2 * sp.pi) * sp.exp((1 - r2) / 2)
    u, v = 1 - g * (y - 5), 1 + g * (x - 5)
    p = rho ** gam
    W = [rho, rho * u, rho * v, p / (gam - 1) + rho * (u * u + v * v) / 2]
    pts = [(5.3, 4.6), (4.1, 5.9)]
    D = np.zeros((len(pts), 6, 4))
    ref = np.zeros((len(pts), 4, 4))
    for i, (px, py) in enumerate(pts):
        s = {x: px, y: py}
        for q in range(4):
            d = [W[q], sp.diff(W[q], x), sp.diff(W[q], y), sp.diff(W[q], x, 2), sp.diff(W[q], x, y),
                 sp.diff(W[q], y, 2)]
            dv = [float(sp.N(e.subs(s), 30)) for e in d]
            D[i, :, q] = dv
            ref[i, :, q] = [-(dv[1] + dv[2]), -(dv[3] + dv[4]), -(dv[4] + dv[5]), dv[3] + 2 * dv[4] + dv[5]]
    out = O.lax_wendroff(2, D)
    assert np.allclose(out, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def test_burgers_one_dimensional_reduction():
    """u = U(x + y): u_t = -2 U U', u_tt = 8 U U'^2 + 4 U^2 U''."""
    U, U1, U2 = 0.8, -0.6, 1.7
    D = np.array([[[U], [U1], [U1], [U2], [U2], [U2]]])
    out = O.lax_wendroff(1, D)[0, :, 0]
    assert np.isclose(out[0], -2 * U * U1, rtol=1e-15)
    assert np.isclose(out[3], 8 * U * U1 ** 2 + 4 * U * U * U2, rtol=1e-14)


@pytest.mark.parametrize("eq", [0, 1, 2])
def test_llf_consistency_and_antisymmetry(eq):
    rng = np.random.default_rng(eq)
    m = 4 if eq == 2 else 1
    if eq == 2:
        def rnd():
            r, u, v, p = rng.uniform(0.5, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2)
            return np.array([r, r * u, r * v, p / 0.4 + 0.5 * r * (u * u + v * v)])
    else:
        def rnd():
            return rng.uniform(-1, 1, size=1)
    th = rng.uniform(0, 2 * np.pi)
    n = np.array([np.cos(th), np.sin(th)])
    for _ in range(5):
        a, b = rnd(), rnd()
        alpha = rng.uniform(0.1, 3.0)
        Haa = O.llf_flux(eq, a, a, n, alpha)
        # consistency: H(W, W) = F(W).n, checked against the direct flux
        Wsym = list(a)
        f, g = _sym_flux(eq, [sp.nsimplify(v) for v in Wsym])
        direct = np.array([float(f[q]) * n[0] + float(g[q]) * n[1] for q in range(m)])
        assert np.allclose(Haa, direct, rtol=1e-13, atol=1e-14)
        # antisymmetry: swapping the sides and reversing the normal flips the sign
        H1 = O.llf_flux(eq, a, b, n, alpha)
        H2 = O.llf_flux(eq, b, a, -n, alpha)
        assert np.allclose(H1, -H2, rtol=1e-14, atol=1e-14)


def test_spectral_radius_is_the_largest_eigenvalue_magnitude():
    W = sp.symbols("w0:4")
    f, g = _sym_flux(2, list(W))
    rng = np.random.default_rng(1)
    for _ in range(5):
        r, u, v, p = rng.uniform(0.5, 1.5), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.3, 2)
        st = [r, r * u, r * v, p / 0.4 + 0.5 * r * (u * u + v * v)]
        th = rng.uniform(0, 2 * np.pi)
        n = (np.cos(th), np.sin(th))
        J = (sp.Matrix(f).jacobian(sp.Matrix(W)) * n[0] + sp.Matrix(g).jacobian(sp.Matrix(W)) * n[1])
        Jn = np.array(J.subs(dict(zip(W, st))).evalf(), dtype=float)
        lam = np.abs(np.linalg.eigvals(Jn)).max()
        assert np.isclose(O.spectral_radius(2, np.array(st), n), lam, rtol=1e-10)
    assert np.isclose(O.spectral_radius(1, np.array([-0.7]), (0.6, 0.8)), 0.7 * 1.4, rtol=1e-15)
    assert np.isclose(O.spectral_radius(0, np.array([3.0]), (0.6, -0.8)), 0.2, rtol=1e-14)
