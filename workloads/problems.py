"""Seeded synthetic workloads: initial data, exact solutions and cell averages.

Every array produced here is an *input* (or an exact reference solution) that is
handed unchanged to both the CPU oracle and the GPU library.  The module holds
none of the numerical method: it only evaluates the paper's initial conditions
and integrates them exactly (to quadrature accuracy) over each triangle.

State layout used throughout: ``state[3][m][N]`` float64 with block 0 the cell
averages of W, block 1 the cell averages of W_x and block 2 those of W_y
(the quantities of the paper's eq. (aver)).

Quadrature (input preparation only):
* cell averages of W: Duffy-collapsed 8 x 8 Gauss-Legendre rule per triangle;
* cell averages of W_x, W_y: divergence theorem, 8-point Gauss-Legendre per edge;
* the four-quadrant Riemann data is piecewise constant, so both are computed
  exactly by clipping triangles and splitting edges at the quadrant lines.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from .meshes import Mesh2D, forward_step_mesh, split_square_mesh, unwrapped_triangles, wedge_mesh

EQ_ADVECTION, EQ_BURGERS, EQ_EULER = 0, 1, 2
GAMMA_GAS = 1.4

_gl_x, _gl_w = np.polynomial.legendre.leggauss(8)
_GL_T = 0.5 * (_gl_x + 1.0)          # nodes on [0, 1]
_GL_W = 0.5 * _gl_w                  # weights summing to 1


def _triangle_rule():
    """Duffy-collapsed tensor rule on the reference triangle, weights sum to 1."""
    u, v = np.meshgrid(_GL_T, _GL_T, indexing="ij")
    wu, wv = np.meshgrid(_GL_W, _GL_W, indexing="ij")
    # x = P0 + u (P1 - P0) + u v (P2 - P1); Jacobian 2|K| u
    a1 = (u * (1.0 - v)).ravel()     # barycentric weight of P1
    a2 = (u * v).ravel()             # barycentric weight of P2
    w = (2.0 * wu * wv * u).ravel()
    return a1, a2, w


_TRI_A1, _TRI_A2, _TRI_W = _triangle_rule()


# ----------------------------------------------------------------------------
# pointwise initial data / exact solutions: f(x, y, t) -> (..., m)
# ----------------------------------------------------------------------------

def _prim_to_cons(rho, u, v, p, gamma=GAMMA_GAS):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], axis=-1)


def advection_sine(x, y, t, k=np.pi, a=(1.0, 1.0)):
    """0.5 + sin(k (x + y)) translated with velocity a."""
    return (0.5 + np.sin(k * ((x - a[0] * t) + (y - a[1] * t))))[..., None]


def burgers_sine(x, y, t, k=0.5 * np.pi):
    """Exact solution of u_t + (u^2/2)_x + (u^2/2)_y = 0 with u0 = 0.5 + sin(k(x+y)).

    Characteristics: u = u0(x - u t, y - u t); solved by Newton's method, valid
    before the breaking time 1/k (the paper's Example 4.1 uses T = 0.5/pi)."""
    s = x + y
    u = 0.5 + np.sin(k * s)
    if t == 0.0:
        return u[..., None]
    for _ in range(60):
        arg = k * (s - 2.0 * u * t)
        F = u - 0.5 - np.sin(arg)
        dF = 1.0 + 2.0 * k * t * np.cos(arg)
        du = F / dF
        u = u - du
        if np.max(np.abs(du)) < 1e-15:
            break
    return u[..., None]


def euler_density_wave(x, y, t):
    """Paper Example 4.2: rho = 1 + 0.2 sin(pi/2 (x + y)), u = v = p = 1, translating."""
    rho = 1.0 + 0.2 * np.sin(0.5 * np.pi * ((x - t) + (y - t)))
    one = np.ones_like(rho)
    return _prim_to_cons(rho, one, one, one)


def make_vortex(center=(5.0, 5.0), strength=5.0, period=(10.0, 10.0), gamma=GAMMA_GAS):
    """Paper Example 4.3 isentropic vortex, translating with velocity (1, 1).

    The vortex centre is taken modulo the period (minimal image), which is how
    the periodic initial condition is defined on the torus."""
    cx, cy = center
    Lx, Ly = period

    def f(x, y, t):
        dx = x - (cx + t)
        dy = y - (cy + t)
        dx = dx - Lx * np.round(dx / Lx)
        dy = dy - Ly * np.round(dy / Ly)
        r2 = dx * dx + dy * dy
        e = np.exp(1.0 - r2)
        T = 1.0 - strength ** 2 * (gamma - 1.0) / (8.0 * gamma * np.pi ** 2) * e
        rho = T ** (1.0 / (gamma - 1.0))
        g = strength / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
        u = 1.0 - g * dy
        v = 1.0 + g * dx
        p = rho ** gamma
        return _prim_to_cons(rho, u, v, p, gamma)

    return f


RIEMANN_QUADRANTS = (  # (rho, u, v, p) for quadrants 1..4 (x>0.5,y>0.5), (x<,y>), (x<,y<), (x>,y<)
    (1.5, 0.0, 0.0, 1.5),
    (0.5323, 1.206, 0.0, 0.3),
    (0.138, 1.206, 1.206, 0.029),
    (0.5323, 0.0, 1.206, 0.3),
)


def riemann_state(q, gamma=GAMMA_GAS):
    rho, u, v, p = RIEMANN_QUADRANTS[q]
    return _prim_to_cons(np.float64(rho), np.float64(u), np.float64(v), np.float64(p), gamma)


def riemann_pointwise(x, y, t=0.0, split=(0.5, 0.5)):
    q = np.where(x >= split[0], np.where(y >= split[1], 0, 3), np.where(y >= split[1], 1, 2))
    states = np.stack([riemann_state(k) for k in range(4)])   # (4, 4)
    return states[q]


# ----------------------------------------------------------------------------
# cell averages
# ----------------------------------------------------------------------------

def _chunks(N, size=65536):
    for s in range(0, N, size):
        yield slice(s, min(N, s + size))


def cell_average_states(mesh: Mesh2D, f: Callable, t: float = 0.0) -> np.ndarray:
    """[3][m][N] cell averages of f(., t), f_x and f_y for a smooth f."""
    P = unwrapped_triangles(mesh)
    N = P.shape[0]
    out = None
    for sl in _chunks(N):
        Pc = P[sl]
        P0, P1, P2 = Pc[:, 0, :], Pc[:, 1, :], Pc[:, 2, :]
        X = P0[:, None, :] + _TRI_A1[None, :, None] * (P1 - P0)[:, None, :] \
            + _TRI_A2[None, :, None] * (P2 - P0)[:, None, :]
        vals = f(X[..., 0], X[..., 1], t)                     # (n, q, m)
        m = vals.shape[-1]
        if out is None:
            out = np.zeros((3, m, N))
        out[0, :, sl] = np.einsum("nqm,q->mn", vals, _TRI_W)
        area = 0.5 * ((P1[:, 0] - P0[:, 0]) * (P2[:, 1] - P0[:, 1])
                      - (P1[:, 1] - P0[:, 1]) * (P2[:, 0] - P0[:, 0]))
        gx = np.zeros((m, Pc.shape[0]))
        gy = np.zeros((m, Pc.shape[0]))
        for k in range(3):
            A = Pc[:, k, :]
            B = Pc[:, (k + 1) % 3, :]
            Y = A[:, None, :] + _GL_T[None, :, None] * (B - A)[:, None, :]
            ev = f(Y[..., 0], Y[..., 1], t)                   # (n, 8, m)
            line = np.einsum("nqm,q->mn", ev, _GL_W)          # mean of f along the edge
            gx += line * (B[:, 1] - A[:, 1])[None, :]
            gy -= line * (B[:, 0] - A[:, 0])[None, :]
        out[1, :, sl] = gx / area[None, :]
        out[2, :, sl] = gy / area[None, :]
    return out


def _clip(poly, axis, value, keep_ge):
    """Clip a convex polygon (list of (x, y)) against x_axis >= value (or <)."""
    out = []
    n = len(poly)
    for i in range(n):
        A = poly[i]
        B = poly[(i + 1) % n]
        ina = (A[axis] >= value) if keep_ge else (A[axis] < value)
        inb = (B[axis] >= value) if keep_ge else (B[axis] < value)
        if ina:
            out.append(A)
        if ina != inb:
            s = (value - A[axis]) / (B[axis] - A[axis])
            out.append((A[0] + s * (B[0] - A[0]), A[1] + s * (B[1] - A[1])))
    return out


def _poly_area(poly):
    if len(poly) < 3:
        return 0.0
    a = 0.0
    for i in range(len(poly)):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % len(poly)]
        a += x0 * y1 - x1 * y0
    return 0.5 * a


def riemann_average_states(mesh: Mesh2D, split=(0.5, 0.5)) -> np.ndarray:
    """Exact [3][4][N] averages of the piecewise-constant four-quadrant data."""
    P = unwrapped_triangles(mesh)
    N = P.shape[0]
    cen = P.mean(axis=1)
    out = np.zeros((3, 4, N))
    out[0] = riemann_pointwise(cen[:, 0], cen[:, 1], 0.0, split).T
    sx, sy = split
    straddle = ((P[:, :, 0].min(1) < sx) & (P[:, :, 0].max(1) > sx)) | \
               ((P[:, :, 1].min(1) < sy) & (P[:, :, 1].max(1) > sy))
    states = np.stack([riemann_state(k) for k in range(4)])
    for c in np.nonzero(straddle)[0]:
        tri = [tuple(P[c, k]) for k in range(3)]
        area = _poly_area(tri)
        acc = np.zeros(4)
        for q, (gx, gy) in enumerate(((True, True), (False, True), (False, False), (True, False))):
            part = _clip(_clip(tri, 0, sx, gx), 1, sy, gy)
            acc += _poly_area(part) * states[q]
        out[0, :, c] = acc / area
        gxs = np.zeros(4)
        gys = np.zeros(4)
        for k in range(3):
            A = np.array(tri[k])
            B = np.array(tri[(k + 1) % 3])
            ts = [0.0, 1.0]
            for ax, val in ((0, sx), (1, sy)):
                den = B[ax] - A[ax]
                if den != 0.0:
                    s = (val - A[ax]) / den
                    if 0.0 < s < 1.0:
                        ts.append(s)
            ts = sorted(ts)
            line = np.zeros(4)
            for t0, t1 in zip(ts[:-1], ts[1:]):
                M = A + 0.5 * (t0 + t1) * (B - A)
                line += (t1 - t0) * riemann_pointwise(np.array(M[0]), np.array(M[1]), 0.0, split)
            gxs += line * (B[1] - A[1])
            gys -= line * (B[0] - A[0])
        out[1, :, c] = gxs / area
        out[2, :, c] = gys / area
    return out


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    eq: int
    m: int
    mesh: Mesh2D
    state0: np.ndarray                  # [3][m][N]
    T: float
    cfl: float
    exact: Callable | None = None       # f(x, y, t) -> (..., m), or None
    adv: tuple = (1.0, 1.0)
    extra: dict = field(default_factory=dict)
    walls: int = 0                      # bit s: box side s (x0, x1, y0, y1) is a reflective wall
    # boundary regions, first match wins: (kind, (x0, x1, y0, y1)) with kind one of
    # "transmissive", "wall", "A", "B" (prescribed states) or "moving" (A where the
    # face midpoint has x < shock[0] + shock[1] t, else B); faces in no region
    # follow `walls`
    regions: tuple = ()
    states: tuple = ()                  # (A, B) conservative states of the prescribed boundaries
    shock: tuple = ()                   # (x0, speed) of the moving switch between A and B

    @property
    def bc(self) -> int:
        return 0 if self.mesh.periodic else 1

    def exact_state(self, t: float) -> np.ndarray:
        if self.exact is None:
            raise ValueError(f"{self.name}: no exact solution")
        return cell_average_states(self.mesh, self.exact, t)


def advection_workload(n=20, jitter=0.0, seed=1, T=0.5, cfl=0.3):
    """2-D linear advection u_t + u_x + u_y = 0 on periodic [0,2]^2, u0 = 0.5 + sin(pi(x+y))."""
    mesh = split_square_mesh(n, (0.0, 2.0, 0.0, 2.0), jitter, seed, periodic=True)
    f = advection_sine
    return Workload("advection", EQ_ADVECTION, 1, mesh, cell_average_states(mesh, f), T, cfl, f)


def burgers_workload(n=160, jitter=0.1, seed=2, T=0.5 / np.pi, cfl=0.3, box=(0.0, 4.0, 0.0, 4.0)):
    """2-D Burgers on a periodic square of side 4, u0 = 0.5 + sin(pi(x+y)/2)."""
    mesh = split_square_mesh(n, box, jitter, seed, periodic=True)
    f = burgers_sine
    return Workload("burgers", EQ_BURGERS, 1, mesh, cell_average_states(mesh, f), T, cfl,
                    f if T < 1.0 / np.pi else None)


def density_wave_workload(n=16, jitter=0.1, seed=7, T=1.0, cfl=0.3):
    """Paper Example 4.2 smooth Euler density wave on periodic (-2,2)^2."""
    mesh = split_square_mesh(n, (-2.0, 2.0, -2.0, 2.0), jitter, seed, periodic=True)
    f = euler_density_wave
    return Workload("density_wave", EQ_EULER, 4, mesh, cell_average_states(mesh, f), T, cfl, f)


def vortex_workload(n=320, jitter=0.1, seed=3, T=2.0, cfl=0.3, center=(5.0, 5.0)):
    """Isentropic vortex (strength 5) on background (1,1,1,1) over periodic [0,10]^2."""
    mesh = split_square_mesh(n, (0.0, 10.0, 0.0, 10.0), jitter, seed, periodic=True)
    f = make_vortex(center)
    return Workload("vortex", EQ_EULER, 4, mesh, cell_average_states(mesh, f), T, cfl, f)


def riemann_workload(n=700, jitter=0.2, seed=4, T=0.3, cfl=0.3):
    """Four-quadrant Euler Riemann problem on [0,1]^2 with transmissive boundaries."""
    mesh = split_square_mesh(n, (0.0, 1.0, 0.0, 1.0), jitter, seed, periodic=False)
    return Workload("riemann", EQ_EULER, 4, mesh, riemann_average_states(mesh), T, cfl, None)


def shock_tube_average_states(mesh: Mesh2D, x_split, left, right) -> np.ndarray:
    """Exact [3][4][N] averages of piecewise-constant data that depend on x only:
    primitive states left = (rho, u, v, p) for x < x_split, right beyond."""
    P = unwrapped_triangles(mesh)
    N = P.shape[0]
    WL = _prim_to_cons(*map(np.float64, left))
    WR = _prim_to_cons(*map(np.float64, right))
    out = np.zeros((3, 4, N))
    cen = P.mean(axis=1)
    out[0] = np.where(cen[:, 0][None, :] >= x_split, WR[:, None], WL[:, None])
    straddle = (P[:, :, 0].min(1) < x_split) & (P[:, :, 0].max(1) > x_split)
    for c in np.nonzero(straddle)[0]:
        tri = [tuple(P[c, k]) for k in range(3)]
        area = _poly_area(tri)
        aR = _poly_area(_clip(tri, 0, x_split, True))
        out[0, :, c] = (aR * WR + (area - aR) * WL) / area
        # derivative averages by the divergence theorem: the x-derivative of a
        # step is the jump times the length of the step line inside the cell
        pts = []
        for k in range(3):
            A, B = np.array(tri[k]), np.array(tri[(k + 1) % 3])
            if (A[0] - x_split) * (B[0] - x_split) < 0:
                s = (x_split - A[0]) / (B[0] - A[0])
                pts.append(A[1] + s * (B[1] - A[1]))
        length = abs(pts[1] - pts[0]) if len(pts) == 2 else 0.0
        out[1, :, c] = (WR - WL) * length / area
        out[2, :, c] = 0.0
    return out


def _split_halfplane(poly, a, b, c):
    """Split a convex polygon by the line a x + b y = c: (part < c, part >= c)."""
    lo, hi = [], []
    n = len(poly)
    for i in range(n):
        A = poly[i]
        B = poly[(i + 1) % n]
        fa = a * A[0] + b * A[1] - c
        fb = a * B[0] + b * B[1] - c
        (hi if fa >= 0 else lo).append(A)
        if (fa >= 0) != (fb >= 0):
            s = fa / (fa - fb)
            P = (A[0] + s * (B[0] - A[0]), A[1] + s * (B[1] - A[1]))
            lo.append(P)
            hi.append(P)
    return lo, hi


def piecewise_average_states(mesh: Mesh2D, f: Callable, lines, t: float = 0.0) -> np.ndarray:
    """[3][m][N] cell averages of f, f_x and f_y for f smooth except across the
    straight lines a x + b y = c in ``lines``.  Cells that a line crosses are cut
    into pieces, each integrated with the triangle rule on a fan of triangles;
    the derivative averages are (1/|K|) times the boundary integral of f n,
    with the edges split where the lines cross them (so the jumps count)."""
    out = cell_average_states(mesh, f, t)
    P = unwrapped_triangles(mesh)
    cut = np.zeros(P.shape[0], dtype=bool)
    for a, b, c in lines:
        v = a * P[:, :, 0] + b * P[:, :, 1] - c
        cut |= (v.min(axis=1) < 0) & (v.max(axis=1) > 0)
    for k in np.nonzero(cut)[0]:
        tri = [tuple(P[k, j]) for j in range(3)]
        area = _poly_area(tri)
        pieces = [tri]
        for a, b, c in lines:
            nxt = []
            for pc in pieces:
                for part in _split_halfplane(pc, a, b, c):
                    if len(part) >= 3 and _poly_area(part) > 0.0:
                        nxt.append(part)
            pieces = nxt
        acc = 0.0
        for pc in pieces:
            Q0 = np.array(pc[0])
            for j in range(1, len(pc) - 1):
                Q1, Q2 = np.array(pc[j]), np.array(pc[j + 1])
                ar = 0.5 * ((Q1[0] - Q0[0]) * (Q2[1] - Q0[1]) - (Q1[1] - Q0[1]) * (Q2[0] - Q0[0]))
                X = Q0[None, :] + _TRI_A1[:, None] * (Q1 - Q0)[None, :] + _TRI_A2[:, None] * (Q2 - Q0)[None, :]
                acc = acc + ar * np.einsum("qm,q->m", f(X[:, 0], X[:, 1], t), _TRI_W)
        out[0, :, k] = acc / area
        gx = 0.0
        gy = 0.0
        for j in range(3):
            A, B = np.array(tri[j]), np.array(tri[(j + 1) % 3])
            ts = [0.0, 1.0]
            for a, b, c in lines:
                fa = a * A[0] + b * A[1] - c
                fb = a * B[0] + b * B[1] - c
                if fa != fb:
                    s_ = fa / (fa - fb)
                    if 0.0 < s_ < 1.0:
                        ts.append(s_)
            ts.sort()
            line = 0.0
            for t0, t1 in zip(ts[:-1], ts[1:]):
                Y = A[None, :] + (t0 + (t1 - t0) * _GL_T)[:, None] * (B - A)[None, :]
                line = line + (t1 - t0) * np.einsum("qm,q->m", f(Y[:, 0], Y[:, 1], t), _GL_W)
            gx = gx + line * (B[1] - A[1])
            gy = gy - line * (B[0] - A[0])
        out[1, :, k] = gx / area
        out[2, :, k] = gy / area
    return out


# Shock tubes on a strip with reflective walls at y = y0, y1 (a 1-D Riemann
# problem in 2-D, so that the exact solution is the 1-D one): the Lax problem
# of Sec. 4 (states (rho, u, p) = (0.445, 0.698, 3.528) | (0.5, 0, 0.571) split
# at x = 0, T = 0.16) and Sod's problem ((1, 0, 1) | (0.125, 0, 0.1), T = 0.2).
SHOCK_TUBES = {
    "lax": ((0.445, 0.698, 0.0, 3.528), (0.5, 0.0, 0.0, 0.571), 0.16),
    "sod": ((1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1), 0.2),
}


def shock_tube_workload(name="lax", nx=200, height=0.06, jitter=0.1, seed=8, cfl=0.3):
    """A shock tube on (-0.5, 0.5) x (-height/2, height/2): nx x ny squares of side
    1/nx, transmissive ends, reflective walls on the long sides."""
    left, right, T = SHOCK_TUBES[name]
    ny = max(3, int(round(height * nx)))
    box = (-0.5, 0.5, -0.5 * ny / nx, 0.5 * ny / nx)
    mesh = split_square_mesh((nx, ny), box, jitter, seed, periodic=False)
    return Workload(name, EQ_EULER, 4, mesh, shock_tube_average_states(mesh, 0.0, left, right), T, cfl, None,
                    extra=dict(left=left, right=right, x_split=0.0), walls=0b1100)


def _two_state(WA, WB, a, b, c):
    """Pointwise data: conservative WA where a x + b y < c, WB elsewhere."""
    WA, WB = np.asarray(WA, dtype=np.float64), np.asarray(WB, dtype=np.float64)

    def f(x, y, t):
        side = (a * np.asarray(x) + b * np.asarray(y) - c) < 0
        return np.where(side[..., None], WA, WB)
    return f


def _strip(x0, x1, height, nx, jitter, seed):
    ny = max(3, int(round(height * nx / (x1 - x0))))
    hy = 0.5 * ny * (x1 - x0) / nx
    return split_square_mesh((nx, ny), (x0, x1, -hy, hy), jitter, seed, periodic=False)


# The Shu-Osher problem of Sec. 4: a Mach 3 shock at x = -4 running into a
# density sine wave on (-5, 5) x (-0.1, 0.1), T = 1.8.  Prescribed inflow
# state on the left, transmissive outflow on the right, walls on the long sides.
SHU_OSHER_LEFT = (3.857143, 2.629369, 0.0, 10.333333)


def shu_osher_workload(nx=300, height=0.2, jitter=0.1, seed=9, cfl=0.3, T=1.8):
    mesh = _strip(-5.0, 5.0, height, nx, jitter, seed)
    WL = _prim_to_cons(*map(np.float64, SHU_OSHER_LEFT))

    def f(x, y, t):
        x = np.asarray(x)
        rho = 1.0 + 0.2 * np.sin(5.0 * x)
        right = _prim_to_cons(rho, np.zeros_like(x), np.zeros_like(x), np.ones_like(x))
        return np.where((x < -4.0)[..., None], WL, right)
    st = piecewise_average_states(mesh, f, [(1.0, 0.0, -4.0)])
    x0, y0, y1 = mesh.box[0], mesh.box[2], mesh.box[3]
    return Workload("shu_osher", EQ_EULER, 4, mesh, st, T, cfl, None, walls=0b1100,
                    regions=(("A", (x0, x0, y0, y1)),), states=(tuple(WL), tuple(WL)), shock=(0.0, 0.0))


# Interacting blast waves of Sec. 4 on (0, 1) x (-0.0075, 0.0075), walls all
# round, T = 0.038: rho = 1, u = v = 0, p = 1000 | 0.01 | 100 split at 0.1, 0.9.
def blast_wave_workload(nx=400, height=0.015, jitter=0.1, seed=10, cfl=0.3, T=0.038):
    mesh = _strip(0.0, 1.0, height, nx, jitter, seed)

    def f(x, y, t):
        x = np.asarray(x)
        p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
        z = np.zeros_like(x)
        return _prim_to_cons(np.ones_like(x), z, z, p)
    st = piecewise_average_states(mesh, f, [(1.0, 0.0, 0.1), (1.0, 0.0, 0.9)])
    return Workload("blast_wave", EQ_EULER, 4, mesh, st, T, cfl, None, walls=0b1111)


# Double Mach reflection of Sec. 4 on (0, 4) x (0, 1), T = 0.2: a Mach 10 shock
# through x = 1/6 at 60 degrees to the bottom wall.  State A (behind the shock,
# the conservative values printed in the paper) where y >= sqrt(3) (x - 1/6),
# B = (1.4, 0, 0, 2.5) ahead.  Boundaries: A on the left and on the bottom for
# x < 1/6, wall on the rest of the bottom, transmissive on the right, and on
# the top the exact shock position x_s(t) = 1/6 + (1 + 20 t) / sqrt(3).
DMR_A = (8.0, 57.1597, -33.0012, 563.544)
DMR_B = (1.4, 0.0, 0.0, 2.5)


def double_mach_workload(n=60, jitter=0.1, seed=11, cfl=0.3, T=0.2):
    """n squares per unit length: 4n x n split squares (8 n^2 triangles); n a
    multiple of 6 puts x = 1/6 on the grid."""
    mesh = split_square_mesh((4 * n, n), (0.0, 4.0, 0.0, 1.0), jitter, seed, periodic=False)
    r3 = np.sqrt(3.0)
    st = piecewise_average_states(mesh, _two_state(DMR_A, DMR_B, r3, -1.0, r3 / 6.0), [(r3, -1.0, r3 / 6.0)])
    regions = (("A", (0.0, 1.0 / 6.0, 0.0, 0.0)), ("wall", (1.0 / 6.0, 4.0, 0.0, 0.0)),
               ("moving", (0.0, 4.0, 1.0, 1.0)), ("A", (0.0, 0.0, 0.0, 1.0)))
    return Workload("double_mach", EQ_EULER, 4, mesh, st, T, cfl, None, regions=regions,
                    states=(DMR_A, DMR_B), shock=(1.0 / 6.0 + 1.0 / r3, 20.0 / r3))


# Double Mach reflection over a 30-degree wedge of Sec. 4 on (-1/6, 2.5) x (0, 2),
# T = 0.2: a Mach 10 shock at x = 0 moving right; (rho, u, v, p) = (8, 8.25, 0,
# 116.5) behind it, (1.4, 0, 0, 1) ahead.  Boundaries: behind-shock state on the
# left and on the bottom for x < 0, transmissive on the right, the exact shock
# position x_s(t) = 10 t on the top, walls elsewhere (the wedge).
WEDGE_A = (8.0, 8.25, 0.0, 116.5)
WEDGE_B = (1.4, 0.0, 0.0, 1.0)


def wedge_workload(nx=160, ny=120, jitter=0.1, seed=12, cfl=0.3, T=0.2):
    """nx a multiple of 16 puts the wedge tip x = 0 on the grid."""
    mesh = wedge_mesh(nx, ny, jitter, seed)
    WA = tuple(_prim_to_cons(*map(np.float64, WEDGE_A)))
    WB = tuple(_prim_to_cons(*map(np.float64, WEDGE_B)))
    st = piecewise_average_states(mesh, _two_state(WA, WB, 1.0, 0.0, 0.0), [(1.0, 0.0, 0.0)])
    x0, x1, y0, y1 = mesh.box
    regions = (("A", (x0, 0.0, 0.0, 0.0)), ("A", (x0, x0, y0, y1)), ("moving", (x0, x1, y1, y1)),
               ("transmissive", (x1, x1, y0, y1)), ("wall", (x0, x1, y0, y1)))
    return Workload("wedge", EQ_EULER, 4, mesh, st, T, cfl, None, regions=regions, states=(WA, WB),
                    shock=(0.0, 10.0))


# The forward-facing step of Sec. 4: a Mach 3 wind tunnel (0, 3) x (0, 1) with a
# step of height 0.2 from x = 0.6, uniform (1.4, 3, 0, 1) initially and at the
# inlet, transmissive outlet, walls elsewhere; T = 4.
STEP_A = (1.4, 3.0, 0.0, 1.0)


def forward_step_workload(n=40, jitter=0.1, seed=13, cfl=0.3, T=4.0):
    mesh = forward_step_mesh(n, jitter, seed)
    WA = tuple(_prim_to_cons(*map(np.float64, STEP_A)))
    st = np.zeros((3, 4, mesh.n_cells))
    st[0] = np.asarray(WA)[:, None]
    regions = (("A", (0.0, 0.0, 0.0, 1.0)), ("transmissive", (3.0, 3.0, 0.2, 1.0)),
               ("wall", (0.0, 3.0, 0.0, 1.0)))
    return Workload("forward_step", EQ_EULER, 4, mesh, st, T, cfl, None, regions=regions, states=(WA, WA),
                    shock=(0.0, 0.0))


# A planar Mach 10 shock (the wedge problem's states) running along a strip
# (0, 1) x (0, 0.1) from x = 0.2 at speed 10: an exact travelling solution,
# with the behind-shock state prescribed on the left, transmissive on the right
# and the moving switch on the long sides.
def moving_shock_workload(nx=100, height=0.1, jitter=0.1, seed=14, cfl=0.3, T=0.05):
    ny = max(3, int(round(height * nx)))
    mesh = split_square_mesh((nx, ny), (0.0, 1.0, 0.0, ny / nx), jitter, seed, periodic=False)
    WA = tuple(_prim_to_cons(*map(np.float64, WEDGE_A)))
    WB = tuple(_prim_to_cons(*map(np.float64, WEDGE_B)))
    st = piecewise_average_states(mesh, _two_state(WA, WB, 1.0, 0.0, 0.2), [(1.0, 0.0, 0.2)])
    x0, x1, y0, y1 = mesh.box
    regions = (("A", (x0, x0, y0, y1)), ("moving", (x0, x1, y0, y0)), ("moving", (x0, x1, y1, y1)))
    return Workload("moving_shock", EQ_EULER, 4, mesh, st, T, cfl, None, regions=regions, states=(WA, WB),
                    shock=(0.2, 10.0), extra=dict(x_shock=lambda t: 0.2 + 10.0 * t))


def perturbed_vortex_target_center(seed=5, sigma=0.3, base=(5.0, 5.0)):
    """Centre of the target vortex for the adjoint misfit: base + N(0, sigma^2) per axis."""
    rng = np.random.default_rng(seed)
    d = rng.normal(0.0, sigma, size=2)
    return (base[0] + float(d[0]), base[1] + float(d[1]))


def fd_directions(N, count=32, seed=6):
    """Unit-norm Gaussian directions over a density slice, shape (count, N)."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(count, N))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_state(m, N, seed, scale=1.0, base=1.0):
    """A seeded random positive state [3][m][N] for unit-level parity checks."""
    rng = np.random.default_rng(seed)
    s = np.empty((3, m, N))
    s[0] = base + 0.1 * scale * rng.uniform(-1.0, 1.0, size=(m, N))
    s[1:] = scale * rng.uniform(-1.0, 1.0, size=(2, m, N))
    return s


def near_vacuum_state(wl: Workload, seed, branch="pressure", untie=False):
    """Data on which the positivity (scaling) limiter acts: the workload's cell
    averages with the part below a fifth of the largest density thinned a
    thousandfold, and seeded derivative averages of the size of the averages
    over a cell.  branch "pressure": small density derivative averages, so
    that only the pressure scaling acts (on hundreds of cells of the
    four-quadrant data); "density": the gas at rest with small energy
    derivative averages, so that only the density scaling acts.  untie:
    also perturb the averages (momentum additively) so that no two
    neighbouring cells are equal and no gas is exactly at rest (piecewise
    constant data sit on the ties of the flux viscosity's max and of |u.n|)."""
    s = wl.state0.copy()
    low = s[0, 0] < 0.2 * s[0, 0].max()
    s[:, :, low] *= 1e-3
    if branch == "density":
        s[:, 1:3] = 0.0
    rng = np.random.default_rng(seed)
    g = rng.normal(size=s[1:].shape) * np.abs(s[0])[None] / wl.mesh.h
    scales = (0.05, 1.0, 1.0, 1.0) if branch == "pressure" else (1.0, 0.0, 0.0, 0.05)
    s[1:] = g * np.asarray(scales)[None, :, None]
    if untie:
        s[0] *= 1.0 + 1e-3 * rng.uniform(-1.0, 1.0, s[0].shape)
        s[0, 1:3] += 1e-2 * np.abs(s[0, 0]) * rng.uniform(-1.0, 1.0, s[0, 1:3].shape)
    return s
