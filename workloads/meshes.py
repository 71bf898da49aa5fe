"""Seeded synthetic triangular meshes (split squares with node jitter).

The paper runs on GMSH meshes that are not available; these meshes stand in for
them with the same kind of element (unstructured-looking triangles obtained by
jittering the nodes of a split-square grid).  Nothing here belongs to the
numerical method: the module only produces node coordinates and connectivity.

Conventions
-----------
* Square (i, j) with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) is split
  along the a-c diagonal into the triangles (a, b, c) and (a, c, d); both are
  counter-clockwise.  Triangle 2*(j*n+i) is the lower one, 2*(j*n+i)+1 the
  upper one.
* Periodic meshes are tori: n x n distinct nodes, node (i, j) has index j*n+i and
  triangles reference nodes modulo n.  Coordinates lie in [x0, x1) x [y0, y1);
  a triangle that straddles a seam is unwrapped by the consumer.
* Non-periodic meshes have (n+1) x (n+1) nodes.
* Rectangular meshes (n = (nx, ny)) follow the same rules with nx squares
  along x and ny along y.
* Jitter: nodes strictly inside the box get an independent uniform offset in
  [-f*h, f*h] per coordinate, drawn from ``numpy.random.default_rng(seed)`` as
  one array of shape (rows, cols, 2) in row-major node order; nodes on the box
  boundary (and on the periodic seams) stay on the grid.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh2D:
    nodes: np.ndarray      # (V, 2) float64
    tris: np.ndarray       # (N, 3) int32, counter-clockwise
    box: tuple             # (x0, x1, y0, y1)
    periodic: bool
    n: int                 # squares per side
    h: float               # square side (x direction)

    @property
    def n_cells(self) -> int:
        return int(self.tris.shape[0])


def split_square_mesh(n, box=(0.0, 1.0, 0.0, 1.0), jitter: float = 0.0,
                      seed: int | None = None, periodic: bool = True) -> Mesh2D:
    """Return an n x n split-square mesh of ``box`` (2 n^2 triangles); ``n`` may
    also be a pair (nx, ny) of squares along x and y (2 nx ny triangles)."""
    nx, ny = (n, n) if np.isscalar(n) else (int(n[0]), int(n[1]))
    if nx < 3 or ny < 3:
        raise ValueError("need at least 3 squares per side")
    x0, x1, y0, y1 = map(float, box)
    hx = (x1 - x0) / nx
    hy = (y1 - y0) / ny
    mx = nx if periodic else nx + 1     # node columns
    my = ny if periodic else ny + 1     # node rows
    jj, ii = np.meshgrid(np.arange(my), np.arange(mx), indexing="ij")
    xs = x0 + ii * hx
    ys = y0 + jj * hy
    if jitter and jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-1.0, 1.0, size=(my, mx, 2))
        inner = (ii >= 1) & (ii <= nx - 1) & (jj >= 1) & (jj <= ny - 1)
        xs = xs + np.where(inner, off[..., 0] * jitter * hx, 0.0)
        ys = ys + np.where(inner, off[..., 1] * jitter * hy, 0.0)
    nodes = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)

    def nid(i, j):
        if periodic:
            return (j % ny) * nx + (i % nx)
        return j * (nx + 1) + i

    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    a = nid(I, J)
    b = nid(I + 1, J)
    c = nid(I + 1, J + 1)
    d = nid(I, J + 1)
    tris = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tris[0::2] = np.stack([a, b, c], axis=1)
    tris[1::2] = np.stack([a, c, d], axis=1)
    return Mesh2D(nodes=nodes, tris=tris, box=(x0, x1, y0, y1), periodic=periodic, n=nx, h=hx)


def unwrapped_triangles(mesh: Mesh2D) -> np.ndarray:
    """Vertex coordinates per triangle, (N, 3, 2), seams unwrapped about vertex 0."""
    P = mesh.nodes[mesh.tris]                     # (N, 3, 2)
    if mesh.periodic:
        L = np.array([mesh.box[1] - mesh.box[0], mesh.box[3] - mesh.box[2]])
        d = P - P[:, :1, :]
        d -= L * np.round(d / L)
        P = P[:, :1, :] + d
    return P


def _boundary_nodes(tris: np.ndarray, n_nodes: int) -> np.ndarray:
    """Mask of the nodes on edges that belong to one triangle only."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e.sort(axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    mask = np.zeros(n_nodes, dtype=bool)
    mask[uniq[cnt == 1].ravel()] = True
    return mask


def _jitter_interior(nodes, tris, jitter, seed, hx, hy):
    """Uniform offsets in [-f h, f h] per coordinate, drawn as one (V, 2) array in
    node order, applied to the nodes on no boundary edge."""
    if not jitter or jitter <= 0.0:
        return nodes
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, size=nodes.shape)
    inner = ~_boundary_nodes(tris, nodes.shape[0])
    out = nodes.copy()
    out[inner, 0] += off[inner, 0] * jitter * hx
    out[inner, 1] += off[inner, 1] * jitter * hy
    return out


def forward_step_mesh(n: int, jitter: float = 0.0, seed: int | None = None) -> Mesh2D:
    """The wind tunnel (0, 3) x (0, 1) with the step [0.6, 3] x [0, 0.2] removed:
    split squares of side 1/n (n a multiple of 5, so the step corner is a node),
    interior nodes jittered (nodes on the tunnel walls, the step, the inlet and
    the outlet stay on the grid).  Nodes are renumbered to the ones in use."""
    if n % 5 or n < 5:
        raise ValueError("n must be a positive multiple of 5")
    full = split_square_mesh((3 * n, n), (0.0, 3.0, 0.0, 1.0), 0.0, None, periodic=False)
    cen = full.nodes[full.tris].mean(axis=1)
    keep = ~((cen[:, 0] > 0.6) & (cen[:, 1] < 0.2))
    tris = full.tris[keep]
    used = np.unique(tris)
    remap = -np.ones(full.nodes.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    tris = remap[tris].astype(np.int32)
    nodes = full.nodes[used]
    h = 1.0 / n
    nodes = _jitter_interior(nodes, tris, jitter, seed, h, h)
    return Mesh2D(nodes=nodes, tris=tris, box=(0.0, 3.0, 0.0, 1.0), periodic=False, n=3 * n, h=h)


def wedge_mesh(nx: int, ny: int, jitter: float = 0.0, seed: int | None = None,
               x0: float = -1.0 / 6.0, x1: float = 2.5, top: float = 2.0,
               angle_deg: float = 30.0) -> Mesh2D:
    """The region over a wedge: x in (x0, x1), y from b(x) to ``top`` with
    b(x) = 0 for x <= 0 and x tan(angle) beyond.  A mapped grid of nx columns
    (x = 0 must be a grid line: nx (0 - x0) / (x1 - x0) an integer) and ny rows
    evenly spaced between b(x) and top; each quadrilateral is split along the
    diagonal from its lower-left corner.  Interior nodes are jittered by up to
    f times the local spacing."""
    k = nx * (0.0 - x0) / (x1 - x0)
    if abs(k - round(k)) > 1e-9:
        raise ValueError("x = 0 must be a grid line")
    t = np.tan(np.radians(angle_deg))
    xs = x0 + (x1 - x0) * np.arange(nx + 1) / nx
    xs[int(round(k))] = 0.0
    b = np.where(xs > 0.0, xs * t, 0.0)
    jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = xs[ii]
    Y = b[ii] + (top - b[ii]) * jj / ny
    nodes = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    nid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    a, bb, c, d = nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)
    tris = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tris[0::2] = np.stack([a, bb, c], axis=1)
    tris[1::2] = np.stack([a, c, d], axis=1)
    if jitter and jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-1.0, 1.0, size=(ny + 1, nx + 1, 2))
        inner = (ii >= 1) & (ii <= nx - 1) & (jj >= 1) & (jj <= ny - 1)
        hx = (x1 - x0) / nx
        hy = (top - b[ii]) / ny
        Xj = X + np.where(inner, off[..., 0] * jitter * hx, 0.0)
        Yj = Y + np.where(inner, off[..., 1] * jitter * hy, 0.0)
        nodes = np.stack([Xj.ravel(), Yj.ravel()], axis=1).astype(np.float64)
    return Mesh2D(nodes=nodes, tris=tris, box=(x0, x1, 0.0, top), periodic=False, n=nx, h=(x1 - x0) / nx)
