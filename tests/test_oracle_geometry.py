"""Oracle pins for the mesh and geometry (closed forms and invariants)."""
import numpy as np
import pytest

from oracle import OracleMesh
from workloads import split_square_mesh

pytestmark = pytest.mark.usefixtures("oracle_lib")


@pytest.mark.parametrize("periodic", [True, False])
def test_areas_normals_and_neighbours(periodic):
    box = (-1.0, 2.0, 0.5, 3.5)
    mesh = split_square_mesh(9, box, jitter=0.2, seed=11, periodic=periodic)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=0 if periodic else 1, box=box)
    g = om.geometry()
    N = om.N
    assert N == 2 * 9 * 9
    # the cells tile the box
    assert np.isclose(g["area"].sum(), 9.0, rtol=1e-13)
    # each closed triangle: sum of n_e |e| = 0 (divergence theorem for a constant)
    closure = (g["normal"] * g["length"][..., None]).sum(axis=1)
    assert np.abs(closure).max() < 1e-13
    # unit normals
    assert np.allclose(np.linalg.norm(g["normal"], axis=-1), 1.0, atol=1e-14)
    # Euler characteristic: E = 3N/2 on a torus; E = (3N + boundary)/2 otherwise
    nb = g["nbr"]
    nbd = int((nb < 0).sum())
    assert om.E == (3 * N + nbd) // 2
    if periodic:
        assert nbd == 0
    else:
        assert nbd == 4 * 9
    # neighbour relation is symmetric, normals opposite, translations antisymmetric
    for k in range(N):
        for f in range(3):
            j = nb[k, f]
            if j < 0:
                continue
            back = np.nonzero(nb[j] == k)[0]
            assert back.size >= 1
            ok = False
            for fb in back:
                if np.allclose(g["normal"][j, fb], -g["normal"][k, f], atol=1e-13) and \
                        np.allclose(g["shift"][j, fb], -g["shift"][k, f], atol=1e-12):
                    ok = True
            assert ok
    # centroids are vertex means in the cell's own frame
    V = om.cell_vertices()
    assert np.allclose(V.mean(axis=1), np.stack([g["cx"], g["cy"]], 1), atol=1e-14)


def test_periodic_translations_are_box_multiples():
    box = (0.0, 4.0, 0.0, 4.0)
    mesh = split_square_mesh(8, box, jitter=0.1, seed=3)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box)
    sh = om.geometry()["shift"].reshape(-1, 2)
    assert np.allclose(sh / 4.0, np.round(sh / 4.0), atol=1e-12)
    assert (np.abs(sh) > 1).any()      # seams are crossed


def test_orientation_is_normalised():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(5, box, jitter=0.1, seed=1, periodic=False)
    tris = mesh.tris.copy()
    tris[::3] = tris[::3, ::-1]          # flip every third triangle to clockwise
    a = OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=1, box=box).geometry()
    b = OracleMesh(mesh.nodes, tris, eq=0, bc=1, box=box).geometry()
    assert np.allclose(a["area"], b["area"], rtol=1e-15)
    assert (b["area"] > 0).all()


def test_bad_meshes_are_rejected():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(4, box, periodic=False)
    # boundary edge in periodic mode
    with pytest.raises(ValueError):
        OracleMesh(mesh.nodes, mesh.tris, eq=0, bc=0, box=box)
    # degenerate triangle
    nodes = mesh.nodes.copy()
    tris = mesh.tris.copy()
    tris[0] = [tris[0, 0], tris[0, 1], tris[0, 1]]
    with pytest.raises(ValueError):
        OracleMesh(nodes, tris, eq=0, bc=1, box=box)
    # non-manifold edge: a third triangle on an existing edge
    extra = np.vstack([mesh.tris, mesh.tris[:1]])
    with pytest.raises(ValueError):
        OracleMesh(mesh.nodes, extra, eq=0, bc=1, box=box)
