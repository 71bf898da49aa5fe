"""Host-side tests of the HIP library (no GPU needed).

* the shared library loads and exports every symbol declared in include/hwe.h;
* argument and mesh validation return the documented statuses;
* the host precompute (host-only handles, device = -1): the Step-1 map
  reproduces quadratics exactly and agrees with the oracle's least squares,
  the Morton permutation is a permutation, moments match the oracle's cells.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import OracleMesh
from workloads import cell_average_states, split_square_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_10809_amd", "libhwe.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhwe.so not built (run __graft_entry__.build())")


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "hwe.h")).read()
    return sorted(set(re.findall(r"^(?:hwe_status|const char\s*\*)\s*(hwe_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2607_10809_amd import _lib
    L = _lib.load_library()
    names = _header_symbols()
    assert "hwe_step" in names and "hwe_step_adjoint" in names and "hwe_mesh_init" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.exported_symbols()) == names


def _host_mesh(mesh, eq="burgers", bc=None, **kw):
    from paper_2607_10809_amd.hwe import Mesh
    bc = bc or ("periodic" if mesh.periodic else "transmissive")
    return Mesh(mesh.nodes, mesh.tris, eq=eq, bc=bc, box=mesh.box, device=-1, **kw)


def test_error_statuses():
    from paper_2607_10809_amd._lib import HweError
    from paper_2607_10809_amd.hwe import Mesh
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(4, box, periodic=False)
    with pytest.raises(HweError) as e:       # boundary edge under periodic boundaries
        Mesh(mesh.nodes, mesh.tris, eq="burgers", bc="periodic", box=box, device=-1)
    assert e.value.status == -2
    bad = mesh.tris.copy()
    bad[3] = [bad[3, 0], bad[3, 0], bad[3, 1]]
    with pytest.raises(HweError) as e:       # degenerate triangle
        Mesh(mesh.nodes, bad, eq="burgers", bc="transmissive", box=box, device=-1)
    assert e.value.status == -2
    with pytest.raises(HweError) as e:       # empty mesh
        Mesh(mesh.nodes, mesh.tris[:0], eq="burgers", bc="transmissive", box=box, device=-1)
    assert e.value.status == -1
    with pytest.raises(HweError) as e:       # non-manifold edge
        Mesh(mesh.nodes, np.vstack([mesh.tris, mesh.tris[:1]]), eq="burgers", bc="transmissive", box=box,
             device=-1)
    assert e.value.status == -2
    for bad_opts in (dict(eq="euler", gas_gamma=0.5), dict(eq="burgers", time_rule=2),
                     dict(eq="burgers", deriv_weight=0.0), dict(eq="burgers", deriv_weight=float("nan")),
                     dict(eq="burgers", positivity=True), dict(eq="burgers", walls=4),
                     dict(eq="euler", walls=16), dict(eq="burgers", edge_rule=4)):
        with pytest.raises(HweError) as e:   # bad options
            Mesh(mesh.nodes, mesh.tris, bc="transmissive", box=box, device=-1, **bad_opts)
        assert e.value.status == -1, bad_opts
    m = Mesh(mesh.nodes, mesh.tris, eq="burgers", bc="transmissive", box=box, device=-1)
    from paper_2607_10809_amd import _lib
    L = _lib.load_library()
    st = L.hwe_step(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64), C.c_double(0.1),
                    C.c_void_p())
    assert st == -6                             # host-only handle: no device work
    st = L.hwe_step_noalloc(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64),
                            C.c_double(0.1), C.c_void_p())
    assert st == -6
    st = L.hwe_step_keep(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64),
                         C.c_double(0.1), C.c_void_p(4096), C.c_void_p())
    assert st == -6
    st = L.hwe_step_keep(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64),
                         C.c_double(0.1), C.c_void_p(), C.c_void_p())
    assert st == -1                             # null reconstruction buffer
    st = L.hwe_step_adjoint_kept(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(), C.c_void_p(48),
                                 C.c_void_p(64), C.c_void_p(80), C.c_void_p(96), C.c_double(0.1), C.c_void_p())
    assert st == -1
    st = L.hwe_step_keep(m.handle, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64),
                         C.c_double(0.1), C.c_void_p(4104), C.c_void_p())
    assert st == -1                             # reconstruction buffer not 16-byte aligned
    st = L.hwe_debug_edge(m.handle, C.c_void_p(4096), C.c_void_p(16), C.c_double(0.1), C.c_void_p(8200),
                          C.c_void_p(9000), C.c_void_p())
    assert st == -1                             # flux buffer not 16-byte aligned
    assert m.N == 32 and m.m == 1


def test_morton_permutation_and_geometry_match_the_oracle():
    box = (0.0, 3.0, 0.0, 3.0)
    mesh = split_square_mesh(9, box, jitter=0.2, seed=3)
    hm = _host_mesh(mesh)
    assert np.array_equal(np.sort(hm.perm), np.arange(hm.N))
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box)
    g = om.geometry()
    area = hm.host_array(2)
    cen = hm.host_array(1)
    assert np.allclose(area, g["area"][hm.perm], rtol=1e-14)
    assert np.allclose(cen[0], g["cx"][hm.perm], atol=1e-13)
    assert np.allclose(cen[1], g["cy"][hm.perm], atol=1e-13)
    # consecutive internal cells are spatially close (Morton order)
    step = np.hypot(np.diff(cen[0]), np.diff(cen[1]))
    assert np.median(step) < 2.0 * 3.0 / 9


@pytest.mark.parametrize("make", ["double_mach", "wedge", "forward_step", "shu_osher", "shock_tube"])
def test_boundary_kinds_match_the_oracle(make):
    from paper_2607_10809_amd.hwe import Mesh
    import workloads
    wl = {"double_mach": lambda: workloads.double_mach_workload(n=12),
          "wedge": lambda: workloads.wedge_workload(nx=32, ny=12),
          "forward_step": lambda: workloads.forward_step_workload(n=10),
          "shu_osher": lambda: workloads.shu_osher_workload(nx=60),
          "shock_tube": lambda: workloads.shock_tube_workload("lax", nx=40)}[make]()
    hm = Mesh.from_workload(wl, device=-1)
    om = OracleMesh.from_workload(wl)
    ok = om.face_kinds()                       # caller order, (N, 3)
    lk = hm.host_array(5).astype(np.int64)     # internal order, (3, N)
    assert np.array_equal(lk, ok[hm.perm].T)
    assert (lk >= 0).sum() > 0


def test_bad_boundary_regions_are_rejected():
    from paper_2607_10809_amd._lib import HweError
    from paper_2607_10809_amd.hwe import Mesh
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(4, box, periodic=False)
    good = (("A", (0.0, 0.0, 0.0, 1.0)),)
    st = ((1.0, 0.0, 0.0, 2.5), (1.0, 0.0, 0.0, 2.5))
    Mesh(mesh.nodes, mesh.tris, eq="euler", bc="transmissive", box=box, device=-1, regions=good, states=st)
    from paper_2607_10809_amd.hwe import hwe_mesh_init, make_opts
    o = make_opts("euler", "transmissive", box, device=-1, regions=good, states=st)
    o.n_regions = 9                                                           # too many regions
    with pytest.raises(HweError) as e:
        hwe_mesh_init(mesh.nodes, mesh.tris, o)
    assert e.value.status == -1
    for kw in (dict(eq="euler", regions=((7, box),), states=st),              # unknown kind
               dict(eq="burgers", regions=(("wall", box),)),                  # walls need Euler
               dict(eq="euler", regions=(("A", (0.0, float("nan"), 0.0, 1.0)),), states=st),
               dict(eq="euler", regions=(("A", (1.0, 0.0, 0.0, 1.0)),), states=st),   # x0 > x1
               dict(eq="euler", regions=good, states=((float("inf"), 0.0, 0.0, 1.0), st[1])),
               dict(eq="euler", regions=good, states=st, shock=(0.0, float("nan")))):
        with pytest.raises(HweError) as e:
            Mesh(mesh.nodes, mesh.tris, bc="transmissive", box=box, device=-1, **kw)
        assert e.value.status == -1, kw
    pm = split_square_mesh(4, box, periodic=True)
    with pytest.raises(HweError) as e:                                        # regions need boundaries
        Mesh(pm.nodes, pm.tris, eq="euler", bc="periodic", box=box, device=-1, regions=good, states=st)
    assert e.value.status == -1


def test_factored_step1_tables_equal_the_map():
    """The device tables hold the Step-1 map as Md (dW columns), Z and Q with
    the V and Y columns equal to Z^T Q."""
    mesh = split_square_mesh(8, (0.0, 1.0, 0.0, 1.0), jitter=0.25, seed=4, periodic=False)
    hm = _host_mesh(mesh)
    P1 = hm.host_array(0).reshape(5, 11, hm.N)
    F = hm.host_array(6)
    Md = F[0:15].reshape(5, 3, hm.N)
    Z = F[15:25].reshape(2, 5, hm.N)
    Q = F[25:41].reshape(2, 8, hm.N)
    assert np.array_equal(Md, P1[:, 0:3])
    ZQ = np.einsum("kjn,kvn->jvn", Z, Q)
    scale = np.abs(P1[:, 3:]).max(axis=(0, 1))
    assert (np.abs(ZQ - P1[:, 3:]).max(axis=(0, 1)) / scale).max() <= 1e-13


def _apply_p1(hm, state_caller):
    """Apply the library's Step-1 map to a caller-order state (component 0)."""
    T = hm.host_array(0).reshape(5, 11, hm.N)
    nb = hm.host_array(4).astype(np.int64)
    s = state_caller[:, 0, hm.perm]                      # internal order
    W, V, Y = s[0], s[1], s[2]
    c = np.zeros((5, hm.N))
    for i in range(hm.N):
        if (nb[:, i] < 0).any():
            continue
        n = nb[:, i]
        x = np.concatenate([W[n] - W[i], [V[i]], V[n], [Y[i]], Y[n]])
        c[:, i] = T[:, :, i] @ x
    return c, (nb >= 0).all(axis=0)


def test_step1_map_reproduces_quadratics():
    box = (0.0, 1.0, 0.0, 1.0)
    mesh = split_square_mesh(8, box, jitter=0.25, seed=6, periodic=False)
    hm = _host_mesh(mesh, bc="transmissive")
    a = dict(c0=0.2, cx=0.7, cy=-1.2, cxx=1.3, cxy=0.45, cyy=-0.8)
    q = lambda x, y: a["c0"] + a["cx"] * x + a["cy"] * y + a["cxx"] * x * x + a["cxy"] * x * y + a["cyy"] * y * y
    s = cell_average_states(mesh, lambda x, y, t: q(x, y)[..., None])
    c, ok = _apply_p1(hm, s)
    cen = hm.host_array(1)
    for i in np.nonzero(ok)[0]:
        x0, y0 = cen[0, i], cen[1, i]
        expect = [a["cx"] + 2 * a["cxx"] * x0 + a["cxy"] * y0, a["cy"] + a["cxy"] * x0 + 2 * a["cyy"] * y0,
                  a["cxx"], a["cxy"], a["cyy"]]
        assert np.allclose(c[:, i], expect, atol=1e-10), (i, c[:, i], expect)


def test_step1_map_agrees_with_the_oracle_least_squares():
    box = (0.0, 2.0, 0.0, 2.0)
    mesh = split_square_mesh(7, box, jitter=0.3, seed=8, periodic=True)
    hm = _host_mesh(mesh)
    om = OracleMesh(mesh.nodes, mesh.tris, eq=1, bc=0, box=box)
    rng = np.random.default_rng(4)
    s = np.empty((3, 1, om.N))
    s[0, 0] = rng.uniform(0.5, 1.5, om.N)
    s[1:, 0] = rng.uniform(-2, 2, (2, om.N))
    c, ok = _apply_p1(hm, s)
    mom = hm.host_array(3)
    for i in range(0, hm.N, 5):
        k = hm.perm[i]
        p = om.recon_cell(s, k)["p"][0, 0]     # monomial coefficients about the centroid
        mono = np.array([c[0, i], c[1, i], c[2, i], c[3, i], c[4, i]])
        assert np.allclose(mono, p[1:], rtol=1e-9, atol=1e-10 * np.abs(p[1:]).max()), (i, mono, p)
        # constant term: Wbar - c3 Mxx - c4 Mxy - c5 Myy
        a0 = s[0, 0, k] - c[2, i] * mom[0, i] - c[3, i] * mom[1, i] - c[4, i] * mom[2, i]
        assert np.isclose(a0, p[0], rtol=1e-12)


def test_set_time_and_capture_refusals():
    """hwe_set_time takes finite times only; a captured step sequence refuses
    meshes whose boundary switch moves with time (host-side checks)."""
    from paper_2607_10809_amd._lib import HweError
    from paper_2607_10809_amd.hwe import Mesh
    import workloads
    wl = workloads.double_mach_workload(n=6)
    hm = Mesh.from_workload(wl, device=-1)
    hm.set_time(0.05)
    with pytest.raises(HweError) as e:
        hm.set_time(float("nan"))
    assert e.value.status == -1
    with pytest.raises(ValueError):
        hm.capture_steps(None, None, 1e-3, 4)           # moving switch: launches would be frozen
    with pytest.raises(ValueError):
        hm.capture_steps(None, None, 1e-3, 3)           # odd step count
