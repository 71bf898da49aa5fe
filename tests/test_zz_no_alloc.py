"""GPU test of hwe_step_noalloc, the step whose scratch is the library's static
device array (for callers that cannot allocate), against hwe_step: the same
results, bit for bit, on consecutive calls whose second input is smaller than
the first (the array keeps the previous call's contents), and a clear refusal
of a mesh whose scratch exceeds the array."""
import ctypes as C

import numpy as np
import pytest

from workloads import burgers_workload, riemann_workload, vortex_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _both(mesh, state, dt):
    """One step of each entry point through the C ABI on the same input."""
    import torch
    from paper_2607_10809_amd import _lib
    L = _lib.load_library()
    w, g = mesh.to_device(state)
    wa, ga = mesh.empty_state()
    wb, gb = mesh.empty_state()
    wb.fill_(np.nan)
    gb.fill_(np.nan)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.hwe_step(mesh.handle, _p(w), _p(g), _p(wa), _p(ga), C.c_double(dt), st))
    _lib.check(L.hwe_step_noalloc(mesh.handle, _p(w), _p(g), _p(wb), _p(gb), C.c_double(dt), st))
    torch.cuda.synchronize()
    return (wa, ga), (wb, gb)


CASES = [
    ("vortex fp64", lambda: vortex_workload(n=96), "fp64", {}),       # 18,432 triangles
    ("vortex fp64", lambda: vortex_workload(n=40), "fp64", {}),       # then 3,200
    ("vortex mixed", lambda: vortex_workload(n=96), "mixed", {}),
    ("vortex mixed", lambda: vortex_workload(n=40), "mixed", {}),
    ("riemann limited fp64", lambda: riemann_workload(n=80), "fp64", {"positivity": True}),
    ("riemann limited fp64", lambda: riemann_workload(n=30), "fp64", {"positivity": True}),
    ("burgers fp64", lambda: burgers_workload(n=120), "fp64", {}),
    ("burgers fp64", lambda: burgers_workload(n=50), "fp64", {}),
]


@pytest.mark.parametrize("k", range(0, len(CASES), 2))
def test_noalloc_step_equals_step_on_two_calls_the_second_smaller(k):
    import torch
    from paper_2607_10809_amd.hwe import Mesh
    for name, make, prec, kw in CASES[k:k + 2]:
        wl = make()
        mesh = Mesh.from_workload(wl, precision=prec, **kw)
        dt = 0.25 * mesh.max_dt(mesh.to_device(wl.state0)[0], wl.cfl)
        print(f"{name}: N = {mesh.N}, dt = {dt:.3e}", flush=True)
        (wa, ga), (wb, gb) = _both(mesh, wl.state0, dt)
        assert torch.equal(wa, wb), name
        assert torch.equal(ga, gb), name
        # and after a second step from the new state
        state1 = mesh.to_host(wa, ga)
        (wa, ga), (wb, gb) = _both(mesh, state1, dt)
        assert torch.equal(wa, wb) and torch.equal(ga, gb), name
        mesh.close()


def test_noalloc_refuses_a_mesh_beyond_the_static_scratch():
    """360 x 360 split squares, Euler, FP64: 259,200 cells need 74.6 MB of
    step scratch, more than the 64 MiB array; hwe_step still runs, and a small
    mesh's hwe_step_noalloc works after the refusal."""
    import torch
    from paper_2607_10809_amd import _lib
    from paper_2607_10809_amd.hwe import Mesh
    L = _lib.load_library()
    wl = vortex_workload(n=360)
    mesh = Mesh.from_workload(wl, precision="fp64")
    w, g = mesh.to_device(wl.state0)
    wo, go = mesh.empty_state()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.hwe_step_noalloc(mesh.handle, _p(w), _p(g), _p(wo), _p(go), C.c_double(1e-3), st)
    assert rc == -1, rc
    msg = L.hwe_last_error().decode()
    assert "bytes of step scratch" in msg and str(64 << 20) in msg, msg
    _lib.check(L.hwe_step(mesh.handle, _p(w), _p(g), _p(wo), _p(go), C.c_double(1e-3), st))
    torch.cuda.synchronize()
    mesh.close()
    wl = vortex_workload(n=24)
    small = Mesh.from_workload(wl, precision="fp64")
    (wa, ga), (wb, gb) = _both(small, wl.state0, 1e-3)
    assert torch.equal(wa, wb) and torch.equal(ga, gb)
