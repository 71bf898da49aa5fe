"""Python binding of the hwe C ABI with torch tensors for device memory and streams.

Functions with the C names (``hwe_mesh_init``, ``hwe_step``, ``hwe_step_adjoint``)
forward their arguments to the library unchanged; :class:`Mesh` adds buffer
management and the caller <-> internal (Morton) cell order maps.  Every step of
the method runs in the HIP library; nothing here computes any part of it.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import BCS, BND_KINDS, EQUATIONS, MAX_REGIONS, PRECISIONS, HweOpts, check, load_library


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_opts(eq="euler", bc="periodic", box=(0.0, 1.0, 0.0, 1.0), precision="fp64", adv=(1.0, 1.0),
              gas_gamma=1.4, lin_w=(0.94, 0.02, 0.02, 0.02), eps=1e-8, linear_weights=False, device=0,
              positivity=False, time_rule=0, deriv_weight=1.0, walls=0, regions=(), states=(), shock=(),
              edge_rule=2) -> HweOpts:
    """Options of a mesh handle.  regions: boundary regions, first match wins,
    as (kind, (x0, x1, y0, y1)) with kind "transmissive", "wall", "A", "B" or
    "moving"; states: the conservative states (A, B); shock: (x0, speed) of the
    moving switch."""
    L = load_library()
    o = HweOpts()
    check(L.hwe_opts_default(C.byref(o)))
    o.eq = EQUATIONS[eq] if isinstance(eq, str) else int(eq)
    o.bc = BCS[bc] if isinstance(bc, str) else int(bc)
    o.prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.linear_weights = 1 if linear_weights else 0
    o.box[:] = [float(v) for v in box]
    o.adv[:] = [float(v) for v in adv]
    o.gas_gamma = float(gas_gamma)
    o.lin_w[:] = [float(v) for v in lin_w]
    o.eps = float(eps)
    o.device = int(device)
    o.positivity = 1 if positivity else 0
    o.time_rule = int(time_rule)
    o.deriv_weight = float(deriv_weight)
    o.walls = int(walls)
    regions = list(regions)
    if len(regions) > MAX_REGIONS:
        raise ValueError(f"at most {MAX_REGIONS} boundary regions")
    o.n_regions = len(regions)
    for r, (kind, rect) in enumerate(regions):
        o.regions[r].kind = BND_KINDS[kind] if isinstance(kind, str) else int(kind)
        o.regions[r].box[:] = [float(v) for v in rect]
    for a, st in enumerate(list(states)[:2]):
        st = [float(v) for v in st]
        o.bstate[a][:len(st)] = st
    if shock:
        o.shock_x0, o.shock_speed = float(shock[0]), float(shock[1])
    o.edge_rule = int(edge_rule)
    return o


def hwe_mesh_init(nodes, tris, opts: HweOpts) -> C.c_void_p:
    L = load_library()
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    h = C.c_void_p()
    check(L.hwe_mesh_init(nodes.ctypes.data_as(C.POINTER(C.c_double)), nodes.shape[0],
                          tris.ctypes.data_as(C.POINTER(C.c_int32)), tris.shape[0], C.byref(opts), C.byref(h)))
    return h


def hwe_step(handle, wbar_in, grad_in, wbar_out, grad_out, dt, stream=None):
    check(load_library().hwe_step(handle, _ptr(wbar_in), _ptr(grad_in), _ptr(wbar_out), _ptr(grad_out),
                                  float(dt), _stream(stream)))


def hwe_step_noalloc(handle, wbar_in, grad_in, wbar_out, grad_out, dt, stream=None):
    check(load_library().hwe_step_noalloc(handle, _ptr(wbar_in), _ptr(grad_in), _ptr(wbar_out), _ptr(grad_out),
                                          float(dt), _stream(stream)))


def hwe_step_adjoint(handle, wbar_n, grad_n, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt, stream=None):
    check(load_library().hwe_step_adjoint(handle, _ptr(wbar_n), _ptr(grad_n), _ptr(lam_wbar_np1),
                                          _ptr(lam_grad_np1), _ptr(lam_wbar_n), _ptr(lam_grad_n), float(dt),
                                          _stream(stream)))


def hwe_step_keep(handle, wbar_in, grad_in, wbar_out, grad_out, dt, recon_out, stream=None):
    check(load_library().hwe_step_keep(handle, _ptr(wbar_in), _ptr(grad_in), _ptr(wbar_out), _ptr(grad_out),
                                       float(dt), _ptr(recon_out), _stream(stream)))


def hwe_step_adjoint_kept(handle, wbar_n, grad_n, recon_n, lam_wbar_np1, lam_grad_np1, lam_wbar_n, lam_grad_n, dt,
                          stream=None):
    check(load_library().hwe_step_adjoint_kept(handle, _ptr(wbar_n), _ptr(grad_n), _ptr(recon_n),
                                               _ptr(lam_wbar_np1), _ptr(lam_grad_np1), _ptr(lam_wbar_n),
                                               _ptr(lam_grad_n), float(dt), _stream(stream)))


class Mesh:
    """A triangular mesh on one GPU with the scheme's options.

    State tensors (internal cell order): ``wbar`` float64 (m, N) and ``grad``
    (2, m, N) of float64 (``precision='fp64'``) or float32 (``'mixed'``).
    """

    def __init__(self, nodes, tris, eq="euler", bc="periodic", box=(0.0, 1.0, 0.0, 1.0), precision="fp64",
                 device=0, **kw):
        self.opts = make_opts(eq, bc, box, precision, device=device, **kw)
        self.precision = precision
        self._L = load_library()
        self._h = hwe_mesh_init(nodes, tris, self.opts)
        N, E, m = C.c_int64(), C.c_int64(), C.c_int32()
        check(self._L.hwe_mesh_info(self._h, C.byref(N), C.byref(E), C.byref(m)))
        self.N, self.E, self.m = N.value, E.value, m.value
        perm = np.empty(self.N, dtype=np.int64)
        check(self._L.hwe_mesh_cell_perm(self._h, perm.ctypes.data_as(C.POINTER(C.c_int64))))
        self.perm = perm                       # internal i -> caller perm[i]
        self.device = torch.device("cuda", device) if device >= 0 else None
        self.gdtype = torch.float64 if precision == "fp64" else torch.float32

    @classmethod
    def from_workload(cls, wl, precision="fp64", device=0, **kw):
        bc = "periodic" if wl.mesh.periodic else "transmissive"
        eq = {0: "advection", 1: "burgers", 2: "euler"}[wl.eq]
        if getattr(wl, "walls", 0) and "walls" not in kw:
            kw["walls"] = wl.walls
        for key in ("regions", "states", "shock"):
            if getattr(wl, key, None) and key not in kw:
                kw[key] = getattr(wl, key)
        return cls(wl.mesh.nodes, wl.mesh.tris, eq=eq, bc=bc, box=wl.mesh.box, precision=precision,
                   device=device, adv=wl.adv, **kw)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.hwe_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ state maps
    def to_device(self, state):
        """Caller-order numpy state [3][m][N] -> (wbar, grad) tensors in internal order."""
        s = np.asarray(state, dtype=np.float64)[:, :, self.perm]
        wbar = torch.from_numpy(np.ascontiguousarray(s[0])).to(self.device)
        grad = torch.from_numpy(np.ascontiguousarray(s[1:])).to(self.device, dtype=self.gdtype)
        return wbar, grad

    def to_host(self, wbar, grad):
        """(wbar, grad) tensors in internal order -> caller-order numpy [3][m][N] float64."""
        out = np.empty((3, self.m, self.N))
        out[0][:, self.perm] = wbar.detach().double().cpu().numpy()
        out[1:][:, :, self.perm] = grad.detach().double().cpu().numpy()
        return out

    def empty_state(self):
        return (torch.empty((self.m, self.N), dtype=torch.float64, device=self.device),
                torch.empty((2, self.m, self.N), dtype=self.gdtype, device=self.device))

    def _check_state(self, wbar, grad):
        if wbar.dtype != torch.float64 or wbar.shape != (self.m, self.N) or not wbar.is_contiguous():
            raise ValueError("wbar must be a contiguous float64 tensor of shape (m, N)")
        if grad.dtype != self.gdtype or grad.shape != (2, self.m, self.N) or not grad.is_contiguous():
            raise ValueError(f"grad must be a contiguous {self.gdtype} tensor of shape (2, m, N)")
        if wbar.device != self.device or grad.device != self.device:
            raise ValueError("state tensors must live on the mesh's device")

    # ------------------------------------------------------------ the step
    def set_time(self, t):
        """Time of the state given to the next steps (moving boundary states)."""
        check(self._L.hwe_set_time(self._h, float(t)))

    def step(self, wbar, grad, dt, out=None, stream=None, keep=None, t=None):
        """One step (from time t, if given).  keep: a buffer from empty_recon()
        that receives the step's reconstruction (for a later
        adjoint(..., recon=keep))."""
        if t is not None:
            self.set_time(t)
        self._check_state(wbar, grad)
        wo, go = out if out is not None else self.empty_state()
        self._check_state(wo, go)
        if keep is None:
            hwe_step(self._h, wbar, grad, wo, go, dt, stream)
        else:
            self._check_recon(keep)
            hwe_step_keep(self._h, wbar, grad, wo, go, dt, keep, stream)
        return wo, go

    def empty_recon(self):
        """Buffer for one step's reconstruction: the library's cell-major
        [N][6][m] record of the coefficients a0..a5 (gdtype)."""
        return torch.empty((self.N, 6, self.m), dtype=self.gdtype, device=self.device)

    def _check_recon(self, R):
        if R.dtype != self.gdtype or R.shape != (self.N, 6, self.m) or not R.is_contiguous():
            raise ValueError(f"recon must be a contiguous {self.gdtype} tensor of shape (N, 6, m)")
        if R.device != self.device:
            raise ValueError("recon must live on the mesh's device")

    def run(self, wbar, grad, dt, nsteps, stream=None, t0=None):
        """nsteps steps of size dt with two ping-pong buffers (from time t0,
        if given); returns the final state."""
        a = (wbar, grad)
        if nsteps <= 0:
            return a
        b = self.empty_state()
        c = self.empty_state() if nsteps > 1 else None
        for k in range(nsteps):
            if t0 is not None:
                self.set_time(t0 + k * dt)
            dst = b if k % 2 == 0 else c
            hwe_step(self._h, a[0], a[1], dst[0], dst[1], dt, stream)
            a = dst
        return a

    def run_to(self, wbar, grad, T, cfl, every=50, stream=None):
        """Advance to time T with dt = cfl * min inradius / max signal speed,
        recomputed on the device from the current state every ``every`` steps
        (the last step is clipped to end at T).  Returns (wbar, grad, steps)."""
        bufs = [(wbar, grad), self.empty_state(), self.empty_state()]
        cur, t, steps = 0, 0.0, 0
        while T - t > 1e-14 * T:
            dt = self.max_dt(bufs[cur][0], cfl, stream)
            for _ in range(every):
                h = min(dt, T - t)
                if h <= 1e-14 * T:
                    break
                nxt = 1 if cur != 1 else 2
                self.set_time(t)
                hwe_step(self._h, bufs[cur][0], bufs[cur][1], bufs[nxt][0], bufs[nxt][1], h, stream)
                cur = nxt
                t += h
                steps += 1
        return bufs[cur][0], bufs[cur][1], steps

    def capture_steps(self, a, b, dt, nsteps):
        """Record nsteps (even) steps of size dt that ping-pong between the
        state buffers a and b (a -> b -> a ...) into a HIP graph; replaying it
        advances the state held in a by nsteps steps.  The launches are
        recorded once, so the mesh must not depend on the time (no moving
        boundary switch)."""
        if nsteps <= 0 or nsteps % 2:
            raise ValueError("nsteps must be positive and even")
        if any(self.opts.regions[r].kind == BND_KINDS["moving"] for r in range(self.opts.n_regions)):
            raise ValueError("a captured step cannot follow a moving boundary switch")
        self._check_state(*a)
        self._check_state(*b)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for k in range(nsteps):
                    src, dst = (a, b) if k % 2 == 0 else (b, a)
                    hwe_step(self._h, src[0], src[1], dst[0], dst[1], dt, s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        return g

    def adjoint(self, wbar, grad, lam_wbar, lam_grad, dt, out=None, stream=None, recon=None, t=None):
        """J^T lam at the state (wbar, grad) (of the step from time t, if
        given).  recon: the buffer that step(wbar, grad, ..., keep=recon)
        filled; skips the reconstruction."""
        if t is not None:
            self.set_time(t)
        self._check_state(wbar, grad)
        self._check_state(lam_wbar, lam_grad)
        lw, lg = out if out is not None else self.empty_state()
        if recon is None:
            hwe_step_adjoint(self._h, wbar, grad, lam_wbar, lam_grad, lw, lg, dt, stream)
        else:
            self._check_recon(recon)
            hwe_step_adjoint_kept(self._h, wbar, grad, recon, lam_wbar, lam_grad, lw, lg, dt, stream)
        return lw, lg

    def max_dt(self, wbar, cfl, stream=None):
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        check(self._L.hwe_max_dt(self._h, _ptr(wbar), float(cfl), _ptr(out), _stream(stream)))
        return float(out.item())

    def check_state(self, wbar, stream=None):
        out = torch.empty(1, dtype=torch.int32, device=self.device)
        check(self._L.hwe_check_state(self._h, _ptr(wbar), _ptr(out), _stream(stream)))
        return int(out.item())

    def debug_recon(self, wbar, grad, stream=None):
        """R - Wbar coefficients a0..a5 per cell and component, as a (6, m, N) view
        of the library's cell-major [N][6][m] record."""
        R = torch.empty((self.N, 6, self.m), dtype=self.gdtype, device=self.device)
        check(self._L.hwe_debug_recon(self._h, _ptr(wbar), _ptr(grad), _ptr(R), _stream(stream)))
        return R.permute(1, 2, 0)

    def debug_edge(self, recon, wbar, dt, stream=None):
        """The edge stage alone from a reconstruction (the (N, 6, m) record of
        empty_recon / step(..., keep=)): (F, G), each (E, m) in the library's
        edge order; F float64, G of the mesh's real type."""
        self._check_recon(recon)
        F = torch.empty((self.E, self.m), dtype=torch.float64, device=self.device)
        G = torch.empty((self.E, self.m), dtype=self.gdtype, device=self.device)
        check(self._L.hwe_debug_edge(self._h, _ptr(recon), _ptr(wbar), float(dt), _ptr(F), _ptr(G),
                                     _stream(stream)))
        return F, G

    def profile_begin(self, n_steps):
        check(self._L.hwe_profile_begin(self._h, int(n_steps)))

    def profile_end(self):
        """Summed per-kernel milliseconds (recon, edge, update) and the step count."""
        ms = (C.c_double * 3)()
        n = C.c_int32()
        check(self._L.hwe_profile_end(self._h, ms, C.byref(n)))
        return [ms[0], ms[1], ms[2]], n.value

    def host_array(self, which):
        sizes = {0: (55, self.N), 1: (2, self.N), 2: (self.N,), 3: (3, self.N), 4: (3, self.N), 5: (3, self.N), 6: (41, self.N), 7: (3, self.N),
                 8: (2, self.E)}
        out = np.empty(sizes[which])
        check(self._L.hwe_debug_host_array(self._h, int(which), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out
