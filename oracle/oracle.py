"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hwe_oracle.cpp")
_LIB = os.path.join(_HERE, "libhwe_oracle.so")

OPTS_DEFAULT = dict(adv=(1.0, 1.0), gas_gamma=1.4, lin_w=(0.94, 0.02, 0.02, 0.02), eps=1e-8,
                    linear_only=0, positivity=0, time_rule=0, deriv_weight=1.0, walls=0,
                    regions=(), states=((0.0,) * 4, (0.0,) * 4), shock=(0.0, 0.0), edge_rule=2)

# boundary kinds of a region
BND_KINDS = {"transmissive": 0, "wall": 1, "A": 2, "B": 3, "moving": 4}


class _Opts(C.Structure):
    _fields_ = [("eq", C.c_int), ("bc", C.c_int), ("box", C.c_double * 4), ("adv", C.c_double * 2),
                ("gas_gamma", C.c_double), ("lin_w", C.c_double * 4), ("eps", C.c_double),
                ("linear_only", C.c_int), ("positivity", C.c_int), ("time_rule", C.c_int),
                ("deriv_weight", C.c_double), ("walls", C.c_int), ("nreg", C.c_int),
                ("reg_kind", C.c_int * 8), ("reg_box", (C.c_double * 4) * 8), ("bstate", (C.c_double * 4) * 2),
                ("shock_x0", C.c_double), ("shock_speed", C.c_double), ("edge_rule", C.c_int)]


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP, -O2, no machine-specific flags: the
    build travels to other hosts)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def use_native_build(dest_dir):
    """Compile the oracle for the host it runs on (g++ -O3 -march=native
    -fopenmp) into dest_dir and load that build; must precede any other use of
    the oracle in the process.  Products are not contracted into fused
    multiply-adds (-ffp-contract=off), so the build computes what the portable
    one does, rounding for rounding.  Returns the compile command."""
    global _LIB
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    lib = os.path.join(dest_dir, "libhwe_oracle_native.so")
    cmd = ["g++", "-O3", "-march=native", "-ffp-contract=off", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o",
           lib, _SRC]
    subprocess.check_call(cmd)
    _LIB = lib
    return " ".join(cmd[:6])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_mesh_new.restype = C.c_void_p
        L.or_mesh_new.argtypes = [dp, C.c_int64, C.POINTER(C.c_int32), C.c_int64, C.POINTER(_Opts),
                                  C.POINTER(C.c_int)]
        L.or_mesh_free.argtypes = [C.c_void_p]
        L.or_mesh_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]
        L.or_geometry.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.or_cell_vertices.argtypes = [C.c_void_p, dp]
        L.or_face_kinds.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.or_step.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int]
        L.or_step_cells.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int64), C.c_int64, dp, C.c_double, C.c_int]
        L.or_run.argtypes = [C.c_void_p, dp, C.c_double, C.c_int64, C.c_int]
        L.or_set_time.argtypes = [C.c_void_p, C.c_double]
        L.or_jvp.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int64, C.c_int]
        L.or_vjp.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int64, C.c_int]
        L.or_count_flops.argtypes = [C.c_void_p, dp, C.c_double, dp]
        L.or_recon_cell.argtypes = [C.c_void_p, dp, C.c_int64, dp, dp, dp, dp]
        L.or_eval_recon.argtypes = [C.c_void_p, dp, C.c_int64, dp, C.c_int64, dp]
        L.or_recon_theta.argtypes = [C.c_void_p, dp, C.c_int64, dp]
        L.or_lax_wendroff.argtypes = [C.POINTER(_Opts), dp, C.c_int64, dp]
        L.or_llf.argtypes = [C.POINTER(_Opts), dp, dp, C.c_double, C.c_double, C.c_double, dp]
        L.or_spectral_radius.restype = C.c_double
        L.or_spectral_radius.argtypes = [C.POINTER(_Opts), dp, C.c_double, C.c_double]
        L.or_max_dt.restype = C.c_double
        L.or_max_dt.argtypes = [C.c_void_p, dp, C.c_double]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _opts(eq, bc=0, box=(0.0, 1.0, 0.0, 1.0), **kw):
    o = dict(OPTS_DEFAULT)
    o.update(kw)
    s = _Opts()
    s.eq = int(eq)
    s.bc = int(bc)
    s.box[:] = [float(v) for v in box]
    s.adv[:] = [float(v) for v in o["adv"]]
    s.gas_gamma = float(o["gas_gamma"])
    s.lin_w[:] = [float(v) for v in o["lin_w"]]
    s.eps = float(o["eps"])
    s.linear_only = int(o["linear_only"])
    s.positivity = int(o["positivity"])
    s.time_rule = int(o["time_rule"])
    s.deriv_weight = float(o["deriv_weight"])
    s.walls = int(o["walls"])
    regs = list(o["regions"])
    if len(regs) > 8:
        raise ValueError("at most 8 boundary regions")
    s.nreg = len(regs)
    for r, (kind, rect) in enumerate(regs):
        s.reg_kind[r] = BND_KINDS[kind]
        s.reg_box[r][:] = [float(v) for v in rect]
    for a in range(2):
        st = list(o["states"][a]) + [0.0] * (4 - len(o["states"][a]))
        s.bstate[a][:] = [float(v) for v in st]
    s.shock_x0, s.shock_speed = float(o["shock"][0]), float(o["shock"][1])
    s.edge_rule = int(o["edge_rule"])
    return s


def _m(eq):
    return 4 if eq == 2 else 1


class OracleMesh:
    """Oracle view of a triangular mesh plus the scheme options."""

    def __init__(self, nodes, tris, eq, bc=0, box=(0.0, 1.0, 0.0, 1.0), **kw):
        L = _load()
        self.eq = eq
        self.m = _m(eq)
        self._o = _opts(eq, bc, box, **kw)
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        st = C.c_int(0)
        h = L.or_mesh_new(_p(nodes), nodes.shape[0], tris.ctypes.data_as(C.POINTER(C.c_int32)),
                          tris.shape[0], C.byref(self._o), C.byref(st))
        if not h:
            raise ValueError(f"oracle: mesh rejected (status {st.value})")
        self._h = C.c_void_p(h)
        N, E, m = C.c_int64(), C.c_int64(), C.c_int32()
        L.or_mesh_sizes(self._h, C.byref(N), C.byref(E), C.byref(m))
        self.N, self.E = N.value, E.value

    @classmethod
    def from_workload(cls, wl, **kw):
        if getattr(wl, "walls", 0) and "walls" not in kw:
            kw["walls"] = wl.walls
        for key in ("regions", "states", "shock"):
            if getattr(wl, key, None) and key not in kw:
                kw[key] = getattr(wl, key)
        return cls(wl.mesh.nodes, wl.mesh.tris, wl.eq, wl.bc, wl.mesh.box, adv=wl.adv, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_mesh_free(h)
            self._h = None

    # ------------------------------------------------------------- queries
    def geometry(self):
        N = self.N
        area, cx, cy = np.empty(N), np.empty(N), np.empty(N)
        faces = np.empty((N, 3, 6))
        _lib.or_geometry(self._h, _p(area), _p(cx), _p(cy), _p(faces))
        return dict(area=area, cx=cx, cy=cy, normal=faces[..., 0:2], length=faces[..., 2],
                    nbr=faces[..., 3].astype(np.int64), shift=faces[..., 4:6])

    def face_kinds(self):
        """(N, 3) int32: boundary kind of each face (BND_KINDS values), -1 inside."""
        out = np.empty((self.N, 3), dtype=np.int32)
        _lib.or_face_kinds(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def cell_vertices(self):
        out = np.empty((self.N, 3, 2))
        _lib.or_cell_vertices(self._h, _p(out))
        return out

    def _check_state(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64)
        if s.shape != (3, self.m, self.N):
            raise ValueError(f"state must be (3, {self.m}, {self.N}), got {s.shape}")
        return s

    # ------------------------------------------------------------- the step
    def step(self, s, dt, nthreads=0, t=0.0):
        """One step from the state s at time t (t matters for moving boundary states only)."""
        s = self._check_state(s)
        out = np.empty_like(s)
        _lib.or_set_time(self._h, float(t))
        st = _lib.or_step(self._h, _p(s), _p(out), float(dt), int(nthreads))
        if st:
            raise RuntimeError(f"oracle step failed ({st})")
        return out

    def step_cells(self, s, cells, dt, nthreads=0, t=0.0):
        s = self._check_state(s)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((3, self.m, cells.size))
        _lib.or_set_time(self._h, float(t))
        st = _lib.or_step_cells(self._h, _p(s), cells.ctypes.data_as(C.POINTER(C.c_int64)), cells.size,
                                _p(out), float(dt), int(nthreads))
        if st:
            raise RuntimeError(f"oracle step_cells failed ({st})")
        return out

    def run(self, s, dt, nsteps, nthreads=0, t=0.0):
        """nsteps steps of size dt from the state s at time t."""
        s = self._check_state(s).copy()
        _lib.or_set_time(self._h, float(t))
        st = _lib.or_run(self._h, _p(s), float(dt), int(nsteps), int(nthreads))
        if st:
            raise RuntimeError(f"oracle run failed ({st})")
        return s

    def run_to(self, s, T, dt, nthreads=0):
        """Steps of size dt from t = 0 with the last one clipped so that the run ends at T."""
        n = int(np.floor(T / dt + 1e-12))
        s = self.run(s, dt, n, nthreads)
        rem = T - n * dt
        if rem > 1e-14 * T:
            s = self.step(s, rem, nthreads, t=n * dt)
        return s

    def jvp(self, s, ds, dt, nsteps, nthreads=0, t=0.0):
        s = self._check_state(s).copy()
        ds = self._check_state(ds).copy()
        _lib.or_set_time(self._h, float(t))
        st = _lib.or_jvp(self._h, _p(s), _p(ds), float(dt), int(nsteps), int(nthreads))
        if st:
            raise RuntimeError(f"oracle jvp failed ({st})")
        return s, ds

    def vjp(self, s, lam, dt, nsteps, nthreads=0, t=0.0):
        """Reverse mode: J^T lam for nsteps steps of size dt from the state s
        at time t (lam: the adjoint of the final state)."""
        s = self._check_state(s).copy()
        lam = self._check_state(lam).copy()
        _lib.or_set_time(self._h, float(t))
        st = _lib.or_vjp(self._h, _p(s), _p(lam), float(dt), int(nsteps), int(nthreads))
        if st:
            raise RuntimeError(f"oracle vjp failed ({st})")
        return lam

    COUNT_STAGES = ("recon", "limiter", "alpha", "eval", "lax_wendroff", "flux", "update")

    def count_flops(self, s, dt, t=0.0):
        """Floating-point operations of one step by stage (see or_count_flops):
        the live +, -, *, / and square roots (those a result of the step
        depends on through arithmetic; values that only decide a branch, such
        as the losing spectral radius of the flux viscosity, are not counted).
        Each interior edge's flux work is counted from both of its cells."""
        s = self._check_state(s)
        out = np.zeros(len(self.COUNT_STAGES))
        _lib.or_set_time(self._h, float(t))
        if _lib.or_count_flops(self._h, _p(s), float(dt), _p(out)):
            raise RuntimeError("oracle count failed")
        return dict(zip(self.COUNT_STAGES, out))

    def recon_cell(self, s, k):
        s = self._check_state(s)
        m = self.m
        p = np.empty((4, m, 6))
        beta = np.empty((m, 4))
        omega = np.empty((m, 4))
        cen = np.empty(2)
        st = _lib.or_recon_cell(self._h, _p(s), int(k), _p(p), _p(beta), _p(omega), _p(cen))
        if st:
            raise RuntimeError("oracle recon failed")
        return dict(p=p, beta=beta, omega=omega, centroid=cen)

    def recon_theta(self, s, k):
        s = self._check_state(s)
        th = np.empty(self.m)
        if _lib.or_recon_theta(self._h, _p(s), int(k), _p(th)):
            raise RuntimeError("oracle recon failed")
        return th

    def eval_recon(self, s, k, xy):
        s = self._check_state(s)
        xy = np.ascontiguousarray(np.atleast_2d(xy), dtype=np.float64)
        out = np.empty((xy.shape[0], self.m, 6))
        st = _lib.or_eval_recon(self._h, _p(s), int(k), _p(xy), xy.shape[0], _p(out))
        if st:
            raise RuntimeError("oracle eval_recon failed")
        return out

    def max_dt(self, s, cfl):
        s = self._check_state(s)
        return float(_lib.or_max_dt(self._h, _p(s), float(cfl)))


def lax_wendroff(eq, D, **kw):
    """D: (np, 6, m) = W, Wx, Wy, Wxx, Wxy, Wyy -> (np, 4, m) = Wt, Wtx, Wty, Wtt."""
    L = _load()
    o = _opts(eq, **kw)
    D = np.ascontiguousarray(D, dtype=np.float64)
    out = np.empty((D.shape[0], 4, D.shape[2]))
    L.or_lax_wendroff(C.byref(o), _p(D), D.shape[0], _p(out))
    return out


def llf_flux(eq, Wi, We, n, alpha, **kw):
    L = _load()
    o = _opts(eq, **kw)
    Wi = np.ascontiguousarray(Wi, dtype=np.float64)
    We = np.ascontiguousarray(We, dtype=np.float64)
    out = np.empty(_m(eq))
    L.or_llf(C.byref(o), _p(Wi), _p(We), float(n[0]), float(n[1]), float(alpha), _p(out))
    return out


def spectral_radius(eq, W, n, **kw):
    L = _load()
    o = _opts(eq, **kw)
    W = np.ascontiguousarray(W, dtype=np.float64)
    return float(L.or_spectral_radius(C.byref(o), _p(W), float(n[0]), float(n[1])))
