"""Helpers shared by the GPU tests: run the HIP path and compare with the oracle."""
from __future__ import annotations

import numpy as np


def rel_max(a, b):
    """Per (block, component) max|a - b| / max|b| over cells; returns the max over all."""
    num = np.abs(a - b).max(axis=-1)
    den = np.abs(b).max(axis=-1)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


def rel_l1(a, b, area):
    """Area-weighted L1 distance relative to the L1 norm of b, max over (block, component)."""
    num = (np.abs(a - b) * area).sum(axis=-1)
    den = (np.abs(b) * area).sum(axis=-1)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


def steps_to(T, dt):
    n = int(np.floor(T / dt + 1e-12))
    rem = T - n * dt
    return n, (rem if rem > 1e-14 * T else 0.0)


def gpu_run(mesh, state0, dt, nsteps, rem=0.0, t0=0.0):
    """Run the HIP path from a caller-order state at time t0; return caller-order numpy state."""
    import torch
    w, g = mesh.to_device(state0)
    w, g = mesh.run(w, g, dt, nsteps, t0=t0)
    if rem > 0.0:
        w, g = mesh.step(w, g, rem, t=t0 + nsteps * dt)
    torch.cuda.synchronize()
    return mesh.to_host(w, g)


def gpu_run_to(mesh, state0, T, dt):
    n, rem = steps_to(T, dt)
    return gpu_run(mesh, state0, dt, n, rem)
