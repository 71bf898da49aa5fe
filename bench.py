"""Benchmark of the explicit ADER-HWENO step on one MI355X.

Workload: 2-D Euler (gamma = 1.4) isentropic vortex of strength 5 on the
periodic square [0,10]^2, 320 x 320 split squares with +-0.1h seeded node
jitter (204,800 triangles).  A step is one call of hwe_step (reconstruction,
edge and update kernels) on state already resident in HBM.

Prints one JSON line: cell-steps/s of the FP64 step (``value``), the mixed
(FP32 bulk) step and its speedup, the adjoint/forward time ratio, the roofline
of the dominant kernel measured live with HIP events, and the CPU oracle timed
on the host cores on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic bytes of one Euler cell-step in FP64 (mixed): the state read and
# written once, the reconstruction tables, geometry and connectivity once, 1.5
# edge records per cell (73 table entries per cell; the factored tables of
# this library hold 53).
ALG_BYTES_PER_CELL_STEP = {"fp64": 976, "mixed": 542}
# Algorithmic FP64 operations of the Euler edge stage per edge: the oracle's
# live operation count (the arithmetic a result of the step depends on) of the
# flux viscosity (15), the Lax-Wendroff procedure (3,232) and the Taylor
# values, normal fluxes and quadratures (757) for the edge's two sides and two
# Gauss points, evaluated once; the evaluation of the reconstruction at the
# points is left out (the oracle evaluates the four candidates, the edge kernel
# the combined polynomial).  The CPU leg recounts it with the oracle
# (cpu_baseline.oracle_flops) and tests/test_oracle_reverse.py checks this
# constant against the oracle.
EDGE_ALG_FLOP_PER_EDGE = 4004
# Algorithmic FP64 operations of one whole Euler cell-step by the same count
# (reconstruction 1,483 per cell, the four edge stages 5,412 per edge, 1.5
# edges per cell, update 16 per cell).
ALG_FLOP_PER_CELL_STEP = 9617
# FP64 flops the Euler edge kernel executes per edge (two sides x two Gauss
# points: evaluation of R, Lax-Wendroff jets, three offset fluxes, side terms,
# LLF combination), from the SQ_INSTS_VALU_FLOPS_FP64 counter x 64 lanes / E on
# the 204,800-triangle mesh; the arithmetic has no data-dependent paths on
# interior edges.
EDGE_FP64_FLOP_PER_EDGE = 3493
# timed repeats of the K steps; the value is their median
REPEATS = 5
CSRC = os.path.join(ROOT, "paper_2607_10809_amd", "csrc")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_euler_vortex_204800.md")


def source_digest():
    """sha256 (first 16 hex digits) over the kernel sources, sorted by name."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` (e.g. 'recon_kernel<2, double>') from the
    committed counter summary, or None when the kernel sources have changed since
    the counters were taken (the summary records the source digest)."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"source digest: `([0-9a-f]+)`", text)
    if not m or m.group(1) != source_digest():
        return None
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) > 5 and cells[1] == kernel:
            try:
                return int(cells[5])
            except ValueError:
                return None
    return None


def measured_valu_busy(kernel):
    """Fraction of VALU issue slots busy for ``kernel`` from the committed counter
    summary (SQ_INSTS_VALU x 4 cycles over the kernel's duration), or None when
    the kernel sources have changed since the counters were taken."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"source digest: `([0-9a-f]+)`", text)
    if not m or m.group(1) != source_digest():
        return None
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) > 8 and cells[1] == kernel and cells[8].endswith("%"):
            return round(float(cells[8][:-1]) / 100.0, 2)
    return None


def copy_bandwidth(nbytes=1 << 30, reps=20):
    """Device-to-device copy rate (bytes read + written per second) of a 1 GiB buffer."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def kernel_bytes(N, E, m, s, positivity=False):
    """Algorithmic bytes per launch of the three kernels (each array once).

    s = bytes of the bulk real type (8 FP64, 4 mixed).  Counts the per-cell and
    per-edge arrays each kernel must read or write at least once (with the
    positivity limiter, recon also reads the six edge Gauss points per cell).
    """
    recon = N * (m * 8 + 2 * m * s + 12 + 41 * s + 9 * s + 8 + 3 * s + 6 * m * s + (96 if positivity else 0))
    edge = E * (8 + 24 + 8 * s + m * 8 + m * s) + N * (6 * m * s + m * 8)
    update = N * (m * 8 + 12 + 12 + 6 * s + 8 + m * 8 + 2 * m * s) + E * (m * 8 + m * s)
    return {"recon": recon, "edge": edge, "update": update}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_leg(wl, steps, warmup, precision):
    import torch
    from paper_2607_10809_amd.hwe import Mesh
    mesh = Mesh.from_workload(wl, precision=precision)
    w0, g0 = mesh.to_device(wl.state0)
    dt = mesh.max_dt(w0, wl.cfl)
    bufs = [(w0.clone(), g0.clone()), mesh.empty_state()]
    stream = torch.cuda.current_stream()

    def run(k, start=0):
        for i in range(k):
            a, b = bufs[(start + i) % 2], bufs[(start + i + 1) % 2]
            mesh.step(a[0], a[1], dt, out=b)
        return start + k

    pos = run(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # eager: one Python call per step
    ev0.record(stream)
    pos = run(steps, pos)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_eager = ev0.elapsed_time(ev1)
    # the timed region: the same steps recorded once into a HIP graph of
    # `chunk` steps and replayed (no host work between the kernels)
    chunk = 100 if steps % 100 == 0 else (steps if steps % 2 == 0 else 0)
    reps = []
    if chunk:
        a = bufs[pos % 2]
        b = bufs[(pos + 1) % 2]
        graph = mesh.capture_steps(a, b, dt, chunk)
        graph.replay()                      # warm replay
        torch.cuda.synchronize()
        for _ in range(REPEATS):
            t_wall0 = time.perf_counter()
            ev0.record(stream)
            for _ in range(steps // chunk):
                graph.replay()
            ev1.record(stream)
            torch.cuda.synchronize()
            reps.append((ev0.elapsed_time(ev1), time.perf_counter() - t_wall0))
        del graph
    else:
        for _ in range(REPEATS):
            t_wall0 = time.perf_counter()
            ev0.record(stream)
            pos = run(steps, pos)
            ev1.record(stream)
            torch.cuda.synchronize()
            reps.append((ev0.elapsed_time(ev1), time.perf_counter() - t_wall0))
    reps.sort()
    ms, t_wall = reps[len(reps) // 2]
    rep_ms = [r[0] for r in reps]
    flags = mesh.check_state(bufs[pos % 2][0])
    # per-kernel durations with events around each kernel (separate profiled loop)
    nprof = min(steps, 2000)
    mesh.profile_begin(nprof)
    pos = run(nprof, pos)
    kms, nk = mesh.profile_end()
    torch.cuda.synchronize()
    return dict(mesh=mesh, dt=dt, ms=ms, ms_eager=ms_eager, graph_chunk=chunk, wall=t_wall, flags=flags,
                kernel_ms=[k / nk for k in kms], rep_ms=rep_ms)


def adjoint_leg(wl, nsteps=200, ckpt=20, precision="fp64"):
    """C5: misfit gradient through a checkpointed rollout; backward/forward time."""
    import torch
    from paper_2607_10809_amd.autograd import rollout
    from paper_2607_10809_amd.hwe import Mesh
    from workloads import cell_average_states, make_vortex, perturbed_vortex_target_center
    mesh = Mesh.from_workload(wl, precision=precision)
    w0, g0 = mesh.to_device(wl.state0)
    dt = mesh.max_dt(w0, wl.cfl)
    tw, tg = mesh.to_device(cell_average_states(wl.mesh, make_vortex(center=perturbed_vortex_target_center())))
    tgt = mesh.run(tw, tg, dt, nsteps)[0][0].clone()
    stream = torch.cuda.current_stream()

    def once():
        w = w0.clone().requires_grad_(True)
        g = g0.clone().requires_grad_(True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        e[0].record(stream)
        wT, gT = rollout(mesh, w, g, dt, nsteps, ckpt)
        e[1].record(stream)
        loss = 0.5 * ((wT[0] - tgt) ** 2).sum()
        loss.backward()
        e[2].record(stream)
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])

    once()
    runs = sorted((once() for _ in range(3)), key=lambda fb: fb[1] / fb[0])
    f, b = runs[1]                          # the run with the median ratio
    # the gradient itself (density slice, caller order), for the mixed-vs-FP64 error
    w = w0.clone().requires_grad_(True)
    g = g0.clone().requires_grad_(True)
    wT, gT = rollout(mesh, w, g, dt, nsteps, ckpt)
    (0.5 * ((wT[0] - tgt) ** 2).sum()).backward()
    torch.cuda.synchronize()
    grad_rho = mesh.to_host(w.grad, g.grad.double())[0, 0]
    # per-step kernel time: adjoint step vs forward step on the same state
    la, lg = mesh.empty_state()
    la.normal_()
    lg.normal_()
    out = mesh.empty_state()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    for _ in range(100):
        mesh.step(w0, g0, dt, out=out)
    ev[1].record(stream)
    for _ in range(100):
        mesh.adjoint(w0, g0, la, lg, dt, out=out)
    ev[2].record(stream)
    torch.cuda.synchronize()
    fs, as_ = ev[0].elapsed_time(ev[1]) / 100, ev[1].elapsed_time(ev[2]) / 100
    return {"forward_ms": f, "backward_ms": b, "ratio": b / f, "runs": 3, "steps": nsteps, "ckpt": ckpt,
            "step_us": fs * 1e3, "adjoint_step_us": as_ * 1e3, "per_step_ratio": as_ / fs, "_grad": grad_rho}


def mixed_error_leg(wl):
    """Error of the mixed path against the FP64 path: both run the vortex to its
    final time T with the same fixed step (the FP64 mesh's CFL step, last step
    clipped); relative max norms per (block, component) of the cell averages
    and of the derivative averages."""
    import torch
    from paper_2607_10809_amd.hwe import Mesh
    res, dt = {}, None
    for prec in ("fp64", "mixed"):
        mesh = Mesh.from_workload(wl, precision=prec)
        w, g = mesh.to_device(wl.state0)
        if dt is None:
            dt = mesh.max_dt(w, wl.cfl)
        n = int(np.floor(wl.T / dt + 1e-12))
        rem = wl.T - n * dt
        w, g = mesh.run(w, g, dt, n)
        if rem > 1e-14 * wl.T:
            w, g = mesh.step(w, g, rem, t=n * dt)
        torch.cuda.synchronize()
        res[prec] = mesh.to_host(w, g)
        del mesh
    a, b = res["mixed"], res["fp64"]

    def rel(x, y):
        den = np.abs(y).max(axis=-1)
        return float((np.abs(x - y).max(axis=-1) / np.where(den == 0, 1.0, den)).max())

    return {"T": wl.T, "steps": n + (1 if rem > 1e-14 * wl.T else 0), "dt": dt,
            "wbar_rel_max": rel(a[:1], b[:1]), "grad_rel_max": rel(a[1:], b[1:]), "bound_wbar": 2e-5}


def cpu_model():
    """The host CPU as lscpu describes it (model, sockets, cores, threads,
    clock), else /proc/cpuinfo's model name."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                     "CPU max MHz", "L3 cache"):
                info[k] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "Model name" not in info:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    info["Model name"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info or None


def cpu_leg(wl, budget_s=12.0, budget_1t_s=5.0):
    """The oracle on the host cores (all of OMP_NUM_THREADS, then one thread),
    compiled for this host (g++ -O3 -march=native -ffp-contract=off -fopenmp) into a temporary
    directory; and the oracle's live operation count of one step."""
    import tempfile
    from oracle import oracle as orc
    build = orc.use_native_build(tempfile.mkdtemp(prefix="hwe_oracle_"))
    from oracle import OracleMesh
    from workloads import vortex_workload
    small = vortex_workload(n=16)
    oc = OracleMesh.from_workload(small)
    c = oc.count_flops(small.state0, oc.max_dt(small.state0, small.cfl))
    per_edge = {k: c[k] / (2 * oc.E) for k in ("alpha", "eval", "lax_wendroff", "flux")}
    flops = {"per_cell": {"recon": c["recon"] / oc.N, "update": c["update"] / oc.N},
             "per_edge": {k: round(v, 2) for k, v in per_edge.items()},
             "edge_stage_per_edge": round(per_edge["alpha"] + per_edge["lax_wendroff"] + per_edge["flux"], 1),
             "per_cell_step": round((c["recon"] + c["update"]) / oc.N + sum(per_edge.values()) * oc.E / oc.N, 1),
             "mesh": f"vortex, 16x16 split squares ({oc.N} triangles), one step"}
    del oc
    om = OracleMesh.from_workload(wl)
    dt = om.max_dt(wl.state0, wl.cfl)

    def timed(budget, nthreads):
        s = om.step(wl.state0, dt, nthreads)      # warm-up
        t0 = time.perf_counter()
        n = 0
        while n == 0 or time.perf_counter() - t0 < budget:
            s = om.step(s, dt, nthreads)
            n += 1
        return n, time.perf_counter() - t0

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n, el = timed(budget_s, cores)
    n1, el1 = timed(budget_1t_s, 1)
    return dict(value=om.N * n / el, unit="cell-steps/s", cores=cores, kind="oracle",
                sample=f"{n} full FP64 steps of the 204,800-triangle vortex mesh after one warm-up step "
                       f"({el:.1f} s wall)",
                one_thread={"value": om.N * n1 / el1, "steps": n1, "seconds": round(el1, 2)},
                build=build, cpu_model=cpu_model(), oracle_flops=flops)


def small_configs_leg(steps=500, warmup=20):
    """Throughput of the two small configurations: linear advection on 800
    triangles (C1; launch-bound) and Burgers on 51,200 jittered triangles (C2),
    each precision, as HIP-graph replays of the step."""
    import torch
    from paper_2607_10809_amd.hwe import Mesh
    from workloads import advection_workload, burgers_workload
    out = {}
    for name, wl in (("advection_800", advection_workload()), ("burgers_51200", burgers_workload())):
        res = {"triangles": wl.mesh.n_cells}
        for prec in ("fp64", "mixed"):
            mesh = Mesh.from_workload(wl, precision=prec)
            w0, g0 = mesh.to_device(wl.state0)
            dt = mesh.max_dt(w0, wl.cfl)
            a, b = (w0.clone(), g0.clone()), mesh.empty_state()
            for _ in range(warmup // 2):
                mesh.step(a[0], a[1], dt, out=b)
                mesh.step(b[0], b[1], dt, out=a)
            graph = mesh.capture_steps(a, b, dt, 100)
            graph.replay()
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps // 100):
                graph.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (steps // 100 * 100)
            res[prec] = {"value": mesh.N / (ms * 1e-3), "us_per_step": round(ms * 1e3, 2)}
            del graph, mesh
        out[name] = res
    return out


def c4_leg(steps, warmup):
    """Throughput on the 980,000-triangle Riemann problem (positivity limiter on):
    its step moves ~1 GB in FP64, far more than the 256 MB Infinity Cache."""
    import torch
    from paper_2607_10809_amd.hwe import Mesh
    from workloads import riemann_workload
    wl = riemann_workload()
    out = {"workload": "euler 2-D Riemann problem, [0,1]^2 transmissive, 700x700 split squares +-0.2h jitter "
                       "seed 4 (980,000 triangles), positivity limiter", "steps": steps}
    for prec in ("fp64", "mixed"):
        mesh = Mesh.from_workload(wl, precision=prec, positivity=True)
        w0, g0 = mesh.to_device(wl.state0)
        dt = mesh.max_dt(w0, 0.2)
        bufs = [(w0, g0), mesh.empty_state()]
        for i in range(warmup):
            mesh.step(bufs[i % 2][0], bufs[i % 2][1], dt, out=bufs[(i + 1) % 2])
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(warmup, warmup + steps):
            mesh.step(bufs[i % 2][0], bufs[i % 2][1], dt, out=bufs[(i + 1) % 2])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        mesh.profile_begin(steps)
        for i in range(steps):
            mesh.step(bufs[i % 2][0], bufs[i % 2][1], dt, out=bufs[(i + 1) % 2])
        kms, nk = mesh.profile_end()
        torch.cuda.synchronize()
        kb = kernel_bytes(mesh.N, mesh.E, mesh.m, 8 if prec == "fp64" else 4, positivity=True)
        out[prec] = {"value": mesh.N / (ms * 1e-3), "ms_per_step": ms,
                     "step_GBps": round(sum(kb.values()) / (ms * 1e-3) / 1e9, 1),
                     "kernels": {n: {"us": round(t / nk * 1e3, 2), "GBps": round(kb[n] / (t / nk * 1e-3) / 1e9, 1)}
                                 for n, t in zip(("recon", "edge", "update"), kms)}}
        del mesh, bufs, w0, g0
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--n", type=int, default=320, help="squares per side (default: 320 -> 204,800 triangles)")
    ap.add_argument("--forward-only", action="store_true",
                    help="skip the adjoint, copy and 980,000-triangle legs (for counter runs)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 980,000-triangle Riemann leg and the two small configurations")
    ap.add_argument("--no-error", action="store_true",
                    help="skip the run of both precisions to the vortex's final time (mixed-vs-FP64 error)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 20 device copies of 256 MiB (reference for HBM byte counters)")
    ap.add_argument("--c4-only", action="store_true",
                    help="only the 980,000-triangle Riemann leg (for counter runs); prints its JSON")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 20}), flush=True)
        return
    from paper_2607_10809_amd import _lib
    _lib.load_library()
    if args.c4_only:
        print(json.dumps({"riemann_980k": c4_leg(args.steps, args.warmup)}), flush=True)
        return
    from workloads import vortex_workload

    log("building workload ...")
    wl = vortex_workload(n=args.n)
    N = wl.mesh.n_cells
    log(f"N = {N}; FP64 leg ...")
    f64 = gpu_leg(wl, args.steps, args.warmup, "fp64")
    log(f"FP64: {f64['ms'] / args.steps * 1e3:.1f} us/step; kernels (ms) {f64['kernel_ms']}")
    mix = gpu_leg(wl, args.steps, args.warmup, "mixed")
    log(f"mixed: {mix['ms'] / args.steps * 1e3:.1f} us/step; kernels (ms) {mix['kernel_ms']}")
    adj = adjm = c4 = copy_gbps = merr = small = None
    if not args.forward_only:
        if not args.no_error:
            log("mixed vs FP64 at T ...")
            merr = mixed_error_leg(wl)
        if not args.no_c4:
            log("980,000-triangle Riemann leg ...")
            c4 = c4_leg(200, 10)
            small = small_configs_leg()
        copy_gbps = copy_bandwidth()
        adj = adjoint_leg(wl)
        log(f"adjoint (FP64, 200 steps, checkpoint 20): forward {adj['forward_ms']:.1f} ms, backward "
            f"{adj['backward_ms']:.1f} ms, ratio {adj['ratio']:.2f}; per step {adj['adjoint_step_us']:.1f} us vs "
            f"{adj['step_us']:.1f} us")
        adjm = adjoint_leg(wl, precision="mixed")
        ga, gb = adjm.pop("_grad"), adj.pop("_grad")
        adjm["gradient_error_vs_fp64"] = {"rel_l2": float(np.linalg.norm(ga - gb) / np.linalg.norm(gb)),
                                          "rel_max": float(np.abs(ga - gb).max() / np.abs(gb).max())}
    E, m = f64["mesh"].E, f64["mesh"].m
    value = N * args.steps / (f64["ms"] * 1e-3)
    value_mixed = N * args.steps / (mix["ms"] * 1e-3)

    names = ["recon", "edge", "update"]
    kb64 = kernel_bytes(N, E, m, 8)
    kbm = kernel_bytes(N, E, m, 4)
    per_kernel = {}
    for tag, leg, kb in (("fp64", f64, kb64), ("mixed", mix, kbm)):
        per_kernel[tag] = {n: {"us": round(t * 1e3, 2), "alg_bytes": int(kb[n]),
                               "GBps": round(kb[n] / (t * 1e-3) / 1e9, 1)}
                           for n, t in zip(names, leg["kernel_ms"])}
    # roofline of the dominant FP64 kernel: recon and update are bound by HBM,
    # the edge kernel by FP64 VALU issue (two thirds of the issue slots busy
    # against a third of HBM)
    dom = names[int(np.argmax(f64["kernel_ms"]))]
    t_dom = f64["kernel_ms"][names.index(dom)] * 1e-3
    gbps = kb64[dom] / t_dom / 1e9
    if dom == "edge":
        tflops = EDGE_ALG_FLOP_PER_EDGE * E / t_dom / 1e12
        xtflops = EDGE_FP64_FLOP_PER_EDGE * E / t_dom / 1e12
        roofline = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
                    "per_launch_flops": int(EDGE_ALG_FLOP_PER_EDGE * E),
                    "flops_per_unit": {"per_edge": EDGE_ALG_FLOP_PER_EDGE,
                                       "source": "oracle live operation count: viscosity + Lax-Wendroff + "
                                                 "Taylor values and fluxes, two sides x two Gauss points"},
                    "executed": {"per_launch_flops": int(EDGE_FP64_FLOP_PER_EDGE * E), "TFLOPs": round(xtflops, 2),
                                 "frac": round(xtflops / FP64_VECTOR_PEAK_TFLOPS, 4),
                                 "source": "SQ_INSTS_VALU_FLOPS_FP64 x 64 / E"},
                    "algorithmic_GBps": round(gbps, 1)}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbps / HBM_PEAK_GBS, 4)}
    roofline.update({"traffic": measured_traffic(f"{dom}_kernel<2, double>"), "kernel": f"{dom}_kernel<2, double>",
                     "per_launch_bytes": int(kb64[dom]), "source_digest": source_digest()})
    if dom == "edge":
        roofline["valu_busy"] = measured_valu_busy("edge_kernel<2, double>")
    if copy_gbps:
        roofline["measured_copy_GBps"] = round(copy_gbps, 1)
        roofline["hbm_frac_of_copy"] = round(gbps / copy_gbps, 4)
    # the HBM-bound reconstruction kernel, reported beside the dominant one
    t_rec = f64["kernel_ms"][0] * 1e-3
    rec_gbps = kb64["recon"] / t_rec / 1e9
    roofline["hbm_kernel"] = {"kernel": "recon_kernel<2, double>", "bound": "hbm", "achieved": round(rec_gbps, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(rec_gbps / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic("recon_kernel<2, double>"),
                              "per_launch_bytes": int(kb64["recon"])}
    if copy_gbps:
        roofline["hbm_kernel"]["frac_of_copy"] = round(rec_gbps / copy_gbps, 4)
    step_bytes = sum(kb64.values())
    ms64, msm = f64["ms"] / args.steps, mix["ms"] / args.steps
    step_roofline = {
        "hbm": {prec: {"alg_bytes_per_cell_step": ALG_BYTES_PER_CELL_STEP[prec],
                       "achieved_GBps": round(v * ALG_BYTES_PER_CELL_STEP[prec] / 1e9, 1),
                       "frac": round(v * ALG_BYTES_PER_CELL_STEP[prec] / 1e9 / HBM_PEAK_GBS, 4)}
                for prec, v in (("fp64", value), ("mixed", value_mixed))},
        "alu_fp64": {"alg_flops_per_cell_step": ALG_FLOP_PER_CELL_STEP,
                     "achieved_TFLOPs": round(value * ALG_FLOP_PER_CELL_STEP / 1e12, 2),
                     "frac": round(value * ALG_FLOP_PER_CELL_STEP / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4)}}
    out = {
        "metric": "cell-steps/s FP64 vs FP32 + adjoint/forward time ratio, Euler 204,800 tris",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "repeats": {"count": REPEATS, "statistic": "median",
                    "ms_per_step": {"fp64": [round(r / args.steps, 5) for r in f64["rep_ms"]],
                                    "mixed": [round(r / args.steps, 5) for r in mix["rep_ms"]]}},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"euler isentropic vortex, periodic [0,10]^2, {args.n}x{args.n} split squares "
                               f"+-0.1h jitter seed 3 ({N} triangles)", "cells": N, "edges": E,
                   "dt": f64["dt"], "parallelism": "1 GPU"},
        "mixed": {"value": value_mixed, "ms_per_step": msm, "dtype": "f32 bulk + f64 averages/weights",
                  "speedup_vs_fp64": value_mixed / value, "error_vs_fp64": merr},
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": {"fp64": adj, "mixed": adjm,
                    "workload": "misfit 0.5|rho(T)-rho_target|^2, 200 steps, checkpoint every 20, same mesh"},
        "step_alg_bytes": {"fp64": int(step_bytes), "mixed": int(sum(kbm.values()))},
        "step_GBps": {"fp64": round(step_bytes / (f64["ms"] / args.steps * 1e-3) / 1e9, 1),
                      "mixed": round(sum(kbm.values()) / (mix["ms"] / args.steps * 1e-3) / 1e9, 1)},
        "kernels": per_kernel,
        "roofline": roofline,
        "step_roofline": step_roofline,
        "state_flags": {"fp64": f64["flags"], "mixed": mix["flags"]},
        "riemann_980k": c4,
        "small_configs": small,
        "hip_graph": {"steps_per_graph": f64["graph_chunk"],
                      "eager_ms_per_step": {"fp64": round(f64["ms_eager"] / args.steps, 5),
                                            "mixed": round(mix["ms_eager"] / args.steps, 5)}},
    }
    if not args.no_cpu:
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_leg(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
