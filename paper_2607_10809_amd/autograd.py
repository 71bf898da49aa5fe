"""Differentiable multi-step rollout of the HIP step with step checkpointing.

``rollout(mesh, wbar0, grad0, dt, n_steps, ckpt)`` runs ``n_steps`` explicit
steps (hwe_step) and returns the final state; its backward pass applies the
hand-written adjoint (hwe_step_adjoint) in reverse.  Only every ``ckpt``-th
state is kept during the forward pass; the backward pass recomputes each
segment of ``ckpt`` steps from its checkpoint, keeping the reconstruction
of every recomputed step (hwe_step_keep), then walks it backwards with the
adjoint that reuses them (hwe_step_adjoint_kept), the recomputation of the
next segment overlapping the adjoints of the current one.  The last state of a
segment is never stepped during the recomputation, so its reconstruction is
rebuilt by the adjoint itself.  The last segment is not recomputed at all: the
forward pass keeps its states and reconstructions as it computes them (ckpt
states and ckpt reconstructions beyond the checkpoints), and the backward pass
walks them first.  The time step is a constant (not differentiated); step k
runs from time t0 + k dt (read by moving boundary states).
"""
from __future__ import annotations

import torch


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, wbar0, grad0, mesh, dt, n_steps, ckpt, t0, overlap, keep_last):
        if ckpt <= 0:
            raise ValueError("ckpt must be positive")
        checkpoints = [(wbar0.detach().clone(), grad0.detach().clone())]
        cur = (checkpoints[0][0], checkpoints[0][1])
        bufs = [mesh.empty_state(), mesh.empty_state()]
        last_start = ((n_steps - 1) // ckpt) * ckpt if n_steps > 0 else 0
        kept_states, kept_recon = [], []
        for k in range(n_steps):
            if keep_last and k >= last_start:
                # the last segment: every state and reconstruction stays
                kept_states.append(cur)
                nxt = mesh.empty_state()
                kept_recon.append(mesh.empty_recon())
                mesh.step(cur[0], cur[1], dt, out=nxt, keep=kept_recon[-1], t=t0 + k * dt)
            else:
                nxt = bufs[k % 2]
                mesh.step(cur[0], cur[1], dt, out=nxt, t=t0 + k * dt)
            cur = nxt
            if (k + 1) % ckpt == 0 and k + 1 < n_steps:
                checkpoints.append((cur[0].clone(), cur[1].clone()))
        ctx.mesh, ctx.dt, ctx.n_steps, ctx.ckpt, ctx.t0 = mesh, dt, n_steps, ckpt, t0
        ctx.overlap = overlap
        ctx.checkpoints = checkpoints
        ctx.kept = (kept_states, kept_recon) if keep_last and n_steps > 0 else None
        return cur[0].clone(), cur[1].clone()

    @staticmethod
    def backward(ctx, lw, lg):
        mesh, dt, n, ckpt, t0 = ctx.mesh, ctx.dt, ctx.n_steps, ctx.ckpt, ctx.t0
        lam = (lw.contiguous().to(torch.float64), lg.contiguous().to(mesh.gdtype))
        nseg = len(ctx.checkpoints)
        seg_len = min(ckpt, n)
        out = [mesh.empty_state(), mesh.empty_state()]
        # Segment s - 1 is recomputed on a second stream while the adjoints of
        # segment s run on the caller's stream; the two alternate between two
        # preallocated sets of segment buffers (states and kept
        # reconstructions).  The recomputations stay ordered on their stream,
        # so the handle's forward scratch is never shared by two of them, and
        # the adjoints use scratch of their own.
        nsets = 2 if nseg > 1 else 1
        sets = [([mesh.empty_state() for _ in range(seg_len - 1)], [mesh.empty_recon() for _ in range(seg_len - 1)])
                for _ in range(nsets)]
        main = torch.cuda.current_stream(mesh.device)
        side = torch.cuda.Stream(device=mesh.device) if (ctx.overlap and nseg > 1) else main
        side.wait_stream(main)
        free = [None] * nsets

        def recompute(s):
            start, length = s * ckpt, min(ckpt, n - s * ckpt)
            j = s % nsets
            if free[j] is not None:
                side.wait_event(free[j])
            st, rc = sets[j]
            states = [ctx.checkpoints[s]]
            for k in range(length - 1):
                states.append(mesh.step(states[-1][0], states[-1][1], dt, out=st[k], keep=rc[k],
                                        t=t0 + (start + k) * dt, stream=side))
            ev = torch.cuda.Event()
            ev.record(side)
            return states, rc[:length - 1], ev

        # the last segment as the forward pass kept it (every reconstruction),
        # or recomputed (all but the last one)
        pending = (*ctx.kept, None) if ctx.kept is not None else recompute(nseg - 1)
        ctx.kept = None
        flip = 0
        for s in reversed(range(nseg)):
            states, rc, ready = pending
            if s > 0:
                pending = recompute(s - 1)
            if ready is not None:
                main.wait_event(ready)
            start, length = s * ckpt, min(ckpt, n - s * ckpt)
            for k in reversed(range(length)):
                dst = out[flip]
                flip ^= 1
                R = rc[k] if k < len(rc) else None
                mesh.adjoint(states[k][0], states[k][1], lam[0], lam[1], dt, out=dst, recon=R, t=t0 + (start + k) * dt)
                lam = dst
            done = torch.cuda.Event()
            done.record(main)
            free[s % nsets] = done
            ctx.checkpoints[s] = None
        main.wait_stream(side)
        return lam[0].clone(), lam[1].clone(), None, None, None, None, None, None, None


def rollout(mesh, wbar0, grad0, dt, n_steps, ckpt=20, t0=0.0, overlap=True, keep_last=True):
    """Final state after n_steps steps from time t0; differentiable with
    respect to (wbar0, grad0).  overlap: recompute the next segment on a
    second stream during the adjoints of the current one; keep_last: keep the
    last segment's states and reconstructions from the forward pass instead of
    recomputing them.  The gradient is the same bits either way."""
    return Rollout.apply(wbar0, grad0, mesh, float(dt), int(n_steps), int(ckpt), float(t0), bool(overlap),
                         bool(keep_last))
