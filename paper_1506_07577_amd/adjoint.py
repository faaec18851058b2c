"""Differentiable implicit-Euler trajectories on the HIP path.

`trajectory(sim, d0, v0, E_tet)` runs `sim.steps` implicit-Euler steps
(ebbx_implicit_step) and is a torch.autograd.Function: its backward pass
runs the per-step vector-Jacobian product (ebbx_implicit_step_vjp: the
adjoint masked PCG solve, K w, T[v, w] and the per-tet Young's-modulus
gradient), newest step first, and returns dL/dd0, dL/dv0 and dL/dE_tet.

Checkpointing: the forward pass keeps (d, v) only at steps 0, k, 2k, ...
(k = sim.checkpoint_every; 0 keeps every state).  The backward pass
recomputes each segment from its checkpoint, then reverses it.  With a
deterministic scatter strategy (block or seg) the recomputed states are
bitwise equal to the forward ones, so the gradient does not depend on k.

Everything here is orchestration: every arithmetic step of the forward and
backward passes runs in libebbx.so; torch supplies the buffers.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import ebbx


@dataclass
class Simulation:
    """A fixed integration schedule on one Fem (vertex vectors in library order)."""
    fem: "ebbx.Fem"
    steps: int
    dt: float
    tol: float = 1e-10
    maxit: int = 2000
    checkpoint_every: int = 5
    g: Sequence[float] = (0.0, 0.0, -9.81)
    precond: int = ebbx.PRECOND_JACOBI
    check_status: bool = True
    alpha: float = 0.0   # Rayleigh damping D = alpha M - beta K
    beta: float = 0.0


class SolverError(RuntimeError):
    pass


def _check_stats(stats: list, what: str):
    """Raise if any step's device report says inverted / not SPD / NaN; one sync."""
    if not stats:
        return
    allst = torch.stack(stats).cpu()
    for i in range(allst.shape[0]):
        raw = allst[i].numpy().tobytes()
        rec = ebbx.StepStats.from_buffer_copy(raw)
        if rec.status not in (ebbx.OK,):
            raise SolverError(f"{what}: step {i} reported status {rec.status} "
                              f"(iters {rec.iters}, rel_res {rec.rel_res:.3e}, inverted {rec.n_inverted})")


def _step(sim: Simulation, d, v, stats):
    st = sim.fem.implicit_step(d, v, sim.dt, g=sim.g, tol=sim.tol, maxit=sim.maxit, precond=sim.precond,
                               alpha=sim.alpha, beta=sim.beta)
    if stats is not None:
        stats.append(st)


def _apply_material(sim: Simulation, E_tet: Optional[torch.Tensor]):
    if E_tet is not None:
        sim.fem.set_material(E_tet=E_tet, nu_tet=None, E=0.0, nu=sim.fem.nu)


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d0, v0, E_tet, sim: Simulation):
        fem = sim.fem
        _apply_material(sim, E_tet)
        k = sim.checkpoint_every if sim.checkpoint_every > 0 else 1
        d = d0.detach().clone()
        v = v0.detach().clone()
        ckpt = {0: (d.clone(), v.clone())}
        stats = [] if sim.check_status else None
        for n in range(sim.steps):
            _step(sim, d, v, stats)
            if (n + 1) % k == 0 and n + 1 < sim.steps:
                ckpt[n + 1] = (d.clone(), v.clone())
        if sim.check_status:
            _check_stats(stats, "trajectory forward")
        ctx.sim = sim
        ctx.ckpt = ckpt
        ctx.final = (d.clone(), v.clone())
        ctx.E_tet = E_tet
        ctx.nt = fem.nt
        return d, v

    @staticmethod
    def backward(ctx, gdT, gvT):
        sim = ctx.sim
        fem = sim.fem
        _apply_material(sim, ctx.E_tet)
        gx = torch.zeros_like(ctx.final[0]) if gdT is None else gdT.contiguous().clone()
        gv = torch.zeros_like(ctx.final[1]) if gvT is None else gvT.contiguous().clone()
        want_E = ctx.E_tet is not None and ctx.needs_input_grad[2]
        E_bar = torch.zeros(max(ctx.nt, 1), dtype=torch.float64, device=gx.device) if want_E else None
        stats = [] if sim.check_status else None
        starts = sorted(ctx.ckpt.keys())
        ends = starts[1:] + [sim.steps]
        for s0, end in reversed(list(zip(starts, ends))):
            # recompute states s0 .. end-1; v_end comes from the next checkpoint (or the final state)
            d, v = (t.clone() for t in ctx.ckpt[s0])
            states = [(d.clone(), v.clone())]
            for _ in range(s0, end - 1):
                _step(sim, d, v, stats)
                states.append((d.clone(), v.clone()))
            v_next = ctx.ckpt[end][1] if end in ctx.ckpt else ctx.final[1]
            for n in range(end - 1, s0 - 1, -1):
                d_n = states[n - s0][0]
                v_np1 = v_next
                d_bar, v_bar, st = fem.step_vjp(d_n, v_np1, gx, gv, sim.dt, tol=sim.tol, maxit=sim.maxit,
                                                precond=sim.precond, E_bar=E_bar, g=sim.g, alpha=sim.alpha,
                                                beta=sim.beta)
                if stats is not None:
                    stats.append(st)
                gx, gv = d_bar, v_bar
                v_next = states[n - s0][1]
        if sim.check_status:
            _check_stats(stats, "trajectory backward")
        E_grad = E_bar[: ctx.nt] if want_E else None
        return gx, gv, E_grad, None


def trajectory(sim: Simulation, d0: torch.Tensor, v0: torch.Tensor, E_tet: Optional[torch.Tensor] = None):
    """(d_T, v_T) after sim.steps implicit steps from (d0, v0).

    d0, v0: (3, nv) FP64 CUDA tensors in library vertex order.  E_tet: (nt,)
    FP64 per-tet Young's modulus in library tet order, or None for the Fem's
    current material.  Differentiable with respect to d0, v0 and E_tet.
    """
    return _Trajectory.apply(d0, v0, E_tet, sim)


def position_loss(X: torch.Tensor, d_T: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """L = ||X + d_T - target||^2 summed over all vertices (inputs (3, nv))."""
    r = X + d_T - target
    return (r * r).sum()
