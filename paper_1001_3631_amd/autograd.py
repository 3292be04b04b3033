"""torch.autograd.Function over the engine: waveform = evolve(Phi0, Pi0, A).

Forward runs the HIP stepper; backward runs the HIP adjoint sweep
(teuk_adjoint_*), so gradients with respect to the initial data and the
source amplitude cost one reverse sweep.  The loss may be any real function
of the waveform; torch hands its gradient in the same convention the adjoint
uses (dL/dRe + i dL/dIm).
"""

import torch

from .engine import Engine


class TeukEvolve(torch.autograd.Function):
    """w = TeukEvolve.apply(phi0, pi0, amplitude, engine, nsteps).

    phi0, pi0: complex128 (nth, nr) on the device; amplitude: 0-dim float64
    tensor (used when the engine has a source attached); returns the
    (nsteps, nth) waveform at the extraction radius."""

    @staticmethod
    def forward(ctx, phi0, pi0, amplitude, engine, nsteps):
        if not isinstance(engine, Engine):
            raise TypeError("engine must be a paper_1001_3631_amd.engine.Engine")
        engine.set_state(phi0.detach().contiguous(), pi0.detach().contiguous())
        if engine.has_source:
            engine.set_amplitude(float(amplitude))
        w = engine.step(int(nsteps))
        ctx.engine = engine
        ctx.nsteps = int(nsteps)
        return w

    @staticmethod
    def backward(ctx, gw):
        eng, n = ctx.engine, ctx.nsteps
        gw = gw.detach().contiguous()
        eng.adjoint_begin(n, gw=gw)
        eng.adjoint_step(n, gw)
        lp, lq, dA = eng.adjoint_get(want_dA=eng.has_source)
        gA = torch.tensor(dA if dA is not None else 0.0, dtype=torch.float64, device=lp.device)
        return lp, lq, gA, None, None


def evolve(phi0, pi0, amplitude, engine, nsteps):
    """Differentiable evolution; see TeukEvolve."""
    return TeukEvolve.apply(phi0, pi0, amplitude, engine, nsteps)


class TeukEvolveCheckpointed(torch.autograd.Function):
    """(w, L_s) = TeukEvolveCheckpointed.apply(phi0, pi0, amplitude, engine, nsteps, state_loss, interval,
    snapshots).

    Like TeukEvolve, plus the state loss
    L_s = weight * sum_{n=n_lo..n_hi} sum_rect |Phi^n|^2 (state_loss dict), whose
    gradient needs the intermediate states: the forward keeps a snapshot every
    `interval` iterations (0 = ceil(sqrt(nsteps))) and the backward recomputes
    each segment before sweeping it in reverse; or, with snapshots = s >= 1,
    at most s snapshots placed by the binomial schedule."""

    @staticmethod
    def forward(ctx, phi0, pi0, amplitude, engine, nsteps, state_loss, interval=0, snapshots=0):
        engine.set_state(phi0.detach().contiguous(), pi0.detach().contiguous())
        if engine.has_source:
            engine.set_amplitude(float(amplitude))
        w, ls = engine.forward_checkpointed(int(nsteps), interval, state_loss, snapshots=int(snapshots))
        ctx.engine = engine
        # the engine keeps the snapshots of its latest forward only
        ctx.generation = engine.checkpoint_generation
        return w, torch.tensor(ls, dtype=torch.float64, device=w.device)

    @staticmethod
    def backward(ctx, gw, gls):
        eng = ctx.engine
        if ctx.generation != eng.checkpoint_generation:
            raise RuntimeError("the engine ran another checkpointed forward since this one: its snapshots "
                               "are gone; use one engine per checkpointed evolution in a graph")
        gw = gw.detach().contiguous() if gw is not None else None
        dls = float(gls) if gls is not None else 0.0
        gp, gq, dA = eng.backward_checkpointed(gw, dls)
        gA = torch.tensor(dA, dtype=torch.float64, device=gp.device)
        return gp, gq, gA, None, None, None, None, None
