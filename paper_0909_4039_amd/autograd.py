"""torch.autograd.Function over the library's forward steps and reverse sweep.

``waveform(solver, phi0, pi0, r0, amp, n_steps, rstar_obs)`` evolves the
initial data (Phi0, Pi0) for n_steps Lax-Wendroff steps (paper Eqs. 13-14)
with the particle source at orbit radius r0 and amplitude amp, and returns
the waveform w^0..w^n at rstar_obs as an (n_steps + 1, n_theta) complex128
tensor.  Its backward pass calls the library's reverse sweep
(``teuk_adjoint``), which returns dL/dPhi0, dL/dPi0, dL/dr0 and dL/damp.

Memory: the step is affine in (Phi, Pi) with coefficients that depend on
neither the state nor the step, so the reverse sweep needs no forward state
at all.  Nothing is saved for backward beyond the scalar parameters:
the sqrt(N)-checkpointing that a nonlinear step would need (sqrt(N) stored
states plus one recomputed forward sweep) is replaced by zero stored states
and no recomputation, and the backward costs one sweep of the same size as
the forward.

``waveform_moving(solver, phi0, pi0, traj, amp, n_steps, rstar_obs)`` does
the same for a moving source that follows an orbit table (r0, phi) at
every half step (an inspiral, the paper's Fig. 1).  Its backward pass
(``teuk_adjoint_moving``) returns the gradient for every table row, so a
differentiable orbit law chains through it.

``waveform(..., spin=a)`` also differentiates with respect to the Kerr spin.
The spin enters the step operator itself, so that gradient needs the
forward states: the library keeps sqrt(N) of them and recomputes the rest
(``teuk_param_gradient``).

Gradient convention: torch's for complex tensors (for L = |z|^2 the
gradient is 2z), which is dL/dRe + i dL/dIm, the library's convention.
"""
from __future__ import annotations

import torch


class TeukWaveform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, pi0, r0, amp, solver, n_steps, rstar_obs, t_start):
        if solver.prec != 64:
            raise ValueError("the differentiable waveform needs an FP64 solver")
        sig = solver.source[2:] if solver.source is not None else (2.0, 2.0)
        r0f, ampf = float(r0), float(amp)
        solver.set_source(r0f, ampf, *sig)
        solver.set_trajectory(None)   # a fixed orbit
        solver.set_state(phi0.detach(), pi0.detach())
        solver.set_time(float(t_start), 0)
        wave = solver.set_observer(rstar_obs, int(n_steps) + 1)
        solver.step(int(n_steps))
        cur = torch.cuda.current_stream(solver.device)
        cur.wait_stream(solver.stream)   # the steps ran on the solver's stream
        out = wave.clone()
        wave.record_stream(cur)
        solver.clear_observer()
        ctx.solver = solver
        ctx.args = (r0f, ampf, sig, int(n_steps), float(rstar_obs), float(t_start))
        ctx.r0_meta = (r0.dtype, r0.device) if torch.is_tensor(r0) else (torch.float64, phi0.device)
        ctx.amp_meta = (amp.dtype, amp.device) if torch.is_tensor(amp) else (torch.float64, phi0.device)
        return out

    @staticmethod
    def backward(ctx, g):
        solver = ctx.solver
        r0f, ampf, sig, n, robs, t0 = ctx.args
        # the solver may have been used in between: restore this call's source
        solver.set_source(r0f, ampf, *sig)
        solver.set_trajectory(None)
        dphi, dpi, dr0, damp = solver.adjoint(g, n, robs, t0)
        need = ctx.needs_input_grad
        return (dphi if need[0] else None, dpi if need[1] else None,
                torch.tensor(dr0, dtype=ctx.r0_meta[0], device=ctx.r0_meta[1]) if need[2] else None,
                torch.tensor(damp, dtype=ctx.amp_meta[0], device=ctx.amp_meta[1]) if need[3] else None,
                None, None, None, None)


class TeukWaveformSpin(torch.autograd.Function):
    """TeukWaveform with the Kerr spin as one more input.  The solver's tables
    are built for one spin, so ``spin`` must equal the solver's a; its
    gradient comes from the library's checkpointed parameter gradient
    (``teuk_param_gradient``), which keeps sqrt(N) forward states, since the
    spin enters the step operator itself."""

    @staticmethod
    def forward(ctx, phi0, pi0, r0, amp, spin, solver, n_steps, rstar_obs, t_start, h):
        a = float(solver.params["a"])
        if abs(float(spin) - a) > 1e-14 * max(1.0, abs(a)):
            raise ValueError(f"spin {float(spin)!r} differs from the solver's a = {a!r}: build the solver at this spin")
        out = TeukWaveform.forward(ctx, phi0, pi0, r0, amp, solver, n_steps, rstar_obs, t_start)
        ctx.init = (phi0.detach().clone(), pi0.detach().clone())
        ctx.h = h
        ctx.spin_meta = (spin.dtype, spin.device) if torch.is_tensor(spin) else (torch.float64, phi0.device)
        return out

    @staticmethod
    def backward(ctx, g):
        dphi, dpi, dr0, damp = TeukWaveform.backward(ctx, g)[:4]
        dspin = None
        if ctx.needs_input_grad[4]:
            _, _, _, n, robs, t0 = ctx.args
            v = ctx.solver.param_gradient("a", g, n, robs, ctx.init[0], ctx.init[1], h=ctx.h, t_start=t0)
            dspin = torch.tensor(v, dtype=ctx.spin_meta[0], device=ctx.spin_meta[1])
        return dphi, dpi, dr0, damp, dspin, None, None, None, None, None


def waveform(solver, phi0, pi0, r0, amp, n_steps, rstar_obs, t_start=0.0, spin=None, spin_h=1e-6):
    """Differentiable waveform w^0..w^n (see the module docstring).  With
    ``spin`` (equal to the solver's a) the spin is differentiable too, by the
    checkpointed sweep (step size ``spin_h`` of its central difference)."""
    if spin is None:
        return TeukWaveform.apply(phi0, pi0, r0, amp, solver, n_steps, rstar_obs, t_start)
    return TeukWaveformSpin.apply(phi0, pi0, r0, amp, spin, solver, n_steps, rstar_obs, t_start, spin_h)


class TeukWaveformMoving(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, pi0, traj, amp, solver, n_steps, rstar_obs):
        if solver.prec != 64:
            raise ValueError("the differentiable waveform needs an FP64 solver")
        import numpy as np
        sig = solver.source[2:] if solver.source is not None else (2.0, 2.0)
        tab = np.ascontiguousarray(traj.detach().to("cpu", torch.float64).numpy())
        ampf = float(amp)
        n = int(n_steps)
        # a source must be set before the table; its radius is overridden by the table
        solver.set_source(float(tab[0, 0]), ampf, *sig)
        solver.set_state(phi0.detach(), pi0.detach())
        solver.set_time(0.0, 0)
        solver.set_trajectory(tab)
        wave = solver.set_observer(rstar_obs, n + 1)
        solver.step(n)
        cur = torch.cuda.current_stream(solver.device)
        cur.wait_stream(solver.stream)
        out = wave.clone()
        wave.record_stream(cur)
        solver.clear_observer()
        ctx.solver = solver
        ctx.args = (tab, ampf, sig, n, float(rstar_obs))
        ctx.traj_meta = (traj.dtype, traj.device, tuple(traj.shape))
        ctx.amp_meta = (amp.dtype, amp.device) if torch.is_tensor(amp) else (torch.float64, phi0.device)
        return out

    @staticmethod
    def backward(ctx, g):
        solver = ctx.solver
        tab, ampf, sig, n, robs = ctx.args
        # the solver may have been used in between: restore this call's source and table
        solver.set_source(float(tab[0, 0]), ampf, *sig)
        solver.set_trajectory(tab)
        dphi, dpi, dtraj, damp = solver.adjoint_moving(g, n, robs)
        dt, dev, shape = ctx.traj_meta
        full = torch.zeros(shape, dtype=torch.float64)
        full[: 2 * n] = torch.from_numpy(dtraj)
        need = ctx.needs_input_grad
        return (dphi if need[0] else None, dpi if need[1] else None, full.to(dev, dt) if need[2] else None,
                torch.tensor(damp, dtype=ctx.amp_meta[0], device=ctx.amp_meta[1]) if need[3] else None,
                None, None, None)


def waveform_moving(solver, phi0, pi0, traj, amp, n_steps, rstar_obs):
    """Differentiable waveform w^0..w^n of a moving source.

    ``traj`` is the orbit table (n_half, 2), row k = (r0, phi) at t = k dt/2,
    n_half >= 2 n_steps; the run starts at t = 0 from (phi0, pi0).  Its
    gradient is dL/dr0_k, dL/dphi_k per row (rows past 2 n_steps get zero), so
    any differentiable orbit law that produced the table (a torch function of
    the initial radius or the mass ratio) chains through autograd."""
    return TeukWaveformMoving.apply(phi0, pi0, traj, amp, solver, n_steps, rstar_obs)
