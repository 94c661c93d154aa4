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
        dphi, dpi, dr0, damp = solver.adjoint(g, n, robs, t0)
        return (dphi, dpi, torch.tensor(dr0, dtype=ctx.r0_meta[0], device=ctx.r0_meta[1]),
                torch.tensor(damp, dtype=ctx.amp_meta[0], device=ctx.amp_meta[1]), None, None, None, None)


def waveform(solver, phi0, pi0, r0, amp, n_steps, rstar_obs, t_start=0.0):
    """Differentiable waveform w^0..w^n (see the module docstring)."""
    return TeukWaveform.apply(phi0, pi0, r0, amp, solver, n_steps, rstar_obs, t_start)
