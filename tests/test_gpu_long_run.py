"""A long run with the circular-orbit source on the r* grid of the Kerr
a = 0.9 source workload (8192 r* nodes over [-100, 400], m = 2, s = -2,
r0 = 10), 64 theta rows, through the GPU path to T = 440 M.  The oracle
cannot run this long at this size, so the test checks properties that the
method fixes at any size:

- the state stays finite and the field inside r* = 200 does not grow;
- once the switch-on burst has passed, the waveform at r* = 100 is the
  steady response of a stable linear system driven by the circular-orbit
  source (Sec. 2.1): constant modulus, rotating at the source frequency
  m Omega (time dependence e^{-i m Omega t}).

The window t in [360, 440] M lies after the burst has passed r* = 100 (the
modulus has settled to 3e-4) and before its echo from the r* = 400
boundary can return; over its last 40 M the modulus keeps settling.

The case keeps the Courant number dt/dr* (0.024, with dt set by the theta
operator) in the range where the scheme damps poorly resolved r* modes.
With 256 theta rows (dt/dr* = 0.006) and the 2-cell source, a poorly
resolved mode at the potential peak grows from t ~ 100 M; that
configuration is not a case here.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_long_run_settles_to_the_driven_response():
    import torch
    from paper_0909_4039_amd import inputs
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    nr, nth, rmin, rmax, a, M, m, s = 8192, 64, -100.0, 400.0, 0.9, 1.0, 2, -2
    r0, robs, T = 10.0, 100.0, 440.0
    dt = suggest_dt(nr, nth, rmin, rmax, a, M, m, s, 1_200_000)
    chunk = int(round(1.0 / dt))            # one waveform sample per M
    n_chunks = int(np.ceil(T / (chunk * dt)))
    rs, _ = inputs.grid(nr, nth, rmin, rmax)
    inner = int(np.searchsorted(rs, 200.0))
    sol = Solver(nr, nth, rmin, rmax, a, M, m, s, dt)
    zero = np.zeros((nth, nr), dtype=np.complex128)
    sol.set_state(zero, zero)
    sol.set_source(r0, 1.0)
    sol.autotune(5)
    ws, peak = [], {}
    for i in range(n_chunks):
        sol.step(chunk)
        ws.append(sol.extract(robs)[nth // 2].clone())
        if (i + 1) % 40 == 0 or i + 1 == n_chunks:
            torch.cuda.synchronize()
            peak[i + 1] = float(sol.phi[:, :inner].abs().max())
            print(f"[gpu] long run {nr}x{nth}: t = {(i + 1) * chunk * dt:.1f} M, "
                  f"max |Phi| inside r* = 200: {peak[i + 1]:.4e}", flush=True)
    torch.cuda.synchronize()
    sol.check_finite()
    w = torch.stack(ws).cpu().numpy()
    t = (np.arange(len(ws)) + 1) * chunk * dt
    sol.close()
    Omega = np.sqrt(M) / (r0 ** 1.5 + a * np.sqrt(M))
    sel = (t >= 360.0) & (t <= 440.0)
    mod = np.abs(w[sel])
    slope = np.polyfit(t[sel], np.unwrap(np.angle(w[sel])), 1)[0]
    spread = (mod.max() - mod.min()) / mod.mean()
    late = np.abs(w[(t >= 400.0) & (t <= 440.0)])
    late_spread = (late.max() - late.min()) / late.mean()
    print(f"[gpu] steady window: |w| mean {mod.mean():.4e}, spread {spread:.2e} (last 40 M: {late_spread:.2e}); "
          f"phase rate {slope:.7f} against -m Omega = {-m * Omega:.7f}", flush=True)
    assert mod.mean() > 0.0
    assert spread < 1e-3, spread
    assert late_spread < 0.5 * spread, (late_spread, spread)
    assert abs(slope + m * Omega) < 1e-4 * m * Omega, (slope, -m * Omega)
    ks = sorted(peak)
    assert peak[ks[-1]] <= 2.0 * max(peak[k] for k in ks if k <= ks[-1] // 2), peak
