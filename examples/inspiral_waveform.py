"""The m = 1..4 modes of one inspiral, stepped together in one batch, with
the waveform recorded at an extraction radius and written to a .npz file.

    python examples/inspiral_waveform.py [--out waveform.npz] [--small]

A particle of mass ratio q spirals in on Kerr (a = 0.9) from r0 = 10 under
the quadrupole decay law of paper_0909_4039_amd.inputs.inspiral_trajectory;
each azimuthal mode is an independent 2+1 problem (the m-mode ansatz, Sec. 2
of the paper), so the batch runs them side by side with bitwise the results
of separate single-mode runs.  The batch's watchdog is on, so a runaway
value stops the run with TEUK_EUNSTABLE instead of filling the file with it.
"""
import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(out=None, small=False, q=1e-4, a=0.9, r_start=10.0, rstar_obs=None):
    import torch
    from paper_0909_4039_amd import batch as B
    from paper_0909_4039_amd import inputs
    from paper_0909_4039_amd.solver import suggest_dt
    nr, nth, rmin, rmax = (1024, 32, -100.0, 400.0) if small else (8192, 128, -100.0, 400.0)
    n_steps = 2000 if small else 100_000
    if rstar_obs is None:
        # the field leaves the orbit (r* = 12.8 M at r0 = 10) at light speed: read it
        # where it arrives well within the run (about 20 M, resp. 130 M of evolution)
        rstar_obs = 20.0 if small else 100.0
    modes = (1, 2, 3, 4)
    # one dt for all modes: the most restrictive of the per-mode rules
    dt = min(suggest_dt(nr, nth, rmin, rmax, a, 1.0, m, -2, n_steps) for m in modes)
    descs = [B.make_desc(nr, nth, rmin, rmax, a, m, dt, r0=r_start, amp=1.0, rstar_obs=rstar_obs)
             for m in modes]
    bt = B.Batch(descs, n_steps)
    traj = inputs.inspiral_trajectory(r_start, a, 1.0, q, dt, n_steps)
    for i in range(len(modes)):
        bt.set_trajectory(i, traj)
    bt.autotune(5)
    bt.set_watchdog(True, 1e8)
    chunk = max(1, n_steps // 10)
    for done in range(0, n_steps, chunk):
        bt.step(min(chunk, n_steps - done))
        bt.synchronize()
        print(f"step {min(done + chunk, n_steps)} of {n_steps}, t = {min(done + chunk, n_steps) * dt:.2f} M",
              flush=True)
    bt.synchronize()
    waves = np.stack([w.cpu().numpy() for w in bt.waves])          # (modes, n_steps + 1, n_theta)
    t = np.arange(n_steps + 1) * dt
    bt.close()
    if out:
        np.savez_compressed(out, t=t, waves=waves, modes=np.array(modes), r0=traj[::2, 0], dt=dt,
                            rstar_obs=rstar_obs)
    return t, waves, traj


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default="waveform.npz")
    ap.add_argument("--small", action="store_true", help="a small grid and 2000 steps")
    args = ap.parse_args()
    t, waves, traj = run(args.out, args.small)
    print(f"wrote {args.out}: {waves.shape[0]} modes, {waves.shape[1]} samples to t = {t[-1]:.2f} M; "
          f"r0 from {traj[0, 0]:.4f} to {traj[-1, 0]:.4f}")


if __name__ == "__main__":
    main()
