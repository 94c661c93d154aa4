"""Write the expected values of the long-run parity tests (tests/test_gpu_long_parity.py).

Calls only the oracle (oracle/) and the seeded input generators
(paper_0909_4039_amd/inputs.py); nothing here touches the GPU path.  Each case
runs the oracle over a workload's full run length (or, for the 32768 x 1024
grid, a window holding the whole domain of dependence of 200 columns after
2000 steps) and stores, compressed:
  - the time step and the inputs' recipe (sizes, seeds, source, observer);
  - the recorded waveform (the field read at a fixed r*, Sec. 2.2, Fig. 1)
    on a stride of steps and theta rows;
  - Phi and Pi of the final state on a sample of rows and columns whose
    strides (13 rows, 29 columns) are prime to every tile width the kernels
    use, so every position within a tile is sampled;
  - the final state's full-grid L2 norms and four random projections
    <w_k, u> of it (weights from inputs.projection_weights), which see every
    point of the grid.

Run from the repository root:  python tests/golden/make_long_runs.py [case ...]
The oracle uses every core (OpenMP); the four cases take about 85 minutes
on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0909_4039_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROW_STRIDE, COL_STRIDE = 13, 29
N_PROJ = 4

# The Kerr a = 0.9 source workload (8192 x 256) over its first 5000 steps from
# smooth seeded data, and over its full 50,000 steps as specified (zero data,
# source on; about an hour on 8 cores); the adjoint workload (4096 x 256,
# a = 0.6, pulse plus source) over its full 20,000 steps; and the largest grid
# (32768 x 1024, a = 0.99) over 2000 steps on a window centred on the source.
CASES = {
    "kerr_a0.9_source_8192x256": dict(
        nr=8192, nth=256, rmin=-100.0, rmax=400.0, a=0.9, m=2, s=-2, r0=10.0, amp=1.0,
        dt_steps=50000, n=5000, robs=20.0, data={"kind": "smooth", "seed": 21},
        wave_step_stride=100, wave_row_stride=4),
    "kerr_a0.9_source_8192x256_full": dict(
        nr=8192, nth=256, rmin=-100.0, rmax=400.0, a=0.9, m=2, s=-2, r0=10.0, amp=1.0,
        dt_steps=50000, n=50000, robs=20.0, data={"kind": "zero"},
        wave_step_stride=100, wave_row_stride=8),
    "adjoint_a0.6_4096x256": dict(
        nr=4096, nth=256, rmin=-100.0, rmax=400.0, a=0.6, m=2, s=-2, r0=10.0, amp=1.0,
        dt_steps=20000, n=20000, robs=30.0, data={"kind": "pulse", "center": 20.0, "width": 4.0, "seed": 4},
        wave_step_stride=200, wave_row_stride=4),
    "kerr_a0.99_source_32768x1024_window": dict(
        nr=32768, nth=1024, rmin=-100.0, rmax=400.0, a=0.99, m=2, s=-2, r0=8.0, amp=1.0,
        dt_steps=100000, n=2000, robs=10.5, data={"kind": "smooth", "seed": 55},
        window=(7223 - 2100, 4200, 0, 1024), wave_step_stride=20, wave_row_stride=8),
}


def initial_data(c):
    d = c["data"]
    if d["kind"] == "zero":
        z = np.zeros((c["nth"], c["nr"]), np.complex128)
        return z, z.copy()
    if d["kind"] == "smooth":
        return inputs.smooth_random_state(c["nr"], c["nth"], c["rmin"], c["rmax"], seed=d["seed"])
    return inputs.pulse(c["nr"], c["nth"], c["rmin"], c["rmax"], c["m"], d["center"], d["width"],
                        inputs.seeded_amplitude(d["seed"]))




def make(name):
    c = CASES[name]
    t0 = time.time()
    dt = oracle.stable_dt(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], c["dt_steps"])
    phi, pi = initial_data(c)
    win = c.get("window")
    if win is not None:
        i0, ni, j0, nj = win
        sl = (slice(j0, j0 + nj), slice(i0, i0 + ni))
        phi, pi = np.ascontiguousarray(phi[sl]), np.ascontiguousarray(pi[sl])
    o = oracle.Oracle(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], dt, r0=c["r0"],
                      amp=c["amp"], rstar_obs=c["robs"], window=win)
    print(f"{name}: dt = {dt!r}, {c['n']} steps on {phi.shape[0]} x {phi.shape[1]} points", flush=True)
    op, oq, ow = o.run(phi, pi, c["n"])
    # the region every step kept exact: the whole grid, or the window less n
    # columns per side (all rows are held, so theta loses nothing)
    if win is None:
        c0, c1 = 0, c["nr"]
    else:
        c0, c1 = win[0] + c["n"], win[0] + win[1] - c["n"]
    loc = slice(c0 - (0 if win is None else win[0]), c1 - (0 if win is None else win[0]))
    vp, vq = op[:, loc], oq[:, loc]
    assert np.all(np.isfinite(vp)) and np.all(np.isfinite(vq))
    rows = np.unique(np.r_[np.arange(0, c["nth"], ROW_STRIDE), c["nth"] - 1])
    cols = np.unique(np.r_[np.arange(0, c1 - c0, COL_STRIDE), c1 - c0 - 1])
    wsteps = np.unique(np.r_[np.arange(0, c["n"] + 1, c["wave_step_stride"]), c["n"]])
    wrows = np.arange(0, c["nth"], c["wave_row_stride"])
    proj = []
    for k in range(N_PROJ):
        w = inputs.projection_weights(vp.shape, seed=1000 + k)
        proj.append([np.vdot(w, vp), np.vdot(w, vq)])
    meta = dict(c, name=name, dt=dt, cols=[c0, c1], row_stride=ROW_STRIDE, col_stride=COL_STRIDE,
                n_proj=N_PROJ, proj_seed0=1000, seconds=time.time() - t0)
    np.savez_compressed(
        os.path.join(HERE, f"long_{name}.npz"),
        meta=np.array(json.dumps(meta)),
        rows=rows, cols=cols + c0, wave_steps=wsteps, wave_rows=wrows,
        phi_sample=vp[np.ix_(rows, cols)], pi_sample=vq[np.ix_(rows, cols)],
        wave=ow[np.ix_(wsteps, wrows)],
        norms=np.array([np.linalg.norm(vp), np.linalg.norm(vq)]),
        proj=np.array(proj))
    print(f"{name}: done in {time.time() - t0:.0f} s; |Phi| = {np.linalg.norm(vp):.6e}, "
          f"|wave| = {np.linalg.norm(ow):.6e}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        make(nm)
