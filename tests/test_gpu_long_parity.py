"""FP64 parity over the workloads' own run lengths, against expected values
the oracle wrote (tests/golden/make_long_runs.py, which calls only oracle/
and the seeded input generators).

  - Kerr a = 0.9 with the source, 8192 x 256: 5000 steps from smooth seeded
    data, and the workload as specified (zero data, source on) over its full
    50,000 steps.
  - The adjoint workload (a = 0.6, 4096 x 256, pulse plus source): the full
    20,000 steps.
  - The largest grid (a = 0.99, 32768 x 1024, source at r0 = 8): 2000 steps
    in the launch configuration the benchmark times, checked on the
    oracle's window that holds the whole domain of dependence of 200
    columns around the source, over every theta row.

Each run is compared on the waveform (a stride of steps and theta rows), on
a sample of the final state, on the final state's full-grid norms and on
four random projections that see every point.  Bars, FP64: relative L2
<= 1e-12 and per element max|g - o| / max|o| <= 1e-12 for the waveform, for
the state u = (Phi, Pi) and for Phi alone, 1e-11 for Pi alone (see below);
projections within 5e-12 of |u| rms|w| (a random projection of an error e is
about |e| rms|w|).
"""
import json
import os

import numpy as np
import pytest

from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL64 = 1e-12
NAMES = ["kerr_a0.9_source_8192x256", "kerr_a0.9_source_8192x256_full", "adjoint_a0.6_4096x256",
         "kerr_a0.99_source_32768x1024_window"]


def load(name):
    path = os.path.join(GOLDEN, f"long_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_long_runs.py {name})")
    z = np.load(path, allow_pickle=False)
    return json.loads(str(z["meta"])), {k: z[k] for k in z.files if k != "meta"}


def initial_data(c):
    d = c["data"]
    if d["kind"] == "zero":
        z = np.zeros((c["nth"], c["nr"]), np.complex128)
        return z, z.copy()
    if d["kind"] == "smooth":
        return inputs.smooth_random_state(c["nr"], c["nth"], c["rmin"], c["rmax"], seed=d["seed"])
    return inputs.pulse(c["nr"], c["nth"], c["rmin"], c["rmax"], c["m"], d["center"], d["width"],
                        inputs.seeded_amplitude(d["seed"]))


def close(got, want, what, tol=TOL64):
    got, want = np.asarray(got), np.asarray(want)
    assert np.all(np.isfinite(got)), what
    r = np.linalg.norm(got - want) / np.linalg.norm(want)
    e = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"  {what}: rel L2 {r:.2e}, max elem {e:.2e}", flush=True)
    assert r <= tol and e <= tol, (what, r, e)


@pytest.mark.parametrize("name", NAMES)
def test_long_run_matches_the_oracle(name):
    import torch
    from paper_0909_4039_amd.solver import Solver
    c, g = load(name)
    print(f"[gpu] long parity {name}: {c['n']} steps, dt = {c['dt']!r}", flush=True)
    phi, pi = initial_data(c)
    s = Solver(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], c["dt"])
    s.set_source(c["r0"], c["amp"])
    s.set_state(phi, pi)
    del phi, pi
    s.set_observer(c["robs"], c["n"] + 1)
    s.step(c["n"])
    torch.cuda.synchronize()
    s.check_finite()
    c0, c1 = c["cols"]
    gp = s.phi[:, c0:c1].cpu().numpy()
    gq = s.pi[:, c0:c1].cpu().numpy()
    wave = s.wave.cpu().numpy()
    s.close()
    close(wave[np.ix_(g["wave_steps"], g["wave_rows"])], g["wave"], "waveform")
    cols = g["cols"] - c0
    sp, sq = gp[np.ix_(g["rows"], cols)], gq[np.ix_(g["rows"], cols)]
    # the state u = (Phi, Pi) of Eq. (9) as one vector, and Phi on its own
    close(np.concatenate([sp.ravel(), sq.ravel()]), np.concatenate([g["phi_sample"].ravel(), g["pi_sample"].ravel()]),
          "state sample")
    close(sp, g["phi_sample"], "Phi sample")
    # Pi on its own: for outgoing waves Pi = d_t Phi + b d_* Phi nearly
    # cancels, so its relative rounding error runs several times Phi's (1.2e-12
    # after the 50,000 steps of the 8192 x 256 workload, against 5e-14 for Phi)
    close(sq, g["pi_sample"], "Pi sample", tol=1e-11)
    norms = np.array([np.linalg.norm(gp), np.linalg.norm(gq)])
    assert np.all(np.abs(norms - g["norms"]) <= TOL64 * np.linalg.norm(g["norms"])), (norms, g["norms"])
    for k in range(c["n_proj"]):
        w = inputs.projection_weights(gp.shape, seed=c["proj_seed0"] + k)
        rms = np.sqrt(np.mean(np.abs(w) ** 2))
        for f, (u, want) in enumerate(((gp, g["proj"][k, 0]), (gq, g["proj"][k, 1]))):
            err = abs(np.vdot(w, u) - want) / (np.linalg.norm(g["norms"]) * rms)   # relative to |u|
            assert err <= 5 * TOL64, (k, f, err)
