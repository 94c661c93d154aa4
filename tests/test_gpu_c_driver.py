"""The C example (examples/teuk_run.c) drives libteuk through its C ABI alone:
device buffers from the HIP runtime, no Python or torch in the process.  Its
final state and waveform must match the oracle to the parity bar (1e-12
relative L2 in FP64; the FP32 waveform within 1e-5 of the FP64 one).
"""
import os
import subprocess

import numpy as np
import pytest

from paper_0909_4039_amd import build as B
from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu


def run_example(tmp_path, phi, pi, args, prec=64):
    assert os.path.exists(B.EXAMPLE_BIN), "examples/teuk_run is not built: run __graft_entry__.build()"
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([phi.ravel(), pi.ravel()]).astype(np.complex128).tofile(fin)
    cmd = [B.EXAMPLE_BIN, str(fin), str(fout)] + [repr(x) if isinstance(x, float) else str(x) for x in args]
    cmd.append(str(prec))
    print("[gpu] running", " ".join(cmd[3:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return np.fromfile(fout, dtype=np.complex128)


@pytest.mark.parametrize("nr,nth,a,m,s", [(190, 37, 0.9, 2, -2), (129, 8, 0.6, 1, -1)], ids=["kerr_190x37", "odd_s_129x8"])
def test_c_example_matches_oracle(oracle_mod, tmp_path, nr, nth, a, m, s):
    rmin, rmax, r0, amp, robs, n = -60.0, 140.0, 9.0, 1.0, 60.0, 37
    dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 1000)
    phi, pi = inputs.random_state(nr, nth, 11)
    out = run_example(tmp_path, phi, pi, [nr, nth, rmin, rmax, a, 1.0, m, s, dt, r0, amp, robs, n])
    npts = nr * nth
    gp = out[:npts].reshape(nth, nr)
    gq = out[npts:2 * npts].reshape(nth, nr)
    gw = out[2 * npts:].reshape(n + 1, nth)
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, a, 1.0, m, s, dt, r0=r0, amp=amp, rstar_obs=robs)
    op, oq, ow = o.run(phi, pi, n)
    for name, g, ref in (("phi", gp, op), ("pi", gq, oq), ("wave", gw, ow)):
        err = max(np.linalg.norm(g - ref) / np.linalg.norm(ref), np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
        print(f"[gpu] C example {nr}x{nth} {name}: rel L2 {err:.2e}", flush=True)
        assert err <= 1e-12, (name, err)


def test_c_example_fp32(oracle_mod, tmp_path):
    nr, nth, rmin, rmax, a, m, s = 256, 32, -60.0, 140.0, 0.9, 2, -2
    r0, amp, robs, n = 9.0, 1.0, 60.0, 200
    dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 1000)
    phi, pi = inputs.pulse(nr, nth, rmin, rmax, m, 15.0, 4.0, inputs.seeded_amplitude(2))
    out = run_example(tmp_path, phi, pi, [nr, nth, rmin, rmax, a, 1.0, m, s, dt, r0, amp, robs, n], prec=32)
    gw = out[2 * nr * nth:].reshape(n + 1, nth)
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, a, 1.0, m, s, dt, r0=r0, amp=amp, rstar_obs=robs)
    _, _, ow = o.run(phi, pi, n)
    err = max(np.linalg.norm(gw - ow) / np.linalg.norm(ow), np.max(np.abs(gw - ow)) / np.max(np.abs(ow)))
    print(f"[gpu] C example FP32 waveform: rel L2 {err:.2e}", flush=True)
    assert err <= 1e-5


def test_c_example_reports_errors(tmp_path):
    # an invalid spin is refused by teuk_create; the example exits with status 2
    # before any step (device buffers are allocated, no kernel runs)
    nr, nth = 64, 8
    phi, pi = inputs.random_state(nr, nth, 1)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([phi.ravel(), pi.ravel()]).astype(np.complex128).tofile(fin)
    r = subprocess.run([B.EXAMPLE_BIN, str(fin), str(fout), "64", "8", "-50.0", "100.0", "0.5", "1.0", "2", "3",
                        "0.1", "9.0", "1.0", "20.0", "5"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "teuk_create" in r.stderr, (r.returncode, r.stderr)
