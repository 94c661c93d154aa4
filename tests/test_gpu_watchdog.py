"""The watchdog of teuk_set_watchdog: scans inside teuk_step for values not
below a bound (or not finite), reported as the sticky TEUK_EUNSTABLE by a
later call.  The conditions are forced from the host (a NaN written into the
bound state, a bound below the state's size) or come from a configuration
with a known growing mode; every kernel runs to its normal end.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def small_solver(prec=64):
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    nr, nth, rmin, rmax, a, m, s = 190, 37, -60.0, 140.0, 0.9, 2, -2
    dt = suggest_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 1000)
    sol = Solver(nr, nth, rmin, rmax, a, 1.0, m, s, dt, prec=prec)
    sol.set_source(9.0, 1.0)
    return sol


@pytest.mark.parametrize("prec", [64, 32])
def test_watchdog_leaves_results_bitwise_unchanged(prec):
    import torch
    phi, pi = inputs.random_state(190, 37, 3)
    out = []
    for every in (0, 7, 1):
        sol = small_solver(prec)
        sol.set_state(phi, pi)
        sol.set_observer(60.0, 42)
        sol.set_watchdog(every, 1e30)
        sol.step(41)
        torch.cuda.synchronize()
        assert sol.status() == _lib.OK
        out.append((sol.phi.cpu().numpy(), sol.pi.cpu().numpy(), sol.wave.cpu().numpy()))
        sol.close()
    for o in out[1:]:
        for x, y in zip(out[0], o):
            assert np.array_equal(x, y)


def test_watchdog_reports_a_nan_written_into_the_state():
    import torch
    sol = small_solver()
    phi, pi = inputs.random_state(190, 37, 4)
    phi[20, 100] = np.nan
    sol.set_state(phi, pi)
    sol.set_watchdog(5, 0.0)
    sol.step(12)                      # scans at steps 5 and 10
    torch.cuda.synchronize()
    assert sol.status() == _lib.EUNSTABLE
    with pytest.raises(_lib.TeukError) as e:
        sol.step(1)
    assert e.value.code == _lib.EUNSTABLE and "at step 5" in str(e.value)
    sol.close()


def test_watchdog_bound_and_reset():
    import torch
    sol = small_solver()
    phi, pi = inputs.random_state(190, 37, 5)   # |parts| of order 1
    sol.set_state(phi, pi)
    sol.set_watchdog(4, 1e6)
    sol.step(9)
    torch.cuda.synchronize()
    assert sol.status() == _lib.OK
    sol.set_watchdog(4, 0.5)                     # below the state's size: the next scan trips
    sol.step(3)                                  # step 9 -> 12: a scan at 12
    torch.cuda.synchronize()
    with pytest.raises(_lib.TeukError) as e:
        sol.step(1)
    assert e.value.code == _lib.EUNSTABLE and "at step 12" in str(e.value)
    # the error is sticky: no reset clears it
    with pytest.raises(_lib.TeukError):
        sol.set_watchdog(0, 0.0)
    sol.close()
    # an unread finding is dropped by a new setting
    sol = small_solver()
    sol.set_state(phi, pi)
    sol.set_watchdog(2, 0.5)
    sol.step(2)
    torch.cuda.synchronize()
    sol.set_watchdog(0, 0.0)
    sol.step(2)
    torch.cuda.synchronize()
    assert sol.status() == _lib.OK
    sol.close()
    with pytest.raises(_lib.TeukError) as e:
        small_solver().set_watchdog(-1, 1.0)
    assert e.value.code == _lib.EINVAL


@pytest.mark.parametrize("nr,nth,trips", [(4096, 256, True), (8192, 64, False)], ids=["4096x256", "8192x64"])
def test_watchdog_catches_the_growing_mode(nr, nth, trips):
    """The circular-orbit source at r0 = 10 (2 cells wide) on r* in [-100, 400]
    with a = 0.9 and 256 theta rows (dt/dr* = 0.003) seeds a poorly resolved
    mode at the potential peak.  |Phi| reaches about 70 by t = 100 M and 2e4 by
    150 M; Pi, which carries the mode's r* derivative, is larger by about
    2/dr*, so the bound 1e3 is passed between t = 80 and 150 M.  With 64 theta
    rows and 8192 r* nodes (dt/dr* = 0.024) the run stays below it."""
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    rmin, rmax, a, m, s = -100.0, 400.0, 0.9, 2, -2
    dt = suggest_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 1_200_000)
    sol = Solver(nr, nth, rmin, rmax, a, 1.0, m, s, dt)
    zero = np.zeros((nth, nr), dtype=np.complex128)
    sol.set_state(zero, zero)
    sol.set_source(10.0, 1.0)
    every = int(round(2.0 / dt))               # a scan every 2 M
    sol.set_watchdog(every, 1e3)
    n_total = int(200.0 / dt)
    chunk = 25 * every
    for done in range(0, n_total, chunk):
        try:
            sol.step(min(chunk, n_total - done))
        except _lib.TeukError as e:
            assert e.code == _lib.EUNSTABLE
            break
        torch.cuda.synchronize()
        print(f"[gpu] watchdog run {nr}x{nth}: t = {(done + chunk) * dt:.0f} M, status {sol.status()}", flush=True)
    torch.cuda.synchronize()
    status = sol.status()
    msg = _lib.lib().teuk_last_error(sol._ctx).decode()
    print(f"[gpu] watchdog {nr}x{nth}: status {status} {msg}", flush=True)
    if trips:
        assert status == _lib.EUNSTABLE
        step = int(msg.rsplit("at step ", 1)[1])
        assert 80.0 <= step * dt <= 150.0, step * dt
    else:
        assert status == _lib.OK
    sol.close()


def test_batch_watchdog_names_the_instance():
    import torch
    from paper_0909_4039_amd import batch as B
    from paper_0909_4039_amd.solver import suggest_dt
    descs = []
    for m, (nr, nth) in zip((1, 2, 3), ((160, 24), (200, 33), (140, 20))):
        dt = suggest_dt(nr, nth, -60.0, 140.0, 0.5, 1.0, m, -2, 200)
        descs.append(B.make_desc(nr, nth, -60.0, 140.0, 0.5, m, dt, r0=9.0, amp=1.0, rstar_obs=60.0))
    states = [inputs.random_state(d.grid.n_rstar, d.grid.n_theta, 20 + i) for i, d in enumerate(descs)]
    # reference: no watchdog
    ref = B.Batch(descs, 40)
    for i, (p, q) in enumerate(states):
        ref.set_state(i, p, q)
    ref.step(10)
    torch.cuda.synchronize()
    want = [ref.phi(i).cpu().numpy() for i in range(3)]
    ref.close()
    bt = B.Batch(descs, 40)
    for i, (p, q) in enumerate(states):
        bt.set_state(i, p, q)
    bt.set_watchdog(True, 1e30)
    bt.step(10)
    torch.cuda.synchronize()
    assert bt.status() == _lib.OK
    for i in range(3):
        assert np.array_equal(bt.phi(i).cpu().numpy(), want[i])
    # a NaN written into instance 1 is named with the step of the scan
    p1 = bt.phi(1)
    p1[5, 50] = float("nan")
    torch.cuda.synchronize()
    bt.step(4)
    torch.cuda.synchronize()
    with pytest.raises(_lib.TeukError) as e:
        bt.step(1)
    assert e.value.code == _lib.EUNSTABLE
    assert "instance 1" in str(e.value) and "at step 14" in str(e.value), str(e.value)
    bt.close()
