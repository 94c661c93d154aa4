"""Checkpoint and resume: Solver.state_dict / load_state_dict around
teuk_get_clock / teuk_set_clock and teuk_set_trajectory.  A run of 2n steps
equals n steps, a checkpoint written with torch.save and read back with
torch.load(weights_only=True) into a fresh solver, and n more steps, bit for
bit, for a fixed orbit and for an inspiral.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu

NR, NTH, RMIN, RMAX, A, M, MM, S = 190, 37, -60.0, 140.0, 0.9, 1.0, 2, -2


def make(dt, prec=64):
    from paper_0909_4039_amd.solver import Solver
    return Solver(NR, NTH, RMIN, RMAX, A, M, MM, S, dt, prec=prec)


@pytest.mark.parametrize("inspiral,prec", [(False, 64), (True, 64), (True, 32)],
                         ids=["fixed_orbit", "inspiral", "inspiral_fp32"])
def test_resume_from_a_saved_checkpoint_is_bitwise(tmp_path, inspiral, prec):
    import torch
    from paper_0909_4039_amd.solver import suggest_dt
    n = 30
    dt = suggest_dt(NR, NTH, RMIN, RMAX, A, M, MM, S, 1000)
    phi, pi = inputs.random_state(NR, NTH, 31)
    a = make(dt, prec)
    a.set_source(9.0, 1.0)
    if inspiral:
        a.set_trajectory(inputs.inspiral_trajectory(9.0, A, M, 0.05, dt, 2 * n))
    a.set_state(phi, pi)
    a.step(n)
    torch.save(a.state_dict(), tmp_path / "ckpt.pt")
    a.set_observer(60.0, n + 1)
    a.step(n)
    torch.cuda.synchronize()
    want = (a.phi.cpu().numpy(), a.pi.cpu().numpy(), a.wave.cpu().numpy(), a.get_time(), a.get_clock())
    a.close()

    b = make(dt, prec)
    b.load_state_dict(torch.load(tmp_path / "ckpt.pt", weights_only=True))
    b.set_observer(60.0, n + 1)
    b.step(n)
    torch.cuda.synchronize()
    got = (b.phi.cpu().numpy(), b.pi.cpu().numpy(), b.wave.cpu().numpy(), b.get_time(), b.get_clock())
    for x, y in zip(want[:3], got[:3]):
        assert np.array_equal(x, y)
    assert got[3] == want[3]
    # the resumed run keeps the saved run's time base (rebasing it at the
    # checkpoint would round the later step times, so the source's phases,
    # differently)
    assert got[4] == want[4]
    # a checkpoint of another run does not load
    c = make(dt, 96 - prec)                       # the other precision
    with pytest.raises(ValueError):
        c.load_state_dict(torch.load(tmp_path / "ckpt.pt", weights_only=True))
    b.close()
    c.close()


def test_checkpoint_after_relabelling_the_step_keeps_the_orbit(tmp_path):
    # set_time relabels steps; the orbit table stays attached to the same
    # steps, so a checkpoint taken after a relabel holds the unused entries.
    import torch
    from paper_0909_4039_amd.solver import suggest_dt
    n = 24
    dt = suggest_dt(NR, NTH, RMIN, RMAX, A, M, MM, S, 1000)
    phi, pi = inputs.random_state(NR, NTH, 32)
    a = make(dt)
    a.set_source(9.0, 1.0)
    a.set_trajectory(inputs.inspiral_trajectory(9.0, A, M, 0.05, dt, 3 * n))
    a.set_state(phi, pi)
    a.step(n)
    t, _ = a.get_time()
    a.set_time(t, 1000)                 # relabel the current step
    a.step(n // 2)
    torch.save(a.state_dict(), tmp_path / "ckpt.pt")
    a.step(n)
    torch.cuda.synchronize()
    want = (a.phi.cpu().numpy(), a.pi.cpu().numpy(), a.get_time())
    a.close()

    b = make(dt)
    d = torch.load(tmp_path / "ckpt.pt", weights_only=True)
    assert d["step"] == 1000 + n // 2
    assert d["trajectory"].shape[0] == 2 * (3 * n - n - n // 2) + 1
    b.load_state_dict(d)
    b.step(n)
    torch.cuda.synchronize()
    got = (b.phi.cpu().numpy(), b.pi.cpu().numpy(), b.get_time())
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])
    assert got[2] == want[2]
    b.close()


def test_clock_calls():
    # teuk_get_clock / teuk_set_clock: step k's time is t0 + (k - step0) dt;
    # set_time(t, s) is set_clock(t, s, s); a non-finite t0 is refused; the
    # orbit table stays attached to the same steps across a clock change
    import torch
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.solver import suggest_dt
    dt = suggest_dt(NR, NTH, RMIN, RMAX, A, M, MM, S, 1000)
    a = make(dt)
    a.set_source(9.0, 1.0)
    a.set_state(*inputs.random_state(NR, NTH, 33))
    assert a.get_clock() == (0.0, 0, 0)
    a.step(3)
    assert a.get_clock() == (0.0, 0, 3) and a.get_time() == (3 * dt, 3)
    a.set_clock(1.25, 10, 14)
    assert a.get_clock() == (1.25, 10, 14)
    assert a.get_time() == (1.25 + 4 * dt, 14)
    a.step(2)
    assert a.get_time() == (1.25 + 6 * dt, 16)
    a.set_time(2.5, 7)
    assert a.get_clock() == (2.5, 7, 7) and a.get_time() == (2.5, 7)
    with pytest.raises(TeukError) as e:
        a.set_clock(float("nan"), 0, 0)
    assert e.value.code == -1
    assert a.get_clock() == (2.5, 7, 7)
    # the orbit table: 4 steps' entries from the current step; moving the
    # current step by set_clock moves the table's first step with it
    a.set_trajectory(inputs.inspiral_trajectory(9.0, A, M, 0.05, dt, 4))
    a.set_clock(0.0, 0, 100)
    a.step(4)
    with pytest.raises(TeukError):
        a.step(1)                        # past the table
    torch.cuda.synchronize()
    a.check_finite()
    a.close()


def test_autotune_cache_reuses_a_choice(tmp_path):
    import torch
    from paper_0909_4039_amd import tune_cache
    from paper_0909_4039_amd.solver import suggest_dt
    dt = suggest_dt(NR, NTH, RMIN, RMAX, A, M, MM, S, 1000)
    path = str(tmp_path / "tune.json")
    a = make(dt)
    choice = a.autotune(3, cache=path)
    form = a.get_tiling()[1]
    a.close()
    k = tune_cache.key(torch.cuda.get_device_name(0), 64, (NTH, NR), "step")
    assert tune_cache.lookup(path, k) == list(choice) + [form]
    # a planted entry is applied as it is, without trials
    tune_cache.store(path, k, (5, 1))
    b = make(dt)
    assert b.autotune(3, cache=path) == (5, 1)
    assert b.get_tiling()[0] == 5 and b.get_blocking() == 1
    b.close()
