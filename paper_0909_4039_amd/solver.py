"""Python binding of libteuk: one m-mode Teukolsky solver on one GPU.

PyTorch provides the device memory (the four state tensors, the waveform
buffer) and the stream; every step of the method runs in the library's HIP
kernels.  Argument marshalling only.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import FP64, TeukGrid, check


def suggest_dt(nr, nth, rstar_min, rstar_max, a, M, m, s, n_steps) -> float:
    g = TeukGrid(nr, nth, rstar_min, rstar_max)
    out = ctypes.c_double(0.0)
    check(_lib.lib().teuk_suggest_dt(ctypes.byref(g), a, M, m, s, int(n_steps), ctypes.byref(out)))
    return out.value


def rstar_of_r(r, a, M=1.0) -> float:
    return _lib.lib().teuk_rstar_of_r(r, a, M)


def delta_of_rstar(rstar, a, M=1.0) -> float:
    return _lib.lib().teuk_delta_of_rstar(rstar, a, M)


class Solver:
    """Lax-Wendroff evolution of (Phi, Pi) for one (a, M, m, s) mode.

    State tensors are complex128 (prec=64) or complex64 (prec=32, and prec=48:
    FP32 storage with FP64 arithmetic) of shape
    (n_theta, n_rstar), r* contiguous, owned by this object and bound to the
    library; ``phi``/``pi`` return the pair that holds the latest state.
    """

    def __init__(self, nr, nth, rstar_min, rstar_max, a, M, m, s, dt, prec=64, device=None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("teuk.Solver needs a GPU")
        self.device = torch.device(device if device is not None else "cuda:0")
        self.prec = int(prec)
        self.dtype = torch.complex128 if self.prec == FP64 else torch.complex64
        self.shape = (int(nth), int(nr))
        self.params = dict(nr=nr, nth=nth, rstar_min=rstar_min, rstar_max=rstar_max, a=a, M=M, m=m, s=s, dt=dt)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            with torch.cuda.stream(self.stream):  # zero fill ordered before the library's launches
                self._bufs = [torch.zeros(self.shape, dtype=self.dtype, device=self.device) for _ in range(4)]
            g = TeukGrid(nr, nth, rstar_min, rstar_max)
            ctx = ctypes.c_void_p()
            check(_lib.lib().teuk_create(ctypes.byref(g), a, M, m, s, dt, self.prec,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
            self._ctx = ctx
            check(_lib.lib().teuk_bind_state(self._ctx, *[b.data_ptr() for b in self._bufs]), self._ctx)
        self.wave = None
        self.source = None
        self.trajectory = None

    # ------------------------------------------------------------ state
    def _cur(self):
        return check_int(_lib.lib().teuk_current(self._ctx))

    @property
    def phi(self):
        return self._bufs[2 * self._cur()]

    @property
    def pi(self):
        return self._bufs[2 * self._cur() + 1]

    def set_state(self, phi, pi):
        """Copy (phi, pi) into the current state buffers (on the solver's stream,
        ordered after work already queued on the caller's current stream)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            self.phi.copy_(torch.as_tensor(phi).to(self.device, self.dtype))
            self.pi.copy_(torch.as_tensor(pi).to(self.device, self.dtype))

    def state_dict(self):
        """A checkpoint from which a fresh Solver of the same grid, mode, dt and
        precision continues this run bit for bit: host copies of the current
        state, the time, the clock (see get_clock) and step count, the source,
        and the part of the orbit table not used yet.  Tensors and plain
        Python values only, so ``torch.save`` / ``torch.load(weights_only=True)``
        round-trip it."""
        self.stream.synchronize()
        t, step = self.get_time()
        t0, step0, _ = self.get_clock()
        d = {"params": dict(self.params, prec=self.prec), "phi": self.phi.cpu(), "pi": self.pi.cpu(),
             "t": t, "step": step, "t0": t0, "step0": step0, "source": self.source, "trajectory": None}
        if self.trajectory is not None:
            used = 2 * (step - self._traj_step0)   # entries consumed by the steps taken since the table was set
            if used < 0:
                raise RuntimeError("the orbit table starts after the current step")
            d["trajectory"] = torch.from_numpy(self.trajectory[used:].copy())
        return d

    def load_state_dict(self, d):
        """Continue from a ``state_dict`` of a run with the same grid, mode, dt
        and precision (ValueError otherwise).  The observer is not part of it."""
        mine = dict(self.params, prec=self.prec)
        if {k: d["params"].get(k) for k in mine} != mine:
            raise ValueError(f"checkpoint of {d['params']} does not match this solver {mine}")
        self.set_state(d["phi"], d["pi"])
        # the clock's base, not the current time: the steps that follow form
        # their times (and the source's phases) as the saved run would have
        self.set_clock(d["t0"], d["step0"], d["step"])
        if d["source"] is not None:
            self.set_source(*d["source"])
        self.set_trajectory(None if d["trajectory"] is None else d["trajectory"].numpy())

    # ------------------------------------------------------------ physics
    def set_source(self, r0, amp, sigma_r_cells=2.0, sigma_th_cells=2.0):
        check(_lib.lib().teuk_set_source(self._ctx, r0, amp, sigma_r_cells, sigma_th_cells), self._ctx)
        self.source = (float(r0), float(amp), float(sigma_r_cells), float(sigma_th_cells))

    def set_trajectory(self, r0_phase):
        """Moving source: r0_phase[k] = (r0, phi) at t_now + k dt/2 (numpy (n, 2)); None: fixed orbit."""
        if r0_phase is None:
            check(_lib.lib().teuk_set_trajectory(self._ctx, None, 0), self._ctx)
            self.trajectory = None
            return
        import numpy as np
        tab = np.ascontiguousarray(r0_phase, dtype=np.float64)
        if tab.ndim != 2 or tab.shape[1] != 2:
            raise ValueError("r0_phase must have shape (n, 2)")
        check(_lib.lib().teuk_set_trajectory(self._ctx, tab.ctypes.data_as(ctypes.c_void_p), tab.shape[0]),
              self._ctx)
        self.trajectory = tab
        self._traj_step0 = self.get_time()[1]

    def set_observer(self, rstar_obs, capacity_rows):
        """Record the waveform at rstar_obs into a new (capacity_rows, n_theta) tensor."""
        with torch.cuda.stream(self.stream):
            self.wave = torch.zeros((int(capacity_rows), self.shape[0]), dtype=self.dtype, device=self.device)
        check(_lib.lib().teuk_set_observer(self._ctx, rstar_obs, self.wave.data_ptr(), int(capacity_rows)),
              self._ctx)
        return self.wave

    def clear_observer(self):
        check(_lib.lib().teuk_set_observer(self._ctx, 0.0, None, 0), self._ctx)
        self.wave = None

    def step(self, n):
        check(_lib.lib().teuk_step(self._ctx, int(n)), self._ctx)

    def extract(self, rstar_obs):
        with torch.cuda.stream(self.stream):
            out = torch.empty((self.shape[0],), dtype=self.dtype, device=self.device)
        check(_lib.lib().teuk_extract(self._ctx, rstar_obs, out.data_ptr()), self._ctx)
        return out

    def get_time(self):
        t = ctypes.c_double()
        n = ctypes.c_int64()
        check(_lib.lib().teuk_get_time(self._ctx, ctypes.byref(t), ctypes.byref(n)), self._ctx)
        return t.value, n.value

    def set_time(self, t, step):
        """Relabel the current step and time.  As in the library, the orbit
        table stays attached to the same steps, so its first step moves by the
        same amount."""
        old = self.get_time()[1]
        check(_lib.lib().teuk_set_time(self._ctx, float(t), int(step)), self._ctx)
        if self.trajectory is not None:
            self._traj_step0 += int(step) - old

    def get_clock(self):
        """(t0, step0, step): the time base (t0 at step step0) from which step
        k's time is t0 + (k - step0) dt, and the current step."""
        t0 = ctypes.c_double()
        n0 = ctypes.c_int64()
        n = ctypes.c_int64()
        check(_lib.lib().teuk_get_clock(self._ctx, ctypes.byref(t0), ctypes.byref(n0), ctypes.byref(n)), self._ctx)
        return t0.value, n0.value, n.value

    def set_clock(self, t0, step0, step):
        """Set the time base and the current step (see get_clock); the orbit
        table moves with the current step as in set_time."""
        old = self.get_time()[1]
        check(_lib.lib().teuk_set_clock(self._ctx, float(t0), int(step0), int(step)), self._ctx)
        if self.trajectory is not None:
            self._traj_step0 += int(step) - old

    def set_tiling(self, rows_per_wave, order=0):
        check(_lib.lib().teuk_set_tiling(self._ctx, int(rows_per_wave), int(order)), self._ctx)

    def set_blocking(self, steps_per_launch):
        """Fuse 1 or 2 steps per kernel launch (bitwise identical results)."""
        check(_lib.lib().teuk_set_blocking(self._ctx, int(steps_per_launch)), self._ctx)

    def get_blocking(self):
        return check_int(_lib.lib().teuk_get_blocking(self._ctx))

    def autotune(self, launches_per_trial=20, cache=None):
        """Pick the fastest (theta rows per wave, steps per launch, launch form)
        by timing trial launches on the bound state; returns (rows,
        steps_per_launch) and ``get_tiling`` reports the form (order).  Results
        of ``step`` are bitwise identical for every choice.  With a cache file
        (``cache`` or the TEUK_TUNE_CACHE environment variable) a choice found
        earlier for this grid, precision and GPU model is applied without
        trials, and a new one is recorded."""
        from . import tune_cache
        path = tune_cache.cache_path(cache)
        k_ = tune_cache.key(torch.cuda.get_device_name(self.device), self.prec, self.shape, "step")
        hit = tune_cache.lookup(path, k_)
        if hit is not None and len(hit) in (2, 3):
            self.set_tiling(hit[0], hit[2] if len(hit) == 3 else 0)
            self.set_blocking(hit[1])
            return hit[0], hit[1]
        r = ctypes.c_int32()
        k = ctypes.c_int32()
        check(_lib.lib().teuk_autotune(self._ctx, int(launches_per_trial), ctypes.byref(r), ctypes.byref(k)),
              self._ctx)
        tune_cache.store(path, k_, (r.value, k.value, self.get_tiling()[1]))
        return r.value, k.value

    def get_tiling(self):
        r = ctypes.c_int32()
        o = ctypes.c_int32()
        check(_lib.lib().teuk_get_tiling(self._ctx, ctypes.byref(r), ctypes.byref(o)), self._ctx)
        return r.value, o.value

    def set_adjoint_tiling(self, rows_per_wave=0, steps_per_launch=1):
        """Tile shape of the reverse sweep (rows 0: follow the step kernel's)."""
        check(_lib.lib().teuk_set_adjoint_tiling(self._ctx, int(rows_per_wave), int(steps_per_launch)), self._ctx)

    def get_adjoint_tiling(self):
        r = ctypes.c_int32()
        k = ctypes.c_int32()
        check(_lib.lib().teuk_get_adjoint_tiling(self._ctx, ctypes.byref(r), ctypes.byref(k)), self._ctx)
        return r.value, k.value

    def adjoint_workspace_bytes(self):
        return check_int(_lib.lib().teuk_adjoint_workspace_bytes(self._ctx))

    def adjoint_autotune(self, launches_per_trial=10):
        """Pick the fastest reverse-sweep tiling by timing trial reverse steps
        on the bound state (left unchanged); returns (rows, steps_per_launch)."""
        r = ctypes.c_int32()
        k = ctypes.c_int32()
        check(_lib.lib().teuk_adjoint_autotune(self._ctx, int(launches_per_trial), ctypes.byref(r),
                                               ctypes.byref(k)), self._ctx)
        return r.value, k.value

    def adjoint(self, dL_dwave, n_steps, rstar_obs, t_start=0.0):
        """Reverse sweep of the library (FP64): gradients of a real loss of the
        waveform w^0..w^n recorded at rstar_obs from initial data at t_start.

        ``dL_dwave`` is (n_steps + 1, n_theta) complex, dL/dRe w + i dL/dIm w.
        Returns (dL/dPhi0, dL/dPi0, dL/dr0, dL/damp) in the same convention;
        the source is the one last given to ``set_source``.
        """
        n = int(n_steps)
        g = torch.as_tensor(dL_dwave).to(self.device, torch.complex128).contiguous()
        if g.shape != (n + 1, self.shape[0]):
            raise ValueError(f"dL_dwave has shape {tuple(g.shape)}, expected {(n + 1, self.shape[0])}")
        nbytes = self.adjoint_workspace_bytes()
        ws = torch.empty((nbytes + 255) // 8 + 32, dtype=torch.float64, device=self.device)
        base = ws.data_ptr()
        off = (-base) % 256
        dphi = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        dpi = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        dr0 = ctypes.c_double()
        damp = ctypes.c_double()
        with torch.cuda.device(self.device):
            # the library works on its own stream; order it after the producers of g
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            check(_lib.lib().teuk_adjoint(self._ctx, float(rstar_obs), g.data_ptr(), n, float(t_start),
                                          ctypes.c_void_p(base + off), int(ws.numel() * 8 - off),
                                          dphi.data_ptr(), dpi.data_ptr(), ctypes.byref(dr0), ctypes.byref(damp)),
                  self._ctx)
        return dphi, dpi, dr0.value, damp.value

    def adjoint_moving(self, dL_dwave, n_steps, rstar_obs):
        """Reverse sweep for the orbit table of ``set_trajectory`` (FP64), the
        forward run having started at its first entry.  Returns (dL/dPhi0,
        dL/dPi0, dL/dtraj, dL/damp) with dL/dtraj a float64 numpy array
        (2 n_steps, 2): row e = (dL/dr0_e, dL/dphi_e)."""
        import numpy as np
        n = int(n_steps)
        g = torch.as_tensor(dL_dwave).to(self.device, torch.complex128).contiguous()
        if g.shape != (n + 1, self.shape[0]):
            raise ValueError(f"dL_dwave has shape {tuple(g.shape)}, expected {(n + 1, self.shape[0])}")
        nbytes = self.adjoint_workspace_bytes()
        ws = torch.empty((nbytes + 255) // 8 + 32, dtype=torch.float64, device=self.device)
        base = ws.data_ptr()
        off = (-base) % 256
        dphi = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        dpi = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        dtraj = np.zeros((max(2 * n, 1), 2), dtype=np.float64)
        damp = ctypes.c_double()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            check(_lib.lib().teuk_adjoint_moving(self._ctx, float(rstar_obs), g.data_ptr(), n,
                                                 ctypes.c_void_p(base + off), int(ws.numel() * 8 - off),
                                                 dphi.data_ptr(), dpi.data_ptr(),
                                                 dtraj.ctypes.data_as(ctypes.c_void_p), ctypes.byref(damp)),
                  self._ctx)
        return dphi, dpi, dtraj[:2 * n], damp.value

    def param_gradient(self, param, dL_dwave, n_steps, rstar_obs, phi0, pi0, h=None, t_start=0.0,
                       checkpoint_interval=0, want_initial=False):
        """Gradient of a real waveform loss with respect to one parameter of the
        problem ("a", "M", "r0" or "amp"), by the library's checkpointed
        reverse sweep from the initial data (phi0, pi0) at t_start (FP64, fixed
        orbit).  dL_dwave is (n_steps + 1, n_theta) complex, as for ``adjoint``.
        h is the central-difference step of one time step's parameter
        derivative (default 1e-6 max(1, |p|)).  Returns dL/dp, or
        (dL/dp, dL/dPhi0, dL/dPi0) with want_initial."""
        names = {"a": _lib.PARAM_A, "M": _lib.PARAM_M, "r0": _lib.PARAM_R0, "amp": _lib.PARAM_AMP}
        if param not in names:
            raise ValueError(f"param must be one of {sorted(names)}")
        value = {"a": self.params["a"], "M": self.params["M"],
                 "r0": self.source[0] if self.source else 0.0, "amp": self.source[1] if self.source else 0.0}[param]
        if h is None:
            h = 1e-6 * max(1.0, abs(value))
        n = int(n_steps)
        g = torch.as_tensor(dL_dwave).to(self.device, torch.complex128).contiguous()
        if g.shape != (n + 1, self.shape[0]):
            raise ValueError(f"dL_dwave has shape {tuple(g.shape)}, expected {(n + 1, self.shape[0])}")
        p0 = torch.as_tensor(phi0).to(self.device, torch.complex128).contiguous()
        q0 = torch.as_tensor(pi0).to(self.device, torch.complex128).contiguous()
        if p0.shape != self.shape or q0.shape != self.shape:
            raise ValueError(f"initial data must have shape {self.shape}")
        nbytes = check_int(_lib.lib().teuk_param_gradient_workspace_bytes(self._ctx, n, int(checkpoint_interval)))
        ws = torch.empty((nbytes + 255) // 8 + 32, dtype=torch.float64, device=self.device)
        base = ws.data_ptr()
        off = (-base) % 256
        dphi = torch.empty(self.shape, dtype=torch.complex128, device=self.device) if want_initial else None
        dpi = torch.empty(self.shape, dtype=torch.complex128, device=self.device) if want_initial else None
        out = ctypes.c_double()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            check(_lib.lib().teuk_param_gradient(self._ctx, names[param], float(h), float(rstar_obs), g.data_ptr(), n,
                                                 float(t_start), p0.data_ptr(), q0.data_ptr(),
                                                 int(checkpoint_interval), ctypes.c_void_p(base + off),
                                                 int(ws.numel() * 8 - off), ctypes.byref(out),
                                                 dphi.data_ptr() if want_initial else None,
                                                 dpi.data_ptr() if want_initial else None), self._ctx)
        return (out.value, dphi, dpi) if want_initial else out.value

    def check_finite(self):
        """Raise TeukError(EUNSTABLE) if the state holds NaN or Inf."""
        check(_lib.lib().teuk_check_finite(self._ctx), self._ctx)

    def set_watchdog(self, every_steps, max_abs=0.0):
        """Scan the state every ``every_steps`` steps during ``step`` for values
        not below ``max_abs`` in magnitude (0: non-finite only); a finding makes
        later calls raise TeukError(EUNSTABLE).  0 turns it off."""
        check(_lib.lib().teuk_set_watchdog(self._ctx, int(every_steps), float(max_abs)), self._ctx)

    def status(self):
        return _lib.lib().teuk_status(self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.lib().teuk_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_int(v):
    if v < 0:
        raise _lib.TeukError(v)
    return v
