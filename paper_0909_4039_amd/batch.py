"""Python binding of libteuk's batches: many independent m-modes stepped by
one persistent launch per step (FP64), optionally replayed from a captured
HIP graph.  PyTorch provides the device memory and the stream; argument
marshalling only.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import TeukDesc, TeukError, TeukGrid


def _check(code, b=None):
    if code < 0:
        msg = _lib.lib().teuk_batch_last_error(b).decode() if b else ""
        raise TeukError(code, msg)
    return code


def make_desc(nr, nth, rstar_min, rstar_max, a, m, dt, s=-2, M=1.0, r0=0.0, amp=0.0, rstar_obs=None,
              sigma_r_cells=2.0, sigma_th_cells=2.0) -> TeukDesc:
    if rstar_obs is None:
        rstar_obs = 0.5 * (rstar_min + rstar_max)
    return TeukDesc(TeukGrid(int(nr), int(nth), float(rstar_min), float(rstar_max)), float(a), float(M), int(m),
                    int(s), float(dt), float(r0), float(amp), float(sigma_r_cells), float(sigma_th_cells),
                    float(rstar_obs))


class Batch:
    """Instances described by ``descs`` (``make_desc``), each with its own
    state tensors (complex128, (n_theta, n_rstar)) and a waveform tensor of
    ``wave_rows`` rows (default max_steps + 1; 0: no recording)."""

    def __init__(self, descs, max_steps, wave_rows=None, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("teuk.Batch needs a GPU")
        self.device = torch.device(device if device is not None else "cuda:0")
        self.n = len(descs)
        self.descs = list(descs)
        rows = int(max_steps) + 1 if wave_rows is None else int(wave_rows)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device)   # default priority; graph capture needs a real stream
            arr = (TeukDesc * self.n)(*self.descs)
            b = ctypes.c_void_p()
            _check(_lib.lib().teuk_batch_create(self.n, arr, int(max_steps), ctypes.c_void_p(self.stream.cuda_stream),
                                                ctypes.byref(b)))
            self._b = b
            self._bufs, self.waves = [], []
            for i, d in enumerate(self.descs):
                shape = (d.grid.n_theta, d.grid.n_rstar)
                bufs = [torch.zeros(shape, dtype=torch.complex128, device=self.device) for _ in range(4)]
                w = torch.zeros((rows, shape[0]), dtype=torch.complex128, device=self.device) if rows > 0 else None
                self._bufs.append(bufs)
                self.waves.append(w)
                _check(_lib.lib().teuk_batch_bind(self._b, i, *[t.data_ptr() for t in bufs],
                                                  w.data_ptr() if w is not None else None, rows), self._b)
            torch.cuda.synchronize(self.device)

    def _cur(self):
        return _check(_lib.lib().teuk_batch_current(self._b), self._b)

    def phi(self, i):
        """Instance i's latest Phi; the batch writes it on its own stream, so
        call ``synchronize`` before reading it on another."""
        return self._bufs[i][2 * self._cur()]

    def pi(self, i):
        return self._bufs[i][2 * self._cur() + 1]

    def set_state(self, i, phi, pi):
        """Copy (phi, pi) into instance i's current pair on the batch's stream,
        ordered after work already queued on the caller's current stream."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            self.phi(i).copy_(torch.as_tensor(phi).to(self.device, torch.complex128))
            self.pi(i).copy_(torch.as_tensor(pi).to(self.device, torch.complex128))

    def set_trajectory(self, i, r0_phase):
        """Moving source for instance i: r0_phase[k] = (r0, phi) at t = k dt/2
        from the batch's step 0 (numpy (n, 2), n >= 2 max_steps); None: its
        fixed orbit."""
        if r0_phase is None:
            _check(_lib.lib().teuk_batch_set_trajectory(self._b, int(i), None, 0), self._b)
            return
        import numpy as np
        tab = np.ascontiguousarray(r0_phase, dtype=np.float64)
        if tab.ndim != 2 or tab.shape[1] != 2:
            raise ValueError("r0_phase must have shape (n, 2)")
        _check(_lib.lib().teuk_batch_set_trajectory(self._b, int(i), tab.ctypes.data_as(ctypes.c_void_p),
                                                    tab.shape[0]), self._b)

    def step(self, n):
        _check(_lib.lib().teuk_batch_step(self._b, int(n)), self._b)

    def capture_graph(self, steps_per_graph):
        _check(_lib.lib().teuk_batch_capture_graph(self._b, int(steps_per_graph)), self._b)

    def set_tiling(self, rows_per_wave, steps_per_launch=2, persistent=True):
        _check(_lib.lib().teuk_batch_set_tiling(self._b, int(rows_per_wave), int(steps_per_launch),
                                                int(bool(persistent))), self._b)

    def autotune(self, launches_per_trial=10):
        """Returns (rows, steps_per_launch, persistent) of the fastest candidate."""
        r = ctypes.c_int32()
        k = ctypes.c_int32()
        p = ctypes.c_int32()
        _check(_lib.lib().teuk_batch_autotune(self._b, int(launches_per_trial), ctypes.byref(r), ctypes.byref(k),
                                              ctypes.byref(p)), self._b)
        return r.value, k.value, bool(p.value)

    def get_step(self):
        v = ctypes.c_int64()
        _check(_lib.lib().teuk_batch_get_step(self._b, ctypes.byref(v)), self._b)
        return v.value

    def set_watchdog(self, on=True, max_abs=0.0):
        """End every ``step`` with a scan of each instance for values not below
        ``max_abs`` in magnitude (0: non-finite only); a finding makes later
        calls raise TeukError(EUNSTABLE)."""
        _check(_lib.lib().teuk_batch_set_watchdog(self._b, int(bool(on)), float(max_abs)), self._b)

    def status(self):
        return _lib.lib().teuk_batch_status(self._b)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "_b", None):
            _lib.lib().teuk_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
