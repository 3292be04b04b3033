"""Python face of the engine: one Engine per (instance, stream).

Thin marshalling over the C ABI (include/teuk.h).  PyTorch only provides
device memory and the stream; every step of the evolution runs in the HIP
library.  Complex fields are torch.complex128 tensors of shape (nth, nr) on
the current HIP device.
"""

import ctypes
import os

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need_device(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128):
        raise TypeError(f"{name} must be a complex128 tensor on the HIP device")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")


def ws_request(source_footprint=(2.0, 2.0, 8.0), adjoint=True):
    """teuk_ws_request: the largest source footprint (sigma_r_cells,
    sigma_th_cells, cutoff_sigmas; None = no source) and whether the adjoint
    area is needed."""
    sr, st, cut = source_footprint if source_footprint is not None else (0.0, 0.0, 0.0)
    return L.WsRequest(float(sr), float(st), float(cut), 1 if adjoint else 0)


def device_buffer(nbytes):
    """Caller-owned device memory for the library: a torch uint8 tensor
    (torch's allocator hands out blocks aligned to at least 256 bytes)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
    if t.data_ptr() % 256 != 0:
        raise RuntimeError("device buffer not 256-byte aligned")
    return t


def grid_desc(g):
    return L.GridDesc(float(g["M"]), float(g["a"]), int(g["s"]), int(g["m"]), int(g["nr"]), int(g["nth"]),
                      float(g["rs_min"]), float(g["rs_max"]), float(g.get("cfl", 0.5)),
                      float(g["rs_max"] if g.get("rs_extract") is None else g["rs_extract"]),
                      float(g.get("ko_eps", 0.5)))


class Engine:
    """One evolving instance.

    Parameters follow teuk_grid_desc: M, a, s, m, nr, nth, rs_min, rs_max,
    cfl, rs_extract, ko_eps.  The context lives in a device workspace that
    this object owns (a torch tensor), sized by teuk_workspace_size for the
    largest source footprint it will take and, with adjoint=True, the
    reverse sweep.
    """

    def __init__(self, M, a, s, m, nr, nth, rs_min, rs_max, cfl=0.5, rs_extract=None,
                 ko_eps=0.5, stream=None, source_footprint=(2.0, 2.0, 8.0), adjoint=True):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the engine needs a HIP device")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        desc = grid_desc(dict(M=M, a=a, s=s, m=m, nr=nr, nth=nth, rs_min=rs_min, rs_max=rs_max, cfl=cfl,
                              rs_extract=rs_extract, ko_eps=ko_eps))
        req = ws_request(source_footprint, adjoint)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.teuk_workspace_size(ctypes.byref(desc), ctypes.byref(req), ctypes.byref(nbytes)))
        self._ws = device_buffer(nbytes.value)
        ctx = ctypes.c_void_p()
        L.check(self._lib.teuk_init_grid(ctypes.byref(desc), ctypes.byref(req),
                                         ctypes.c_void_p(self.stream.cuda_stream), _ptr(self._ws),
                                         nbytes.value, ctypes.byref(ctx)))
        self.ctx = ctx
        self.m = int(m)
        self._orbit = None
        self._orbit_dev = None
        self._ckpt_buf = None
        self._gw = None
        self.checkpoint_generation = 0   # counts forward_checkpointed calls

    @property
    def workspace_bytes(self):
        return self._ws.numel()

    @classmethod
    def _borrowed(cls, lib, ctx, m, stream):
        """View of a context owned elsewhere (a batch instance); close() is a no-op."""
        e = cls.__new__(cls)
        e._lib = lib
        e.stream = stream
        e.ctx = ctx
        e.m = int(m)
        e._orbit = None
        e._orbit_dev = None
        e._ckpt_buf = None
        e._gw = None
        e.checkpoint_generation = 0
        e._borrowed_ctx = True
        return e

    @property
    def has_source(self):
        return self._orbit is not None

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_borrowed_ctx", False):
            self.ctx = None
            return
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self._lib.teuk_destroy(self.ctx)
            self.ctx = None
        # the buffers go only after the context is gone
        self._orbit_dev = None
        self._ckpt_buf = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ------------------------------------------------------------
    @property
    def info(self):
        inf = L.Info()
        L.check(self._lib.teuk_get_info(self.ctx, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in L.Info._fields_}

    @property
    def shape(self):
        i = self.info
        return (i["nth"], i["nr"])

    # -- state --------------------------------------------------------------
    def set_state(self, phi, pi):
        _need_device(phi, self.shape, "phi")
        _need_device(pi, self.shape, "pi")
        L.check(self._lib.teuk_set_state(self.ctx, _ptr(phi), _ptr(pi)))

    def get_state(self):
        nth, nr = self.shape
        phi = torch.empty((nth, nr), dtype=torch.complex128, device="cuda")
        pi = torch.empty_like(phi)
        L.check(self._lib.teuk_get_state(self.ctx, _ptr(phi), _ptr(pi)))
        return phi, pi

    def init_pulse(self, center, width, amplitude=1.0):
        L.check(self._lib.teuk_init_pulse(self.ctx, float(center), float(width), float(amplitude)))

    # -- source -------------------------------------------------------------
    def orbit_circular(self, r0, nsamples, M=1.0, a=None):
        """Orbit samples (nsamples, 3) from the library's own orbit builder."""
        info = self.info
        if a is None:
            raise ValueError("pass the spin a of this instance")
        out = np.zeros((int(nsamples), 3), dtype=np.float64)
        L.check(self._lib.teuk_orbit_circular(float(M), float(a), float(r0), float(info["dt"]),
                                              int(nsamples),
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def orbit_eccentric(self, p, e, nsamples, M=1.0, a=None, chi0=0.0):
        """Eccentric equatorial orbit samples (nsamples, 3): semi-latus rectum
        p, eccentricity e, anomaly chi0 at t = 0 (0 = periapsis)."""
        info = self.info
        if a is None:
            raise ValueError("pass the spin a of this instance")
        out = np.zeros((int(nsamples), 3), dtype=np.float64)
        L.check(self._lib.teuk_orbit_eccentric(float(M), float(a), float(p), float(e), float(chi0),
                                               float(info["dt"]), int(nsamples),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_source(self, orbit, amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0,
                   cutoff_sigmas=8.0):
        if orbit is None:
            L.check(self._lib.teuk_set_source(self.ctx, None))
            self._orbit = None
            self._orbit_dev = None
            return
        orbit = np.ascontiguousarray(orbit, dtype=np.float64).reshape(-1, 3)
        dev = torch.empty(orbit.size, dtype=torch.float64, device="cuda")
        desc = L.SourceDesc(float(amplitude), float(sigma_r_cells), float(sigma_th_cells),
                            float(cutoff_sigmas), orbit.shape[0],
                            orbit.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(dev))
        L.check(self._lib.teuk_set_source(self.ctx, ctypes.byref(desc)))
        self._orbit = orbit
        self._orbit_dev = dev

    def set_amplitude(self, amplitude):
        L.check(self._lib.teuk_set_amplitude(self.ctx, float(amplitude)))

    # -- evolution ----------------------------------------------------------
    def step(self, nsteps, waveform=True, out=None):
        """Take nsteps iterations; returns the (nsteps, nth) waveform or None."""
        nth = self.shape[0]
        w = None
        if waveform:
            w = out if out is not None else torch.empty((int(nsteps), nth), dtype=torch.complex128,
                                                        device="cuda")
            _need_device(w, (int(nsteps), nth), "waveform")
        L.check(self._lib.teuk_step_n(self.ctx, int(nsteps), _ptr(w) if w is not None else None))
        return w

    def extract(self):
        nth = self.shape[0]
        w = torch.empty((nth,), dtype=torch.complex128, device="cuda")
        L.check(self._lib.teuk_extract_waveform(self.ctx, _ptr(w)))
        return w

    @property
    def tuning(self):
        t = L.Tuning()
        L.check(self._lib.teuk_get_tuning(self.ctx, ctypes.byref(t)))
        return {"seg_rows": t.seg_rows, "k_steps": t.k_steps, "adj_seg_rows": t.adj_seg_rows}

    def set_tuning(self, seg_rows, k_steps=1, adj_seg_rows=0):
        """Launch configuration: theta rows per segment and iterations per
        launch of the stepper; theta rows per segment of the adjoint (0 keeps
        the current value)."""
        t = L.Tuning(int(seg_rows), int(k_steps), int(adj_seg_rows))
        L.check(self._lib.teuk_set_tuning(self.ctx, ctypes.byref(t)))

    def autotune(self, cache_path=None):
        """Measure every launch configuration (or take it from the cache file)
        and keep the fastest; returns [(seg_rows, k_steps, us/iteration)],
        fastest first (one entry when served from the cache)."""
        cap = 16
        table = (L.TuneEntry * cap)()
        n = ctypes.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        L.check(self._lib.teuk_autotune(self.ctx, path, table, cap, ctypes.byref(n)))
        return [(table[k].seg_rows, table[k].k_steps, table[k].us_per_iteration) for k in range(n.value)]

    # -- adjoint ------------------------------------------------------------
    def adjoint_begin(self, n_end, lam_phi=None, lam_pi=None, gw=None):
        """lambda := (lam_phi, lam_pi) (None = 0) + dL/dw_{n_end}; clock := n_end."""
        shape = self.shape
        for t, name in ((lam_phi, "lam_phi"), (lam_pi, "lam_pi")):
            if t is not None:
                _need_device(t, shape, name)
        if gw is not None:
            _need_device(gw, (gw.shape[0], shape[0]), "gw")
            if gw.shape[0] < int(n_end):
                raise ValueError("gw needs a row for every forward iteration 1..n_end")
        self._gw = gw
        L.check(self._lib.teuk_adjoint_begin(self.ctx, _ptr(lam_phi) if lam_phi is not None else None,
                                             _ptr(lam_pi) if lam_pi is not None else None, int(n_end),
                                             _ptr(gw) if gw is not None else None))

    def adjoint_step(self, nsteps, gw=None):
        gw = gw if gw is not None else self._gw
        L.check(self._lib.teuk_adjoint_step_n(self.ctx, int(nsteps), _ptr(gw) if gw is not None else None))

    def adjoint_add_state(self, gphi=None, gpi=None):
        L.check(self._lib.teuk_adjoint_add_state(self.ctx, _ptr(gphi) if gphi is not None else None,
                                                 _ptr(gpi) if gpi is not None else None))

    def adjoint_get(self, want_dA=True):
        """(lambda_phi, lambda_pi, dL/dA or None)."""
        nth, nr = self.shape
        p = torch.empty((nth, nr), dtype=torch.complex128, device="cuda")
        q = torch.empty_like(p)
        dA = ctypes.c_double(0.0)
        L.check(self._lib.teuk_adjoint_get(self.ctx, _ptr(p), _ptr(q), ctypes.byref(dA) if want_dA else None))
        return p, q, (dA.value if want_dA else None)

    # -- checkpointed gradient ----------------------------------------------
    def _make_plan(self, nsteps, interval, state_loss, force_recompute, snapshots):
        sl = state_loss or {}
        return L.GradPlan(nsteps=int(nsteps), interval=int(interval), snapshots=int(snapshots),
                          state_weight=float(sl.get("weight", 0.0)),
                          i0=int(sl.get("i0", 0)), i1=int(sl.get("i1", 0)), j0=int(sl.get("j0", 0)),
                          j1=int(sl.get("j1", 0)), n_lo=int(sl.get("n_lo", 0)), n_hi=int(sl.get("n_hi", 0)),
                          force_recompute=1 if force_recompute else 0, ckpt_dev=None, ckpt_bytes=0)

    def _plan(self, nsteps, interval, state_loss, force_recompute, snapshots):
        plan = self._make_plan(nsteps, interval, state_loss, force_recompute, snapshots)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.teuk_checkpoint_size(self.ctx, ctypes.byref(plan), ctypes.byref(nbytes)))
        if self._ckpt_buf is None or self._ckpt_buf.numel() < nbytes.value:
            self._ckpt_buf = None
            self._ckpt_buf = device_buffer(nbytes.value)
        plan.ckpt_dev = self._ckpt_buf.data_ptr()
        plan.ckpt_bytes = self._ckpt_buf.numel()
        return plan

    def checkpoint_bytes(self, nsteps, interval=0, state_loss=None, snapshots=0):
        """Bytes of checkpoint buffer a checkpointed run of nsteps needs
        (uniform schedule, or binomial with `snapshots` slots)."""
        plan = self._make_plan(nsteps, interval, state_loss, False, snapshots)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.teuk_checkpoint_size(self.ctx, ctypes.byref(plan), ctypes.byref(nbytes)))
        return nbytes.value

    def snapshots_for_budget(self, nsteps, budget_bytes, state_loss=None):
        """The most binomial snapshot slots whose checkpoint buffer fits
        budget_bytes (at least 1), capped at nsteps."""
        one = self.checkpoint_bytes(nsteps, state_loss=state_loss, snapshots=1)
        per = self.checkpoint_bytes(nsteps, state_loss=state_loss, snapshots=2) - one
        return int(max(1, min(int(nsteps), 1 + (int(budget_bytes) - one) // per)))

    def forward_checkpointed(self, nsteps, interval=0, state_loss=None, force_recompute=False, snapshots=0):
        """Run nsteps iterations keeping snapshots for the reverse sweep.
        state_loss: dict(weight, i0, i1, j0, j1, n_lo, n_hi) for
        L_s = weight * sum_{n=n_lo..n_hi} sum_rect |Phi^n|^2, or None.
        snapshots 0: a snapshot every `interval` iterations (0: ceil(sqrt));
        snapshots s >= 1: the binomial schedule with at most s snapshots.
        Returns (waveform, L_s)."""
        self._ckpt = self._plan(nsteps, interval, state_loss, force_recompute, snapshots)
        self.checkpoint_generation += 1
        nth = self.shape[0]
        w = torch.empty((int(nsteps), nth), dtype=torch.complex128, device="cuda")
        ls = ctypes.c_double(0.0)
        L.check(self._lib.teuk_forward_checkpointed(self.ctx, ctypes.byref(self._ckpt), _ptr(w), ctypes.byref(ls)))
        return w, ls.value

    def backward_checkpointed(self, gw=None, dL_dLs=1.0):
        """Gradients (dL/dPhi0, dL/dPi0, dL/dA) after forward_checkpointed."""
        nth, nr = self.shape
        if gw is not None:
            _need_device(gw, (self._ckpt.nsteps, nth), "gw")
        gp = torch.empty((nth, nr), dtype=torch.complex128, device="cuda")
        gq = torch.empty_like(gp)
        dA = ctypes.c_double(0.0)
        L.check(self._lib.teuk_backward_checkpointed(self.ctx, ctypes.byref(self._ckpt),
                                                     _ptr(gw) if gw is not None else None, float(dL_dLs),
                                                     _ptr(gp), _ptr(gq), ctypes.byref(dA)))
        return gp, gq, dA.value

    def set_kernel_timing(self, enable):
        L.check(self._lib.teuk_set_kernel_timing(self.ctx, 1 if enable else 0))

    def kernel_timing(self):
        """(summed stencil-launch time in ms, number of timed launches)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.check(self._lib.teuk_kernel_timing(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def check_finite(self):
        L.check(self._lib.teuk_check_finite(self.ctx))


class Batch:
    """Many independent instances stepped together (teuk_batch_*): one
    launch per iteration covering every instance (the default), or one
    persistent graph launch per call (mode, see set_mode).

    grids: list of dicts with Engine's grid parameters.  instances[k] is an
    Engine view of instance k (set_state, init_pulse, get_state, ...)."""

    PERSISTENT = L.BATCH_PERSISTENT
    PER_ITERATION = L.BATCH_PER_ITERATION

    def __init__(self, grids, stream=None, source_footprint=(2.0, 2.0, 8.0), adjoint=False):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the engine needs a HIP device")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        n = len(grids)
        descs = (L.GridDesc * n)()
        for k, g in enumerate(grids):
            descs[k] = grid_desc(g)
        req = ws_request(source_footprint, adjoint)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.teuk_batch_workspace_size(n, descs, ctypes.byref(req), ctypes.byref(nbytes)))
        self._ws = device_buffer(nbytes.value)
        ctx = ctypes.c_void_p()
        L.check(self._lib.teuk_batch_create(n, descs, ctypes.byref(req), ctypes.c_void_p(self.stream.cuda_stream),
                                            _ptr(self._ws), nbytes.value, ctypes.byref(ctx)))
        self.ctx = ctx
        self.instances = []
        for k, g in enumerate(grids):
            ic = ctypes.c_void_p()
            L.check(self._lib.teuk_batch_instance(self.ctx, k, ctypes.byref(ic)))
            self.instances.append(Engine._borrowed(self._lib, ic, g["m"], self.stream))

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            for e in self.instances:
                e.close()
            self._lib.teuk_batch_destroy(self.ctx)
            self.ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def seg_rows(self):
        v = ctypes.c_int32()
        L.check(self._lib.teuk_batch_get_tuning(self.ctx, ctypes.byref(v)))
        return v.value

    def set_tuning(self, seg_rows):
        L.check(self._lib.teuk_batch_set_tuning(self.ctx, int(seg_rows)))

    @property
    def mode(self):
        v = ctypes.c_int32()
        L.check(self._lib.teuk_batch_get_mode(self.ctx, ctypes.byref(v)))
        return v.value

    def set_mode(self, mode):
        """Batch.PERSISTENT or Batch.PER_ITERATION."""
        L.check(self._lib.teuk_batch_set_mode(self.ctx, int(mode)))

    def groups(self):
        """The per-iteration mode's cache-sized groups, as lists of instance
        indices in the order they run (one group when the batch fits the
        last-level cache)."""
        ng = ctypes.c_int32()
        L.check(self._lib.teuk_batch_get_groups(self.ctx, ctypes.byref(ng), None, None))
        first = (ctypes.c_int32 * (ng.value + 1))()
        order = (ctypes.c_int32 * len(self.instances))()
        L.check(self._lib.teuk_batch_get_groups(self.ctx, ctypes.byref(ng), first, order))
        return [list(order[first[g]:first[g + 1]]) for g in range(ng.value)]

    def step(self, nsteps, waveform=True, out=None):
        """nsteps iterations of every instance; returns the per-instance
        (nsteps, nth) waveforms (out, if given), or None."""
        n = len(self.instances)
        ws = None
        arr = None
        if waveform:
            if out is None:
                out = [torch.empty((int(nsteps), e.shape[0]), dtype=torch.complex128, device="cuda")
                       for e in self.instances]
            for t, e in zip(out, self.instances):
                _need_device(t, (int(nsteps), e.shape[0]), "waveform")
            ws = list(out)
            arr = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ws])
        L.check(self._lib.teuk_batch_step_n(self.ctx, int(nsteps), arr))
        return ws

    def sync(self):
        L.check(self._lib.teuk_batch_sync(self.ctx))

    def set_wait_limit(self, seconds):
        """Device wall-clock time a dependency wait of the persistent mode
        may take before the launch gives up (default 2 s)."""
        L.check(self._lib.teuk_batch_set_wait_limit(self.ctx, float(seconds)))

    def abort(self):
        """Make the persistent launches queued from here on exit at once;
        the next sync() raises TEUK_EDEVICE."""
        L.check(self._lib.teuk_batch_abort(self.ctx))

    def autotune(self, cache_path=None):
        """Measure every (mode, seg_rows) (or take it from the cache file) and
        keep the fastest; returns [(seg_rows, mode, us/iteration)], fastest
        first (one entry when served from the cache)."""
        cap = 16
        table = (L.TuneEntry * cap)()
        cnt = ctypes.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        L.check(self._lib.teuk_batch_autotune(self.ctx, path, table, cap, ctypes.byref(cnt)))
        return [(table[k].seg_rows, table[k].batch_mode, table[k].us_per_iteration) for k in range(cnt.value)]


def radiated_flux(ms, waves, dt, stream=None):
    """Radiated energy, linear and z angular momentum (teuk_radiated_flux).

    ms: the m of each waveform; waves: complex128 device tensors of shape
    (nsteps + 1, nth), row n = Phi at the extraction column at t = n dt (row
    0 the initial state).  Returns a (nsteps + 1, 10) float64 device tensor:
    dE/dt, dPx/dt, dPy/dt, dPz/dt, dJz/dt, E, Px, Py, Pz, Jz."""
    lib = L.load()
    n = len(ms)
    rows, nth = waves[0].shape
    for w in waves:
        _need_device(w, (rows, nth), "waveform")
    m_arr = (ctypes.c_int32 * n)(*[int(m) for m in ms])
    p_arr = (ctypes.c_void_p * n)(*[w.data_ptr() for w in waves])
    desc = L.FluxDesc(n, m_arr, p_arr, rows - 1, nth, float(dt))
    nbytes = ctypes.c_size_t()
    L.check(lib.teuk_flux_workspace_size(ctypes.byref(desc), ctypes.byref(nbytes)))
    ws = device_buffer(nbytes.value)
    out = torch.empty((rows, 10), dtype=torch.float64, device="cuda")
    stream = stream if stream is not None else torch.cuda.current_stream()
    L.check(lib.teuk_radiated_flux(ctypes.byref(desc), ctypes.c_void_p(stream.cuda_stream), _ptr(ws),
                                   nbytes.value, _ptr(out)))
    stream.synchronize()        # the workspace tensor goes out of scope here
    return out


def checkpoint_schedule(nsteps, snapshots):
    """The binomial checkpoint schedule (host only): (forward actions,
    backward actions, stats).  Actions are (op, a, b) rows: 0 advance a
    iterations to iteration b, 1 store u^b in slot a, 2 restore slot a
    (u^b), 3 reverse iteration a; stats = (repetitions, iterations
    recomputed by the backward, most slots held at once)."""
    import numpy as np
    lib = L.load()
    out = []
    stats = (ctypes.c_int64 * 3)()
    for phase in (0, 1):
        count = ctypes.c_int64()
        L.check(lib.teuk_checkpoint_schedule(int(nsteps), int(snapshots), phase, None, 0, ctypes.byref(count), None))
        buf = np.zeros((max(count.value, 1), 3), dtype=np.int64)
        L.check(lib.teuk_checkpoint_schedule(int(nsteps), int(snapshots), phase,
                                             buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), count.value,
                                             ctypes.byref(count), stats))
        out.append(buf[:count.value])
    return out[0], out[1], tuple(int(x) for x in stats)
