"""Python front end of the two-fluid FDTD library.

``Simulation`` owns the device buffers as torch tensors (torch supplies device
memory and streams only) and forwards every operation to the C ABI of
``libtfl.so``; all arithmetic of the time step runs in the HIP kernels.
"""
import ctypes
import hashlib
import json

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float64: L.TFL_F64, torch.float32: L.TFL_F32}
_WAVES = {"sin": L.TFL_WAVE_SIN, "gauss": L.TFL_WAVE_GAUSS, "mod_gauss": L.TFL_WAVE_MOD_GAUSS}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Simulation:
    """Two-fluid Maxwell-London FDTD on an nx x ny x nz Yee grid (Sec. 3, Algorithm 1).

    Parameters
    ----------
    shape : (nx, ny, nz)
    spacing : (dx, dy, dz) in m
    dt : time step in s
    theta : weight of the Ohmic term (Algorithm 1 step 3), in [0.5, 1]
    dtype : torch.float64 or torch.float32 (storage and arithmetic of E, H, Js and maps)
    pml : per axis None (periodic) or (lo, hi) absorbing cells (CPML backed by a PEC wall)
    pml_order, pml_scale, kappa_max, alpha_max : CPML grading (tfl_config)
    device : the GPU holding every buffer
    fused : bind a second E, H set (and H-side CPML variables) so that a step runs as one sweep
    edge_classes : after each set_materials, replace the maps read by the E update with one 16-bit
        class per edge and a coefficient table when the grid has few enough distinct materials
        (the number bound is in ``edge_classes`` afterwards, 0 on the map path); results are
        bit-identical either way
    """

    def __init__(self, shape, spacing, dt, theta=1.0, dtype=torch.float64, pml=(None, None, None),
                 pml_order=3.0, pml_scale=1.0, kappa_max=1.0, alpha_max=0.0, device="cuda", fused=True,
                 edge_classes=True):
        if dtype not in _DT:
            raise ValueError("dtype must be torch.float64 or torch.float32")
        self.nx, self.ny, self.nz = (int(v) for v in shape)
        self.shape3 = (self.nz, self.ny, self.nx)
        self.spacing = tuple(float(v) for v in spacing)
        self.dt = float(dt)
        self.theta = float(theta)
        self.dtype = dtype
        self.device = torch.device(device)
        cfg = L.tfl_config()
        cfg.nx, cfg.ny, cfg.nz = self.nx, self.ny, self.nz
        cfg.dx, cfg.dy, cfg.dz = self.spacing
        cfg.dt, cfg.theta, cfg.dtype = self.dt, self.theta, _DT[dtype]
        for a in range(3):
            if pml[a] is None:
                cfg.bc[a] = L.TFL_PERIODIC
            else:
                cfg.bc[a] = L.TFL_CPML
                cfg.pml_lo[a], cfg.pml_hi[a] = int(pml[a][0]), int(pml[a][1])
        cfg.pml_order, cfg.pml_scale, cfg.kappa_max, cfg.alpha_max = pml_order, pml_scale, kappa_max, alpha_max
        self.pml = tuple(pml)
        self._cfg = cfg
        h = ctypes.c_void_p()
        L.call("tfl_create", ctypes.byref(cfg), ctypes.byref(h))
        self._h = h
        z = lambda: torch.zeros(self.shape3, dtype=dtype, device=self.device)  # noqa: E731
        self.E = [z() for _ in range(3)]
        self.H = [z() for _ in range(3)]
        self.J = [z() for _ in range(3)]
        ws, sc, st = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._call("tfl_buffer_sizes", ctypes.byref(ws), ctypes.byref(sc), ctypes.byref(st))
        self.state_bytes = st.value
        self.workspace = torch.zeros(max(ws.value, 1), dtype=torch.uint8, device=self.device)
        self.scratch = torch.zeros(sc.value, dtype=torch.uint8, device=self.device)
        e3, self._ek = L.ptr3([t.data_ptr() for t in self.E])
        h3, self._hk = L.ptr3([t.data_ptr() for t in self.H])
        j3, self._jk = L.ptr3([t.data_ptr() for t in self.J])
        self._call("tfl_bind_state", e3, h3, j3)
        self._call("tfl_bind_workspace", ctypes.c_void_p(self.workspace.data_ptr() if ws.value else 0),
                   ctypes.c_void_p(self.scratch.data_ptr()), _stream())
        # second E, H set for the one-sweep step (fused=False keeps two passes)
        fb = ctypes.c_size_t()
        self._call("tfl_fused_buffer_bytes", ctypes.byref(fb))
        self.fused_buffer = None
        if fused and fb.value:
            self.fused_buffer = torch.empty(fb.value, dtype=torch.uint8, device=self.device)
            self._call("tfl_bind_fused_buffer", ctypes.c_void_p(self.fused_buffer.data_ptr()))
        self.maps = None
        # per-edge coefficient classes for the forward sweeps, built by set_materials when the grid
        # holds few distinct materials (edge_classes=False keeps the per-cell maps path)
        self.use_edge_classes = bool(edge_classes)
        self.class_buffer = None
        self.edge_classes = 0
        self._probes = []
        self._probe_desc = []
        self._sources = []

    # -- plumbing -----------------------------------------------------------
    def _call(self, name, *args):
        return L.call(name, self._h, *args, handle=self._h)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            L.lib().tfl_destroy(h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = torch.as_tensor(a)
        if tuple(t.shape) != self.shape3:
            raise ValueError(f"expected shape {self.shape3}, got {tuple(t.shape)}")
        return t.to(device=self.device, dtype=self.dtype).contiguous()

    # -- set-up -------------------------------------------------------------
    def set_materials(self, eps_r, sigma, inv_lambda2):
        """Per-cell eps_r, sigma_n (S/m) and 1/lambda_L^2 (m^-2); validated and dt-checked on the device."""
        maps = [self._dev(m) for m in (eps_r, sigma, inv_lambda2)]
        self.edge_classes = 0
        self._call("tfl_bind_materials", *[ctypes.c_void_p(m.data_ptr()) for m in maps], _stream())
        self.maps = maps
        if self.use_edge_classes:
            self._bind_edge_classes()

    def _bind_edge_classes(self):
        """Edge-coefficient classes of the bound maps (tfl_bind_edge_classes); stays on the maps path
        when the grid has more distinct materials than the class table holds."""
        if self.class_buffer is None:
            nb = ctypes.c_size_t()
            self._call("tfl_edge_class_bytes", ctypes.byref(nb))
            self.class_buffer = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        n = ctypes.c_int()
        try:
            self._call("tfl_bind_edge_classes", ctypes.c_void_p(self.class_buffer.data_ptr()), ctypes.byref(n),
                       _stream())
        except L.TflError as err:
            if err.code != L.TFL_E_RANGE:
                raise
            self.class_buffer = None
            n.value = 0
        self.edge_classes = n.value

    def set_fields(self, E, H, J=None):
        """Integer-time fields at t = 0 (E^0, H^0, Js^0); converted to the staggered state."""
        for q in range(3):
            self.E[q].copy_(self._dev(E[q]))
            self.H[q].copy_(self._dev(H[q]))
            self.J[q].copy_(self._dev(J[q]) if J is not None else torch.zeros_like(self.J[q]))
        self._call("tfl_set_initial_integer_time", _stream())

    def add_source(self, comp, box, amplitude, waveform="sin", freq=0.0, t0=0.0, tw=1.0):
        s = L.tfl_source()
        s.comp = int(comp)
        for q in range(6):
            s.box[q] = int(box[q])
        s.amplitude, s.waveform = float(amplitude), _WAVES[waveform]
        s.freq, s.t0, s.tw = float(freq), float(t0), float(tw)
        sid = ctypes.c_int()
        self._call("tfl_add_source", ctypes.byref(s), ctypes.byref(sid))
        self._sources.append(s)
        return sid.value

    def add_probe(self, comp, box, capacity, freqs=()):
        freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).reshape(-1))
        series = torch.zeros(max(int(capacity), 1), dtype=torch.float64, device=self.device)
        dft = torch.zeros(max(2 * freqs.size, 1), dtype=torch.float64, device=self.device)
        p = L.tfl_probe()
        p.comp = int(comp)
        for q in range(6):
            p.box[q] = int(box[q])
        p.series = series.data_ptr() if capacity > 0 else None
        p.capacity = int(capacity)
        p.nfreq = int(freqs.size)
        p.freqs = freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if freqs.size else None
        p.dft = dft.data_ptr() if freqs.size else None
        pid = ctypes.c_int()
        self._call("tfl_add_probe", ctypes.byref(p), ctypes.byref(pid))
        self._probes.append((series, dft, int(capacity), int(freqs.size)))
        self._probe_desc.append([int(comp), [int(v) for v in box], int(capacity), [float(f) for f in freqs]])
        return pid.value

    # -- running ------------------------------------------------------------
    def step(self, n=1):
        self._call("tfl_step", ctypes.c_int64(int(n)), _stream())

    SWEEPS = {"auto": 0, "two_pass": 1, "fused": 2, "two_step": 3}

    def set_sweep(self, sweep):
        """Sweep policy: 'auto' (default), 'two_pass', 'fused' or 'two_step' (tfl_set_sweep)."""
        self._call("tfl_set_sweep", ctypes.c_int32(self.SWEEPS[sweep]))

    def sweep_counts(self):
        """Steps of the last step() call on (two passes, fused sweep, two-step sweep)."""
        c = (ctypes.c_int64 * 3)()
        self._call("tfl_sweep_counts", c)
        return tuple(int(v) for v in c)

    def set_nonfinite_check(self, every):
        """Count NaN / Inf values of E, H and Js on the device after every `every`-th step (0: off);
        a step() or forward_checkpointed() that saw any raises TflError with code TFL_E_NONFINITE."""
        self._call("tfl_set_nonfinite_check", ctypes.c_int64(int(every)))

    def profile_step(self, n):
        """Run n steps with HIP events around each pass; returns (H-pass ms, E-pass ms) summed."""
        h, e = ctypes.c_double(), ctypes.c_double()
        self._call("tfl_profile_step", ctypes.c_int64(int(n)), _stream(), ctypes.byref(h), ctypes.byref(e))
        return h.value, e.value

    @property
    def step_index(self):
        v = ctypes.c_int64()
        self._call("tfl_get_step", ctypes.byref(v))
        return v.value

    def set_step(self, n):
        self._call("tfl_set_step", ctypes.c_int64(int(n)))

    # -- read-back ----------------------------------------------------------
    def integer_time_fields(self):
        """(E^n, H^n, Js^n) as new device tensors (Algorithm 1's state at integer time)."""
        Hn = [torch.empty_like(t) for t in self.H]
        Jn = [torch.empty_like(t) for t in self.J]
        h3, hk = L.ptr3([t.data_ptr() for t in Hn])
        j3, jk = L.ptr3([t.data_ptr() for t in Jn])
        self._call("tfl_sync_integer_time", h3, j3, _stream())
        return [t.clone() for t in self.E], Hn, Jn

    def energy(self):
        w, bad = ctypes.c_double(), ctypes.c_int64()
        self._call("tfl_energy", ctypes.byref(w), ctypes.byref(bad), _stream())
        return w.value, bad.value

    def probe(self, pid):
        series, dft, cap, nf = self._probes[pid]
        s = series[:cap].cpu().numpy()
        d = dft[: 2 * nf].cpu().numpy()
        return s, d[0::2] + 1j * d[1::2]

    def save_state(self, dst=None):
        if dst is None:
            dst = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        self._call("tfl_save_state", ctypes.c_void_p(dst.data_ptr()), _stream())
        return dst

    def load_state(self, src):
        self._call("tfl_load_state", ctypes.c_void_p(src.data_ptr()), _stream())

    # -- restart files --------------------------------------------------------
    def _run_description(self):
        """What a saved state belongs to: the problem statement (grid, spacing, dt, theta, storage type,
        boundaries), a hash of the bound maps, the sources and the probes."""
        c = self._cfg
        h = hashlib.sha256()
        for m in self.maps or []:
            h.update(m.cpu().numpy().tobytes())
        src = [[x.comp, list(x.box), x.amplitude, x.waveform, x.freq, x.t0, x.tw] for x in self._sources]
        return dict(shape=[self.nx, self.ny, self.nz], spacing=list(self.spacing), dt=self.dt, theta=self.theta,
                    dtype=str(self.dtype), bc=list(c.bc), pml_lo=list(c.pml_lo), pml_hi=list(c.pml_hi),
                    pml=[c.pml_order, c.pml_scale, c.kappa_max, c.alpha_max], maps_sha256=h.hexdigest(),
                    sources=src, probes=self._probe_desc)

    def save_checkpoint(self, path):
        """Write the run to `path` (NumPy .npz of plain arrays, nothing pickled): the state of
        tfl_save_state (E, H, Js and the CPML variables), the step index, every probe's FP64 series and
        DFT accumulators, and the run's description, which load_checkpoint checks."""
        state = self.save_state().cpu().numpy()
        arrays = {"state": state, "step": np.array([self.step_index], dtype=np.int64),
                  "description": np.frombuffer(json.dumps(self._run_description()).encode(), dtype=np.uint8)}
        for q, (series, dft, _, _) in enumerate(self._probes):
            arrays[f"series{q}"] = series.cpu().numpy()
            arrays[f"dft{q}"] = dft.cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    def load_checkpoint(self, path):
        """Continue a run written by save_checkpoint: this simulation must describe the same run (grid,
        spacing, dt, theta, storage type, boundaries, maps, sources and probes, added in the same order);
        the state, step index and probe buffers are replaced.  Raises ValueError on a mismatch."""
        with np.load(path, allow_pickle=False) as z:
            saved = json.loads(z["description"].tobytes().decode())
            mine = json.loads(json.dumps(self._run_description()))
            if saved != mine:
                diff = sorted(k for k in set(saved) | set(mine) if saved.get(k) != mine.get(k))
                raise ValueError(f"checkpoint belongs to another run (differs in: {', '.join(diff)})")
            state = z["state"]
            if state.size != self.state_bytes:
                raise ValueError(f"checkpoint state has {state.size} bytes, this run {self.state_bytes}")
            self.load_state(torch.from_numpy(np.ascontiguousarray(state)).to(self.device))
            self.set_step(int(z["step"][0]))
            for q, (series, dft, _, _) in enumerate(self._probes):
                series.copy_(torch.from_numpy(z[f"series{q}"]).to(self.device))
                dft.copy_(torch.from_numpy(z[f"dft{q}"]).to(self.device))

    def ringdown_fit(self, pid, start, count, decim=1, order=0, f_hint=0.0):
        """Linear-prediction fit of probe pid's series window; returns dict(f0, alpha, Q, residual,
        order, modes=[(f, alpha), ...])."""
        rq = L.tfl_fit_req()
        rq.start, rq.count, rq.decim, rq.order, rq.f_hint = int(start), int(count), int(decim), int(order), f_hint
        r = L.tfl_fit_result()
        self._call("tfl_ringdown_fit", ctypes.c_int(int(pid)), ctypes.byref(rq), ctypes.byref(r), _stream())
        modes = [(r.modes[2 * q], r.modes[2 * q + 1]) for q in range(r.nmodes)]
        return dict(f0=r.f0, alpha=r.alpha, Q=r.Q, residual=r.residual, order=r.order, modes=modes)

    def esprit_fit(self, pid, start, count, decim=1, order=0, pencil=0, f_hint=0.0):
        """ESPRIT fit of probe pid's series window (pencil 0: min(64, count // 3)); returns
        dict(f0, alpha, Q, residual, order, pencil, modes=[(f, alpha), ...])."""
        rq = L.tfl_fit_req()
        rq.start, rq.count, rq.decim, rq.order, rq.f_hint = int(start), int(count), int(decim), int(order), f_hint
        r = L.tfl_fit_result()
        self._call("tfl_esprit_fit", ctypes.c_int(int(pid)), ctypes.byref(rq), ctypes.c_int32(int(pencil)),
                   ctypes.byref(r), _stream())
        modes = [(r.modes[2 * q], r.modes[2 * q + 1]) for q in range(r.nmodes)]
        M = int(pencil) if pencil else min(64, int(count) // 3)
        return dict(f0=r.f0, alpha=r.alpha, Q=r.Q, residual=r.residual, order=r.order, pencil=M, modes=modes)

    # -- adjoint ------------------------------------------------------------
    @staticmethod
    def _objective(comp, box, f0):
        o = L.tfl_objective()
        o.comp = int(comp)
        for q in range(6):
            o.box[q] = int(box[q])
        o.f0 = float(f0)
        return o

    def adjoint_buffers(self, nsteps, seg):
        """Caller-owned device buffers for a checkpointed run: (checkpoints, snapshots, workspace)."""
        c, s, a = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._call("tfl_adjoint_sizes", ctypes.c_int64(int(nsteps)), ctypes.c_int64(int(seg)), ctypes.byref(c),
                   ctypes.byref(s), ctypes.byref(a))
        mk = lambda n: torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)  # noqa: E731
        return mk(c.value), mk(s.value), mk(a.value)

    def forward_checkpointed(self, objective, nsteps, seg, ckpt):
        """Run nsteps with checkpoints every seg steps; returns F (complex) of the objective
        (comp, box, f0): J = |F|^2, F = sum_n dt exp(-i 2 pi f0 n dt) sum_box E_comp^n."""
        o = self._objective(*objective)
        F = (ctypes.c_double * 2)()
        self._call("tfl_forward_checkpointed", ctypes.byref(o), ctypes.c_int64(int(nsteps)), ctypes.c_int64(int(seg)),
                   ctypes.c_void_p(ckpt.data_ptr()), F, _stream())
        return complex(F[0], F[1])

    def adjoint_nested_buffers(self, nsteps, seg, seg2):
        """Buffers of the three-level schedule: (outer checkpoints, inner checkpoints, snapshots, workspace)."""
        v = [ctypes.c_size_t() for _ in range(4)]
        self._call("tfl_adjoint_nested_sizes", ctypes.c_int64(int(nsteps)), ctypes.c_int64(int(seg)),
                   ctypes.c_int64(int(seg2)), *[ctypes.byref(x) for x in v])
        return tuple(torch.empty(max(x.value, 1), dtype=torch.uint8, device=self.device) for x in v)

    def adjoint_nested(self, objective, nsteps, seg, seg2, ckpt, F, ckpt2, snap, work):
        """Per-cell FP64 gradients of the last checkpointed run, three-level schedule."""
        o = self._objective(*objective)
        Fa = (ctypes.c_double * 2)(F.real, F.imag)
        gl = torch.empty(self.shape3, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.shape3, dtype=torch.float64, device=self.device)
        self._call("tfl_adjoint_nested", ctypes.byref(o), ctypes.c_int64(int(nsteps)), ctypes.c_int64(int(seg)),
                   ctypes.c_void_p(ckpt.data_ptr()), Fa, ctypes.c_int64(int(seg2)), ctypes.c_void_p(ckpt2.data_ptr()),
                   ctypes.c_void_p(snap.data_ptr()), ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(gl.data_ptr()),
                   ctypes.c_void_p(gs.data_ptr()), _stream())
        return gl, gs

    def adjoint(self, objective, nsteps, seg, ckpt, F, snap, work):
        """Per-cell FP64 gradients (dJ/d inv_lambda2, dJ/d sigma_n) of the last checkpointed run."""
        o = self._objective(*objective)
        Fa = (ctypes.c_double * 2)(F.real, F.imag)
        gl = torch.empty(self.shape3, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.shape3, dtype=torch.float64, device=self.device)
        self._call("tfl_adjoint", ctypes.byref(o), ctypes.c_int64(int(nsteps)), ctypes.c_int64(int(seg)),
                   ctypes.c_void_p(ckpt.data_ptr()), Fa, ctypes.c_void_p(snap.data_ptr()),
                   ctypes.c_void_p(work.data_ptr()), ctypes.c_void_p(gl.data_ptr()), ctypes.c_void_p(gs.data_ptr()),
                   _stream())
        return gl, gs
