"""MI355X spin-stepping Bloch simulator (Python binding of libparspin.so).

Every spin of an object is stepped through a sequence of elementary
sequences with analytic Bloch solutions and the rotating-frame transverse
magnetisation of all spins is summed per ADC sample (section 5.1.1).  All
of that runs in hand-written HIP kernels behind the C ABI of
include/parspin.h; this module only marshals arguments.  PyTorch provides
device memory and streams.

    import paper_1305_6861_amd as ps
    ctx = ps.Context()                      # device 0, FP32 stepping
    sig = ctx.simulate(obj, seq)            # torch.complex128 on the GPU

`obj` is a mapping (or object with attributes) of x, y, z, m0, t1, t2, dw:
float32 CUDA tensors, or numpy arrays that are copied to the device.
`seq` exposes dt, m, rf_alpha, rf_phase, rf_shape, n_adc, flags (one entry
per elementary sequence) and shapes (tau, m_sub, alpha, phase).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _binding as _b
from ._binding import PsError, PS_EV_SPOIL, PS_EV_SNAPSHOT, PS_EV_TRAJECTORY

FIELDS = ("x", "y", "z", "m0", "t1", "t2", "dw")

__all__ = ["Context", "Plan", "Ticket", "SchedulerTest", "PsError", "PS_EV_SPOIL", "PS_EV_SNAPSHOT", "count", "pack_sequence",
           "to_device", "kt_extent", "FIELDS"]


class PackedSequence:
    """A sequence marshalled into ps_event / ps_rf_shape arrays (host memory
    kept alive by this object)."""

    def __init__(self, seq):
        n = int(seq.n_events)
        self.n_events = n
        self._events = (_b.ps_event * max(n, 1))()
        if n:
            dt = np.asarray(seq.dt, np.float64)
            m = np.asarray(seq.m, np.float64).reshape(n, 3)
            al = np.asarray(seq.rf_alpha, np.float64)
            ph = np.asarray(seq.rf_phase, np.float64)
            sh = np.asarray(seq.rf_shape, np.int64)
            na = np.asarray(seq.n_adc, np.int64)
            fl = np.asarray(seq.flags, np.int64)
            tr = (np.asarray(seq.trajectory, np.int64) if hasattr(seq, "trajectory")
                  else np.full(n, -1, np.int64))
            if np.any(na < 0) or np.any(na > 0x7FFFFFFF):
                raise PsError(1, "n_adc out of range")
            fl = np.where(tr >= 0, fl | _b.PS_EV_TRAJECTORY, fl)
            rec = np.zeros(n, dtype=np.dtype([("dt", "<f8"), ("m", "<f8", (3,)), ("a", "<f8"), ("p", "<f8"),
                                               ("s", "<i4"), ("n", "<u4"), ("f", "<u4"), ("r", "<u4")]))
            rec["dt"] = dt; rec["m"] = m; rec["a"] = al; rec["p"] = ph
            rec["s"] = sh.astype(np.int32); rec["n"] = na.astype(np.uint32); rec["f"] = fl.astype(np.uint32)
            rec["r"] = np.where(tr >= 0, tr, 0).astype(np.uint32)
            ctypes.memmove(self._events, rec.ctypes.data, rec.nbytes)
        shapes = list(getattr(seq, "shapes", []))
        self._keep = []
        self._shapes = (_b.ps_rf_shape * max(len(shapes), 1))()
        for i, s in enumerate(shapes):
            a = np.ascontiguousarray(s.alpha, np.float64)
            p = np.ascontiguousarray(s.phase, np.float64)
            self._keep += [a, p]
            rec = self._shapes[i]
            rec.n_sub = int(a.shape[0])
            rec.tau = float(s.tau)
            for d in range(3):
                rec.m_sub[d] = float(np.asarray(s.m_sub, np.float64).reshape(3)[d])
            rec.alpha = a.ctypes.data
            rec.phase = p.ctypes.data
        trajs = list(getattr(seq, "trajectories", []))
        self._trajs = (_b.ps_trajectory * max(len(trajs), 1))()
        for i, t in enumerate(trajs):
            k = np.ascontiguousarray(t.k, np.float64).reshape(-1)
            tt = np.ascontiguousarray(t.t, np.float64).reshape(-1)
            self._keep += [k, tt]
            self._trajs[i].n = int(tt.shape[0])
            self._trajs[i].k = k.ctypes.data
            self._trajs[i].t = tt.ctypes.data
        self.struct = _b.ps_sequence(n, ctypes.addressof(self._events), len(shapes), len(trajs),
                                     ctypes.addressof(self._shapes), ctypes.addressof(self._trajs))

    def count(self):
        ns = ctypes.c_int64(); st = ctypes.c_int64()
        _b.check(_b.lib.ps_count(ctypes.byref(self.struct), ctypes.byref(ns), ctypes.byref(st)))
        return int(ns.value), int(st.value)

    def count_snapshots(self) -> int:
        n = ctypes.c_int64()
        _b.check(_b.lib.ps_count_snapshots(ctypes.byref(self.struct), ctypes.byref(n)))
        return int(n.value)


def pack_sequence(seq) -> PackedSequence:
    return seq if isinstance(seq, PackedSequence) else PackedSequence(seq)


def count(seq):
    """(n_samples, n_steps_per_spin) of a sequence, validated by the library."""
    return pack_sequence(seq).count()


def kt_extent(seq, dk, t1: float, t2: float, grey_step: float = 0.0, extent=None) -> dict:
    """Spin spacing the sequence needs (ps_kt_extent, section 5.2): k_max and
    dx_max per axis (cycles/m, m) for lattice steps dk (cycles/m per axis)
    and the reference tissue (t1, t2); grey_step > 0 leaves out outer
    configurations too weak to show at that grey-value step (eq. 5.4 / 5.5).
    With the object's extent (m per axis) also n_spins_min, the isochromats
    one tissue class needs at that spacing (eq. 5.2)."""
    ps = pack_sequence(seq)
    dkv = (ctypes.c_double * 3)(*[float(v) for v in dk])
    ext = None if extent is None else (ctypes.c_double * 3)(*[float(v) for v in extent])
    km = (ctypes.c_double * 3)()
    dx = (ctypes.c_double * 3)()
    n_min = ctypes.c_int64()
    peak = ctypes.c_int64()
    _b.check(_b.lib.ps_kt_extent(ctypes.byref(ps.struct), dkv, float(t1), float(t2), float(grey_step), ext, km, dx,
                                 ctypes.byref(n_min) if ext is not None else None, ctypes.byref(peak)))
    out = {"k_max": np.array(km[:]), "dx_max": np.array(dx[:]), "n_configs_peak": int(peak.value)}
    if ext is not None:
        out["n_spins_min"] = int(n_min.value)
    return out


def to_device(obj, device="cuda"):
    """Spin arrays as contiguous float32 tensors on the device."""
    import torch
    out = {}
    for f in FIELDS:
        v = obj[f] if isinstance(obj, dict) else getattr(obj, f)
        t = v if isinstance(v, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(v, np.float32))
        out[f] = t.to(device=device, dtype=torch.float32).contiguous()
    return out


def _object_struct(dev):
    n = int(dev["x"].numel())
    for f in FIELDS:
        t = dev[f]
        if t.dtype.itemsize != 4 or not t.is_contiguous() or int(t.numel()) != n or not t.is_cuda:
            raise PsError(1, f"field {f} must be a contiguous float32 CUDA tensor of {n} entries")
    return _b.ps_object(n, *[dev[f].data_ptr() if n else 0 for f in FIELDS])


class Context:
    """One library context (device, precision, tiling)."""

    def __init__(self, device: int = 0, precision: int = 32, spins_per_lane: int = 0,
                 max_partial_bytes: int = 0, max_footprint_bytes: int = 0, kernel_timing: bool = False,
                 shape_cache: bool = True, readout_split: bool = True, max_slice_steps: int = 0,
                 autotune: bool = False, serve_graphs: bool = True, matrix_readout: bool = True):
        cfg = _b.ps_config()
        _b.check(_b.lib.ps_config_default(ctypes.byref(cfg)))
        cfg.device = device
        cfg.precision = precision
        cfg.spins_per_lane = spins_per_lane
        cfg.flags = (_b.PS_CFG_KERNEL_TIMING if kernel_timing else 0) | \
            (0 if shape_cache else _b.PS_CFG_NO_SHAPE_CACHE) | \
            (0 if readout_split else _b.PS_CFG_NO_READOUT_SPLIT) | \
            (_b.PS_CFG_AUTOTUNE if autotune else 0) | \
            (0 if serve_graphs else _b.PS_CFG_SERVE_DIRECT) | \
            (0 if matrix_readout else _b.PS_CFG_NO_MATRIX_READOUT)
        if max_partial_bytes:
            cfg.max_partial_bytes = max_partial_bytes
        if max_footprint_bytes:
            cfg.max_footprint_bytes = max_footprint_bytes
        if max_slice_steps:
            cfg.max_slice_steps = max_slice_steps
        h = ctypes.c_void_p()
        _b.check(_b.lib.ps_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h
        self.device = device
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _b.lib.ps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tile(self, n_spins: int):
        """(spins per lane, spins per workgroup) used for an object of n_spins."""
        spl = ctypes.c_int32(); spb = ctypes.c_int64()
        _b.check(_b.lib.ps_tile(self._h, int(n_spins), ctypes.byref(spl), ctypes.byref(spb)))
        return int(spl.value), int(spb.value)

    def tile_for(self, n_spins: int, seq, n_coils: int = 0) -> dict:
        """The tiling a request of this size and sequence gets (ps_tile_for):
        spins per lane, readout-replica mode and whether it comes from the
        tiling table (tuned) or the threshold rule."""
        ps = pack_sequence(seq)
        spl, rep, tuned = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _b.check(_b.lib.ps_tile_for(self._h, int(n_spins), ctypes.byref(ps.struct), int(n_coils),
                                    ctypes.byref(spl), ctypes.byref(rep), ctypes.byref(tuned)))
        return {"spins_per_lane": int(spl.value), "replicas": _b.REPLICA_MODES[int(rep.value)],
                "tuned": bool(tuned.value)}

    def readout_path(self, n_spins: int, seq, spins_per_lane: int, n_coils: int = 0) -> dict:
        """How a request's readouts are summed at this spins-per-lane, planned
        as a simulate call plans it (ps_readout_path): readouts in all, on the
        matrix cores, whether the matrix-only kernel runs the request, and
        its time slices."""
        ps = pack_sequence(seq)
        n, m, mo, sl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _b.check(_b.lib.ps_readout_path(self._h, int(n_spins), ctypes.byref(ps.struct), int(n_coils),
                                        int(spins_per_lane), ctypes.byref(n), ctypes.byref(m), ctypes.byref(mo),
                                        ctypes.byref(sl)))
        return {"readouts": int(n.value), "matrix": int(m.value), "matrix_only": bool(mo.value),
                "slices": int(sl.value)}

    def tune(self, obj, seq, coils=None, force: bool = False) -> dict:
        """Time the candidate tilings of the request's class on the device and
        keep the fastest in the context's tiling table (ps_tune); returns the
        chosen tiling with every candidate's median probe time in ms."""
        import torch
        owned = not (isinstance(obj, dict) and all(isinstance(obj[f], torch.Tensor) and obj[f].is_cuda
                                                   for f in FIELDS))
        dev = to_device(obj, f"cuda:{self.device}") if owned else obj
        torch.cuda.current_stream(self.device).synchronize()
        ps = pack_sequence(seq)
        n_spins = int(dev["x"].numel())
        keep, rx = _receive(coils, n_spins, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        o = _object_struct(dev)
        r = _b.ps_tune_result()
        _b.check(_b.lib.ps_tune(self._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                ctypes.byref(rx) if rx is not None else None,
                                _b.PS_TUNE_FORCE if force else 0, ctypes.byref(r)))
        return {"spins_per_lane": int(r.spins_per_lane), "replicas": _b.REPLICA_MODES[int(r.replicas)],
                "from_table": bool(r.from_table), "best_ms": float(r.best_ms), "rule_ms": float(r.rule_ms),
                "probe_events": int(r.probe_events),
                "candidates": [{"spins_per_lane": int(r.cand_spins_per_lane[i]),
                                "replicas": _b.REPLICA_MODES[int(r.cand_replicas[i])], "ms": float(r.cand_ms[i])}
                               for i in range(int(r.n_candidates))]}

    def kt_simulate(self, obj, tissue_begin, t1, t2, dw, seq, dk, voxel=(0.0, 0.0, 0.0), stream=None):
        """Signal by the K-t engine (ps_kt_simulate): obj's spins (x, y, z, m0;
        ordered tissue by tissue, tissue c holding spins tissue_begin[c] ..
        tissue_begin[c + 1] - 1) with per-tissue t1, t2 (s) and dw (rad/s),
        a sequence whose moments lie on the lattice dk (cycles/m per axis),
        and box voxels of size voxel (m per axis, 0 = point spins) centred
        on the spins.  Returns a complex128 CUDA tensor."""
        import torch
        fields = ("x", "y", "z", "m0")
        dev = {}
        for f in fields:
            v = obj[f] if isinstance(obj, dict) else getattr(obj, f)
            t = v if isinstance(v, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(v, np.float32))
            dev[f] = t.to(device=f"cuda:{self.device}", dtype=torch.float32).contiguous()
        n_spins = int(dev["x"].numel())
        tb = np.ascontiguousarray(tissue_begin, np.int64)
        t1a = np.ascontiguousarray(t1, np.float64)
        t2a = np.ascontiguousarray(t2, np.float64)
        dwa = np.ascontiguousarray(dw, np.float64)
        n_t = int(t1a.size)
        if tb.size != n_t + 1 or t2a.size != n_t or dwa.size != n_t:
            raise PsError(1, "tissue_begin needs n_tissues + 1 entries and t1, t2, dw n_tissues each")
        ps = pack_sequence(seq)
        n_samples, _ = ps.count()
        out = torch.empty(2 * n_samples, dtype=torch.float64, device=f"cuda:{self.device}")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        for t in dev.values():
            t.record_stream(stream)
        o = _b.ps_kt_object(n_t, 0, t1a.ctypes.data, t2a.ctypes.data, dwa.ctypes.data, tb.ctypes.data, n_spins,
                            *[dev[f].data_ptr() if n_spins else 0 for f in fields],
                            (ctypes.c_double * 3)(*[float(v) for v in voxel]))
        dkv = (ctypes.c_double * 3)(*[float(v) for v in dk])
        _b.check(_b.lib.ps_kt_simulate(self._h, ctypes.byref(o), ctypes.byref(ps.struct), dkv,
                                       ctypes.c_void_p(out.data_ptr() if n_samples else 0), n_samples,
                                       ctypes.c_void_p(stream.cuda_stream)))
        return out.view(torch.complex128)

    def tune_save(self, path: str):
        _b.check(_b.lib.ps_tune_save(self._h, str(path).encode()))

    def tune_load(self, path: str) -> int:
        n = ctypes.c_int32()
        _b.check(_b.lib.ps_tune_load(self._h, str(path).encode(), ctypes.byref(n)))
        return int(n.value)

    def tune_clear(self):
        _b.check(_b.lib.ps_tune_clear(self._h))

    def kernel_times(self, capacity: int = 1 << 16):
        """(step-kernel durations in ms in launch order, summed finalize-kernel
        ms) of the launches since the previous call.  Needs a context created
        with kernel_timing=True; synchronises on those launches."""
        buf = (ctypes.c_double * capacity)()
        n = ctypes.c_int64(); fin = ctypes.c_double()
        _b.check(_b.lib.ps_kernel_times(self._h, buf, capacity, ctypes.byref(n), ctypes.byref(fin)))
        return [buf[i] for i in range(min(n.value, capacity))], float(fin.value)

    def valu_peak(self, precision: int = 32) -> float:
        """TFLOP/s of vector FMAs that code built like the kernels attains on
        this context's device (FP32 with packed FP32 disabled, or FP64):
        measurement support for the roofline, not part of the simulation."""
        out = ctypes.c_double()
        _b.check(_b.lib.ps_valu_peak(self._h, int(precision), ctypes.byref(out)))
        return float(out.value)

    def simulate_batch(self, objs, seqs, stream=None):
        """Signals of several requests computed together (one persistent
        launch per spins-per-lane class and time-slice round); each equals,
        bit for bit, what simulate() returns for that request alone."""
        import torch
        if len(objs) != len(seqs):
            raise PsError(1, "objs and seqs differ in length")
        n = len(objs)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        devs, packs, outs = [], [], []
        o_arr = (_b.ps_object * max(n, 1))()
        s_arr = (_b.ps_sequence * max(n, 1))()
        sig_arr = (ctypes.c_void_p * max(n, 1))()
        ns_arr = (ctypes.c_int64 * max(n, 1))()
        for i, (obj, seq) in enumerate(zip(objs, seqs)):
            owned = not (isinstance(obj, dict) and all(isinstance(obj[f], torch.Tensor) and obj[f].is_cuda
                                                       for f in FIELDS))
            dev = to_device(obj, f"cuda:{self.device}") if owned else obj
            if owned:
                for t in dev.values():
                    t.record_stream(stream)
            ps = pack_sequence(seq)
            try:
                ns, _ = ps.count()
            except PsError as e:
                raise PsError(e.status, f"request {i}: {e}") from None
            out = torch.empty(2 * ns, dtype=torch.float64, device=f"cuda:{self.device}")
            devs.append(dev); packs.append(ps); outs.append(out)
            o_arr[i] = _object_struct(dev)
            s_arr[i] = ps.struct
            sig_arr[i] = out.data_ptr() if ns else None
            ns_arr[i] = ns
        _b.check(_b.lib.ps_simulate_batch(self._h, n, o_arr, s_arr, sig_arr, ns_arr,
                                          ctypes.c_void_p(stream.cuda_stream)))
        return [o.view(torch.complex128) for o in outs]

    # ---- served execution -------------------------------------------------
    def submit(self, obj, seq):
        """Queue a request on the context's scheduler; returns a Ticket.  The
        object's device arrays are made ready (current stream synchronised)
        before submission; the output tensor is owned by the ticket."""
        import torch
        owned = not (isinstance(obj, dict) and all(isinstance(obj[f], torch.Tensor) and obj[f].is_cuda
                                                   for f in FIELDS))
        dev = to_device(obj, f"cuda:{self.device}") if owned else obj
        torch.cuda.current_stream(self.device).synchronize()
        ps = pack_sequence(seq)
        ns, _ = ps.count()
        out = torch.empty(2 * ns, dtype=torch.float64, device=f"cuda:{self.device}")
        o = _object_struct(dev)
        t = ctypes.c_uint64()
        _b.check(_b.lib.ps_submit(self._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                  ctypes.c_void_p(out.data_ptr() if ns else 0), ns, ctypes.byref(t)))
        return Ticket(self, int(t.value), out, dev)

    def plan(self, obj, seq, coils=None) -> Plan:
        """Compile once and capture the launches in a HIP graph (ps_plan_create)."""
        return Plan(self, obj, seq, coils)

    def server_stats(self):
        st = _b.ps_server_stats_t()
        _b.check(_b.lib.ps_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def simulate(self, obj, seq, out=None, stream=None, coils=None, snapshots: bool = False):
        """Signal of one request as a complex128 CUDA tensor (stream-ordered
        on `stream`, default torch's current stream).

        coils: optional receive coils, a pair (s_x, s_y) of (n_coils, n_spins)
        arrays or tensors with each coil's transverse sensitivity at each
        spin (ps_simulate_rx); the signal is then (n_coils, n_samples).
        snapshots: also return the magnetisation of every spin after every
        event flagged PS_EV_SNAPSHOT (ps_simulate_ex), a tensor of shape
        (n_snapshots, 3, n_spins) in the stepping precision: the call then
        returns (signal, snapshots)."""
        import torch
        owned = not (isinstance(obj, dict) and all(isinstance(obj[f], torch.Tensor) and obj[f].is_cuda
                                                   for f in FIELDS))
        dev = to_device(obj, f"cuda:{self.device}") if owned else obj
        ps = pack_sequence(seq)
        n_samples, _ = ps.count()
        n_spins = int(dev["x"].numel())
        keep, rx = _receive(coils, n_spins, self.device)
        n_out = rx.n_coils if rx is not None else 1
        if out is None:
            out = torch.empty(2 * n_samples * max(n_out, 1), dtype=torch.float64, device=f"cuda:{self.device}")
        elif out.dtype != torch.float64 or out.numel() != 2 * n_samples * n_out or not out.is_contiguous():
            raise PsError(1, "out must be a contiguous float64 tensor of 2 * n_samples * n_coils entries")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        if owned:   # temporaries must outlive the asynchronous work on `stream`
            for t in dev.values():
                t.record_stream(stream)
        for t in keep:
            t.record_stream(stream)
        o = _object_struct(dev)
        sig_ptr = ctypes.c_void_p(out.data_ptr() if n_samples else 0)
        if snapshots:
            n_snap = ps.count_snapshots()
            snap = torch.empty((n_snap, 3, n_spins), dtype=torch.float32 if self.precision == 32 else torch.float64,
                               device=f"cuda:{self.device}")
            _b.check(_b.lib.ps_simulate_ex(self._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                           ctypes.byref(rx) if rx is not None else None, sig_ptr, n_samples,
                                           ctypes.c_void_p(snap.data_ptr() if snap.numel() else 0), n_snap,
                                           ctypes.c_void_p(stream.cuda_stream)))
        elif rx is None:
            _b.check(_b.lib.ps_simulate(self._h, ctypes.byref(o), ctypes.byref(ps.struct), sig_ptr,
                                        n_samples, ctypes.c_void_p(stream.cuda_stream)))
        else:
            _b.check(_b.lib.ps_simulate_rx(self._h, ctypes.byref(o), ctypes.byref(ps.struct), ctypes.byref(rx),
                                           sig_ptr, n_samples, ctypes.c_void_p(stream.cuda_stream)))
        sig = out.view(torch.complex128)
        if rx is not None:
            sig = sig.view(max(n_out, 0), n_samples)
        return (sig, snap) if snapshots else sig


def simulate_noalloc(ctx: "Context", obj, seq, out, stream=None):
    """ps_simulate_noalloc: the signal of one request computed with the
    library's static device scratch (the call allocates nothing).  obj must
    be device tensors (to_device) and out a float64 tensor of 2 * n_samples
    entries: allocating them is the caller's business."""
    import torch
    ps = pack_sequence(seq)
    n_samples, _ = ps.count()
    if out.dtype != torch.float64 or out.numel() != 2 * n_samples or not out.is_contiguous():
        raise PsError(1, "out must be a contiguous float64 tensor of 2 * n_samples entries")
    if stream is None:
        stream = torch.cuda.current_stream(ctx.device)
    o = _object_struct(obj)
    _b.check(_b.lib.ps_simulate_noalloc(ctx._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                        ctypes.c_void_p(out.data_ptr() if n_samples else 0), n_samples,
                                        ctypes.c_void_p(stream.cuda_stream)))
    return out.view(torch.complex128)


class Plan:
    """A request compiled once with its launches captured in a HIP graph
    (ps_plan_create); launch() replays it.  The object tensors, coil
    sensitivities and the output tensor are fixed at creation; rewrite their
    contents in place between launches to simulate new parameters."""

    def __init__(self, ctx: "Context", obj, seq, coils=None):
        import torch
        self.ctx = ctx
        self.obj = obj if (isinstance(obj, dict) and all(isinstance(obj[f], torch.Tensor) and obj[f].is_cuda
                                                         for f in FIELDS)) else to_device(obj, f"cuda:{ctx.device}")
        ps = pack_sequence(seq)
        self.n_samples, _ = ps.count()
        n_spins = int(self.obj["x"].numel())
        self.coils, rx = _receive(coils, n_spins, ctx.device)
        self.n_out = rx.n_coils if rx is not None else 1
        self.out = torch.zeros(2 * self.n_samples * max(self.n_out, 1), dtype=torch.float64,
                               device=f"cuda:{ctx.device}")
        torch.cuda.synchronize(ctx.device)           # inputs resident before the capture
        o = _object_struct(self.obj)
        h = ctypes.c_void_p()
        _b.check(_b.lib.ps_plan_create(ctx._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                       ctypes.byref(rx) if rx is not None else None,
                                       ctypes.c_void_p(self.out.data_ptr() if self.n_samples else 0),
                                       self.n_samples, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        """Replay on `stream` (default torch's current stream); returns the
        signal tensor (complex128, (n_coils, n_samples) with coils)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.ctx.device)
        _b.check(_b.lib.ps_plan_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))
        sig = self.out.view(torch.complex128)
        return sig.view(self.n_out, self.n_samples) if self.coils else sig

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _b.lib.ps_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class SchedulerTest(Context):
    """A context whose served loop runs with no device (ps_create_scheduler_test):
    iterations write the stand-in pattern (re, im) = (n_spins + sample index,
    slice index) into host signal arrays and take iteration_seconds; the
    iteration numbered fail_iteration reports a device error.  For testing
    admission, batching, cancellation and failure handling on a CPU."""

    def __init__(self, iteration_seconds: float = 0.0, fail_iteration: int = -1, max_footprint_bytes: int = 0,
                 max_slice_steps: int = 0, precision: int = 32):
        cfg = _b.ps_config()
        _b.check(_b.lib.ps_config_default(ctypes.byref(cfg)))
        cfg.precision = precision
        if max_footprint_bytes:
            cfg.max_footprint_bytes = max_footprint_bytes
        if max_slice_steps:
            cfg.max_slice_steps = max_slice_steps
        tb = _b.ps_test_backend(float(iteration_seconds), int(fail_iteration))
        h = ctypes.c_void_p()
        _b.check(_b.lib.ps_create_scheduler_test(ctypes.byref(h), ctypes.byref(cfg), ctypes.byref(tb)))
        self._h = h
        self.device = 0
        self.precision = precision

    def submit(self, obj, seq):
        """Queue a request; its object arrays are host arrays (never read) and
        its signal a host float64 array owned by the ticket."""
        arrs = {f: np.ascontiguousarray(obj[f] if isinstance(obj, dict) else getattr(obj, f), np.float32)
                for f in FIELDS}
        n = int(arrs["x"].shape[0])
        ps = pack_sequence(seq)
        ns, _ = ps.count()
        out = np.full(2 * max(ns, 1), np.nan)
        o = _b.ps_object(n, *[arrs[f].ctypes.data if n else 0 for f in FIELDS])
        t = ctypes.c_uint64()
        _b.check(_b.lib.ps_submit(self._h, ctypes.byref(o), ctypes.byref(ps.struct),
                                  ctypes.c_void_p(out.ctypes.data if ns else 0), ns, ctypes.byref(t)))
        return HostTicket(self, int(t.value), out[:2 * ns], (arrs, ps))


def _receive(coils, n_spins: int, device: int):
    """(kept tensors, ps_receive or None) for a pair (s_x, s_y)."""
    import torch
    if coils is None:
        return [], None
    cs = []
    for c in coils:
        t = torch.as_tensor(c, dtype=torch.float32).to(f"cuda:{device}").contiguous()
        if t.dim() != 2 or t.shape[1] != n_spins:
            raise PsError(1, f"coil sensitivities must have shape (n_coils, {n_spins})")
        cs.append(t)
    if len(cs) != 2 or cs[0].shape != cs[1].shape:
        raise PsError(1, "coils must be a pair (s_x, s_y) of equal shape")
    rx = _b.ps_receive(int(cs[0].shape[0]), 0, cs[0].data_ptr() if cs[0].numel() else 0,
                       cs[1].data_ptr() if cs[1].numel() else 0)
    return cs, rx


class Ticket:
    """Handle of a served request (keeps its device arrays alive)."""

    def __init__(self, ctx: Context, ticket: int, out, dev):
        self.ctx, self.ticket, self._out, self._dev = ctx, ticket, out, dev

    def done(self) -> bool:
        d = ctypes.c_int32()
        _b.check(_b.lib.ps_poll(self.ctx._h, self.ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, timeout_s: float = -1.0):
        """Block until finished; returns the signal (complex128 CUDA tensor)
        or raises PsError with the request's failure status."""
        _b.check(_b.lib.ps_wait(self.ctx._h, self.ticket, float(timeout_s)))
        return self._out.view(__import__("torch").complex128)

    def cancel(self):
        _b.check(_b.lib.ps_cancel(self.ctx._h, self.ticket))

    def info(self) -> dict:
        i = _b.ps_request_info()
        _b.check(_b.lib.ps_request_info(self.ctx._h, self.ticket, ctypes.byref(i)))
        d = {f: getattr(i, f) for f, _ in i._fields_}
        d["state"] = _b.REQ_STATES.get(d["state"], d["state"])
        return d

    def stats(self) -> dict:
        """(ps_stats) t_queue, t_kernel and t_e2e in seconds; -1 where not known yet."""
        q, k, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _b.check(_b.lib.ps_stats(self.ctx._h, self.ticket, ctypes.byref(q), ctypes.byref(k), ctypes.byref(e)))
        return {"t_queue": q.value, "t_kernel": k.value, "t_e2e": e.value}

    def release(self):
        _b.check(_b.lib.ps_release(self.ctx._h, self.ticket))


class HostTicket(Ticket):
    """Ticket of a scheduler-test request: its signal is a host array."""

    def wait(self, timeout_s: float = -1.0):
        _b.check(_b.lib.ps_wait(self.ctx._h, self.ticket, float(timeout_s)))
        return self._out
