"""MI355X-native decorated-particle (Scovel-Weinstein, k = 2) Vlasov-Poisson hot path.

Thin Python binding over the C ABI of include/vp.h (libvp.so, HIP for gfx950).  PyTorch
provides device memory and the stream; every step of the method runs in the HIP kernels.

    eng = Engine("fp32c", max_slots=1)
    eng.admit(0, state, L=..., ng=512, dt=0.05)     # state: dict Q, P, qs, ps, psi
    eng.step(1000)
    d = eng.diagnostics(0)                           # K, W, H, charge, momentum, ...
    st = eng.retire(0)                               # state at the last integer step

There is no CPU fallback: constructing an Engine without the built library or without a
GPU raises.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from ctypes import byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

from . import _lib as L
from ._lib import VPError  # noqa: F401

PRECISIONS = {"fp64": L.VP_FP64, "fp32c": L.VP_FP32_COMP, "fp32": L.VP_FP32,
              "fp32ts": L.VP_FP32_TWOSUM}
FIELDS = ("Q", "P", "qs", "ps", "psi")
MOMENTS = ("Mqq", "Mqp", "Mpp")        # second moments of k = 3 particles


def load_library():
    return L.load()


# Engines still open when the interpreter starts to exit are closed by close_all(), which
# atexit runs before the interpreter tears its objects down: every handle, graph and device
# table of the library is released while the HIP runtime (and any tool attached to it, such
# as a profiler) is fully alive, never from a destructor during shutdown.
_open_engines = weakref.WeakSet()


def close_all():
    """Close every open Engine (and Simulation), after the device has finished its work."""
    engines = list(_open_engines)
    if not engines:
        return
    try:
        import torch
        torch.cuda.synchronize()
    except Exception:
        pass
    for e in engines:
        e.close()


atexit.register(close_all)


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


SOLVERS = {"scan": L.VP_SOLVE_SCAN, "fft": L.VP_SOLVE_FFT}
PROJECTIONS = {"elem": L.VP_PROJ_ELEM, "nodal": L.VP_PROJ_NODAL,
               "consistent": L.VP_PROJ_CONSISTENT}


def make_config(n, ng, L_, dt, precision, sort_every=0, sort_chunk=0, hist_cap=4096,
                solver="scan", projection="elem", monopole_only=False, self_field=True,
                external=None, element_order=1, moment_order=2):
    return L.vp_config(n=int(n), ng=int(ng), precision=_prec(precision), L=float(L_),
                       dt=float(dt), sort_every=int(sort_every), sort_chunk=int(sort_chunk),
                       hist_cap=int(hist_cap),
                       solver=SOLVERS[solver] if isinstance(solver, str) else int(solver),
                       projection=PROJECTIONS[projection] if isinstance(projection, str)
                       else int(projection), monopole_only=1 if monopole_only else 0,
                       no_self_field=0 if self_field else 1,
                       ext_mode=int(external["mode"]) if external else 0,
                       ext_amplitude=float(external["amp"]) if external else 0.0,
                       element_order=int(element_order), moment_order=int(moment_order))


def workspace_bytes(cfg) -> int:
    lib = L.load()
    b = c_size_t()
    L.check(lib.vp_workspace_bytes(byref(cfg), byref(b)), "vp_workspace_bytes")
    return int(b.value)


def wall_clock_hz() -> float:
    """Ticks per second of the device clock that stamps history records (vp_wall_clock_hz)."""
    lib = L.load()
    hz = c_double()
    L.check(lib.vp_wall_clock_hz(byref(hz)), "vp_wall_clock_hz")
    return float(hz.value)


def cluster_markers(Q, P, w, k: int, L_: float, iters: int = 10, init_idx=None, seed: int = 0,
                    return_assign: bool = False, stream=None, batch=None, nbatch: int = 0,
                    batch_idx=None):
    """Decorated particles from markers (the paper's Algorithm 1), on the GPU.

    Q, P, w: marker positions in [0, L), velocities and positive weights (device or host
    arrays, taken as float64).  k clusters from `iters` Lloyd iterations starting at the
    markers init_idx (by default k distinct markers drawn with `seed`).  With `batch`, the
    clusters come from `nbatch` mini-batch updates instead (batches of `batch` marker
    indices drawn with replacement with `seed`, or the given batch_idx of shape
    (nbatch, batch)); `iters` is then not used.  Returns a dict of device float64 tensors
    Q, P, qs, ps, psi (one entry per non-empty cluster), plus `assign` (int32, the final
    cluster of each marker) when return_assign, and `absorbed` (each centre's absorbed
    weight) in the mini-batch case."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the decorated-particle path runs only on the GPU")
    lib = L.load()
    dev = torch.device("cuda")

    def t64(a):
        if isinstance(a, torch.Tensor):
            return a.to(device=dev, dtype=torch.float64).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    def t32(a):
        if isinstance(a, torch.Tensor):
            return a.to(device=dev, dtype=torch.int32).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
    q, p, wt = t64(Q), t64(P), t64(w)
    m = int(q.numel())
    g = torch.Generator().manual_seed(int(seed))
    if init_idx is None:
        init_idx = torch.randperm(m, generator=g)[:int(k)]
    idx = t32(init_idx)
    mini = batch is not None or batch_idx is not None
    if mini:
        if batch_idx is None:
            batch_idx = torch.randint(0, m, (int(nbatch), int(batch)), generator=g)
        bidx = t32(batch_idx)
        if bidx.dim() != 2:
            raise ValueError("batch_idx must have shape (nbatch, batch)")
        nbatch, batch = int(bidx.shape[0]), int(bidx.shape[1])
    b = c_size_t()
    if mini:
        L.check(lib.vp_cluster_minibatch_workspace_bytes(m, int(k), batch, byref(b)),
                "vp_cluster_minibatch_workspace_bytes")
    else:
        L.check(lib.vp_cluster_workspace_bytes(m, int(k), byref(b)), "vp_cluster_workspace_bytes")
    ws = torch.empty(max(256, int(b.value)), dtype=torch.uint8, device=dev)
    out = {f: torch.empty(int(k), dtype=torch.float64, device=dev) for f in FIELDS}
    assign = torch.empty(m, dtype=torch.int32, device=dev) if return_assign else None
    absorbed = torch.empty(int(k), dtype=torch.float64, device=dev) if mini else None
    n = c_int32()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    outs = [c_void_p(out[f].data_ptr()) for f in FIELDS]
    ap = c_void_p(assign.data_ptr()) if assign is not None else None
    if mini:
        L.check(lib.vp_cluster_markers_minibatch(
            c_void_p(q.data_ptr()), c_void_p(p.data_ptr()), c_void_p(wt.data_ptr()), m, int(k),
            c_void_p(idx.data_ptr()), c_void_p(bidx.data_ptr()), batch, nbatch, float(L_),
            c_void_p(ws.data_ptr()), c_void_p(s.cuda_stream), *outs, ap,
            c_void_p(absorbed.data_ptr()), byref(n)), "vp_cluster_markers_minibatch")
    else:
        L.check(lib.vp_cluster_markers(
            c_void_p(q.data_ptr()), c_void_p(p.data_ptr()), c_void_p(wt.data_ptr()), m, int(k),
            c_void_p(idx.data_ptr()), int(iters), float(L_), c_void_p(ws.data_ptr()),
            c_void_p(s.cuda_stream), *outs, ap, byref(n)), "vp_cluster_markers")
    res = {f: out[f][:n.value] for f in FIELDS}
    if return_assign:
        res["assign"] = assign
    if mini:
        res["absorbed"] = absorbed
    return res


class Engine:
    """A set of slots, each holding one simulation instance, advanced together."""

    def __init__(self, precision="fp32c", max_slots: int = 1, device=None, stream=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the decorated-particle path runs only on the GPU")
        self.lib = L.load()
        self.prec = _prec(precision)
        self.dtype = torch.float64 if self.prec == L.VP_FP64 else torch.float32
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_slots = int(max_slots)
        h = c_void_p()
        L.check(self.lib.vp_engine_create(self.prec, self.max_slots,
                                          c_void_p(self.stream.cuda_stream), byref(h)),
                "vp_engine_create")
        self.h = h
        self.slots = {}
        _open_engines.add(self)

    # ---------------------------------------------------------------- slots
    def _tensor(self, a):
        t = self._torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=self.dtype).contiguous().clone()
        return t.from_numpy(np.ascontiguousarray(a)).to(device=self.device, dtype=self.dtype)

    def admit(self, slot: int, state: dict, L_: float, ng: int, dt: float, sort_every: int = 0,
              sort_chunk: int = 0, hist_cap: int = 4096, solver="scan", projection="elem",
              monopole_only: bool = False, self_field: bool = True, external=None,
              element_order: int = 1, moment_order: int = None):
        """Copy `state` (arrays Q, P, qs, ps, psi) to the device and admit it into `slot`.
        monopole_only: plain particle-in-cell particles (p* = q* = 0; qs, ps may be left out
        of `state`, and are zeroed on admission).  self_field=False: the particles feel no
        field of their own (charge e = 0).  external = {"amp": A, "mode": m}: the prescribed
        potential A (1 - cos(2 pi m q / L)).  element_order=2: P2 elements (a vertex and a
        midpoint node per element; phi_h'' from the basis).  moment_order=3 (the default when
        `state` holds Mqq): the particles also carry their second moments Mqq, Mqp, Mpp (k = 3;
        P2 elements only)."""
        t = self._torch
        if moment_order is None:
            moment_order = 3 if "Mqq" in state else 2
        names = FIELDS + (MOMENTS if moment_order == 3 else ())
        tens = {k: self._tensor(state[k]) for k in names if k in state}
        if monopole_only:
            for k in ("qs", "ps"):
                if k not in tens:
                    tens[k] = t.zeros_like(tens["Q"])
        missing = [k for k in names if k not in tens]
        if missing:
            raise ValueError(f"state lacks {missing}")
        n = int(tens["Q"].numel())
        if any(int(v.numel()) != n for v in tens.values()):
            raise ValueError("state arrays differ in length")
        cfg = make_config(n, ng, L_, dt, self.prec, sort_every, sort_chunk, hist_cap, solver,
                          projection, monopole_only, self_field, external, element_order,
                          moment_order)
        ws = t.zeros(workspace_bytes(cfg), dtype=t.uint8, device=self.device)
        if ws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        parts = L.vp_particles(*(c_void_p(tens[k].data_ptr() if k in tens else None)
                                 for k in FIELDS + MOMENTS))
        t.cuda.current_stream(self.device).synchronize()
        L.check(self.lib.vp_admit(self.h, int(slot), byref(cfg), parts, c_void_p(ws.data_ptr())),
                "vp_admit")
        self.slots[int(slot)] = {"tensors": tens, "ws": ws, "cfg": cfg}
        return tens

    def retire(self, slot: int) -> dict:
        """Remove the instance; returns its tensors holding the state at its last integer step."""
        L.check(self.lib.vp_retire(self.h, int(slot)), "vp_retire")
        rec = self.slots.pop(int(slot))
        return rec["tensors"]

    def free_slot(self):
        for s in range(self.max_slots):
            if s not in self.slots:
                return s
        return None

    def state(self, slot: int = 0) -> dict:
        """Device tensors of one slot (P, q* are half a kick ahead until sync_state())."""
        return self.slots[int(slot)]["tensors"]

    def state_numpy(self, slot: int = 0) -> dict:
        self.sync_state()
        self._torch.cuda.synchronize(self.device)
        return {k: v.detach().cpu().numpy() for k, v in self.state(slot).items()}

    # ---------------------------------------------------------------- steps
    def step(self, nsteps: int = 1):
        L.check(self.lib.vp_step(self.h, int(nsteps)), "vp_step")

    def prepare_step(self, nsteps: int):
        """Capture the graphs a later step(nsteps) replays, without stepping."""
        L.check(self.lib.vp_prepare_step(self.h, int(nsteps)), "vp_prepare_step")

    def sync_state(self):
        L.check(self.lib.vp_sync_state(self.h), "vp_sync_state")

    def deposit(self):
        L.check(self.lib.vp_deposit(self.h), "vp_deposit")

    def poisson(self):
        L.check(self.lib.vp_poisson(self.h), "vp_poisson")

    def gather_push(self, kick: float, drift: float):
        L.check(self.lib.vp_gather_push(self.h, float(kick), float(drift)), "vp_gather_push")

    def sort(self, slot: int = 0, want_perm: bool = False):
        t = self._torch
        perm = None
        ptr = None
        if want_perm:
            n = int(self.slots[int(slot)]["cfg"].n)
            perm = t.empty(n, dtype=t.int32, device=self.device)
            ptr = c_void_p(perm.data_ptr())
        L.check(self.lib.vp_sort(self.h, int(slot), ptr), "vp_sort")
        return perm

    def cell_index(self, slot: int = 0):
        t = self._torch
        n = int(self.slots[int(slot)]["cfg"].n)
        cells = t.empty(n, dtype=t.int32, device=self.device)
        L.check(self.lib.vp_cell_index(self.h, int(slot), c_void_p(cells.data_ptr())),
                "vp_cell_index")
        return cells

    # ---------------------------------------------------------------- diagnostics
    def diagnostics(self, slot: int = 0, grid: bool = False, allow_nonfinite: bool = False):
        d = L.vp_diag()
        cfg = self.slots[int(slot)]["cfg"]
        ng = int(cfg.ng)
        na = 2 * ng if int(cfg.element_order) == 2 else ng   # nodes of b~ and Phi
        buf = np.zeros(2 * na + 2 * ng) if grid else None
        ptr = buf.ctypes.data_as(c_void_p) if grid else None
        st = self.lib.vp_diagnostics(self.h, int(slot), byref(d), ptr)
        if not (allow_nonfinite and st == L.VP_ERR_NONFINITE):
            L.check(st, "vp_diagnostics")
        out = d.as_dict()
        out["finite"] = st == L.VP_OK   # False once the instance went NaN / Inf (and froze)
        if grid:
            out.update(bt=buf[:na], Phi=buf[na:2 * na], E=buf[2 * na:2 * na + ng],
                       g=buf[2 * na + ng:])
        return out

    def history(self, slot: int, first: int, count: int, allow_nonfinite: bool = False):
        arr = (L.vp_diag * max(1, int(count)))()
        st = self.lib.vp_history(self.h, int(slot), int(first), int(count), arr)
        if not (allow_nonfinite and st == L.VP_ERR_NONFINITE):
            L.check(st, "vp_history")
        return [arr[i].as_dict() for i in range(int(count))]

    def history_array(self, slot: int, first: int, count: int, allow_nonfinite: bool = False):
        """The same records as history(), as one numpy structured array (a field per
        vp_diag member; no per-record Python objects)."""
        arr = (L.vp_diag * max(1, int(count)))()
        st = self.lib.vp_history(self.h, int(slot), int(first), int(count), arr)
        if not (allow_nonfinite and st == L.VP_ERR_NONFINITE):
            L.check(st, "vp_history")
        dt = np.dtype([(k, np.int64 if k == "step" else np.float64)
                       for k, _ in L.vp_diag._fields_])
        assert dt.itemsize == ctypes.sizeof(L.vp_diag)
        return np.frombuffer(arr, dtype=dt, count=int(count)).copy()

    # ---------------------------------------------------------------- tuning
    def get_tuning(self) -> dict:
        tu = L.vp_tuning()
        L.check(self.lib.vp_get_tuning(self.h, byref(tu)), "vp_get_tuning")
        return tu.as_dict()

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        tu = L.vp_tuning(**cur)
        L.check(self.lib.vp_set_tuning(self.h, byref(tu)), "vp_set_tuning")

    def tune(self, steps_per_trial: int = 20):
        """Time every candidate launch shape on the current slots, keep the fastest."""
        t = self._torch
        b = c_size_t()
        L.check(self.lib.vp_tune_scratch_bytes(self.h, byref(b)), "vp_tune_scratch_bytes")
        scratch = t.empty(max(256, int(b.value)), dtype=t.uint8, device=self.device)
        best = L.vp_tuning()
        us = c_double()
        L.check(self.lib.vp_tune(self.h, c_void_p(scratch.data_ptr()), int(steps_per_trial),
                                 byref(best), byref(us)), "vp_tune")
        return best.as_dict(), float(us.value)

    def occupancy(self):
        s, p = c_int32(), c_int64()
        L.check(self.lib.vp_occupancy(self.h, byref(s), byref(p)), "vp_occupancy")
        return int(s.value), int(p.value)

    def slot_status(self):
        """{slot: (device step, finite)} for every occupied slot, from one device call."""
        n = self.max_slots
        steps = (c_int64 * n)()
        flags = (c_int32 * n)()
        L.check(self.lib.vp_slot_status(self.h, n, steps, flags), "vp_slot_status")
        return {s: (int(steps[s]), not (flags[s] & L.VP_SLOT_NONFINITE))
                for s in range(n) if flags[s] & L.VP_SLOT_OCCUPIED}

    def close(self):
        if getattr(self, "h", None):
            self.lib.vp_destroy(self.h)
            self.h = None
        _open_engines.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation(Engine):
    """One instance: Simulation(state, L, ng, dt, precision)."""

    def __init__(self, state: dict, L_: float, ng: int, dt: float, precision="fp32c",
                 sort_every: int = 0, sort_chunk: int = 0, hist_cap: int = 4096, device=None,
                 stream=None, solver="scan", projection="elem", monopole_only=False,
                 self_field=True, external=None, element_order=1, moment_order=None):
        super().__init__(precision, 1, device, stream)
        self.admit(0, state, L_, ng, dt, sort_every, sort_chunk, hist_cap, solver, projection,
                   monopole_only, self_field, external, element_order, moment_order)
