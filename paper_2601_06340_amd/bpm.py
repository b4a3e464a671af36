"""ctypes binding of libbpm_hip.so (include/bpm.h), argument marshalling only.

Every step of the march runs in the HIP library; this module converts Python
problem dicts (see ``synth``) into the C descriptors, holds the arrays they
point to, and turns status codes into exceptions.  It raises ImportError-like
``BpmError`` at load time if the built library is missing -- there is no CPU
fallback.

torch is imported before the library is loaded so that both share one HIP
runtime; torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch  # noqa: F401  (shares its HIP runtime with the library)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbpm_hip.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_BUDGET, E_PENDING, E_CANCELLED, E_NOTFOUND, \
    E_UNSUPPORTED, E_NUMERIC = range(10)
F64, F32 = 0, 1
PRECISION = {"f64": F64, "f32": F32}
STRAIN = {"none": 0, "poly2": 1, "edge_dislocation": 2, "table": 3}


class BpmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Complex(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Strain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("x_ref_um", C.c_double), ("z_ref_um", C.c_double),
                ("c", C.c_double * 6), ("b_um", C.c_double), ("nu", C.c_double),
                ("u_table", C.POINTER(C.c_double))]


class PlanDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("dx_um", C.c_double), ("dz_um", C.c_double),
                ("x0_um", C.c_double), ("lambda_um", C.c_double), ("d_um", C.c_double),
                ("chi0", Complex), ("chih", Complex), ("chihbar", Complex),
                ("nseg", C.c_int32), ("seg", C.POINTER(C.c_int32)), ("strain", Strain),
                ("det_lo", C.c_int32), ("det_hi", C.c_int32), ("precision", C.c_int32),
                ("split_order", C.c_int32), ("ny", C.c_int32), ("dy_um", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
                ("threads_per_solve", C.c_int32), ("state_bytes", C.c_size_t),
                ("device_bytes", C.c_size_t), ("cell_steps", C.c_double)]


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("chunk_steps", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("plan", C.POINTER(PlanDesc)), ("psi_p0", C.POINTER(Complex)),
                ("psi_m0", C.POINTER(Complex)), ("psi_p_out", C.POINTER(Complex)),
                ("psi_m_out", C.POINTER(Complex))]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("R", C.c_double), ("T", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("cancelled", C.c_int64), ("failed", C.c_int64), ("launches", C.c_int64),
                ("cell_steps_done", C.c_double), ("bytes_in_use", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("wide", C.c_int64), ("rounds", C.c_int64),
                ("active_max", C.c_int64), ("t_device_wait_s", C.c_double),
                ("t_host_s", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("nsolves", C.c_int32), ("nsteps", C.c_int32),
                ("ms", C.c_double * 4)]


SCHEDULES = {"default": 0, "uniform": 1, "mixed": 2, "any": 3}


# name -> (restype, argtypes); every entry point declared in include/bpm.h
SIGNATURES = {
    "bpm_autotune": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(TuneResult)]),
    "bpm_schedule_set": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "bpm_schedule_get": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "bpm_schedule_save": (C.c_int, [C.c_char_p]),
    "bpm_schedule_load": (C.c_int, [C.c_char_p]),
    "bpm_plan_create": (C.c_int, [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]),
    "bpm_plan_destroy": (None, [C.c_void_p]),
    "bpm_plan_info_get": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "bpm_propagate": (C.c_int, [C.c_void_p, C.POINTER(Complex), C.POINTER(Complex), C.POINTER(Complex),
                                C.POINTER(Complex), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "bpm_propagate_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpm_propagate_device_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpm_far_field": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpm_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "bpm_batch_layout": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "bpm_batch_run": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpm_batch_destroy": (None, [C.c_void_p]),
    "bpm_td_assemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpm_server_create": (C.c_int, [C.POINTER(ServerDesc), C.POINTER(C.c_void_p)]),
    "bpm_batch_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.c_int32, C.POINTER(C.c_uint64)]),
    "bpm_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Result)]),
    "bpm_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "bpm_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "bpm_server_drain": (C.c_int, [C.c_void_p, C.c_double]),
    "bpm_server_destroy": (None, [C.c_void_p]),
    "bpm_status_str": (C.c_char_p, [C.c_int]),
    "bpm_last_error": (C.c_char_p, []),
    "bpm_max_nx": (C.c_int32, [C.c_int32]),
}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BpmError(E_DEVICE, "libbpm_hip.so not built (run __graft_entry__.build() or "
                                     "python -m paper_2601_06340_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise BpmError(rc, lib().bpm_last_error().decode())


def _cbuf(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(Complex))


class _Desc:
    """A PlanDesc plus the numpy arrays it points into."""

    def __init__(self, p: dict):
        d = PlanDesc()
        d.nx, d.nz = int(p["nx"]), int(p["nz"])
        d.dx_um, d.dz_um = float(p["dx_um"]), float(p["dz_um"])
        d.x0_um = float(p.get("x0_um", 0.0))
        d.lambda_um, d.d_um = float(p["lambda_um"]), float(p["d_um"])
        for name, key in (("chi0", "chi0"), ("chih", "chih"), ("chihbar", "chihb")):
            v = complex(p.get(key, p["chih"]))
            setattr(d, name, Complex(v.real, v.imag))
        self.seg = np.ascontiguousarray(p["seg"], dtype=np.int32)
        d.ny = int(p.get("ny", 1))
        d.dy_um = float(p.get("dy_um", 0.0))
        if d.ny > 1:   # 3D: [nz][ny][nseg][2]
            d.nseg = int(self.seg.shape[2]) if self.seg.ndim == 4 else 1
        else:
            d.nseg = int(self.seg.shape[1]) if self.seg.ndim == 3 else 1
        d.seg = self.seg.ctypes.data_as(C.POINTER(C.c_int32))
        st = p.get("strain") or {"kind": "none"}
        d.strain.kind = STRAIN[st.get("kind", "none")]
        d.strain.x_ref_um = float(st.get("x_ref_um", 0.0))
        d.strain.z_ref_um = float(st.get("z_ref_um", 0.0))
        for i, c in enumerate(st.get("c", [0.0] * 6)):
            d.strain.c[i] = float(c)
        d.strain.b_um = float(st.get("b_um", 0.0))
        d.strain.nu = float(st.get("nu", 0.0))
        self.utab = None
        if d.strain.kind == STRAIN["table"]:
            self.utab = np.ascontiguousarray(st["u_table"], dtype=np.float64)
            d.strain.u_table = self.utab.ctypes.data_as(C.POINTER(C.c_double))
        d.det_lo = int(p.get("det_lo", 0))
        d.det_hi = int(p.get("det_hi", p["nx"]))
        d.precision = PRECISION[p.get("precision", "f64")]
        d.split_order = int(p.get("split_order", 1))
        self.c = d


class Plan:
    """A device plan (bpm_plan_create)."""

    def __init__(self, problem: dict):
        self._desc = _Desc(problem)
        h = C.c_void_p()
        _check(lib().bpm_plan_create(C.byref(self._desc.c), C.byref(h)))
        self.handle = h
        info = PlanInfo()
        _check(lib().bpm_plan_info_get(h, C.byref(info)))
        self.info = info
        self.nx = info.nx
        self.ny = max(1, int(problem.get("ny", 1)))
        self.cells = self.nx * self.ny              # samples per beam
        self.shape = (self.ny, self.nx) if self.ny > 1 else (self.nx,)
        self.precision = "f32" if info.precision == F32 else "f64"

    @property
    def cdtype(self):
        return torch.complex64 if self.precision == "f32" else torch.complex128

    def propagate(self, psi_p0, psi_m0=None):
        """Blocking march from host arrays.  Returns (psi_p, psi_m, R, T)."""
        a = np.ascontiguousarray(psi_p0, dtype=np.complex128).reshape(-1)
        b = None if psi_m0 is None else np.ascontiguousarray(psi_m0, dtype=np.complex128).reshape(-1)
        op = np.empty(self.cells, np.complex128)
        om = np.empty(self.cells, np.complex128)
        R, T = C.c_double(), C.c_double()
        _check(lib().bpm_propagate(self.handle, _cbuf(a), None if b is None else _cbuf(b),
                                   _cbuf(op), _cbuf(om), C.byref(R), C.byref(T)))
        return op.reshape(self.shape), om.reshape(self.shape), R.value, T.value

    def propagate_device(self, d_in: int, d_out: int, d_rt: int | None = None, stream: int | None = None):
        """Asynchronous march on device buffers (raw pointers, plan precision)."""
        _check(lib().bpm_propagate_device(self.handle, stream, d_in, d_out, d_rt))

    def propagate_device_noalloc(self, d_in: int, d_out: int, d_rt: int | None = None, stream: int | None = None):
        """bpm_propagate_device without any device allocation (the library's static scratch)."""
        _check(lib().bpm_propagate_device_noalloc(self.handle, stream, d_in, d_out, d_rt))

    def far_field_device(self, distance_um: float, d_in: int, d_out: int, stream: int | None = None):
        """Vacuum propagation of a device state over distance_um (bpm_far_field)."""
        _check(lib().bpm_far_field(self.handle, float(distance_um), stream, d_in, d_out))

    def far_field(self, distance_um: float, psi_p, psi_m=None):
        """Host arrays in and out (copies through a device state of the plan's precision)."""
        n = self.cells
        st = torch.zeros(2 * n, dtype=self.cdtype)
        st[:n] = torch.from_numpy(np.asarray(psi_p, np.complex128).reshape(-1)).to(self.cdtype)
        if psi_m is not None:
            st[n:] = torch.from_numpy(np.asarray(psi_m, np.complex128).reshape(-1)).to(self.cdtype)
        d = st.to("cuda")
        self.far_field_device(distance_um, d.data_ptr(), d.data_ptr(), torch.cuda.current_stream().cuda_stream)
        out = d.cpu().to(torch.complex128).numpy()
        return out[:n].reshape(self.shape), out[n:].reshape(self.shape)

    def close(self):
        if getattr(self, "handle", None):
            lib().bpm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many plans marched by one launch per precision (bpm_batch_*)."""

    def __init__(self, plans: list):
        self.plans = list(plans)
        arr = (C.c_void_p * max(1, len(plans)))(*[p.handle for p in plans])
        h = C.c_void_p()
        _check(lib().bpm_batch_create(arr, len(plans), C.byref(h)))
        self.handle = h
        offs = (C.c_size_t * max(1, len(plans)))()
        total = C.c_size_t()
        _check(lib().bpm_batch_layout(h, offs, C.byref(total)))
        self.offsets = [int(offs[i]) for i in range(len(plans))]
        self.total_bytes = int(total.value)

    def run(self, d_in: int, d_out: int, d_rt: int | None = None, stream: int | None = None):
        _check(lib().bpm_batch_run(self.handle, stream, d_in, d_out, d_rt))

    def td_assemble(self, d_state: int, stream: int | None = None) -> torch.Tensor:
        """Time-domain assembly of the batch's exit envelopes (bpm_td_assemble):
        a [2, nx, M] complex tensor on the device."""
        p = self.plans[0]
        out = torch.empty((2, p.nx, len(self.plans)), dtype=p.cdtype, device="cuda")
        _check(lib().bpm_td_assemble(self.handle, stream, d_state, out.data_ptr()))
        return out

    def pack(self, psis: list, device="cuda") -> torch.Tensor:
        """Device byte buffer holding every solve's entrance state at its offset."""
        buf = torch.zeros(self.total_bytes, dtype=torch.uint8, device=device)
        for p, off, (a, b) in zip(self.plans, self.offsets, psis):
            st = torch.zeros(2 * p.cells, dtype=p.cdtype)
            st[: p.cells] = torch.from_numpy(np.asarray(a, np.complex128).reshape(-1)).to(p.cdtype)
            if b is not None:
                st[p.cells:] = torch.from_numpy(np.asarray(b, np.complex128).reshape(-1)).to(p.cdtype)
            raw = st.view(torch.uint8)
            buf[off: off + raw.numel()].copy_(raw.to(device))
        return buf

    def unpack(self, buf: torch.Tensor) -> list:
        """Host (psi_p, psi_m) complex128 arrays of every solve."""
        host = buf.cpu()
        out = []
        for p, off in zip(self.plans, self.offsets):
            nb = 2 * p.cells * (8 if p.precision == "f32" else 16)
            st = host[off: off + nb].view(p.cdtype).numpy().astype(np.complex128)
            out.append((st[: p.cells].reshape(p.shape), st[p.cells:].reshape(p.shape)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().bpm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (bpm_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 512, chunk_steps: int = 256):
        d = ServerDesc(int(hbm_budget_bytes), int(max_slots), int(chunk_steps))
        h = C.c_void_p()
        _check(lib().bpm_server_create(C.byref(d), C.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, problem: dict, psi_p0, psi_m0=None, want_fields: bool = True) -> int:
        desc = _Desc(problem)
        a = np.ascontiguousarray(psi_p0, dtype=np.complex128).reshape(-1)
        b = None if psi_m0 is None else np.ascontiguousarray(psi_m0, dtype=np.complex128).reshape(-1)
        ny = max(1, int(problem.get("ny", 1)))
        shape = (ny, int(problem["nx"])) if ny > 1 else (int(problem["nx"]),)
        op = np.empty(shape, np.complex128) if want_fields else None
        om = np.empty(shape, np.complex128) if want_fields else None
        req = Request(C.pointer(desc.c), _cbuf(a), None if b is None else _cbuf(b),
                      None if op is None else _cbuf(op), None if om is None else _cbuf(om))
        t = C.c_uint64()
        rc = lib().bpm_batch_submit(self.handle, C.byref(req), 1, C.byref(t))
        if rc not in (OK, E_BUDGET):
            _check(rc)
        self._keep[int(t.value)] = (op, om, a, b, desc)
        return int(t.value)

    def poll(self, ticket: int):
        """None while pending, else dict(status, R, T, t_submit, t_admit, t_done, psi_p, psi_m)."""
        r = Result()
        rc = lib().bpm_poll(self.handle, ticket, C.byref(r))
        if rc == E_PENDING:
            return None
        _check(rc)
        op, om = self._keep.get(ticket, (None, None))[:2]
        return {"status": r.status, "R": r.R, "T": r.T, "t_submit": r.t_submit,
                "t_admit": r.t_admit, "t_done": r.t_done, "psi_p": op, "psi_m": om}

    def cancel(self, ticket: int):
        _check(lib().bpm_cancel(self.handle, ticket))

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().bpm_server_stats_get(self.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def drain(self, timeout_s: float = -1.0) -> bool:
        rc = lib().bpm_server_drain(self.handle, float(timeout_s))
        if rc == E_PENDING:
            return False
        _check(rc)
        return True

    def close(self):
        if getattr(self, "handle", None):
            lib().bpm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(precision: str, nx: int, strain_kind: int = 0, nsolves: int = 256, nsteps: int = 200) -> dict:
    """Time every kernel family that can march nx on a synthetic batch, enter the
    fastest into the schedule table (bpm_autotune); returns the choice and times."""
    r = TuneResult()
    _check(lib().bpm_autotune(PRECISION[precision], int(nx), int(strain_kind), int(nsolves), int(nsteps),
                              C.byref(r)))
    names = {v: k for k, v in SCHEDULES.items()}
    return {"schedule": names[r.schedule], "nsolves": r.nsolves, "nsteps": r.nsteps,
            "ms": {names[i]: r.ms[i] for i in range(1, 4) if r.ms[i] > 0}}


def schedule_set(precision: str, nx: int, strain_kind: int, schedule: str):
    _check(lib().bpm_schedule_set(PRECISION[precision], int(nx), int(strain_kind), SCHEDULES[schedule]))


def schedule_get(precision: str, nx: int, strain_kind: int) -> str:
    v = lib().bpm_schedule_get(PRECISION[precision], int(nx), int(strain_kind))
    if v < 0:
        raise BpmError(E_INVALID, "bad schedule key")
    return {v2: k for k, v2 in SCHEDULES.items()}[v]


def schedule_save(path: str):
    _check(lib().bpm_schedule_save(str(path).encode()))


def schedule_load(path: str):
    _check(lib().bpm_schedule_load(str(path).encode()))


def max_nx(precision: str) -> int:
    return int(lib().bpm_max_nx(PRECISION[precision]))


def status_str(rc: int) -> str:
    return lib().bpm_status_str(rc).decode()
