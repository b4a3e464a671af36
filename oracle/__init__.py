"""TEST INFRASTRUCTURE: ctypes wrapper around the FP64 C oracle (``bpm_oracle.c``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this
package imports nothing from the product package.

Problems are passed as plain dicts (the same dicts the input generators in
``paper_2601_06340_amd.synth`` produce), so the oracle and the GPU path see
identical inputs without sharing code.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bpm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STRAIN_KIND = {"none": 0, "poly2": 1, "edge_dislocation": 2, "table": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("nz", C.c_int),
        ("dx_um", C.c_double), ("dz_um", C.c_double), ("x0_um", C.c_double),
        ("lambda_um", C.c_double), ("d_um", C.c_double),
        ("chi0_re", C.c_double), ("chi0_im", C.c_double),
        ("chih_re", C.c_double), ("chih_im", C.c_double),
        ("chihb_re", C.c_double), ("chihb_im", C.c_double),
        ("nseg", C.c_int), ("seg", C.POINTER(C.c_int)),
        ("strain_kind", C.c_int),
        ("x_ref_um", C.c_double), ("z_ref_um", C.c_double),
        ("strain_c", C.c_double * 6),
        ("disl_b_um", C.c_double), ("disl_nu", C.c_double),
        ("u_table", C.POINTER(C.c_double)),
        ("det_lo", C.c_int), ("det_hi", C.c_int),
        ("split_order", C.c_int),
        ("ny", C.c_int), ("dy_um", C.c_double),
    ]


class _Scalars(C.Structure):
    _fields_ = [("k", C.c_double), ("h", C.c_double), ("s", C.c_double),
                ("c", C.c_double), ("dzh", C.c_double),
                ("a0", C.c_double * 2), ("ap", C.c_double * 2), ("am", C.c_double * 2)]


_lib = None


def _open(path: str):
    L = C.CDLL(path)
    cd = C.POINTER(C.c_double)
    L.oracle_fft.argtypes = [cd, C.c_int, C.c_int]
    L.oracle_dft.argtypes = [cd, cd, C.c_int, C.c_int]
    L.oracle_dft.restype = None
    L.oracle_bessel_series.argtypes = [C.c_double, C.c_double, cd, cd]
    L.oracle_bessel_series.restype = None
    L.oracle_exp_series.argtypes = [C.c_double, C.c_double, cd, cd]
    L.oracle_exp_series.restype = None
    L.oracle_coupling.argtypes = [C.POINTER(_Desc), C.c_double, C.c_int, cd, cd, cd]
    L.oracle_propagator_frac.argtypes = [C.POINTER(_Desc), C.c_double, cd, cd]
    L.oracle_split_sequence.argtypes = [C.c_int, cd, cd]
    L.oracle_strain_phase_z.argtypes = [C.POINTER(_Desc), C.c_int, C.c_int, C.c_double]
    L.oracle_strain_phase_z.restype = C.c_double
    L.oracle_td_assemble.argtypes = [C.POINTER(_Desc), C.c_int, cd, cd]
    L.oracle_scalars_get.argtypes = [C.POINTER(_Desc), C.POINTER(_Scalars)]
    L.oracle_propagator.argtypes = [C.POINTER(_Desc), cd, cd]
    L.oracle_strain_phase.argtypes = [C.POINTER(_Desc), C.c_int, C.c_int]
    L.oracle_strain_phase.restype = C.c_double
    L.oracle_propagate.argtypes = [C.POINTER(_Desc), cd, cd, cd, cd]
    L.oracle_propagate_batch.argtypes = [C.POINTER(_Desc), C.c_int, C.POINTER(cd),
                                         cd, cd, C.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _open(_LIB)
    return _lib


def build_variant(src_text: str, out_path: str) -> str:
    """Compile another C text of the oracle (same flags) to ``out_path``.  The
    mutation tests use it to build copies with one deliberate mistake each."""
    c_path = out_path[:-3] + ".c" if out_path.endswith(".so") else out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-I", _HERE, "-o", out_path, c_path, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


@contextlib.contextmanager
def using(path: str):
    """Route every call of this module to another build of the oracle for the
    duration of the block."""
    global _lib
    saved = _lib
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = saved


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Keep:
    """Holds the numpy arrays a descriptor points into."""

    def __init__(self):
        self.refs = []


def _desc(p: dict, keep: _Keep) -> _Desc:
    d = _Desc()
    d.nx, d.nz = int(p["nx"]), int(p["nz"])
    d.dx_um, d.dz_um = float(p["dx_um"]), float(p["dz_um"])
    d.x0_um = float(p.get("x0_um", 0.0))
    d.lambda_um, d.d_um = float(p["lambda_um"]), float(p["d_um"])
    chi0, chih = complex(p["chi0"]), complex(p["chih"])
    chihb = complex(p.get("chihb", chih))
    d.chi0_re, d.chi0_im = chi0.real, chi0.imag
    d.chih_re, d.chih_im = chih.real, chih.imag
    d.chihb_re, d.chihb_im = chihb.real, chihb.imag
    seg = np.ascontiguousarray(p["seg"], dtype=np.int32)
    keep.refs.append(seg)
    d.nseg = int(seg.shape[1]) if seg.ndim == 3 else 1
    d.seg = seg.ctypes.data_as(C.POINTER(C.c_int))
    st = p.get("strain", {"kind": "none"})
    d.strain_kind = STRAIN_KIND[st.get("kind", "none")]
    d.x_ref_um = float(st.get("x_ref_um", 0.0))
    d.z_ref_um = float(st.get("z_ref_um", 0.0))
    cc = st.get("c", [0.0] * 6)
    for i in range(6):
        d.strain_c[i] = float(cc[i])
    d.disl_b_um = float(st.get("b_um", 0.0))
    d.disl_nu = float(st.get("nu", 0.0))
    if d.strain_kind == STRAIN_KIND["table"]:
        ut = np.ascontiguousarray(st["u_table"], dtype=np.float64)
        keep.refs.append(ut)
        d.u_table = _dptr(ut)
    d.det_lo = int(p.get("det_lo", 0))
    d.det_hi = int(p.get("det_hi", p["nx"]))
    d.split_order = int(p.get("split_order", 1))
    d.ny = int(p.get("ny", 1))
    d.dy_um = float(p.get("dy_um", 0.0))
    if d.ny > 1:
        d.nseg = int(seg.shape[2]) if seg.ndim == 4 else 1
    return d


def fft(a: np.ndarray, sign: int = -1) -> np.ndarray:
    x = np.ascontiguousarray(a, dtype=np.complex128).copy()
    rc = lib().oracle_fft(_dptr(x), len(x), sign)
    if rc:
        raise ValueError("oracle_fft failed (%d)" % rc)
    return x


def dft(a: np.ndarray, sign: int = -1) -> np.ndarray:
    x = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.empty_like(x)
    lib().oracle_dft(_dptr(x), _dptr(out), len(x), sign)
    return out


def bessel_series(y: complex):
    j0 = np.zeros(1, np.complex128)
    g = np.zeros(1, np.complex128)
    lib().oracle_bessel_series(complex(y).real, complex(y).imag, _dptr(j0), _dptr(g))
    return complex(j0[0]), complex(g[0])


def exp_series(y: complex):
    """cosh(v) and sinh(v)/v as series in y = v^2."""
    ch = np.zeros(1, np.complex128)
    sh = np.zeros(1, np.complex128)
    lib().oracle_exp_series(complex(y).real, complex(y).imag, _dptr(ch), _dptr(sh))
    return complex(ch[0]), complex(sh[0])


def coupling(p: dict, b: float, form: int):
    """(a0, ap, am) of a coupling sub-step b*dz; form 0 Jacobi-Anger, 1 exponential."""
    keep = _Keep()
    d = _desc(p, keep)
    out = [np.zeros(1, np.complex128) for _ in range(3)]
    if lib().oracle_coupling(C.byref(d), float(b), int(form), *[_dptr(o) for o in out]):
        raise ValueError("invalid problem")
    return tuple(complex(o[0]) for o in out)


def propagator_frac(p: dict, a: float):
    keep = _Keep()
    d = _desc(p, keep)
    pp = np.zeros(d.nx, np.complex128)
    pm = np.zeros(d.nx, np.complex128)
    if lib().oracle_propagator_frac(C.byref(d), float(a), _dptr(pp), _dptr(pm)):
        raise ValueError("invalid problem")
    return pp, pm


def split_sequence(order: int):
    a = np.zeros(8)
    b = np.zeros(8)
    m = lib().oracle_split_sequence(int(order), _dptr(a), _dptr(b))
    return list(a[:m]), list(b[:m])


def strain_phase_z(p: dict, j: int, n: int, z: float) -> float:
    keep = _Keep()
    d = _desc(p, keep)
    return lib().oracle_strain_phase_z(C.byref(d), int(j), int(n), float(z))


def scalars(p: dict) -> dict:
    keep = _Keep()
    d = _desc(p, keep)
    s = _Scalars()
    if lib().oracle_scalars_get(C.byref(d), C.byref(s)):
        raise ValueError("invalid problem")
    cx = lambda v: complex(v[0], v[1])
    return {"k": s.k, "h": s.h, "s": s.s, "c": s.c, "dzh": s.dzh,
            "a0": cx(s.a0), "ap": cx(s.ap), "am": cx(s.am)}


def propagator(p: dict):
    keep = _Keep()
    d = _desc(p, keep)
    n = d.nx
    pp = np.zeros(n, np.complex128)
    pm = np.zeros(n, np.complex128)
    if lib().oracle_propagator(C.byref(d), _dptr(pp), _dptr(pm)):
        raise ValueError("invalid problem")
    return pp, pm


def strain_phase(p: dict, j: int, n: int) -> float:
    keep = _Keep()
    d = _desc(p, keep)
    return lib().oracle_strain_phase(C.byref(d), int(j), int(n))


def propagate(p: dict, psi_p0: np.ndarray, psi_m0: np.ndarray | None = None):
    """Run the full march.  Returns (psi_p, psi_m, R, T)."""
    keep = _Keep()
    d = _desc(p, keep)
    a = np.ascontiguousarray(psi_p0, dtype=np.complex128).copy()
    if psi_m0 is None:
        b = np.zeros_like(a)
    else:
        b = np.ascontiguousarray(psi_m0, dtype=np.complex128).copy()
    R = np.zeros(1)
    T = np.zeros(1)
    rc = lib().oracle_propagate(C.byref(d), _dptr(a), _dptr(b), _dptr(R), _dptr(T))
    if rc:
        raise ValueError("oracle_propagate failed (%d)" % rc)
    return a, b, float(R[0]), float(T[0])


def propagate_batch(problems: list, psi0: list, nthreads: int | None = None):
    """Many independent solves on a thread pool.  psi0[i] = (psi_p0, psi_m0 or None).
    Returns (list of (psi_p, psi_m), R array, T array)."""
    n = len(problems)
    keep = _Keep()
    descs = (_Desc * max(n, 1))()
    bufs = []
    for i, p in enumerate(problems):
        descs[i] = _desc(p, keep)
        pp0, pm0 = psi0[i]
        nx = int(p["nx"])
        buf = np.zeros(2 * nx, np.complex128)
        buf[:nx] = pp0
        if pm0 is not None:
            buf[nx:] = pm0
        bufs.append(buf)
    ptrs = (C.POINTER(C.c_double) * max(n, 1))(*[_dptr(b) for b in bufs])
    R = np.zeros(max(n, 1))
    T = np.zeros(max(n, 1))
    nt = nthreads or os.cpu_count() or 1
    rc = lib().oracle_propagate_batch(descs, n, ptrs, _dptr(R), _dptr(T), int(nt))
    if rc:
        raise ValueError("oracle_propagate_batch failed (%d)" % rc)
    outs = [(b[: len(b) // 2].copy(), b[len(b) // 2:].copy()) for b in bufs]
    return outs, R[:n].copy(), T[:n].copy()


def td_assemble(problems: list, exits: list):
    """Time-domain assembly of M components: exits[m] = (psi_p, psi_m) at the exit
    plane.  Returns out[2][nx][M] (beam, x sample, time sample)."""
    keep = _Keep()
    M = len(problems)
    arr = (_Desc * M)(*[_desc(p, keep) for p in problems])
    nx = int(problems[0]["nx"])
    psi = np.zeros((M, 2, nx), np.complex128)
    for m, (a, b) in enumerate(exits):
        psi[m, 0] = a
        psi[m, 1] = b
    out = np.zeros((2, nx, M), np.complex128)
    if lib().oracle_td_assemble(arr, M, _dptr(psi), _dptr(out)):
        raise ValueError("invalid components")
    return out
