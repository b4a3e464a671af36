"""Seeded synthetic inputs for the two-beam BPM march.

This module builds *inputs* only: incident envelopes, crystal-shape masks (as
per-step index intervals), strain-field parameters and random draws.  It holds
none of the method's arithmetic (no propagators, no coupling, no FFTs), so the
FP64 oracle and the HIP path can both consume what it makes without sharing
code.

Crystal shapes are rasterised here once, on the host, as half-open index
intervals ``[lo, hi)`` per z-step: a cell ``j`` at step ``n`` is inside the
crystal when ``lo <= j < hi`` for one of the step's intervals (the binary mask
Pi(x, z) of Eq. (9)-(10)).

Workload recipes (synthetic stand-ins for the paper's crystals; all numbers in
micrometres unless stated):

* common: lambda = d = 0.95 Angstrom (theta_B = 30 deg, E = 13.051 keV),
  chi0 = -2e-6 + 1e-8j, chih = chihb = -1.5e-6 + 8e-9j.
* ``flat_bragg``  - symmetric Bragg slab, Nx 4096, dx 0.1, Nz 2000, dz 0.05,
  crystal x in [256, 384), Gaussian beam w = 50 at x = 128, 64 angles across
  three Darwin widths around the refraction-shifted peak, detector x < 256.
* ``bent_laue``   - symmetric Laue plate filling z in [0, 200], Nx 16384, dx 0.1,
  Nz 8000, dz 0.025, displacement along h u = (x - Lx/2)(z - 100)/R, R in
  {1, 0.1, 10} m, seeded beam centre, width and angle, detector = window.
* ``disl_bragg``  - asymmetric (10 deg) Bragg trapezoid with one edge dislocation,
  Nx 32768, dx 0.1, Nz 16000, dz 0.05, b = 0.38 nm along h, nu = 0.22, core at a
  seeded depth below the entrance face, half-cell offsets.
* ``td_batch``    - 1024 photon energies of a 20 fs Gaussian pulse with seeded
  spectral phases, each a flat-Bragg solve with Nx in {2048..16384} and Nz in
  [1000, 8000] drawn per component.
* ``serve_mix``   - Poisson request stream mixing the above shapes.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------- constants
LAMBDA_UM = 0.95e-4           # 0.95 Angstrom
D_UM = 0.95e-4                # d-spacing; lambda = d -> theta_B = 30 deg
HC_KEV_ANGSTROM = 12.398419843320026
E0_KEV = HC_KEV_ANGSTROM / 0.95
CHI0 = complex(-2e-6, 1e-8)
CHIH = complex(-1.5e-6, 8e-9)
DARWIN_URAD = 3.464           # full Darwin width of this reflection (urad)
REFRACTION_URAD = 2.309       # refraction shift of the Bragg peak (urad)
SEED_BASE = 2601063400


# ---------------------------------------------------------------- SplitMix64
class SplitMix64:
    """Counter-based 64-bit generator (Steele, Lea & Flood, OOPSLA 2014)."""

    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """53-bit uniform double in [lo, hi)."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))

    def choice(self, seq):
        return seq[self.randint(0, len(seq) - 1)]

    def complex_normal(self, n: int) -> np.ndarray:
        """n complex samples with independent Box-Muller normal parts."""
        out = np.empty(n, np.complex128)
        for i in range(n):
            u1 = max(self.uniform(), 1e-300)
            u2 = self.uniform()
            r = math.sqrt(-2.0 * math.log(u1))
            out[i] = complex(r * math.cos(2 * math.pi * u2), r * math.sin(2 * math.pi * u2))
        return out


# ---------------------------------------------------------------- beams
def gaussian_beam(nx: int, dx: float, xc: float, w: float, tilt_per_um: float,
                  x0: float = 0.0, amplitude: complex = 1.0) -> np.ndarray:
    """exp(-((x-xc)/w)^2) * exp(i*tilt*(x-xc)); w is the 1/e amplitude radius.

    ``tilt_per_um`` is the envelope's transverse wavenumber, i.e.
    k*(sin(theta_B + delta) - sin(theta_B)) for an incidence delta off Bragg.
    """
    x = x0 + dx * np.arange(nx)
    return amplitude * np.exp(-((x - xc) / w) ** 2) * np.exp(1j * tilt_per_um * (x - xc))


def envelope_tilt(lambda_um: float, d_um: float, delta_rad: float,
                  theta_ref: float | None = None) -> float:
    """Transverse wavenumber of an incident plane wave's envelope (um^-1).

    The beam makes angle ``theta_ref + delta`` with the planes; the envelope
    carrier is sin(theta_B) = lambda/(2d) of *this* wavelength.  ``theta_ref``
    defaults to this wavelength's Bragg angle.
    """
    k = 2 * math.pi / lambda_um
    s = lambda_um / (2 * d_um)
    th = math.asin(s) if theta_ref is None else theta_ref
    return k * (math.sin(th + delta_rad) - s)


# ---------------------------------------------------------------- masks
def mask_full(nz: int, nx: int) -> np.ndarray:
    seg = np.zeros((nz, 1, 2), np.int32)
    seg[:, 0, 1] = nx
    return seg


def mask_empty(nz: int) -> np.ndarray:
    return np.zeros((nz, 1, 2), np.int32)


def _index_at_or_above(x: float, x0: float, dx: float) -> int:
    """Smallest j with x0 + j*dx >= x."""
    return int(math.ceil((x - x0) / dx - 1e-9))


def mask_tilted_face(nz: int, nx: int, dx: float, dz: float, xa: float, xb: float, alpha_rad: float,
                     x0: float = 0.0) -> np.ndarray:
    """Bragg-type crystal whose entrance face is tilted by alpha from the z axis:
    crystal where xa + z tan(alpha) <= x < xb at z = n dz (sample j at x0 + j dx)."""
    seg = np.zeros((nz, 1, 2), np.int32)
    for n in range(nz):
        xf = xa + n * dz * math.tan(alpha_rad)
        seg[n, 0] = (max(0, min(nx, int(math.ceil((xf - x0) / dx - 1e-9)))),
                     max(0, min(nx, int(round((xb - x0) / dx)))))
    return seg


def mask_x_slab(nz: int, nx: int, dx: float, xa: float, xb: float, x0: float = 0.0,
                za: float = -math.inf, zb: float = math.inf, dz: float = 1.0) -> np.ndarray:
    """Bragg-type slab: crystal where xa <= x < xb and za <= z < zb."""
    seg = np.zeros((nz, 1, 2), np.int32)
    lo = max(0, min(nx, _index_at_or_above(xa, x0, dx)))
    hi = max(0, min(nx, _index_at_or_above(xb, x0, dx)))
    for n in range(nz):
        z = n * dz
        if za <= z < zb:
            seg[n, 0] = (lo, hi)
    return seg


def mask_z_slab(nz: int, nx: int, dz: float, za: float, zb: float) -> np.ndarray:
    """Laue-type slab: crystal over the whole window where za <= z < zb."""
    seg = np.zeros((nz, 1, 2), np.int32)
    for n in range(nz):
        if za <= n * dz < zb:
            seg[n, 0] = (0, nx)
    return seg


def mask_asym_trapezoid(nz: int, nx: int, dx: float, dz: float, x_face0: float,
                        asymm_deg: float, x_back: float, za: float, zb: float,
                        x0: float = 0.0) -> np.ndarray:
    """Asymmetric Bragg crystal: entrance face x = x_face0 + z*tan(asymm), back
    face x = x_back, crystal for za <= z < zb."""
    ta = math.tan(math.radians(asymm_deg))
    seg = np.zeros((nz, 1, 2), np.int32)
    hi = max(0, min(nx, _index_at_or_above(x_back, x0, dx)))
    for n in range(nz):
        z = n * dz
        if za <= z < zb:
            lo = max(0, min(nx, _index_at_or_above(x_face0 + z * ta, x0, dx)))
            seg[n, 0] = (lo, max(lo, hi))
    return seg


def mask_polygon(nz: int, nx: int, dx: float, dz: float, verts, x0: float = 0.0,
                 nseg: int = 2) -> np.ndarray:
    """Arbitrary simple polygon (list of (x, z) vertices), rasterised by the
    even-odd rule at each (x_j, z_n); up to ``nseg`` intervals per step."""
    seg = np.zeros((nz, nseg, 2), np.int32)
    V = list(verts)
    for n in range(nz):
        z = n * dz
        xs = []
        for (xa, za), (xb, zb) in zip(V, V[1:] + V[:1]):
            if (za <= z < zb) or (zb <= z < za):
                xs.append(xa + (z - za) * (xb - xa) / (zb - za))
        xs.sort()
        k = 0
        for i in range(0, len(xs) - 1, 2):
            if k >= nseg:
                raise ValueError("polygon needs more than %d intervals per step" % nseg)
            lo = max(0, min(nx, _index_at_or_above(xs[i], x0, dx)))
            hi = max(0, min(nx, _index_at_or_above(xs[i + 1], x0, dx)))
            seg[n, k] = (lo, max(lo, hi))
            k += 1
    return seg


# ---------------------------------------------------------------- problems
def base_problem(nx: int, nz: int, dx: float, dz: float, seg: np.ndarray,
                 lambda_um: float = LAMBDA_UM, d_um: float = D_UM,
                 chi0: complex = CHI0, chih: complex = CHIH, chihb: complex | None = None,
                 x0: float = 0.0, det=None, precision: str = "f64", strain=None) -> dict:
    det = (0, nx) if det is None else det
    return {
        "nx": int(nx), "nz": int(nz), "dx_um": float(dx), "dz_um": float(dz),
        "x0_um": float(x0), "lambda_um": float(lambda_um), "d_um": float(d_um),
        "chi0": complex(chi0), "chih": complex(chih),
        "chihb": complex(chih if chihb is None else chihb),
        "seg": seg, "det_lo": int(det[0]), "det_hi": int(det[1]),
        "precision": precision, "strain": strain or {"kind": "none"},
    }


def flat_bragg_scan(n_angles: int = 64, nx: int = 4096, nz: int = 2000, dx: float = 0.1,
                    dz: float = 0.05, precision: str = "f64"):
    """Symmetric Bragg slab angle scan.  Returns list of (problem, psi_p0)."""
    Lx = nx * dx
    xa, xb, xc = 0.625 * Lx, 0.9375 * Lx, 0.3125 * Lx
    seg = mask_x_slab(nz, nx, dx, xa, xb)
    det = (0, _index_at_or_above(xa, 0.0, dx))
    out = []
    for m in range(n_angles):
        delta = (REFRACTION_URAD + (m - (n_angles - 1) / 2) * (3 * DARWIN_URAD / n_angles)) * 1e-6
        p = base_problem(nx, nz, dx, dz, seg, det=det, precision=precision)
        p["delta_rad"] = delta
        psi = gaussian_beam(nx, dx, xc, 50.0, envelope_tilt(LAMBDA_UM, D_UM, delta))
        out.append((p, psi))
    return out


def bent_laue(radii_m=(1.0, 0.1, 10.0), beams_per_radius: int = 1, nx: int = 16384,
              nz: int = 8000, dx: float = 0.1, dz: float = 0.025, thickness: float = 200.0,
              precision: str = "f32", seed: int = SEED_BASE + 1):
    """Symmetric Laue bent plate; u along h = (x - Lx/2)(z - T/2)/R."""
    rng = SplitMix64(seed)
    Lx = nx * dx
    seg = mask_z_slab(nz, nx, dz, 0.0, thickness)
    out = []
    for R in radii_m:
        for _ in range(beams_per_radius):
            xc = rng.uniform(0.4, 0.6) * Lx
            w = rng.uniform(10.0, 50.0)
            delta = rng.uniform(-2.0, 2.0) * DARWIN_URAD * 1e-6
            strain = {"kind": "poly2", "x_ref_um": Lx / 2, "z_ref_um": thickness / 2,
                      "c": [0.0, 0.0, 0.0, 0.0, 1.0 / (R * 1e6), 0.0]}
            p = base_problem(nx, nz, dx, dz, seg, precision=precision, strain=strain)
            p["radius_m"] = R
            psi = gaussian_beam(nx, dx, xc, w, envelope_tilt(LAMBDA_UM, D_UM, delta))
            out.append((p, psi))
    return out


def disl_bragg(nx: int = 32768, nz: int = 16000, dx: float = 0.1, dz: float = 0.05,
               asymm_deg: float = 10.0, precision: str = "f32", seed: int = SEED_BASE + 2,
               scale: float = 1.0, delta_urad: float = REFRACTION_URAD):
    """Asymmetric Bragg trapezoid with one edge dislocation (b along h).

    ``scale`` shrinks every length of the 3276.8 x 800 um layout (for small
    parity cases).  Returns (problem, psi_p0)."""
    rng = SplitMix64(seed)
    ta = math.tan(math.radians(asymm_deg))
    xf0, xback = 1200.0 * scale, 2400.0 * scale
    za, zb = 50.0 * scale, 750.0 * scale
    seg = mask_asym_trapezoid(nz, nx, dx, dz, xf0, asymm_deg, xback, za, zb)
    zf = rng.uniform(300.0, 700.0) * scale
    depth = rng.uniform(2.0, 20.0) * min(1.0, scale * 4)
    ca, sa = math.cos(math.radians(asymm_deg)), math.sin(math.radians(asymm_deg))
    xd = xf0 + zf * ta + depth * ca
    zd = zf - depth * sa
    # half-cell offsets: the core never sits on a grid point
    xd = (math.floor(xd / dx) + 0.5) * dx
    zd = (math.floor(zd / dz) + 0.5) * dz
    strain = {"kind": "edge_dislocation", "x_ref_um": xd, "z_ref_um": zd,
              "b_um": 0.38e-3, "nu": 0.22}
    det = (0, _index_at_or_above(xf0 + zb * ta, 0.0, dx))
    p = base_problem(nx, nz, dx, dz, seg, det=det, precision=precision, strain=strain)
    psi = gaussian_beam(nx, dx, 1000.0 * scale, 50.0 * min(1.0, scale * 4),
                        envelope_tilt(LAMBDA_UM, D_UM, delta_urad * 1e-6))
    return p, psi


def disl_bragg_cores(n_cores: int, nx: int = 32768, nz: int = 16000, dx: float = 0.1, dz: float = 0.05,
                     asymm_deg: float = 10.0, precision: str = "f32", seed: int = SEED_BASE + 2):
    """``n_cores`` solves of the dislocation trapezoid that differ only in the
    seeded core position (one crystal mask, shared).  Returns [(problem, psi_p0)]."""
    base, psi = disl_bragg(nx=nx, nz=nz, dx=dx, dz=dz, asymm_deg=asymm_deg, precision=precision, seed=seed)
    rng = SplitMix64(seed + 1000)
    ta = math.tan(math.radians(asymm_deg))
    ca, sa = math.cos(math.radians(asymm_deg)), math.sin(math.radians(asymm_deg))
    out = []
    for _ in range(n_cores):
        zf = rng.uniform(300.0, 700.0)
        depth = rng.uniform(2.0, 20.0)
        xd = (math.floor((1200.0 + zf * ta + depth * ca) / dx) + 0.5) * dx
        zd = (math.floor((zf - depth * sa) / dz) + 0.5) * dz
        p = dict(base, strain=dict(base["strain"], x_ref_um=xd, z_ref_um=zd))
        out.append((p, psi))
    return out


def cube_3d(nx: int = 512, ny: int = 256, nz: int = 300, dx: float = 0.05, dy: float = 0.05,
            dz: float = 0.05, side: float = 10.0, precision: str = "f32", dislocation: bool = True,
            seed: int = SEED_BASE + 5):
    """3D envelopes: a cube of the given side in a (nx dx) x (ny dy) x (nz dz)
    window (the 300 x 200 x 300 grid of the paper's 3D case padded to powers of
    two), a Gaussian beam in x and y, and optionally an edge dislocation through
    the cube centre (line along y, b = 4 d along h, half-cell offsets).
    Returns (problem, psi_p0 [ny][nx])."""
    rng = SplitMix64(seed)
    Lx, Ly, Lz = nx * dx, ny * dy, nz * dz
    xa, ya, za = 0.3 * Lx, 0.5 * (Ly - side), 0.5 * (Lz - side)
    ja, jb = _index_at_or_above(xa, 0.0, dx), _index_at_or_above(xa + side, 0.0, dx)
    seg = np.zeros((nz, ny, 1, 2), np.int32)
    for n in range(nz):
        if za <= n * dz < za + side:
            for i in range(ny):
                if ya <= i * dy < ya + side:
                    seg[n, i, 0] = (ja, jb)
    strain = None
    if dislocation:
        xd = (math.floor((xa + 0.5 * side + rng.uniform(-0.5, 0.5)) / dx) + 0.5) * dx
        zd = (math.floor((za + 0.5 * side + rng.uniform(-0.5, 0.5)) / dz) + 0.5) * dz
        strain = {"kind": "edge_dislocation", "x_ref_um": xd, "z_ref_um": zd, "b_um": 4 * D_UM, "nu": 0.22}
    p = base_problem(nx, nz, dx, dz, seg, precision=precision, strain=strain)
    p["ny"], p["dy_um"] = ny, dy
    xs = np.arange(nx) * dx
    ys = np.arange(ny) * dy
    g = gaussian_beam(nx, dx, 0.2 * Lx, 3.0, envelope_tilt(LAMBDA_UM, D_UM, REFRACTION_URAD * 1e-6))
    psi = np.exp(-((ys - 0.5 * Ly) / 3.0) ** 2)[:, None] * g[None, :]
    del xs
    return p, psi.astype(np.complex128)


def td_batch(n_comp: int = 1024, sigma_t_fs: float = 20.0, nx_choices=(2048, 4096, 8192, 16384),
             nz_range=(1000, 8000), dx: float = 0.1, dz: float = 0.05, precision: str = "f32",
             seed: int = SEED_BASE + 3):
    """Frequency components of a Gaussian pulse, each its own Bragg solve."""
    rng = SplitMix64(seed)
    hbar_ev_fs = 0.6582119569
    sigma_e_kev = hbar_ev_fs / sigma_t_fs * 1e-3
    de_kev = 12 * sigma_e_kev / n_comp
    theta0 = math.asin(LAMBDA_UM / (2 * D_UM)) + REFRACTION_URAD * 1e-6
    out = []
    for m in range(n_comp):
        E = E0_KEV + (m - (n_comp - 1) / 2) * de_kev
        lam = HC_KEV_ANGSTROM / E * 1e-4
        amp = math.exp(-((E - E0_KEV) ** 2) / (2 * sigma_e_kev ** 2))
        ph = rng.uniform(0.0, 2 * math.pi)
        nx = int(rng.choice(list(nx_choices)))
        nz = rng.randint(nz_range[0], nz_range[1])
        Lx = nx * dx
        xa, xb = 0.625 * Lx, 0.9375 * Lx
        seg = mask_x_slab(nz, nx, dx, xa, xb)
        det = (0, _index_at_or_above(xa, 0.0, dx))
        p = base_problem(nx, nz, dx, dz, seg, lambda_um=lam, det=det, precision=precision)
        p["energy_kev"] = E
        tilt = envelope_tilt(lam, D_UM, theta0 - math.asin(lam / (2 * D_UM)))
        psi = gaussian_beam(nx, dx, 0.3125 * Lx, 50.0, tilt,
                            amplitude=amp * complex(math.cos(ph), math.sin(ph)))
        out.append((p, psi))
    return out


def scaled_geometry(kind: str, nx: int, nz: int, dx: float, dz: float, rng: SplitMix64,
                    precision: str):
    """One request of the serving mix: geometry ``kind`` scaled to the window."""
    Lx, Lz = nx * dx, nz * dz
    delta = rng.uniform(-1.5, 1.5) * DARWIN_URAD * 1e-6 + REFRACTION_URAD * 1e-6
    tilt = envelope_tilt(LAMBDA_UM, D_UM, delta)
    if kind == "flat":
        xa, xb = 0.625 * Lx, 0.9375 * Lx
        seg = mask_x_slab(nz, nx, dx, xa, xb)
        p = base_problem(nx, nz, dx, dz, seg, det=(0, _index_at_or_above(xa, 0, dx)),
                         precision=precision)
        psi = gaussian_beam(nx, dx, 0.3125 * Lx, min(50.0, 0.08 * Lx), tilt)
    elif kind == "bent":
        R = 10 ** rng.uniform(0.0, 1.0)
        seg = mask_full(nz, nx)
        strain = {"kind": "poly2", "x_ref_um": Lx / 2, "z_ref_um": Lz / 2,
                  "c": [0.0, 0.0, 0.0, 0.0, 1.0 / (R * 1e6), 0.0]}
        p = base_problem(nx, nz, dx, dz, seg, precision=precision, strain=strain)
        psi = gaussian_beam(nx, dx, rng.uniform(0.4, 0.6) * Lx,
                            min(rng.uniform(10, 50), 0.05 * Lx), tilt)
    elif kind in ("disl", "trapezoid"):
        xf0, xback = 0.37 * Lx, 0.73 * Lx
        ta = math.tan(math.radians(10.0))
        # the 10-degree entrance face must stay inside the window: a crystal
        # deeper than 0.9 (xback - xf0) / tan(10 deg) is cut to that depth
        za = 0.06 * Lz
        zb = min(0.94 * Lz, za + 0.9 * (xback - xf0) / ta)
        seg = mask_asym_trapezoid(nz, nx, dx, dz, xf0, 10.0, xback, za, zb)
        strain = None
        if kind == "disl":
            zf = za + rng.uniform(0.375, 0.875) * (zb - za)
            depth = rng.uniform(2.0, 20.0)
            xd = (math.floor((xf0 + zf * ta + depth * math.cos(math.radians(10))) / dx) + 0.5) * dx
            zd = (math.floor((zf - depth * math.sin(math.radians(10))) / dz) + 0.5) * dz
            strain = {"kind": "edge_dislocation", "x_ref_um": xd, "z_ref_um": zd,
                      "b_um": 0.38e-3, "nu": 0.22}
        p = base_problem(nx, nz, dx, dz, seg, precision=precision, strain=strain,
                         det=(0, min(nx, _index_at_or_above(xf0 + zb * ta, 0, dx))))
        psi = gaussian_beam(nx, dx, 0.3 * Lx, min(50.0, 0.05 * Lx), tilt)
    else:
        raise ValueError(kind)
    p["kind"] = kind
    return p, psi


def serve_mix(n_req: int = 10000, rate_hz: float = 200.0, log2nx=(10, 16), nz_range=(500, 20000),
              fp64_frac: float = 0.2, dx: float = 0.1, dz: float = 0.05, seed: int = SEED_BASE + 4,
              build=True):
    """Poisson request stream.  Returns a list of dicts with arrival time (s),
    and, if ``build``, the problem and entrance envelope."""
    rng = SplitMix64(seed)
    t = 0.0
    reqs = []
    kinds = ["flat", "bent", "disl", "trapezoid"]
    for i in range(n_req):
        t += -math.log(max(1e-300, 1.0 - rng.uniform())) / rate_hz
        nx = 1 << rng.randint(log2nx[0], log2nx[1])
        nz = rng.randint(nz_range[0], nz_range[1])
        kind = rng.choice(kinds)
        prec = "f64" if rng.uniform() < fp64_frac else "f32"
        r = {"t_arrival": t, "nx": nx, "nz": nz, "kind": kind, "precision": prec,
             "seed": rng.next_u64()}
        if build:
            r["problem"], r["psi_p0"] = scaled_geometry(kind, nx, nz, dx, dz,
                                                        SplitMix64(r["seed"]), prec)
        reqs.append(r)
    return reqs


def random_envelopes(nx: int, seed: int):
    """Random complex psi_p, psi_m (for algebraic pins that need generic fields)."""
    rng = SplitMix64(seed)
    return rng.complex_normal(nx), rng.complex_normal(nx)
