"""Seeded synthetic inputs: sequences, phantoms, coil maps and probe vectors.

This module holds none of the method's arithmetic (no simulation, no encoding,
no Jacobian). It only draws the inputs that the HIP path, the oracle, the tests
and the benchmark all consume, so that both sides see identical arrays.

The paper's own workloads (the BrainWeb phantom, gel-phantom and in-vivo
scanner data of the Methods section) are not available; the generators below
stand in for them with the same structure: a Cartesian transient-state
sequence with a smoothly varying flip train (Supporting Information S1), a
head-like phantom with white/gray matter values of the same order as the
paper's in-vivo table, and complex proton density.

Seeds: phantom 0, noise 1, flip peaks 2, probe vectors 3, surrogate samples 4,
MLP initialisation 5.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SEED_PHANTOM, SEED_NOISE, SEED_FLIPS, SEED_PROBE, SEED_SURR, SEED_MLP = 0, 1, 2, 3, 4, 5


@dataclass
class Problem:
    """Sequence and grid description (mirrors the C struct of the library)."""
    nx: int
    ny: int
    n_tr: int
    n_read: int
    n_states: int
    n_coils: int
    tr: float
    te: float
    t_inv: float
    flip_deg: np.ndarray
    rf_phase: np.ndarray
    ky_line: np.ndarray
    traj: tuple | None = None     # (kx, ky) [n_tr][n_read] cycles per FOV; None = Cartesian
    iso: tuple | None = None      # (flip scale, weight) [n_iso]: balanced isochromat model; None = EPG
    dwell: float = 0.0            # readout sample spacing [s]; > 0: T2 decay and off-resonance during readouts
    db0: np.ndarray | None = None  # [Nv] off-resonance [Hz] (readout dynamics); None = 0
    rd_min_t2: float = 0.005      # readout dynamics on the GPU: T2 [s] and |db0| [Hz] bounds
    rd_max_db0: float = 200.0     # within which its expansion holds FP32 accuracy
    db0_unit: float = 0.0         # > 0: Delta B0 fitted as theta row 5, in units of db0_unit Hz
                                  # (db0 then None; its box is +-rd_max_db0 Hz)

    @property
    def nv(self) -> int:
        return self.nx * self.ny

    @property
    def data_shape(self):
        return (self.n_coils, self.n_tr, self.n_read)


@dataclass
class Workload:
    name: str
    problem: Problem
    theta: np.ndarray             # [5][Nv] ground truth (ln T1, ln T2, B1, Re rho, Im rho)
    coil: np.ndarray | None       # [C][Nv] complex or None
    snr: float | None             # None = noiseless
    n_gn: int
    n_cg: int
    param_mask: int               # bit p set = parameter p reconstructed
    extra: dict = field(default_factory=dict)


def linear_ky(n_tr: int, ny: int) -> np.ndarray:
    """Linear Cartesian order: one phase-encode line per TR, ny lines per sweep."""
    return (np.arange(n_tr) % ny).astype(np.int32)


def flips_config1(n_tr: int = 128) -> np.ndarray:
    """60 |sin(pi n / 128)| degrees."""
    n = np.arange(n_tr, dtype=np.float64)
    return 60.0 * np.abs(np.sin(np.pi * n / 128.0))


def flips_sin2_sweeps(n_tr: int, ny: int, peak_lo=30.0, peak_hi=70.0, seed=SEED_FLIPS):
    """Connected sine-squared waves, one per k-space sweep, starting at zero and
    peaking at the central line, with random peak amplitudes; the largest peak
    is set to peak_hi."""
    n_sweeps = (n_tr + ny - 1) // ny
    rng = np.random.default_rng(seed)
    peaks = rng.uniform(peak_lo, peak_hi, size=n_sweeps)
    peaks[np.argmax(peaks)] = peak_hi
    n = np.arange(n_tr)
    line = n % ny
    return peaks[n // ny] * np.sin(np.pi * line / ny) ** 2


def make_problem(nx, ny, n_tr, n_read, n_states, n_coils=1, tr=0.008, te=0.004,
                 t_inv=0.0, flip_deg=None, rf_phase=None, ky_line=None) -> Problem:
    if flip_deg is None:
        flip_deg = flips_sin2_sweeps(n_tr, ny)
    if rf_phase is None:
        rf_phase = np.zeros(n_tr)
    if ky_line is None:
        ky_line = linear_ky(n_tr, ny)
    return Problem(nx, ny, n_tr, n_read, n_states, n_coils, float(tr), float(te),
                   float(t_inv), np.asarray(flip_deg, dtype=np.float64),
                   np.asarray(rf_phase, dtype=np.float64), np.asarray(ky_line, dtype=np.int32))


GOLDEN_ANGLE_DEG = 180.0 * (np.sqrt(5.0) - 1.0) / 2.0   # about 111.246 degrees


def radial_golden(n_tr: int, n_read: int, nx: int, ny: int) -> tuple:
    """Golden-angle radial sampling: one spoke through the k-space centre per
    TR at angle n * 111.246 degrees, n_read samples spaced nx / n_read (ny /
    n_read) cycles per field of view along x (y), from -nx/2 (-ny/2).
    Returns (kx, ky), each [n_tr][n_read]."""
    phi = np.deg2rad(GOLDEN_ANGLE_DEG) * np.arange(n_tr)
    s = np.arange(n_read) - n_read // 2
    kx = (s * (nx / n_read))[None, :] * np.cos(phi)[:, None]
    ky = (s * (ny / n_read))[None, :] * np.sin(phi)[:, None]
    return kx, ky


def cartesian_traj(prob: "Problem") -> tuple:
    """The Cartesian samples of prob written as a trajectory (cycles per
    field of view): kx = (k - n_read/2) nx / n_read, ky = l(n) - ny/2."""
    kx = np.tile((np.arange(prob.n_read) - prob.n_read // 2) * (prob.nx / prob.n_read), (prob.n_tr, 1))
    ky = np.repeat((prob.ky_line.astype(np.float64) - prob.ny // 2)[:, None], prob.n_read, axis=1)
    return kx, ky


def slice_profile_gaussian(n_iso: int, z_max: float = 1.5) -> tuple:
    """Slice profile of a Gaussian RF envelope for the balanced isochromat
    model: n_iso positions z uniformly spaced over [-z_max, z_max] slice
    thicknesses (cell centres), flip-angle scale exp(-4 ln 2 z^2) (full width
    at half maximum one slice thickness: the small-tip profile of a Gaussian
    pulse is Gaussian) and weight dz (a midpoint sum over z).
    Returns (scale, weight), each [n_iso]."""
    dz = 2.0 * z_max / n_iso
    z = -z_max + dz * (np.arange(n_iso) + 0.5)
    return np.exp(-4.0 * np.log(2.0) * z * z), np.full(n_iso, dz)


def balanced_phases(n_tr: int) -> np.ndarray:
    """RF phase alternating 0 / 180 degrees (the paper's balanced sequence)."""
    return np.pi * (np.arange(n_tr) % 2)


def pack_theta(T1, T2, B1, rho) -> np.ndarray:
    T1, T2, B1, rho = (np.asarray(a).reshape(-1) for a in (T1, T2, B1, rho))
    return np.stack([np.log(T1), np.log(T2), B1.astype(np.float64),
                     rho.real.astype(np.float64), rho.imag.astype(np.float64)])


def iid_maps(nv: int, seed=SEED_PHANTOM, t1=(0.3, 2.5), t2=(0.03, 0.3), b1=1.0):
    """Independent per-voxel maps (the small plain-method case)."""
    rng = np.random.default_rng(seed)
    T1 = rng.uniform(*t1, size=nv)
    T2 = rng.uniform(*t2, size=nv)
    mag = rng.uniform(0.5, 1.0, size=nv)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=nv)
    B1 = np.full(nv, b1) if np.isscalar(b1) else np.asarray(b1)
    return pack_theta(T1, T2, B1, mag * np.exp(1j * ph))


# Tissue classes: (T1 [s], T2 [s], |rho|). White and gray matter are of the
# order of the paper's in-vivo table; the others are plausible stand-ins.
TISSUES = {
    "wm": (0.52, 0.055, 0.70),
    "gm": (0.90, 0.078, 0.85),
    "csf": (3.0, 1.0, 1.0),
    "fat": (0.30, 0.08, 0.90),
    "lesion": (1.2, 0.12, 0.80),
}


def _gauss_blur(img, sigma):
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(img, sigma, mode="wrap")


def _ellipse(X, Y, cx, cy, ax, ay, ang=0.0):
    c, s = np.cos(ang), np.sin(ang)
    xr = (X - cx) * c + (Y - cy) * s
    yr = -(X - cx) * s + (Y - cy) * c
    return (xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0


def brain_phantom(nx, ny, seed=SEED_PHANTOM, b1_range=None):
    """Head-like ellipse phantom: scalp ring, gray matter, white matter core,
    two ventricles, a few random lesions; multiplicative texture
    1 + 0.05 * (unit-std Gaussian-blurred noise, sigma 2 px); smooth rho phase
    (random 2nd-order polynomial spanning about +-pi); rho = 0 outside the head.
    b1_range: None -> B1 = 1, else a blurred random field (sigma nx/8) mapped
    affinely onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    X = (x - nx / 2 + 0.5) / (nx / 2)
    Y = (y - ny / 2 + 0.5) / (ny / 2)
    label = np.full((ny, nx), "", dtype=object)
    head = _ellipse(X, Y, 0, 0, 0.86, 0.94)
    brain = _ellipse(X, Y, 0, 0, 0.78, 0.86)
    wm = _ellipse(X, Y, 0, 0.02, 0.55, 0.65)
    label[head] = "fat"
    label[brain] = "gm"
    label[wm] = "wm"
    for sx in (-1, 1):
        label[_ellipse(X, Y, sx * 0.12, -0.05, 0.07, 0.22, sx * 0.25)] = "csf"
    for _ in range(4):
        cx, cy = rng.uniform(-0.45, 0.45, size=2)
        r = rng.uniform(0.04, 0.09)
        label[_ellipse(X, Y, cx, cy, r, r * rng.uniform(0.7, 1.3))] = "lesion"

    T1 = np.ones((ny, nx))
    T2 = np.full((ny, nx), 0.1)
    mag = np.zeros((ny, nx))
    for name, (t1, t2, pd) in TISSUES.items():
        sel = label == name
        T1[sel], T2[sel], mag[sel] = t1, t2, pd

    def texture():
        g = _gauss_blur(rng.standard_normal((ny, nx)), 2.0)
        return 1.0 + 0.05 * g / g.std()

    T1 = T1 * texture()
    T2 = T2 * texture()
    mag = mag * texture()
    coef = rng.uniform(-1, 1, size=6)
    poly = (coef[0] + coef[1] * X + coef[2] * Y + coef[3] * X * X + coef[4] * X * Y
            + coef[5] * Y * Y)
    poly = poly - poly.mean()
    phase = np.pi * poly / max(np.abs(poly).max(), 1e-12)
    rho = mag * np.exp(1j * phase)
    rho[~head] = 0.0
    if b1_range is None:
        B1 = np.ones((ny, nx))
    else:
        f = _gauss_blur(rng.standard_normal((ny, nx)), nx / 8.0)
        f = (f - f.min()) / (f.max() - f.min())
        B1 = b1_range[0] + (b1_range[1] - b1_range[0]) * f
    return pack_theta(T1, T2, B1, rho), head.reshape(-1)


def coil_maps(nx, ny, n_coils, seed=SEED_PHANTOM + 10):
    """Smooth complex receive sensitivities: Gaussians centred on a circle of
    radius 0.6 FOV (sigma 0.5 FOV) with a linear phase each, scaled so that
    sum_c |C_c|^2 = 1 in every voxel."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    X = (x - nx / 2) / nx
    Y = (y - ny / 2) / ny
    maps = []
    for c in range(n_coils):
        a = 2 * np.pi * c / n_coils
        cx, cy = 0.6 * np.cos(a), 0.6 * np.sin(a)
        amp = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 0.5 ** 2))
        kx, ky = rng.uniform(-2, 2, size=2)
        maps.append(amp * np.exp(1j * (kx * X + ky * Y + rng.uniform(0, 2 * np.pi))))
    maps = np.stack(maps)
    maps /= np.sqrt((np.abs(maps) ** 2).sum(axis=0, keepdims=True))
    return maps.reshape(n_coils, nx * ny).astype(np.complex128)


def n_params(prob: Problem) -> int:
    """Parameter rows: 5, or 6 with Delta B0 fitted."""
    return 6 if (getattr(prob, "db0_unit", 0.0) or 0.0) > 0.0 else 5


def probe_vectors(prob: Problem, param_mask=0b111111, seed=SEED_PROBE):
    """v ~ N(0,1) on the active parameters, w ~ CN(0,1) in data space."""
    rng = np.random.default_rng(seed)
    npar = n_params(prob)
    v = rng.standard_normal((npar, prob.nv))
    for q in range(npar):
        if not (param_mask >> q) & 1:
            v[q] = 0.0
    w = (rng.standard_normal(prob.data_shape) + 1j * rng.standard_normal(prob.data_shape)) / np.sqrt(2)
    return v, w


def unit_noise(prob: Problem, seed=SEED_NOISE):
    """Unscaled iid complex Gaussian noise; the caller scales it so that
    ||signal|| / ||noise|| equals the chosen SNR."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(prob.data_shape) + 1j * rng.standard_normal(prob.data_shape)


# Parameter box for the reconstruction: ln T1, ln T2, B1.
GN_LO = (float(np.log(0.05)), float(np.log(0.005)), 0.5)
GN_HI = (float(np.log(8.0)), float(np.log(4.0)), 1.5)
# Initial guess for the non-linear parameters (Methods, Reconstructions).
INIT_T1, INIT_T2, INIT_B1 = 1.0, 0.1, 1.0


def initial_theta(nv: int) -> np.ndarray:
    return pack_theta(np.full(nv, INIT_T1), np.full(nv, INIT_T2), np.full(nv, INIT_B1),
                      np.zeros(nv, dtype=np.complex128))


def config(idx: int) -> Workload:
    """The five workloads: 1 small plain case, 2 128^2 FP32 case, 3 224^2
    precision case, 4 surrogate (224^2 sequence), 5 256^2 with 8 coils.
    The two small cases hold B1 known (T1, T2, rho fitted); the three large
    ones fit B1 as well."""
    if idx == 1:
        prob = make_problem(32, 32, 128, 32, 16, flip_deg=flips_config1(128))
        return Workload("32x32, 128 TRs, Nk 32, K 16, 1 coil", prob, iid_maps(prob.nv),
                        None, None, 5, 10, 0b11011)
    if idx == 2:
        prob = make_problem(128, 128, 1024, 256, 32)
        th, head = brain_phantom(128, 128)
        return Workload("128x128 phantom, 1024 TRs, Nk 256, K 32, SNR 50", prob, th, None,
                        50.0, 10, 20, 0b11011, {"head": head})
    if idx in (3, 4):
        prob = make_problem(224, 224, 1120, 448, 32)
        th, head = brain_phantom(224, 224, b1_range=(0.8, 1.2))
        # All five parameters reconstructed, B1 included (as for the paper's
        # scanner data); B1-known fits pass param_mask 0b11011 themselves.
        return Workload("224x224 phantom, 1120 TRs, Nk 448, K 32", prob, th, None, None,
                        10, 20, 0b11111, {"head": head})
    if idx == 5:
        prob = make_problem(256, 256, 1280, 512, 32, n_coils=8)
        th, head = brain_phantom(256, 256, b1_range=(0.8, 1.2))
        return Workload("256x256 phantom, 8 coils, 1280 TRs, Nk 512, K 32, SNR 50", prob, th,
                        coil_maps(256, 256, 8), 50.0, 15, 30, 0b11111, {"head": head})
    raise ValueError(idx)


# Surrogate network: training box for (T1 [s], T2 [s], B1) and initialisation.
SURR_BOX_T1 = (0.1, 5.0)
SURR_BOX_T2 = (0.01, 2.0)
SURR_BOX_B1 = (0.7, 1.3)
SURR_LO = (float(np.log(SURR_BOX_T1[0])), float(np.log(SURR_BOX_T2[0])), SURR_BOX_B1[0])
SURR_HI = (float(np.log(SURR_BOX_T1[1])), float(np.log(SURR_BOX_T2[1])), SURR_BOX_B1[1])


def surrogate_samples(n, seed=SEED_SURR):
    """Training inputs: T1 and T2 log-uniform, B1 uniform over the box.
    Returns theta rows (ln T1, ln T2, B1) as [3][n]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(SURR_LO[0], SURR_HI[0], n), rng.uniform(SURR_LO[1], SURR_HI[1], n),
                     rng.uniform(SURR_LO[2], SURR_HI[2], n)])


def mlp_init_params(n_tr, width=256, depth=4, seed=SEED_MLP):
    """Uniform Glorot-style weights, zero biases, packed as W1 [width][3], b1,
    (W [width][width], b) per further hidden layer, Wout [8 n_tr][width], bout."""
    rng = np.random.default_rng(seed)
    shapes = [(width, 3), (width,)] + [(width, width), (width,)] * (depth - 1) + \
        [(8 * n_tr, width), (8 * n_tr,)]
    parts = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s).reshape(-1))
        else:
            parts.append(np.zeros(s[0]))
    return np.concatenate(parts)


def shrink(prob: Problem, **kw) -> Problem:
    return replace(prob, **kw)
