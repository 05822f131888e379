"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library.

This module holds no arithmetic of the indexing method: it only draws the
random quantities that a synthetic experiment needs (grain orientations and
positions, perturbed starting grains) and states the experiment presets.
Random numbers that the method itself consumes inside a simulation (ray
noise, outlier positions, spot order) are NOT drawn here: both sides derive
them from the Philox4x32-10 counter-based generator, keyed by the seed below
and by the spot's identity, each side with its own implementation.

Units: millimetres, Angstrom, radians (degrees only in the preset fields that
say so).  Grains are FP64 unit quaternions (w, x, y, z) with w >= 0 and FP64
positions.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 240406478


@dataclasses.dataclass(frozen=True)
class Detector:
    """A flat square detector: centre, unit normal, two in-plane unit axes, side."""
    center: tuple
    normal: tuple
    axis1: tuple
    axis2: tuple
    size: float


TRANSMISSION_150 = Detector((150.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                            (0.0, 0.0, 1.0), 200.0)
BACKSCATTER_150 = Detector((-150.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                           (0.0, 0.0, 1.0), 200.0)


@dataclasses.dataclass(frozen=True)
class Preset:
    """One synthetic experiment: lattice, band, sample, scan, noise, solver knobs."""
    name: str
    a: float                 # cubic lattice constant, Angstrom
    centering: str           # 'P', 'I' (BCC) or 'F' (FCC) extinction rule
    n_max: int               # largest h^2+k^2+l^2 in the plane list
    lam_min: float           # band, Angstrom
    lam_max: float
    n_grains: int
    n_rot: int               # number of sample rotations about z
    domega_deg: float        # rotation step, degrees (omega_t = t * step)
    sigma_mm: float          # spot noise on the detector, mm
    outlier_frac: float      # outliers per (rotation, detector) as a fraction of true spots
    eps_start: float         # entropic temperature schedule, mm^2
    eps_end: float
    n_stages: int
    iters_per_stage: int
    n_candidates: int = 0
    radius_mm: float = 2.5   # sample cylinder (axis z)
    height_mm: float = 5.0
    detectors: tuple = (TRANSMISSION_150, BACKSCATTER_150)
    index: int = 0

    @property
    def seed(self) -> int:
        return BASE_SEED + self.index

    @property
    def distance(self) -> float:
        """Detector distance D that converts the mm noise to an angle."""
        return float(abs(self.detectors[0].center[0]))


def _schedule(sigma):
    return 111.0 * sigma * sigma, 1.11 * sigma * sigma


TINY = Preset("tiny", 2.87, "I", 14, 1.0, 3.5, 5, 12, 15.0, 0.3, 0.10,
              10.0, 0.1, 5, 4, index=0)
MEDIUM = Preset("medium", 2.87, "I", 30, 1.0, 4.0, 100, 60, 3.0, 1.0, 0.30,
                *_schedule(1.0), 5, 4, n_candidates=100_000, index=1)
LEARNED = Preset("learned", 2.87, "I", 30, 1.0, 4.0, 1000, 60, 3.0, 1.0, 0.70,
                 *_schedule(1.0), 5, 4, n_candidates=1 << 20, index=3)
# The learned-scale sample at the paper's fiducial noise and outlier level
# (Sec. 7: sigma = 0.4 mm on the detector, outliers 10% of the spot count).
LEARNED_FIDUCIAL = Preset("learned_fiducial", 2.87, "I", 30, 1.0, 4.0, 1000, 60, 3.0, 0.4, 0.10,
                          *_schedule(0.4), 5, 4, index=5)
STRESS = Preset("stress", 3.52, "F", 40, 0.8, 5.0, 2000, 90, 2.0, 1.5, 0.50,
                *_schedule(1.5), 5, 4, index=4)
PRESETS = {p.name: p for p in (TINY, MEDIUM, LEARNED, LEARNED_FIDUCIAL, STRESS)}


def batching_samples(n_samples=64, seed=BASE_SEED + 2):
    """Presets of the uneven multi-sample batch: grains U{50..400}, rotations
    U{24..90} over 180 degrees, lattice in {2.87 I, 3.52 F, 4.05 F}, sigma
    U(0.3, 1.5) mm, outliers U(0, 0.5)."""
    rng = np.random.default_rng(seed)
    lattices = [(2.87, "I"), (3.52, "F"), (4.05, "F")]
    out = []
    for s in range(n_samples):
        a, cen = lattices[int(rng.integers(0, 3))]
        n_grains = int(rng.integers(50, 401))
        n_rot = int(rng.integers(24, 91))
        sigma = float(rng.uniform(0.3, 1.5))
        frac = float(rng.uniform(0.0, 0.5))
        out.append(Preset(f"batch{s}", a, cen, 30, 1.0, 4.0, n_grains, n_rot,
                          180.0 / n_rot, sigma, frac, *_schedule(sigma), 5, 4,
                          index=1000 + s))
    return out


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform rotations: normalised 4-D Gaussian vectors, sign fixed to w >= 0."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def random_positions(rng: np.random.Generator, n: int, radius: float, height: float) -> np.ndarray:
    """Uniform points in the cylinder r <= radius, |z| <= height/2, axis z."""
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n))
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    z = (rng.uniform(0.0, 1.0, n) - 0.5) * height
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def random_grains(preset: Preset, n: int | None = None, seed: int | None = None):
    """Ground-truth grains of a preset: (quaternions [n,4], positions [n,3]), FP64."""
    rng = np.random.default_rng(preset.seed if seed is None else seed)
    n = preset.n_grains if n is None else n
    q = random_quaternions(rng, n)
    x = random_positions(rng, n, preset.radius_mm, preset.height_mm)
    return q, x


def _qmul(a, b):
    w1, x1, y1, z1 = a.T
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=1)


def perturb_grains(q, x, angle_deg, shift_mm, seed):
    """Starting grains near the truth: each orientation is turned by exactly
    angle_deg about a random axis (left-multiplied) and each position moved by
    exactly shift_mm in a random direction."""
    rng = np.random.default_rng(seed)
    n = q.shape[0]
    ax = rng.standard_normal((n, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    h = math.radians(angle_deg) / 2.0
    dq = np.concatenate([np.full((n, 1), math.cos(h)), math.sin(h) * ax], axis=1)
    q2 = _qmul(dq, q)
    q2 /= np.linalg.norm(q2, axis=1, keepdims=True)
    q2[q2[:, 0] < 0] *= -1.0
    dx = rng.standard_normal((n, 3))
    dx /= np.linalg.norm(dx, axis=1, keepdims=True)
    return q2, x + shift_mm * dx


def to_f32_exact(a) -> np.ndarray:
    """Round to FP32 and promote back to FP64 exactly (what both sides consume)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
