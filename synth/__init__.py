"""Seeded synthetic disk clusters for the sound-soft multiple-scattering workloads.

This module only draws inputs: disk centers, radii, per-disk truncation orders,
wavenumbers and angle grids.  It holds none of the scattering arithmetic, so both
the CPU oracle (``oracle/``) and the HIP path may consume its output.

Draw protocol (every workload):
  * RNG: ``numpy.random.default_rng(seed)`` (PCG64); independent instances use
    child generators from ``SeedSequence(seed).spawn(n)``.
  * Per instance: all radii first (one vectorised draw), then the centers one
    disk at a time: a candidate ``rng.uniform(lo, hi, 2)`` is accepted iff its
    edge gap to every accepted disk is at least ``gap``; at most 10**6
    candidates per disk, else ``RuntimeError``.
  * Angle grids are uniform: ``2*pi*j/n`` for ``j = 0..n-1``.

Disks must be disjoint (paper section 2: the scatterers are bounded and
disjoint), which the rejection rule guarantees for ``gap > 0``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Cluster", "random_disks", "uniform_angles", "tiny", "one_rhs", "multi_rhs",
    "uneven_instances", "differentiation", "perturb", "small_random",
]


@dataclass
class Cluster:
    """One scattering configuration: M disks, wavenumber k, truncation N_p."""
    centers: np.ndarray          # [M, 2] float64
    radii: np.ndarray            # [M] float64
    n_modes: np.ndarray          # [M] int32, N_p (2 N_p + 1 modes per disk)
    k: float
    betas: np.ndarray = field(default_factory=lambda: np.zeros(1))   # incidence angles
    thetas: np.ndarray = field(default_factory=lambda: np.zeros(0))  # far-field angles
    name: str = ""

    @property
    def M(self) -> int:
        return int(self.radii.shape[0])

    @property
    def n_tot(self) -> int:
        return int(np.sum(2 * self.n_modes + 1))


def uniform_angles(n: int) -> np.ndarray:
    """Uniform grid 2*pi*j/n, j = 0..n-1 (float64)."""
    return 2.0 * math.pi * np.arange(n, dtype=np.float64) / n


def random_disks(rng: np.random.Generator, M: int, r_lo: float, r_hi: float,
                 box_lo: float, box_hi: float, gap: float,
                 max_tries: int = 10**6) -> tuple[np.ndarray, np.ndarray]:
    """Seeded rejection placement of M disks with radii U[r_lo, r_hi].

    Centers are uniform in [box_lo, box_hi]^2 (disks may protrude).  A
    candidate is accepted iff |O - O_i| >= a + a_i + gap for all accepted i.
    """
    if r_lo == r_hi:
        radii = np.full(M, float(r_lo))
    else:
        radii = rng.uniform(r_lo, r_hi, M)
    centers = np.empty((M, 2))
    for p in range(M):
        a = radii[p]
        for _ in range(max_tries):
            c = rng.uniform(box_lo, box_hi, 2)
            if p == 0:
                break
            d = np.hypot(centers[:p, 0] - c[0], centers[:p, 1] - c[1])
            if np.all(d >= a + radii[:p] + gap):
                break
        else:
            raise RuntimeError(f"could not place disk {p} after {max_tries} tries")
        centers[p] = c
    return centers, radii


def _ceil_rule(k: float, radii: np.ndarray, extra: int) -> np.ndarray:
    # Truncation rule N_p = ceil(k a_p) + extra, as fixed by the workload.
    return (np.ceil(k * radii) + extra).astype(np.int32)


def tiny() -> Cluster:
    """4 unit disks at (0,0),(3,0),(0,3),(3,3); k = 2 pi; N_p = 15; beta = 0;
    360 far-field angles."""
    centers = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 3.0], [3.0, 3.0]])
    return Cluster(centers, np.ones(4), np.full(4, 15, np.int32), 2.0 * math.pi,
                   np.zeros(1), uniform_angles(360), "tiny")


def one_rhs(seed: int = 2, M: int = 400) -> Cluster:
    """M = 400 disks of radius 0.5 in [0,60]^2, gap 0.2; k = 2 pi; N_p = 12;
    incidence pi/4; 720 far-field angles."""
    rng = np.random.default_rng(seed)
    centers, radii = random_disks(rng, M, 0.5, 0.5, 0.0, 60.0, 0.2)
    return Cluster(centers, radii, np.full(M, 12, np.int32), 2.0 * math.pi,
                   np.array([math.pi / 4]), uniform_angles(720), "one_rhs")


def multi_rhs(seed: int = 3, M: int = 1000, R: int = 256, box: float = 150.0) -> Cluster:
    """M = 1000 disks, radii U[0.3,1.0] in [0,150]^2, gap 0.1; k = 10;
    N_p = ceil(k a_p) + 10; R = 256 uniform incidence angles."""
    rng = np.random.default_rng(seed)
    centers, radii = random_disks(rng, M, 0.3, 1.0, 0.0, box, 0.1)
    k = 10.0
    return Cluster(centers, radii, _ceil_rule(k, radii, 10), k, uniform_angles(R),
                   uniform_angles(360), "multi_rhs")


def uneven_instances(seed: int = 4, n_inst: int = 512, R: int = 8,
                     m_lo: int = 10, m_hi: int = 200) -> list[Cluster]:
    """Independent instances: M ~ U{m_lo..m_hi}, radii U[0.2,1.0], square of
    side sqrt(pi sum a^2 / 0.2) (20% area fraction), gap 0.1, k ~ U[1,20],
    N_p = ceil(k a_p) + 8, R = 8 incidence angles."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(n_inst)):
        rng = np.random.default_rng(child)
        M = int(rng.integers(m_lo, m_hi + 1))
        k = float(rng.uniform(1.0, 20.0))
        radii = rng.uniform(0.2, 1.0, M)
        side = math.sqrt(math.pi * float(np.sum(radii ** 2)) / 0.2)
        centers = np.empty((M, 2))
        for p in range(M):
            a = radii[p]
            for _ in range(10**6):
                c = rng.uniform(0.0, side, 2)
                if p == 0:
                    break
                d = np.hypot(centers[:p, 0] - c[0], centers[:p, 1] - c[1])
                if np.all(d >= a + radii[:p] + 0.1):
                    break
            else:
                raise RuntimeError("placement failed")
            centers[p] = c
        out.append(Cluster(centers, radii, _ceil_rule(k, radii, 8), k,
                           uniform_angles(R), uniform_angles(64), f"inst{i}"))
    return out


def perturb(rng: np.random.Generator, base: Cluster, sc: float = 0.05, sr: float = 0.02,
            min_gap: float = 0.05, min_r: float = 0.05) -> Cluster:
    """Target geometry: centers + N(0, sc^2), radii + N(0, sr^2); redrawn until
    every edge gap >= min_gap and every radius >= min_r.  N_p follows the same
    ceil rule (recomputed from the perturbed radii by the caller if needed)."""
    M = base.M
    for _ in range(10**4):
        c = base.centers + rng.normal(0.0, sc, (M, 2))
        r = base.radii + rng.normal(0.0, sr, M)
        if np.min(r) < min_r:
            continue
        d = np.hypot(c[:, None, 0] - c[None, :, 0], c[:, None, 1] - c[None, :, 1])
        g = d - r[:, None] - r[None, :]
        np.fill_diagonal(g, np.inf)
        if np.min(g) >= min_gap:
            return Cluster(c, r, base.n_modes.copy(), base.k, base.betas, base.thetas,
                           base.name + "_target")
    raise RuntimeError("perturbation failed")


def differentiation(seed: int = 5, n_cfg: int = 32, M: int = 100, R: int = 64,
                    n_rec: int = 64) -> list[tuple[Cluster, Cluster]]:
    """(base, target) pairs: M = 100 disks, radii U[0.4,0.8] in [0,40]^2, gap
    0.2, k = 8, N_p = ceil(8 a_p) + 8, 64 incidence angles and 64 receivers.
    Target = base perturbed (sigma 0.05 on centers, 0.02 on radii); the
    target's N_p follows the same rule from its own radii."""
    out = []
    for child in np.random.SeedSequence(seed).spawn(n_cfg):
        rng = np.random.default_rng(child)
        centers, radii = random_disks(rng, M, 0.4, 0.8, 0.0, 40.0, 0.2)
        k = 8.0
        base = Cluster(centers, radii, _ceil_rule(k, radii, 8), k, uniform_angles(R),
                       uniform_angles(n_rec), "diff")
        tgt = perturb(rng, base)
        tgt.n_modes = _ceil_rule(k, tgt.radii, 8)
        out.append((base, tgt))
    return out


def dort_example(n_alpha: int = 512) -> Cluster:
    """Three small sound-soft disks of the time-reversal example: centers
    (0,20), (10,-10), (-10,-20), radii 0.02, 0.01, 0.005, k = 2 pi;
    N_p = ceil(k a_p) + 3 = 4; mirror angles 2 pi j / n_alpha (incidences and,
    shifted by pi, receivers)."""
    centers = np.array([[0.0, 20.0], [10.0, -10.0], [-10.0, -20.0]])
    radii = np.array([0.02, 0.01, 0.005])
    k = 2.0 * math.pi
    al = uniform_angles(n_alpha)
    return Cluster(centers, radii, _ceil_rule(k, radii, 3), k, al, al + math.pi, "dort")


def penetrable_example(spacing: float = 3.0, half: int = 10) -> Cluster:
    """Penetrable lattice: unit disks on a (2 half + 1)^2 square lattice of the
    given spacing centered on the origin, with the row and the column through
    the origin removed (400 disks for half = 10); k+ = 1 (k- = 2 is the
    workload's interior wavenumber); N_p = 8; one point source at the origin;
    720 far-field angles."""
    g = spacing * np.arange(-half, half + 1)
    g = g[g != 0.0]
    X, Y = np.meshgrid(g, g, indexing="ij")
    centers = np.stack([X.ravel(), Y.ravel()], 1)
    M = centers.shape[0]
    return Cluster(centers, np.ones(M), np.full(M, 8, np.int32), 1.0, np.zeros(1),
                   uniform_angles(720), "penetrable")


def small_random(seed: int, M: int, r_lo: float, r_hi: float, box: float, gap: float,
                 k: float, extra: int, R: int = 1, n_theta: int = 64) -> Cluster:
    """Small seeded cluster for tests: N_p = ceil(k a_p) + extra."""
    rng = np.random.default_rng(seed)
    centers, radii = random_disks(rng, M, r_lo, r_hi, 0.0, box, gap)
    return Cluster(centers, radii, _ceil_rule(k, radii, extra), k, uniform_angles(R),
                   uniform_angles(n_theta), f"small{seed}")
