"""Seeded synthetic-input generators shared by the oracle's data script, the tests and the bench.

This module holds no arithmetic of the method itself: it only names the workloads (sizes, counts,
iteration numbers) and draws raw random numbers from seeded ``numpy.random.Generator`` streams.
Everything that evaluates the head model, the projector or MLEM lives elsewhere.

Workloads (the paper's simulation study, Sec. "Simulation Studies", uses 128x128 grids, projections
over the full angular range and Poisson noise; its phantoms are not published, so a seeded phantom
family stands in for them):

* ``smoke_n64``      64x64 image at 0.4 cm, 64 angles over 360 deg x 64 bins, 1e5 counts, one
                     candidate (the true head), 20 MLEM iterations.
* ``plain_n128``     128x128 at 0.2 cm, 128 angles x 128 bins, 5e5 counts, one candidate, 50 iterations.
* ``batch256_n128``  the 128 slice above, 256 random candidates, 30 iterations plus the objective.
* ``grad64_n128``    the 128 slice above, 64 random candidates (own stream), 20 iterations,
                     objective and gradient, checkpoint every 5 iterations.
* ``paper72_n128``   the paper's angular sampling: 128x128 at 0.2 cm, 72 angles over 360 deg x 128
                     bins, 5e5 counts, simulated on a 2x finer grid (no inverse crime), 256 random
                     candidates, 30 iterations plus the objective.
* ``uneven48``       48 slices with N in {96,128,192,256}, angles in {64,96,128,256}, bins = N,
                     pixel = 25.6/N cm, counts log-uniform in [1e5, 2e6], 32 candidates each,
                     40 iterations plus objective and gradient.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Iterator, List, Tuple

import numpy as np

# True head used to simulate every slice: Legendre coefficients c_0..c_5 (cm), brain and cranium
# attenuation (1/cm) and the fixed cranium thickness delta_R (cm).
TRUE_C = (7.5, 0.0, 1.2, 0.0, -0.3, 0.0)
TRUE_MU_B = 0.150
TRUE_MU_C = 0.250
DELTA_R = 0.8

# Candidate prior: c_0 ~ U[6.5, 8.5], c_1..c_5 ~ U[-1.5, 1.5] (cm), mu_b ~ U[0.13, 0.17],
# mu_c ~ U[0.20, 0.30] (1/cm).
CAND_LO = np.array([6.5, -1.5, -1.5, -1.5, -1.5, -1.5, 0.13, 0.20])
CAND_HI = np.array([8.5, 1.5, 1.5, 1.5, 1.5, 1.5, 0.17, 0.30])

# Phantom: three hot disks of radius U[0.8, 1.5] cm at four times the background activity.
N_DISKS = 3
DISK_R_LO, DISK_R_HI = 0.8, 1.5
BACKGROUND_ACTIVITY = 1.0
DISK_ACTIVITY = 4.0


@dataclass(frozen=True)
class SliceSpec:
    """One sinogram slice: image n x n with the given pixel (cm), n_angles over 360 deg, n_bins bins,
    n_samples samples per ray (spacing = pixel), total expected counts, and its seed."""
    n: int
    n_angles: int
    n_bins: int
    n_samples: int
    pixel: float
    counts: float
    seed: int
    # independent seed stream for this slice (phantom, noise, candidates)
    stream: Tuple[int, ...] = ()
    # data simulated on a grid this many times finer than the reconstruction grid (1: the same grid)
    oversample: int = 1
    # true head (c_0..c_5, mu_b, mu_c) of this slice; empty: the default true head
    true_theta: Tuple[float, ...] = ()


@dataclass(frozen=True)
class Workload:
    name: str
    slices: Tuple[SliceSpec, ...]
    n_cand: int
    n_iter: int
    ckpt_every: int = 0          # 0: forward only
    cand_seed_offset: int = 0    # candidates come from seed + offset's candidate stream
    true_candidate_only: bool = False


def _slice(n, na, counts, seed, pixel=None):
    return SliceSpec(n=n, n_angles=na, n_bins=n, n_samples=n,
                     pixel=float(pixel if pixel is not None else 25.6 / n),
                     counts=float(counts), seed=seed)


def workload(name: str, seed: int = 0) -> Workload:
    if name == "smoke_n64":
        return Workload(name, (_slice(64, 64, 1e5, seed, 0.4),), 1, 20, true_candidate_only=True)
    if name == "plain_n128":
        return Workload(name, (_slice(128, 128, 5e5, seed, 0.2),), 1, 50, true_candidate_only=True)
    if name == "batch256_n128":
        return Workload(name, (_slice(128, 128, 5e5, seed, 0.2),), 256, 30)
    if name == "grad64_n128":
        return Workload(name, (_slice(128, 128, 5e5, seed, 0.2),), 64, 20, ckpt_every=5,
                        cand_seed_offset=1)
    if name == "paper72_n128":
        sl = SliceSpec(n=128, n_angles=72, n_bins=128, n_samples=128, pixel=0.2, counts=5e5, seed=seed,
                       stream=(72,), oversample=2)
        return Workload(name, (sl,), 256, 30)
    if name == "uneven48":
        return Workload(name, tuple(uneven_layout(seed, 48)), 32, 40, ckpt_every=5)
    raise KeyError(name)


WORKLOADS = ("smoke_n64", "plain_n128", "batch256_n128", "grad64_n128", "paper72_n128", "uneven48")


# Three true heads of the BOAC-vs-NAC study (cases A, B, C), inside the candidate box.
STUDY_HEADS = (
    (7.5, 0.0, 1.2, 0.0, -0.3, 0.0, 0.150, 0.250),
    (7.8, 0.3, 0.9, -0.2, -0.2, 0.1, 0.145, 0.260),
    (7.2, -0.2, 1.4, 0.1, -0.4, -0.1, 0.155, 0.235),
)


def study_cases(seed: int = 0) -> List[SliceSpec]:
    """The study's slices: the paper's geometry (128^2, 72 angles over 360 deg), data simulated on a
    2x finer grid, 5e5 counts, one true head and phantom seed stream per case."""
    return [SliceSpec(n=128, n_angles=72, n_bins=128, n_samples=128, pixel=0.2, counts=5e5, seed=seed,
                      stream=(9, k), oversample=2, true_theta=tuple(h)) for k, h in enumerate(STUDY_HEADS)]


def slice_truth(spec: SliceSpec) -> np.ndarray:
    return np.array(spec.true_theta, dtype=np.float64) if spec.true_theta else true_candidate()


def streams(seed: int, stream: Tuple[int, ...] = ()):
    """(phantom, noise, candidate) generators of one slice, from SeedSequence(seed) or a spawned key."""
    ss = np.random.SeedSequence(seed, spawn_key=tuple(stream))
    a, b, c = ss.spawn(3)
    return np.random.Generator(np.random.PCG64(a)), np.random.Generator(np.random.PCG64(b)), \
        np.random.Generator(np.random.PCG64(c))


def candidate_stream(seed: int, stream: Tuple[int, ...] = ()) -> np.random.Generator:
    return streams(seed, stream)[2]


def draw_candidates(rng: np.random.Generator, count: int) -> np.ndarray:
    """count x 8 candidates (c_0..c_5, mu_b, mu_c), drawn candidate by candidate in that order."""
    u = rng.random((count, 8))
    return CAND_LO + (CAND_HI - CAND_LO) * u


def true_candidate() -> np.ndarray:
    return np.array(list(TRUE_C) + [TRUE_MU_B, TRUE_MU_C], dtype=np.float64)


def disk_proposals(rng: np.random.Generator) -> Iterator[Tuple[float, float, float]]:
    """Endless (u_radius, u_x, u_y) triples in [0,1)^3; the phantom builder maps and accepts them."""
    while True:
        u = rng.random(3)
        yield float(u[0]), float(u[1]), float(u[2])


def uneven_layout(seed: int, n_slices: int) -> List[SliceSpec]:
    """Slices of the uneven batch: N and angle count drawn uniformly and independently from their sets,
    counts log-uniform in [1e5, 2e6]; each slice gets its own spawned seed stream."""
    ss = np.random.SeedSequence([seed, 5])
    layout = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    ns = layout.choice([96, 128, 192, 256], size=n_slices)
    nas = layout.choice([64, 96, 128, 256], size=n_slices)
    counts = np.exp(layout.uniform(np.log(1e5), np.log(2e6), size=n_slices))
    out = []
    for s in range(n_slices):
        out.append(SliceSpec(n=int(ns[s]), n_angles=int(nas[s]), n_bins=int(ns[s]),
                             n_samples=int(ns[s]), pixel=25.6 / float(ns[s]),
                             counts=float(counts[s]), seed=seed, stream=(5, s)))
    return out


def workload_candidates(w: Workload, seed: int = 0) -> List[np.ndarray]:
    """Per-slice candidate arrays [C, 8] (float64) of a workload."""
    out = []
    for sl in w.slices:
        if w.true_candidate_only:
            out.append(true_candidate()[None, :].repeat(w.n_cand, axis=0))
            continue
        rng = candidate_stream(sl.seed + w.cand_seed_offset, sl.stream)
        out.append(draw_candidates(rng, w.n_cand))
    return out
