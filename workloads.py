"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only *draws numbers and names shapes*; it contains none of the
integrator's arithmetic (no operators, no reaction terms, no equilibria).
Both the oracle and the HIP path receive exactly these arrays.

Memory layout of every field produced here: C-contiguous
``[species][n3][n2][n1]`` (2D geometries drop ``n3``), i.e. the first grid
coordinate of the paper is the fastest-varying index, matching the paper's
vectorisation ``w_{i+(j-1)n+(k-1)n^2}`` (Section 2, eqs. (disk)-(cylinder)).

Randomness: the paper seeds MATLAB's generator; that stream cannot be
reproduced here, so every draw uses ``numpy.random.default_rng(seed)`` with
the seeds listed in each workload, and the perturbations are one-sided
uniform ``U(0,1)`` as in the paper's Section 5.3 and 5.6 initial data.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

GEOMETRIES = ("disk", "sphere", "ball", "cylinder", "disk_lambda")


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic problem instance family.

    ``n`` is the grid in the paper's coordinate order:
      disk and disk_lambda (n_rho, n_theta); sphere (n_theta, n_phi);
      ball (n_rho, n_theta, n_phi); cylinder (n_rho, n_theta, n_z).
    ``reaction`` names the kinetics ("schnakenberg" or "ais3": a 3-species
    activator-inhibitor-substrate system); ``params`` are its constants,
    ``diff`` the per-species diffusion coefficients.
    """

    name: str
    geometry: str
    n: Tuple[int, ...]
    reaction: str
    params: Tuple[float, ...]
    diff: Tuple[float, ...]
    tau: float
    steps: int
    seed: int
    amplitude: float = 1e-3
    extent: Tuple[float, float] = (1.0, 1.0)  # (rho_*, z_*); disk_lambda: (rho_*, lambda)
    batch: int = 1

    @property
    def n_species(self) -> int:
        return len(self.diff)

    @property
    def grid_points(self) -> int:
        return int(np.prod(self.n))

    @property
    def dof(self) -> int:
        """Degrees of freedom counted over all species and instances."""
        return self.grid_points * self.n_species * self.batch

    def field_shape(self) -> Tuple[int, ...]:
        return (self.n_species,) + tuple(reversed(self.n))


# Schnakenberg constants (a, b) and diffusion (d_u, d_v) of the activator-
# inhibitor workloads; the 3-species model constants are (a, b, kappa, mu).
SCHNAK = (0.1, 0.9)
AIS3 = (0.1, 0.9, 0.5, 1.0)
# anomalous-diffusion disk (Section 5.3): (alpha_2, beta_1, alpha_1) and lambda
SCHNAK_ANOMALOUS = (0.14, 1.34, 500.0)
ANOMALOUS_LAMBDA = -1.95

WORKLOADS: Dict[str, Workload] = {
    "disk_32x64": Workload("disk_32x64", "disk", (32, 64), "schnakenberg",
                           SCHNAK, (1.0, 20.0), 1e-2, 100, seed=2),
    "ball_64x64x128": Workload("ball_64x64x128", "ball", (64, 64, 128),
                               "schnakenberg", SCHNAK, (1.0, 20.0), 5e-3,
                               500, seed=3),
    "cylinder_100x100x100": Workload("cylinder_100x100x100", "cylinder",
                                     (100, 100, 100), "ais3", AIS3,
                                     (1.0, 10.0, 40.0), 2e-3, 1000, seed=4),
    "sphere_256x512": Workload("sphere_256x512", "sphere", (256, 512),
                               "schnakenberg", SCHNAK, (1.0, 20.0), 1e-2,
                               2000, seed=1000, batch=64),
    "sphere_128x256": Workload("sphere_128x256", "sphere", (128, 256),
                               "schnakenberg", SCHNAK, (1.0, 20.0), 1e-2,
                               2000, seed=1064, batch=32),
    "disk_256x512": Workload("disk_256x512", "disk", (256, 512),
                             "schnakenberg", SCHNAK, (1.0, 20.0), 1e-2, 400,
                             seed=6),
    # Section 5.3: anomalous diffusion Delta_lambda, lambda = -1.95, on the
    # unit disk with Dirichlet data at the equilibrium; kinetics alpha_1 (b, c)
    # with (alpha_2, beta_1, alpha_1) = (0.14, 1.34, 500), d = (1, delta = 50),
    # t_* = 2.5 in m = 25000 steps, perturbation 1e-5 U(0, 1)
    "disk_lambda_160x160": Workload("disk_lambda_160x160", "disk_lambda", (160, 160),
                                    "schnakenberg_scaled", SCHNAK_ANOMALOUS, (1.0, 50.0),
                                    1e-4, 25000, seed=8, amplitude=1e-5,
                                    extent=(1.0, ANOMALOUS_LAMBDA)),
}


# Section 5.5: bulk-surface Schnakenberg, ball (u, v) + its surface (r, s).
# Grid (n_rho, n_theta, n_phi) = (30, 50, 30), t_* = 15 in m = 150000 steps,
# perturbations 1e-3 N(0, 1) per point and species (the paper's draw).
BULK_SURFACE = dict(name="ball_sphere_30x50x30", n=(30, 50, 30), tau=1e-4, steps=150000, seed=9,
                    amplitude=1e-3)


def bulk_surface_perturbations(n: Tuple[int, int, int], seed: int, amplitude: float = 1e-3):
    """(bulk [2][n3][n2][n1], surface [2][n3][n2]) deviations, amplitude * N(0, 1)."""
    rng = np.random.default_rng(seed)
    bulk = amplitude * rng.standard_normal((2, n[2], n[1], n[0]))
    surf = amplitude * rng.standard_normal((2, n[2], n[1]))
    return bulk, surf


# Section 5.6: bulk-surface DIB model, cylinder (n_rho, n_theta, n_z) =
# (140, 140, 25) of radius 15 and height 25 with its bottom disk (140, 140);
# t_* = 250 in m = 10000 steps; the bulk starts at its equilibrium and the
# surface species at theirs plus 1e-2 U(0, 1) per point.
BULK_SURFACE_CYLINDER = dict(name="cylinder_disk_140x140x25", n=(140, 140, 25), extent=(15.0, 25.0),
                             tau=0.025, steps=10000, seed=10, amplitude=1e-2)


def bulk_surface_cylinder_perturbations(n: Tuple[int, int, int], seed: int, amplitude: float = 1e-2):
    """(bulk [2][n3][n2][n1] zeros, surface [2][n2][n1] amplitude * U(0, 1))."""
    rng = np.random.default_rng(seed)
    return np.zeros((2, n[2], n[1], n[0])), amplitude * rng.random((2, n[1], n[0]))


def scaled(w: Workload, n: Tuple[int, ...], steps: Optional[int] = None,
           name: Optional[str] = None) -> Workload:
    """Same physics on a different grid (used for small parity cases)."""
    return dataclasses.replace(w, n=tuple(n), steps=w.steps if steps is None else steps,
                               name=name or f"{w.geometry}_{'x'.join(map(str, n))}")


def perturbation(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Initial deviation from the homogeneous steady state.

    ``amplitude * U(0,1)`` per grid point and species, float64, layout
    ``[species][n3][n2][n1]``.
    """
    rng = np.random.default_rng(w.seed if seed is None else seed)
    return w.amplitude * rng.random(w.field_shape())


def batch_perturbations(w: Workload) -> np.ndarray:
    """``[batch][species][...]``: instance ``b`` uses seed ``w.seed + b``."""
    return np.stack([perturbation(w, w.seed + b) for b in range(w.batch)])


def sphere_batch_params(n_instances: int, seed: int = 5) -> np.ndarray:
    """Per-instance ``(a, b, d_v)`` drawn from U[0.05,0.2] x U[0.7,1.1] x U[10,40]."""
    rng = np.random.default_rng(seed)
    lo = np.array([0.05, 0.7, 10.0])
    hi = np.array([0.2, 1.1, 40.0])
    return lo + (hi - lo) * rng.random((n_instances, 3))


def target_pattern(w: Workload, seed: int = 7) -> np.ndarray:
    """Deviation field of the seeded target used by the gradient workload."""
    return perturbation(w, seed)[0]


def random_field(shape: Tuple[int, ...], seed: int, scale: float = 1.0,
                 centred: bool = True) -> np.ndarray:
    """Generic seeded test field (U(-1,1) if centred else U(0,1)), float64."""
    rng = np.random.default_rng(seed)
    x = rng.random(shape)
    return scale * (2.0 * x - 1.0 if centred else x)


def list_workloads() -> List[str]:
    return sorted(WORKLOADS)
