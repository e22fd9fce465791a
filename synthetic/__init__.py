"""Seeded synthetic optimal-transport instances.

This module only draws inputs: two histograms on square pixel grids and the
integer pixel coordinates the squared-Euclidean cost is generated from.  It
holds none of the solver's arithmetic, so both the CPU oracle and the HIP
library can consume it without sharing any method code.

The paper measures on the DOTmark image collection (Section 5.1), which is not
available here; these generators stand in for it with densities of the same
shapes and sizes:

* ``gaussian_mixture``  -- sum of isotropic Gaussian bumps plus a floor
  (stands in for the "simulations based on probability distributions" classes);
* ``white_noise``       -- i.i.d. uniform pixels plus a floor;
* ``cauchy_mixture``    -- heavy-tailed bumps w / (1 + r^2/s^2) plus a floor.

Conventions (fixed so that every consumer sees identical arrays):

* ``numpy.random.default_rng(seed)`` (PCG64) for every draw;
* instance ``k`` of a family uses ``seed_a = 1_000_003*k + 1`` for the source
  histogram and ``seed_b = 1_000_003*k + 2`` for the target histogram;
* bump centres are continuous uniform on ``[0, side-1]^2``, weights uniform on
  ``[0.5, 1]``, bumps are unnormalised with peak value equal to the weight;
* the floor is added before normalising to total mass 1;
* pixel ``i`` sits at integer coordinates ``(i // side, i % side)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Instance",
    "grid_coords",
    "gaussian_mixture",
    "white_noise",
    "cauchy_mixture",
    "instance_seeds",
    "make_instance",
    "config_instance",
    "batch_instances",
    "CONFIGS",
]


@dataclass
class Instance:
    """One Kantorovich problem: masses ``a`` (m), ``b`` (n) and coordinates.

    ``xs`` is (m, 2) int32, ``xt`` is (n, 2) int32; the cost of moving a unit
    of mass from source i to target j is the integer squared Euclidean distance
    between ``xs[i]`` and ``xt[j]``.
    """

    a: np.ndarray
    b: np.ndarray
    xs: np.ndarray
    xt: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.a.shape[0])

    @property
    def n(self) -> int:
        return int(self.b.shape[0])


def grid_coords(side: int) -> np.ndarray:
    """Integer coordinates of the pixels of a ``side x side`` image."""
    i = np.arange(side * side, dtype=np.int64)
    return np.stack([i // side, i % side], axis=1).astype(np.int32)


def _grid_xy(side: int):
    c = grid_coords(side).astype(np.float64)
    return c[:, 0], c[:, 1]


def _normalise(d: np.ndarray, floor: float) -> np.ndarray:
    d = d + floor
    return (d / d.sum()).astype(np.float64)


def gaussian_mixture(side: int, components: int, seed: int, floor: float = 1e-3,
                     sigma_range=(1.0, 4.0)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y = _grid_xy(side)
    d = np.zeros(side * side, dtype=np.float64)
    for _ in range(components):
        cx, cy = rng.uniform(0.0, side - 1.0, size=2)
        sig = rng.uniform(*sigma_range)
        w = rng.uniform(0.5, 1.0)
        d += w * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sig * sig))
    return _normalise(d, floor)


def white_noise(side: int, seed: int, floor: float = 1e-3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _normalise(rng.uniform(0.0, 1.0, size=side * side), floor)


def cauchy_mixture(side: int, components: int, seed: int, floor: float = 1e-4,
                   scale_range=(2.0, 16.0)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x, y = _grid_xy(side)
    d = np.zeros(side * side, dtype=np.float64)
    for _ in range(components):
        cx, cy = rng.uniform(0.0, side - 1.0, size=2)
        s = rng.uniform(*scale_range)
        w = rng.uniform(0.5, 1.0)
        d += w / (1.0 + ((x - cx) ** 2 + (y - cy) ** 2) / (s * s))
    return _normalise(d, floor)


def instance_seeds(k: int):
    return 1_000_003 * k + 1, 1_000_003 * k + 2


# Workload families.  Sizes follow the paper's resolutions (Table 1) and the
# density shapes above.
CONFIGS = {
    # 16x16 grids, 3 Gaussian bumps, 10 seeds, FP64.
    "c1": dict(side=16, family="gauss", components=3, seeds=10, floor=1e-3),
    # 64x64 grids, 5 Gaussian bumps, 5 seeds, FP64.
    "c2": dict(side=64, family="gauss", components=5, seeds=5, floor=1e-3),
    # 128x128 white noise, 3 seeds, mixed precision.
    "c3": dict(side=128, family="noise", components=0, seeds=3, floor=1e-3),
    # 512 instances of side U{8..32}, 1-5 Gaussian bumps.
    "c4": dict(side=None, family="gauss_batch", components=None, seeds=512, floor=1e-3),
    # 256x256, 4 Cauchy bumps, 2 seeds.
    "c5": dict(side=256, family="cauchy", components=4, seeds=2, floor=1e-4),
}


def make_instance(side: int, family: str, components: int, k: int,
                  floor: float | None = None, name: str = "") -> Instance:
    sa, sb = instance_seeds(k)
    if family == "gauss":
        fl = 1e-3 if floor is None else floor
        a = gaussian_mixture(side, components, sa, fl)
        b = gaussian_mixture(side, components, sb, fl)
    elif family == "noise":
        fl = 1e-3 if floor is None else floor
        a = white_noise(side, sa, fl)
        b = white_noise(side, sb, fl)
    elif family == "cauchy":
        fl = 1e-4 if floor is None else floor
        a = cauchy_mixture(side, components, sa, fl)
        b = cauchy_mixture(side, components, sb, fl)
    else:
        raise ValueError(f"unknown family {family!r}")
    xy = grid_coords(side)
    return Instance(a=a, b=b, xs=xy, xt=xy.copy(), name=name or f"{family}{side}_k{k}")


def config_instance(cfg: str, k: int = 0) -> Instance:
    """Instance ``k`` of one of the workload families in ``CONFIGS``."""
    c = CONFIGS[cfg]
    if c["family"] == "gauss_batch":
        return batch_instances(k + 1)[k]
    return make_instance(c["side"], c["family"], c["components"], k, c["floor"],
                         name=f"{cfg}_k{k}")


def batch_instances(count: int = 512, side_range=(8, 32), comp_range=(1, 5),
                    first: int = 0) -> list[Instance]:
    """Instances of uneven grid sizes for batched solves.

    Instance k draws its side in ``side_range`` and its number of bumps in
    ``comp_range`` (both inclusive) from ``default_rng(1_000_003*k + 3)``;
    its histograms then follow the Gaussian-mixture recipe with the usual
    per-instance seeds.
    """
    out = []
    for k in range(first, first + count):
        rng = np.random.default_rng(1_000_003 * k + 3)
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        comp = int(rng.integers(comp_range[0], comp_range[1] + 1))
        out.append(make_instance(side, "gauss", comp, k, 1e-3, name=f"batch_k{k}"))
    return out
