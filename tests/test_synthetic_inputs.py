"""The seeded input generators follow their stated recipe (CPU).

Each workload family stands in for the paper's DOTmark images (Section 5.1)
at the paper's grid sizes (Table 1).  These checks pin what the tests and the
bench rely on.  Sizes are the grid's pixel counts. Marginals are positive
histograms of mass 1 with the family's floor. Instances are reproducible
from their index, and source and target are drawn independently. The
batched family spreads over its side and bump ranges. Coordinates are the
integer pixel positions in row-major order.
"""
import numpy as np
import pytest

from synthetic import (CONFIGS, batch_instances, cauchy_mixture, config_instance,
                       gaussian_mixture, grid_coords, white_noise)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3", "c5"])
def test_family_sizes_mass_and_floor(cfg):
    c = CONFIGS[cfg]
    inst = config_instance(cfg, 0)
    side = c["side"]
    assert inst.m == inst.n == side * side
    for h in (inst.a, inst.b):
        assert h.dtype == np.float64 and h.shape == (side * side,)
        assert abs(h.sum() - 1.0) <= 1e-12
        assert h.min() > 0.0
        # the floor is added before normalising, and no pixel of the raw
        # density exceeds (number of bumps, or 1 for noise) + floor, so every
        # pixel keeps at least floor / (n * (bumps + floor)) of the mass
        k = max(c["components"], 1)
        assert h.min() >= c["floor"] / (side * side * (k + c["floor"]))
    assert np.array_equal(inst.xs, grid_coords(side)) and np.array_equal(inst.xt, inst.xs)


def test_coordinates_are_row_major_integer_pixels():
    xy = grid_coords(5)
    assert xy.dtype == np.int32 and xy.shape == (25, 2)
    assert xy[0].tolist() == [0, 0] and xy[1].tolist() == [0, 1] and xy[5].tolist() == [1, 0]
    assert xy[24].tolist() == [4, 4]


def test_instances_are_reproducible_and_sides_independent():
    a0 = config_instance("c2", 1)
    a1 = config_instance("c2", 1)
    assert np.array_equal(a0.a, a1.a) and np.array_equal(a0.b, a1.b)
    assert not np.array_equal(a0.a, a0.b)
    assert not np.array_equal(a0.a, config_instance("c2", 2).a)


def test_gaussian_bumps_peak_at_their_centres():
    # one bump, no floor to speak of: the histogram's maximum is the pixel
    # nearest the drawn centre
    d = gaussian_mixture(32, 1, seed=11, floor=1e-12)
    rng = np.random.default_rng(11)
    cx, cy = rng.uniform(0.0, 31.0, size=2)
    i = int(np.argmax(d))
    assert abs(i // 32 - cx) <= 0.5 + 1e-9 and abs(i % 32 - cy) <= 0.5 + 1e-9


def test_white_noise_is_flat_on_average():
    d = white_noise(128, seed=5)
    # i.i.d. U[0,1] + 1e-3, normalised: mean 1/n, relative spread of a
    # uniform variable (1/sqrt(3) of its mean)
    n = d.size
    assert abs(d.mean() - 1.0 / n) <= 1e-15
    rel_sd = d.std() / d.mean()
    assert abs(rel_sd - 1.0 / np.sqrt(3.0)) <= 0.02


def test_cauchy_bumps_are_heavy_tailed():
    # 1 / (1 + r^2 / s^2) keeps a fraction of its peak far from the centre,
    # where a Gaussian of the same scale has none
    side = 256
    c = cauchy_mixture(side, 4, seed=3, floor=1e-4)
    g = gaussian_mixture(side, 4, seed=3, floor=1e-4, sigma_range=(2.0, 16.0))
    assert abs(c.sum() - 1.0) <= 1e-12
    # mass outside the densest tenth of the pixels
    def tail(h):
        return np.sort(h)[: int(0.9 * h.size)].sum()
    assert tail(c) > 2.0 * tail(g)


def test_batch_family_spreads_over_its_ranges():
    insts = batch_instances(512)
    sides = np.array([int(round(np.sqrt(i.m))) for i in insts])
    assert all(i.m == i.n == s * s for i, s in zip(insts, sides))
    assert sides.min() == 8 and sides.max() == 32
    assert len(set(sides.tolist())) == 25  # every side in 8..32 occurs
    for i in insts[:16]:
        assert abs(i.a.sum() - 1.0) <= 1e-12 and i.a.min() > 0.0
    # instance k is the same whether drawn alone or within a batch
    k = 37
    alone = batch_instances(1, first=k)[0]
    assert np.array_equal(alone.a, insts[k].a) and np.array_equal(alone.b, insts[k].b)
    assert config_instance("c4", 3).m == insts[3].m
