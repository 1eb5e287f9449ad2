"""Seeded input generators: reproducibility, distributions, layout, geometry."""
import math

import numpy as np
import pytest

from paper_2510_20507_amd import synth


def test_seeded_reproducible_and_subset_consistent():
    a = synth.rayleigh_sweep(B_per_p=3)
    b = synth.rayleigh_sweep(B_per_p=3)
    np.testing.assert_array_equal(a.H, b.H)
    np.testing.assert_array_equal(a.V0, b.V0)
    np.testing.assert_array_equal(a.alpha, b.alpha)
    s = a.subset([4, 1])
    i4 = a.instance(4)
    j0 = s.instance(0)
    np.testing.assert_array_equal(i4["H"][0], j0["H"][0])
    np.testing.assert_array_equal(i4["V0"][0], j0["V0"][0])


def test_sweep_layout_and_power():
    b = synth.rayleigh_sweep(B_per_p=2)
    assert b.batch == 8
    assert list(b.P) == pytest.approx([1, 1, 10, 10, 100, 100, 1000, 1000])
    for i in range(b.batch):
        inst = b.instance(i)
        assert inst["H"][0].shape == (64, 64)
        assert inst["V0"][0].shape == (64, 64)
        p = np.vdot(inst["V0"][0], inst["V0"][0]).real
        assert p == pytest.approx(inst["P"][0], rel=1e-12)
        assert np.all((inst["alpha"] >= 0.5) & (inst["alpha"] <= 1.5))
    assert b.h_off[1] == 64 * 64 and b.v_off[1] == 64 * 64


def test_cn01_moments():
    rng = np.random.default_rng(0)
    x = synth.cn01(rng, 400000)
    assert np.mean(np.abs(x) ** 2) == pytest.approx(1.0, rel=1e-2)
    assert abs(np.mean(x)) < 1e-2
    assert np.mean(x.real ** 2) == pytest.approx(0.5, rel=2e-2)
    assert abs(np.mean(x * x)) < 1e-2          # circular symmetry: E[x^2] = 0


def test_single_small_shapes():
    b = synth.single_small()
    inst = b.instance(0)
    assert (inst["M"], inst["U"], inst["N"], inst["d"]) == (8, 4, 2, 2)
    assert inst["H"][0].shape == (8, 8)
    assert inst["P"][0] == 10.0 and np.all(inst["alpha"] == 1) and np.all(inst["sigma2"] == 1)


def test_hexcell_geometry_and_scales():
    b = synth.hexcell_batch(B=40)
    sites = synth.hex_sites()
    assert np.allclose(np.linalg.norm(sites[1:], axis=1), 500.0)
    for i in range(b.batch):
        inst = b.instance(i)
        assert inst["C"] == 7
        assert inst["M"] in (16, 32, 64, 128)
        assert inst["N"] in (1, 2, 4) and inst["d"] == min(inst["N"], 2)
        assert all(2 <= u <= 12 for u in inst["cell_users"])
        assert len(inst["H"]) == 7
        for c in range(7):
            assert inst["H"][c].shape == (inst["U"] * inst["N"], inst["M"])
            assert inst["V0"][c].shape == (inst["M"], inst["cell_users"][c] * inst["d"])
            assert np.vdot(inst["V0"][c], inst["V0"][c]).real == pytest.approx(synth.HEX_P_W)
        assert inst["sigma2"][0] == pytest.approx(3.98e-14, rel=1e-2)
        # received power per antenna: between 35 m without shadowing (+4 sigma)
        # and the farthest site with -4 sigma shadowing
        gains = np.array([np.mean(np.abs(inst["H"][c]) ** 2) for c in range(7)])
        pl_min = synth.pathloss_db(35.0) - 4 * 8
        pl_max = synth.pathloss_db(1500.0) + 4 * 8
        g_db = -10 * np.log10(gains)
        assert np.all(g_db > pl_min - 6) and np.all(g_db < pl_max + 6)


def test_uniform_in_hexagon():
    rng = np.random.default_rng(1)
    R = 500 / math.sqrt(3)
    pts = np.array([synth._uniform_in_hexagon(rng, R, 35.0) for _ in range(4000)])
    r = np.linalg.norm(pts, axis=1)
    assert r.min() >= 35.0 and r.max() <= R + 1e-9
    # area-uniform: compare the mean distance with a fine deterministic grid
    # over the same region (hexagon minus the 35 m disc)
    g = np.linspace(-R, R, 1201)
    X, Y = np.meshgrid(g, g)
    h = R * math.sqrt(3) / 2
    inside = (np.abs(Y) <= h) & (math.sqrt(3) * np.abs(X) + np.abs(Y) <= math.sqrt(3) * R)
    rr = np.hypot(X, Y)
    inside &= rr >= 35.0
    assert np.mean(r) == pytest.approx(rr[inside].mean(), rel=0.02)
    # and the fraction of points within R/2 matches the area fraction
    assert np.mean(r <= R / 2) == pytest.approx(np.mean(rr[inside] <= R / 2), abs=0.03)


def test_pathloss_formula_values():
    assert synth.pathloss_db(1000.0) == pytest.approx(128.1)
    assert synth.pathloss_db(100.0) == pytest.approx(128.1 - 37.6)
