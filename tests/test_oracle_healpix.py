"""Pins of the oracle's HEALPix geometry against properties the published
pixelization fixes (equal areas: Sec. 4.1 footnote; NESTED children and the
bit-shift bundle map: Sec. 3.1)."""
import numpy as np
import pytest

from oracle import healpix as hp


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16])
def test_counts_and_equal_area_rings(N):
    rt = hp.ring_table(N)
    assert rt["n"].sum() == 12 * N * N
    assert rt["first"][0] == 0
    assert np.array_equal(rt["first"][1:], np.cumsum(rt["n"])[:-1])
    # cap area above each ring centre = pixel area x (pixels in earlier rings
    # + half of this ring), which is what equal-area pixels with centres on
    # the ring require
    omega = 4 * np.pi / (12 * N * N)
    cap = 2 * np.pi * (1 - rt["z"])
    expect = omega * (rt["first"] + rt["n"] / 2)
    assert np.allclose(cap, expect, rtol=0, atol=1e-13)
    # north/south mirror symmetry and shared longitudes
    assert np.allclose(rt["z"], -rt["z"][::-1], atol=1e-15)
    assert np.array_equal(rt["n"], rt["n"][::-1])
    assert np.allclose(rt["phi0"], rt["phi0"][::-1])


def test_base_resolution():
    z, phi, _ = hp.pix2ang_ring(1, np.arange(12))
    assert np.allclose(z, [2 / 3] * 4 + [0] * 4 + [-2 / 3] * 4)
    assert np.allclose(phi[:4], np.pi / 4 + np.arange(4) * np.pi / 2)
    assert np.allclose(phi[4:8], np.arange(4) * np.pi / 2)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 32])
def test_nest_ring_bijection_and_ang2pix(N):
    p = np.arange(12 * N * N)
    r = hp.nest2ring(N, p)
    assert np.array_equal(np.sort(r), p)
    assert np.array_equal(hp.ring2nest(N, r), p)
    z, phi, _ = hp.pix2ang_nest(N, p)
    assert np.array_equal(hp.ang2pix_nest(N, z, phi), p)
    # the per-pixel RING -> NESTED map agrees with the full permutation
    assert np.array_equal(hp.ring2nest_pix(N, p), hp.ring2nest(N, p))


@pytest.mark.parametrize("N", [2, 4, 8])
def test_children_are_nearest_finer_pixels(N):
    """NESTED children 4p..4p+3 at 2N are the four finer pixels nearest to
    the parent centre (the parent centre is their common vertex)."""
    zc, pc, sc = hp.pix2ang_nest(N, np.arange(12 * N * N))
    vc = hp.vec(zc, pc, sc)
    zf, pf, sf = hp.pix2ang_nest(2 * N, np.arange(48 * N * N))
    vf = hp.vec(zf, pf, sf)
    d = vc @ vf.T
    nearest = np.sort(np.argsort(-d, axis=1)[:, :4], axis=1)
    expect = 4 * np.arange(12 * N * N)[:, None] + np.arange(4)[None, :]
    assert np.array_equal(nearest, expect)


def test_ang2pix_hierarchy_random_points():
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, 20000)
    phi = rng.uniform(0, 2 * np.pi, 20000)
    for N in [1, 2, 8, 64]:
        a = hp.ang2pix_nest(N, z, phi)
        b = hp.ang2pix_nest(2 * N, z, phi)
        assert np.array_equal(b >> 2, a)
    # a point is never far from its pixel's centre
    N = 16
    p = hp.ang2pix_nest(N, z, phi)
    zc, pc, sc = hp.pix2ang_nest(N, p)
    cosd = np.sum(hp.vec(z, phi) * hp.vec(zc, pc, sc), axis=1)
    assert np.all(np.arccos(np.clip(cosd, -1, 1)) < 1.4 * np.sqrt(4 * np.pi / (12 * N * N)))


def test_degrade_conserves_mass():
    rng = np.random.default_rng(1)
    m = rng.normal(size=12 * 64)
    d = hp.degrade_nest_mean(8, 2, m)
    assert np.isclose(d.sum() * 16, m.sum())
    assert np.allclose(hp.degrade_nest_mean(8, 8, m), m)


def test_interpolation():
    N = 8
    rt = hp.ring_table(N)
    npx = 12 * N * N
    rng = np.random.default_rng(2)
    m = rng.normal(size=npx)
    # exact at pixel centres
    z, phi, s = hp.pix2ang_ring(N, np.arange(npx))
    th = np.arctan2(s, z)
    assert np.allclose(hp.interp(N, m, th, phi), m, atol=1e-12)
    # reproduces a + b theta between the first and last ring
    f = 0.3 + 1.7 * np.arctan2(s, z)
    tq = rng.uniform(rt["theta"][0], rt["theta"][-1], 500)
    pq = rng.uniform(0, 2 * np.pi, 500)
    assert np.allclose(hp.interp(N, f, tq, pq), 0.3 + 1.7 * tq, atol=1e-12)
    # weights sum to one everywhere, including the polar caps
    tq = rng.uniform(0, np.pi, 2000)
    pix, w = hp.interp_weights(N, tq, rng.uniform(0, 2 * np.pi, 2000))
    assert np.allclose(w.sum(axis=0), 1.0)
    assert np.all(w >= -1e-15)
    # above the first ring the pole carries the ring mean
    v = hp.interp(N, m, np.array([0.0]), np.array([1.0]))
    assert np.isclose(v[0], m[:4].mean())
