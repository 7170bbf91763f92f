"""Pins of the oracle's power spectra of a ray state (oracle/spectra.py):
closed forms and identities, not its own formulas retyped.

* Y_20: its shear is gamma_1 = 3 sqrt(5/(16 pi)) sin^2 theta, gamma_2 = 0
  (worked out by hand from U_tt = f'', U_pp = cot f'), whose only mode is
  E_20 = N_2 / 2 = sqrt(6);
* random potentials: the shear built by the (separately pinned) derivative
  synthesis analyses to E_lm = N_l psi_lm / 2 and B = 0, and turning it by
  45 degrees swaps the two (B' = E, E' = -B);
* the maps of a ray state: eq. invmagmat inverted exactly for rays at their
  pixel centres; transport along a meridian leaves the components alone;
  any transport keeps kappa, omega and |gamma|;
* a spectrum of single modes by hand.

Tolerances: HEALPix quadrature is not exact; at Nside 32 the spin-2
analysis of fields band-limited at l <= 8 reproduces the coefficients to
about 4e-4 of the largest (the spin-0 analysis of the same potential's
convergence: 2e-4), an error that falls as Nside^-2."""
import numpy as np
import pytest

from oracle import healpix as hp
from oracle import sht
from oracle import spectra as osp


def nl(l):
    return np.sqrt(np.maximum((l - 1.0) * l * (l + 1.0) * (l + 2.0), 0.0))


def test_y20_shear_is_pure_e():
    N, lmax = 32, 8
    z, ph, s = hp.pix2ang_ring(N, np.arange(12 * N * N))
    g1 = 3.0 * np.sqrt(5.0 / (16.0 * np.pi)) * s * s
    E, B = osp.spin2_map2alm(N, lmax, g1, np.zeros_like(g1))
    i20 = sht.alm_index(lmax, 2, 0)
    assert abs(E[i20] - np.sqrt(6.0)) < 1e-4 * np.sqrt(6.0)
    rest = np.delete(E, i20)
    assert np.abs(rest).max() < 1e-4 * np.sqrt(6.0)
    assert np.abs(B).max() < 1e-4 * np.sqrt(6.0)


def random_psi(lmax, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(sht.nalm(lmax)) + 1j * rng.standard_normal(sht.nalm(lmax))
    l, m = sht.lm_arrays(lmax)
    a[m == 0] = a[m == 0].real
    a[l < 2] = 0.0
    return a


@pytest.mark.parametrize("seed", [1, 2])
def test_potential_shear_round_trip_and_rotation(seed):
    """The error of the round trip is HEALPix quadrature: below 1e-3 at
    Nside 32 and falling as Nside^-2 (at least 3.5x from Nside 32 to 64)."""
    lmax = 8
    psi = random_psi(lmax, seed)
    l, _ = sht.lm_arrays(lmax)
    want = 0.5 * nl(l) * psi
    scale = np.abs(want).max()
    errs = []
    for N in (32, 64):
        d = sht.derivative_maps(N, lmax, psi)
        g1 = 0.5 * (d["U_tt"] - d["U_pp"])
        g2 = d["U_tp"]
        E, B = osp.spin2_map2alm(N, lmax, g1, g2)
        errs.append(max(np.abs(E - want).max(), np.abs(B).max()) / scale)
        E2, B2 = osp.spin2_map2alm(N, lmax, -g2, g1)
        np.testing.assert_allclose(B2, E, atol=1e-13 * scale)
        np.testing.assert_allclose(E2, -B, atol=1e-13 * scale)
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 3.5, errs


def fields_matrix(k, g1, g2, w):
    return np.array([1 - k - g1, -g2 + w, -g2 - w, 1 - k + g1])


def centre_state(N):
    n = 12 * N * N
    z, ph, s = hp.pix2ang_nest(N, np.arange(n))
    return np.arctan2(s, z), ph


def test_fields_at_pixel_centres_invert_invmagmat():
    N = 4
    n = 12 * N * N
    rng = np.random.default_rng(5)
    k, g1, g2, w = rng.standard_normal((4, n)) * 0.1
    th, ph = centre_state(N)
    f = osp.fields_from_rays(N, th, ph, fields_matrix(k, g1, g2, w))
    r = hp.nest2ring(N, np.arange(n))
    for got, want in zip(f, (k, g1, g2, w)):
        np.testing.assert_allclose(got[r], want, atol=1e-14)


def test_fields_transport_invariants():
    N = 4
    n = 12 * N * N
    rng = np.random.default_rng(6)
    k, g1, g2, w = rng.standard_normal((4, n)) * 0.1
    th, ph = centre_state(N)
    A = fields_matrix(k, g1, g2, w)
    r = hp.nest2ring(N, np.arange(n))
    # along the meridian: theta-hat and phi-hat are parallel transported
    dth = 0.01 * np.where(th < np.pi / 2, 1.0, -1.0)
    f = osp.fields_from_rays(N, th + dth, ph, A)
    for got, want in zip(f, (k, g1, g2, w)):
        np.testing.assert_allclose(got[r], want, atol=1e-13)
    # an arbitrary small displacement rotates gamma only
    f = osp.fields_from_rays(N, th + 0.02, ph + 0.05, A)
    np.testing.assert_allclose(f[0][r], k, atol=1e-13)
    np.testing.assert_allclose(f[3][r], w, atol=1e-13)
    np.testing.assert_allclose(np.hypot(f[1][r], f[2][r]), np.hypot(g1, g2), atol=1e-13)
    assert np.abs(f[1][r] - g1).max() > 1e-4


def test_spectrum_by_hand():
    lmax = 4
    a = np.zeros(sht.nalm(lmax), complex)
    a[sht.alm_index(lmax, 3, 1)] = 1 + 1j
    a[sht.alm_index(lmax, 3, 0)] = 2.0
    a[sht.alm_index(lmax, 0, 0)] = 0.5
    cl = osp.spectrum(lmax, a)
    np.testing.assert_allclose(cl, [0.25, 0, 0, (4.0 + 2 * 2.0) / 7.0, 0], atol=1e-15)
