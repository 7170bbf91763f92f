"""Pins of the oracle's SHT (Sec. 3.2: analysis, -l(l+1) psi_lm = kappa_lm,
synthesis, pure-SHT derivatives) against the mathematics: orthonormality,
library Legendre functions, brute-force Y_lm sums, single-harmonic and
closed-form lens solutions (App. A, App. E)."""
import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

from oracle import healpix as hp
from oracle import sht


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, np.sqrt(1 - x * x), w


@pytest.mark.parametrize("lmax,ms", [(40, [0, 1, 5, 40]), (1400, [1300, 1400])])
def test_legendre_orthonormal_gauss(lmax, ms):
    """2 pi sum_k w_k lambda_lm lambda_l'm = delta_ll' on Gauss-Legendre
    nodes; at lmax 1400 the high-m functions underflow float64 near the
    poles and exercise the scaled recurrence."""
    x, s, w = _gl(lmax + 1)
    l, m = sht.lm_arrays(lmax)
    keep = np.isin(m, ms)
    lam = np.zeros((keep.sum(), x.size))
    idx = {int(i): k for k, i in enumerate(np.nonzero(keep)[0])}
    for k, L in sht.lambda_diagonals(lmax, x, s):
        for mm in ms:
            if mm <= lmax - k:
                lam[idx[sht.alm_index(lmax, mm + k, mm)]] = L[mm]
    for mm in ms:
        rows = lam[m[keep] == mm]
        G = 2 * np.pi * (rows * w) @ rows.T
        assert np.abs(G - np.eye(rows.shape[0])).max() < 1e-12


def test_legendre_against_scipy():
    lmax = 30
    x, s, _ = _gl(17)
    lam = sht.lambda_table(lmax, x, s)
    l, m = sht.lm_arrays(lmax)
    # m = 0: sqrt((2l+1)/4pi) P_l
    ref0 = np.sqrt((2 * np.arange(lmax + 1) + 1) / (4 * np.pi))[:, None] * \
        eval_legendre(np.arange(lmax + 1)[:, None], x[None, :])
    assert np.allclose(lam[: lmax + 1], ref0, atol=1e-13)
    # all m: Y_lm(theta, 0) from scipy (includes the Condon-Shortley phase)
    th = np.arccos(x)
    for k in range(l.size):
        ref = sph_harm_y(l[k], m[k], th, 0.0).real
        assert np.allclose(lam[k], ref, atol=1e-12), (l[k], m[k])


def test_legendre_mirror_parity():
    lmax = 60
    x, s, _ = _gl(20)
    a = sht.lambda_table(lmax, x, s)
    b = sht.lambda_table(lmax, -x, s)
    l, m = sht.lm_arrays(lmax)
    assert np.allclose(b, ((-1.0) ** (l + m))[:, None] * a, atol=1e-12)


def test_ring_transforms_direct_sum():
    N, lmax = 4, 37              # lmax above every ring length: aliasing
    rt = hp.ring_table(N)
    rng = np.random.default_rng(3)
    f = rng.normal(size=12 * N * N)
    F = sht.ring_forward(N, lmax, f)
    G = rng.normal(size=F.shape) + 1j * rng.normal(size=F.shape)
    out = sht.ring_inverse(N, G)
    ms = np.arange(lmax + 1)
    for r in range(rt["n"].size):
        n, p0 = rt["n"][r], rt["first"][r]
        phi = rt["phi0"][r] + 2 * np.pi * np.arange(n) / n
        ref = np.exp(-1j * ms[:, None] * phi[None, :]) @ f[p0:p0 + n]
        assert np.allclose(F[r], ref, atol=1e-12)
        c = np.where(ms == 0, 1.0, 2.0)
        ref_inv = np.real((c * G[r])[None, :] * np.exp(1j * phi[:, None] * ms[None, :])).sum(1)
        assert np.allclose(out[p0:p0 + n], ref_inv, atol=1e-11)


@pytest.mark.parametrize("N,lmax", [(4, 9), (8, 16)])
def test_synthesis_bruteforce(N, lmax):
    rng = np.random.default_rng(N)
    l, m = sht.lm_arrays(lmax)
    alm = rng.normal(size=l.size) + 1j * rng.normal(size=l.size)
    alm[m == 0] = alm[m == 0].real
    mp = sht.alm2map(N, lmax, alm)
    z, ph, s = hp.pix2ang_ring(N, np.arange(12 * N * N))
    th = np.arctan2(s, z)
    ref = np.zeros_like(mp)
    for k in range(l.size):
        ref += (sph_harm_y(l[k], m[k], th, ph) * alm[k]).real * (1 if m[k] == 0 else 2)
    assert np.abs(mp - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_analysis_recovers_bandlimited():
    """HEALPix quadrature is not exact; with lmax <= N and Jacobi
    iterations the analysis converges to the input a_lm."""
    N, lmax = 16, 16
    rng = np.random.default_rng(7)
    l, m = sht.lm_arrays(lmax)
    alm = rng.normal(size=l.size) + 1j * rng.normal(size=l.size)
    alm[m == 0] = alm[m == 0].real
    mp = sht.alm2map(N, lmax, alm)
    e0 = np.abs(sht.map2alm(N, lmax, mp) - alm).max()
    e3 = np.abs(sht.map2alm(N, lmax, mp, iters=3) - alm).max()
    assert e0 < 0.05
    assert e3 < 1e-4 and e3 < e0 / 100


def test_poisson_single_harmonic():
    lmax = 20
    for (L, M) in [(1, 0), (2, 0), (5, 3), (20, 20)]:
        a = np.zeros(sht.nalm(lmax), complex)
        a[sht.alm_index(lmax, L, M)] = 0.7 - 0.2j if M else 0.7
        p = sht.poisson(lmax, a)
        assert np.isclose(p[sht.alm_index(lmax, L, M)], -2 * a[sht.alm_index(lmax, L, M)] / (L * (L + 1)))
    a = np.zeros(sht.nalm(lmax), complex)
    a[0] = 3.0
    assert sht.poisson(lmax, a)[0] == 0


def test_Y20_Y10_closed_forms():
    """kappa = Y_20 gives gamma_1 = -sqrt(5/16pi) sin^2(theta), gamma_2 = 0
    and kappa_rec = Y_20; kappa = Y_10 gives zero shear (App. A formulas)."""
    N, lmax = 16, 32
    z, ph, s = hp.pix2ang_ring(N, np.arange(12 * N * N))
    a = np.zeros(sht.nalm(lmax), complex)
    a[sht.alm_index(lmax, 2, 0)] = 1.0
    d = sht.derivative_maps(N, lmax, sht.poisson(lmax, a))
    g1 = 0.5 * (d["U_tt"] - d["U_pp"])
    assert np.allclose(g1, -np.sqrt(5 / (16 * np.pi)) * s * s, atol=1e-13)
    assert np.abs(d["U_tp"]).max() < 1e-13
    assert np.allclose(0.5 * (d["U_tt"] + d["U_pp"]),
                       np.sqrt(5 / (16 * np.pi)) * (3 * z * z - 1), atol=1e-13)
    # gradient: psi = -Y20/3, d/dtheta
    assert np.allclose(d["g_t"], -(1 / 3) * np.sqrt(5 / (16 * np.pi)) * (-6 * z * s), atol=1e-13)
    a = np.zeros(sht.nalm(lmax), complex)
    a[sht.alm_index(lmax, 1, 0)] = 1.0
    d = sht.derivative_maps(N, lmax, sht.poisson(lmax, a))
    assert np.abs(d["U_tt"] - d["U_pp"]).max() < 1e-13
    assert np.abs(d["U_tp"]).max() < 1e-13


def test_E_mode_ratio_single_l():
    """For a single-l field: int |gamma|^2 / int kappa^2 = (l-1)(l+2)/(l(l+1))
    and the reconstructed convergence equals the input."""
    N, lmax, L = 32, 16, 6
    rng = np.random.default_rng(11)
    l, m = sht.lm_arrays(lmax)
    a = np.where(l == L, rng.normal(size=l.size) + 1j * rng.normal(size=l.size), 0)
    a[m == 0] = a[m == 0].real
    kap = sht.alm2map(N, lmax, a)
    d = sht.derivative_maps(N, lmax, sht.poisson(lmax, a))
    g1, g2 = 0.5 * (d["U_tt"] - d["U_pp"]), d["U_tp"]
    assert np.allclose(0.5 * (d["U_tt"] + d["U_pp"]), kap, atol=1e-12)
    ratio = np.sum(g1 ** 2 + g2 ** 2) / np.sum(kap ** 2)
    assert abs(ratio / ((L - 1) * (L + 2) / (L * (L + 1))) - 1) < 2e-3


def _epanechnikov(theta, sigma):
    """Closed forms of App. E for the Epanechnikov kernel at the pole, for
    the equation lap Psi = K - 1/(4 pi):  returns (K, dPsi/dtheta, gamma_1)."""
    sinc = lambda x: np.sinc(x)
    Nn = 2 * np.pi * (sinc(sigma / (2 * np.pi)) ** 2 - 2 * sinc(sigma / np.pi) + 1)
    c = np.cos(theta)
    K = np.where(theta < sigma, (1 - (theta / sigma) ** 2) / Nn, 0.0)
    h = ((theta / sigma) ** 2 * (-2 * sinc(theta / np.pi) + c + sinc(theta / 2 / np.pi) ** 2)
         + 1 - c) / (Nn * (1 - c)) - 1 / (4 * np.pi)
    inside = theta < sigma
    dpsi = np.where(inside, h * (1 - c) / np.sin(theta),
                    np.sin(theta) / (4 * np.pi * (1 - c)))
    g1 = np.where(inside, -0.5 * (2 * c / (1 + c) * h - K + 1 / (4 * np.pi)),
                  -(1 + c) / (8 * np.pi * (1 - c)))
    return K, dpsi, g1


def test_epanechnikov_normalisation():
    from scipy.integrate import quad
    for sigma in [0.05, 0.3, 1.0]:
        v, _ = quad(lambda t: 2 * np.pi * _epanechnikov(t, sigma)[0] * np.sin(t), 0, sigma)
        assert abs(v - 1) < 1e-12


@pytest.mark.parametrize("lmax,tol_g,tol_s", [(48, 1e-3, 0.02), (96, 2e-4, 0.006)])
def test_epanechnikov_pure_sht(lmax, tol_g, tol_s):
    """The pure-SHT solve of an Epanechnikov kernel at the pole matches the
    App. E deflection and shear, with an error that falls as lmax grows
    (the kernel has a kink at theta = sigma)."""
    sigma, N = 0.6, 64
    x, w = np.polynomial.legendre.leggauss(400)
    t = 0.5 * sigma * (x + 1)
    wt = 0.5 * sigma * w
    kstd = 0.5 * _epanechnikov(t, sigma)[0]          # standard convergence
    lam = sht.lambda_table(lmax, np.cos(t), np.sin(t))
    a = np.zeros(sht.nalm(lmax), complex)
    a[: lmax + 1] = 2 * np.pi * lam[: lmax + 1] @ (kstd * np.sin(t) * wt)
    d = sht.derivative_maps(N, lmax, sht.poisson(lmax, a))
    z, ph, s = hp.pix2ang_ring(N, np.arange(12 * N * N))
    th = np.arctan2(s, z)
    _, dpsi, g1 = _epanechnikov(th, sigma)
    sel = (th > 0.15) & (np.abs(th - sigma) > 0.15) & (th < 2.5)
    scale = np.abs(dpsi[sel]).max()
    assert np.abs(d["g_t"][sel] - dpsi[sel]).max() < tol_g * scale
    assert np.abs(d["g_p"]).max() < 1e-12
    g1m = 0.5 * (d["U_tt"] - d["U_pp"])
    assert np.abs(g1m[sel] - g1[sel]).max() < tol_s * np.abs(g1[sel]).max()


def test_derivative_maps_ring_subset():
    """derivative_maps on a subset of rings is the full computation at those
    rings' pixels (polar caps, belt edges, equator)."""
    N, lmax = 16, 40
    rng = np.random.default_rng(21)
    a = rng.standard_normal(sht.nalm(lmax)) + 1j * rng.standard_normal(sht.nalm(lmax))
    l, m = sht.lm_arrays(lmax)
    a[m == 0] = a[m == 0].real
    p = sht.poisson(lmax, a)
    full = sht.derivative_maps(N, lmax, p)
    rings = [0, 1, 14, 15, 16, 31, 47, 48, 61, 62]
    sub = sht.derivative_maps(N, lmax, p, rings=rings)
    pix = sht.ring_pixels(N, rings)
    assert pix.size == sum(min(r + 1, 4 * N - r - 1, N) * 4 for r in rings)
    for k in full:
        np.testing.assert_allclose(sub[k], full[k][pix], rtol=1e-13, atol=1e-13 * np.abs(full[k]).max())
