"""Pins of the oracle's galaxy-image grid search (Sec. 2.3, Sec. 3.3,
App. D) to geometry and to closed forms:
* the triangles over the HEALPix pixel centres tile the sphere: all of
  positive orientation, 2 N_pix - 4 of them (Euler), total area 4 pi;
* every direction lies in exactly one triangle;
* without lensing the grid search returns each source as its own image;
* a smoothed point mass (the Epanechnikov kernel of App. E) on one lens
  plane: the source reconstructed from the found image by the exact lens
  mapping is within 0.2 arcsec of the true source (the bound of the paper's
  weak-lensing image test);
* the radial propagation to the galaxy distance and the Jacobian step."""
import numpy as np
import pytest

from oracle import healpix as hp
from oracle import images as im
from oracle import rays as orays
from oracle.mg import basis

ARCSEC = np.pi / 180 / 3600


def _ang(a, b):
    """Angle between unit vectors, accurate for small angles."""
    return np.arctan2(np.linalg.norm(np.cross(a, b)), np.dot(a, b))


@pytest.mark.parametrize("N", [1, 2, 4, 8, 32])
def test_triangles_tile_the_sphere(N):
    t = im.all_triangles(N)
    assert len(t) == 2 * 12 * N * N - 4
    v = im.pixel_vectors(N, t.ravel()).reshape(-1, 3, 3)
    a = im.spherical_area(v[:, 0], v[:, 1], v[:, 2])
    assert a.min() > 0
    assert abs(a.sum() - 4 * np.pi) < 1e-11
    # every edge is shared by exactly two triangles, in opposite directions
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    fwd = {tuple(x) for x in e}
    assert len(fwd) == len(e)
    assert all((b, a_) in fwd for a_, b in fwd)


def _contains(v, g):
    """g inside the spherical triangle v (3 x 3 rows, counter-clockwise)."""
    return all(np.dot(np.cross(v[i], v[(i + 1) % 3]), g) >= 0 for i in range(3))


def test_every_direction_in_one_triangle():
    N = 4
    t = im.all_triangles(N)
    v = im.pixel_vectors(N, t.ravel()).reshape(-1, 3, 3)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((300, 3))
    g /= np.linalg.norm(g, axis=1)[:, None]
    for x in g:
        hits = sum(_contains(v[k], x) for k in range(len(t)))
        assert hits == 1


def test_ring_predecessor_integer_rule():
    """The merge apex: the last vertex of the other ring strictly before in
    azimuth, against a direct float comparison."""
    N = 16
    for q in range(0, 4 * N - 2, 7):
        fa, na, sa = im.ring_info(N, q)
        fb, nb, sb = im.ring_info(N, q + 1)
        pa = 2 * np.pi * (np.arange(na) + sa / 2) / na
        pb = 2 * np.pi * (np.arange(nb) + sb / 2) / nb
        for j in range(na):
            k = int(im._pred(j, na, sa, nb, sb))
            before = np.nonzero(pb < pa[j])[0]
            assert k == (before.max() if before.size else nb - 1)


@pytest.mark.parametrize("N", [8, 64])
def test_no_lensing_images_are_sources(N):
    rng = np.random.default_rng(11)
    g = rng.standard_normal((40, 3))
    g /= np.linalg.norm(g, axis=1)[:, None]
    src_of = lambda pix: im.pixel_vectors(N, pix)
    for x in g:
        img, tri, b = im.find_image(N, x, src_of, 2.0 / N)
        assert np.all(b >= 0) and abs(b.sum() - 1) < 1e-14
        assert _ang(img, x) < 1e-14


def test_propagate_least_root():
    n = np.array([0.0, 0.0, 1.0])
    beta = np.array([0.6, 0.0, 0.8])
    out = im.propagate(n, beta, 100.0, 120.0)
    x = 100.0 * n
    lam = -x @ beta + np.sqrt((x @ beta) ** 2 + 120.0 ** 2 - 100.0 ** 2)
    y = x + lam * beta
    assert np.allclose(out, y / np.linalg.norm(y), atol=1e-15)
    # backward (galaxy in front of the plane's radius): lambda < 0
    back = im.propagate(n, beta, 100.0, 90.0)
    lam = -x @ beta + np.sqrt((x @ beta) ** 2 + 90.0 ** 2 - 100.0 ** 2)
    y = x + lam * beta
    assert lam < 0 and np.allclose(back, y / np.linalg.norm(y), atol=1e-15)


def _epan_dpsi(theta, sigma):
    """dPsi/dtheta of App. E for the Epanechnikov kernel at the pole (unit
    mass, lap Psi = K - 1/(4 pi))."""
    sinc = np.sinc
    Nn = 2 * np.pi * (sinc(sigma / (2 * np.pi)) ** 2 - 2 * sinc(sigma / np.pi) + 1)
    c = np.cos(theta)
    h = ((theta / sigma) ** 2 * (-2 * sinc(theta / np.pi) + c + sinc(theta / 2 / np.pi) ** 2)
         + 1 - c) / (Nn * (1 - c)) - 1 / (4 * np.pi)
    return np.where(theta < sigma, h * (1 - c) / np.sin(theta),
                    np.sin(theta) / (4 * np.pi * (1 - c)))


def test_smoothed_point_mass_images():
    """One lens plane holding an Epanechnikov-smoothed point mass (smoothing
    length 13.74 arcmin, peak deflection about 0.5 arcmin, weak lensing);
    rays on an Nside 2048 grid.  For random sources near the lens the grid
    search finds an image whose exact lens mapping lands within 0.2 arcsec
    of the source."""
    N = 2048
    sigma = 13.74 / 60 * np.pi / 180
    L = hp.vec(np.cos(1.1), 2.0)                       # lens direction
    chi = np.array([1000.0, 2000.0])                   # plane, source radius
    tt = np.linspace(1e-4, 3 * sigma, 2000)
    amp = (0.5 / 60 * np.pi / 180) / np.abs(_epan_dpsi(tt, sigma)).max()

    def source_of(n):
        """The exact single-plane mapping of an image direction: deflect
        toward the lens at the plane (d = -grad psi), move to the source
        radius."""
        r = orays.Ray(*hp.vec2ang(n))
        ct = np.clip(n @ L, -1, 1)
        th = np.arccos(ct)
        e = n * ct - L                                 # away from the lens
        e = e / np.linalg.norm(e)
        tn, pn = hp.vec2ang(n)
        et, ep = basis(np.cos(tn), pn)
        d = amp * _epan_dpsi(th, sigma)
        g = np.array([d * (e @ et), d * (e @ ep)])
        orays.ray_step(r, chi, 0, g, np.zeros((2, 2)))
        return r.n

    src_of = lambda pix: np.array([source_of(v) for v in im.pixel_vectors(N, pix)])
    rng = np.random.default_rng(21)
    worst = 0.0
    for _ in range(12):
        # a source within 1.5 smoothing lengths of the lens
        off = rng.uniform(0.05, 1.5) * sigma
        ax = np.cross(L, [0.0, 0.0, 1.0])
        ax /= np.linalg.norm(ax)
        ax = orays.rodrigues(L, rng.uniform(0, 2 * np.pi), ax)
        gsrc = orays.rodrigues(ax, off, L)
        img, tri, b = im.find_image(N, gsrc, src_of, 2.0 / 60 * np.pi / 180)
        err = _ang(source_of(img), gsrc)
        worst = max(worst, err)
        # the image moved away from the lens relative to the source
        assert _ang(img, L) > _ang(gsrc, L)
    print("worst reconstructed-source error %.3g arcsec" % (worst / ARCSEC))
    assert worst < 0.2 * ARCSEC


def test_image_jacobian_uniform_rays():
    """Rays with one Jacobian pair everywhere and no deflection: eq. gatraj
    exactly, the transport between coincident positions being the identity."""
    N = 16
    A = np.array([[0.9, 0.05], [0.02, 1.1]])
    Ap = np.array([[0.95, 0.01], [0.0, 1.02]])
    rng = np.random.default_rng(5)
    for _ in range(5):
        g = rng.standard_normal(3)
        g /= np.linalg.norm(g)
        out = im.image_jacobian(N, g, lambda p: A, lambda p: Ap, lambda p: g, 0.3)
        assert np.allclose(out, 0.7 * Ap + 0.3 * A, atol=1e-14)
