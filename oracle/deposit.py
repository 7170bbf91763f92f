"""Epanechnikov deposition of particles onto a HEALPix map, for the FP64
CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Sec. 3.2 of the paper smooths the mass of every N-body particle of a lens
plane with the Epanechnikov kernel normalised on the sphere,
    K(theta; sigma) = [1 - (theta / sigma)^2] / N(sigma)   for theta < sigma,
    N(sigma) = 2 pi (sinc^2(sigma / 2 pi) - 2 sinc(sigma / pi) + 1),
    sinc(x) = sin(pi x) / (pi x),
bins the kernel over the HEALPix map and enforces exact mass conservation.

Readings (the paper does not spell out the binning):
* a particle's weight on pixel p is K at the angle between the particle
  and the pixel centre, over all pixel centres closer than sigma, divided
  by the sum of those values: every particle's weights add up to one;
* a particle whose sigma reaches no pixel centre puts all its mass in the
  pixel that contains it;
* the map holds mass per unit area: kappa(p) = sum_i w_i W_i(p) / Omega_pix,
  Omega_pix = 4 pi / N_pix, with w_i in convergence times steradian, so
  sum_p kappa(p) Omega_pix = sum_i w_i exactly (up to rounding);
* angles are taken as atan2(|a x b|, a . b), accurate at any separation.
"""
import numpy as np

from . import healpix as hp


def kernel(theta, sigma):
    """K(theta; sigma), the normalised Epanechnikov kernel (0 beyond sigma)."""
    sinc = np.sinc                                   # sin(pi x) / (pi x)
    nrm = 2 * np.pi * (sinc(sigma / (2 * np.pi)) ** 2 - 2 * sinc(sigma / np.pi) + 1)
    return np.where(theta < sigma, (1 - (theta / sigma) ** 2) / nrm, 0.0)


def _deposit_one(nside, out, cand, V, t, p, w, sg):
    """One particle's weight onto out (mass per pixel) over the candidate
    pixel centres cand (unit vectors V), which hold every centre within
    sigma."""
    n = hp.vec(np.cos(t), p, np.sin(t))
    ang = np.arctan2(np.linalg.norm(np.cross(V, n), axis=1), V @ n)
    sel = np.nonzero(ang < sg)[0]
    k = kernel(ang[sel], sg)
    if sel.size == 0 or k.sum() == 0.0:
        own = hp.nest2ring(nside, hp.ang2pix_nest(nside, np.cos(t), p))
        out[own] += w
    else:
        out[cand[sel]] += w * k / k.sum()


def deposit(nside, theta, phi, weight, sigma, pixels=None):
    """RING map of the particles' kappa (mass per steradian).  `pixels`
    (RING indices) limits the pixel centres tried, for large grids: it must
    hold every pixel centre within sigma of every particle."""
    npix = hp.npix(nside)
    cand = np.arange(npix) if pixels is None else np.asarray(pixels)
    z, ph, s = hp.pix2ang_ring(nside, cand)
    V = hp.vec(z, ph, s)
    out = np.zeros(npix)
    for t, p, w, sg in zip(theta, phi, weight, sigma):
        _deposit_one(nside, out, cand, V, t, p, w, sg)
    return out / (4 * np.pi / npix)


def local_pixels(nside, theta, phi, radius, rt=None):
    """RING indices of a superset of the pixel centres within radius of
    (theta, phi): the rings whose colatitude is within radius of theta and,
    in each, the pixels within the azimuth range that the haversine allows,
    sin^2(dphi / 2) <= sin^2(radius / 2) / (sin theta sin theta_ring), widened
    by two pixels (all of a ring when that range reaches around it)."""
    rt = hp.ring_table(nside) if rt is None else rt
    th_r = np.arccos(np.clip(rt["z"], -1.0, 1.0))
    out = []
    for r in np.nonzero(np.abs(th_r - theta) <= radius)[0]:
        nr, first = int(rt["n"][r]), int(rt["first"][r])
        ss = np.sin(theta) * np.sin(th_r[r])
        q = np.sin(0.5 * radius) ** 2 / ss if ss > 0 else np.inf
        half = 2.0 * np.arcsin(np.sqrt(q)) if q < 1.0 else np.inf
        if half >= np.pi:
            out.append(first + np.arange(nr))
            continue
        step = 2 * np.pi / nr
        j0 = int(np.floor((phi - half - rt["phi0"][r]) / step)) - 2
        j1 = int(np.ceil((phi + half - rt["phi0"][r]) / step)) + 2
        if j1 - j0 + 1 >= nr:
            out.append(first + np.arange(nr))
        else:
            out.append(first + np.mod(np.arange(j0, j1 + 1), nr))
    return np.unique(np.concatenate(out)) if out else np.zeros(0, dtype=np.int64)


def deposit_sparse(nside, theta, phi, weight, sigma):
    """deposit() for large grids with few particles: the same arithmetic,
    each particle over its local pixels (local_pixels within sigma plus two
    pixel sizes, which hold every centre within sigma)."""
    npix = hp.npix(nside)
    rt = hp.ring_table(nside)
    pix = np.sqrt(4 * np.pi / npix)
    out = np.zeros(npix)
    for t, p, w, sg in zip(theta, phi, weight, sigma):
        cand = local_pixels(nside, t, p, sg + 2 * pix, rt)
        z, ph, s = hp.pix2ang_ring(nside, cand)
        _deposit_one(nside, out, cand, hp.vec(z, ph, s), t, p, w, sg)
    return out / (4 * np.pi / npix)
