"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This module holds random draws and the input recipe only: no
part of the lens-plane solve or the ray propagation is computed here.

The paper measures on N-body light cones (Table 1) that are not available;
Gaussian and lognormal fields with C_l proportional to l^-2 stand in for the
lens-plane convergence.  The recipe:
* a_lm drawn in HEALPix order idx = m (2 lmax + 1 - m) / 2 + l from
  numpy.random.default_rng(seed): re = N(0,1)[n_lm], then im = N(0,1)[n_lm];
  a_l0 = sqrt(C_l) re, a_lm = sqrt(C_l / 2) (re + i im) for m > 0;
  C_l = A l^-2 for 2 <= l <= lmax, 0 below, with A fixing the pixel variance
  sigma^2 = sum_l (2l+1)/(4 pi) C_l;
* the map is the synthesis of these a_lm (done by the caller with its own
  transform), lognormal variant exp(g) - mean(exp(g));
* for multiplane runs each plane is scaled so that the Gaussian field's
  rms deflection is 1 arcmin (alpha_rms^2 = sum_l (2l+1)/(4 pi) 4 C_l /
  (l (l+1))), which keeps rays within a few arcmin of their bundle;
* positions uniform on the sphere: cos(theta) ~ U[-1, 1], phi ~ U[0, 2 pi).
"""
import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def lm_order(lmax):
    """(l, m) of every a_lm slot in HEALPix order."""
    ls, ms = [], []
    for m in range(lmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def cl_amplitude(lmax, sigma):
    """A such that C_l = A l^-2 (2 <= l <= lmax) has pixel variance sigma^2."""
    l = np.arange(2, lmax + 1, dtype=np.float64)
    return sigma ** 2 / np.sum((2 * l + 1) / (4 * np.pi * l * l))


def gaussian_alm(lmax, seed, sigma=None, amplitude=None):
    """Complex128 a_lm of a Gaussian field with C_l = A l^-2, l >= 2."""
    if amplitude is None:
        amplitude = 1.0 if sigma is None else cl_amplitude(lmax, sigma)
    l, m = lm_order(lmax)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(l.size)
    im = rng.standard_normal(l.size)
    cl = np.where(l >= 2, amplitude / np.maximum(l, 1.0) ** 2, 0.0)
    alm = np.where(m == 0, np.sqrt(cl) * re,
                   np.sqrt(cl / 2.0) * (re + 1j * im)).astype(np.complex128)
    return alm


def deflection_scale(lmax, sigma, alpha_rms=ARCMIN):
    """s_m that brings the Gaussian field's rms deflection to alpha_rms."""
    A = cl_amplitude(lmax, sigma)
    l = np.arange(2, lmax + 1, dtype=np.float64)
    a2 = np.sum((2 * l + 1) / (4 * np.pi) * 4.0 * A / l ** 2 / (l * (l + 1)))
    return alpha_rms / np.sqrt(a2)


def uniform_sphere(n, seed):
    """(theta, phi) uniform on the sphere."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.arccos(z), phi


def galaxy_redshifts(n, seed, zmin=0.3, zmax=1.5):
    """Galaxy positions and redshifts: uniform on the sphere, z ~ U[zmin, zmax]."""
    theta, phi = uniform_sphere(n, seed)
    rng = np.random.default_rng(seed + 1)
    return theta, phi, rng.uniform(zmin, zmax, n)


def multiplane_sigmas(nplanes=20, lo=0.1, hi=0.6):
    """Lognormal sigma_g per plane, growing linearly with plane index."""
    return lo + (hi - lo) * np.arange(nplanes) / max(nplanes - 1, 1)


def c4_nsides(nplanes=32, seed=4):
    """HEALPix resolution of each plane of the batched-precision workload:
    drawn uniformly from {512, 1024, 2048}."""
    rng = np.random.default_rng(seed)
    return [(512, 1024, 2048)[k] for k in rng.integers(0, 3, nplanes)]


def particle_cone(n, seed, nside, halo_fraction=0.5, halo_radius=2e-3):
    """Synthetic particles of one lens plane (the N-body light cones of the
    paper's Table 1 are not available): a uniform field population and
    clustered particles around halo centres, with Pareto-distributed (index
    1) halo occupations and Gaussian angular profiles of width halo_radius
    rad.  Equal weights summing to 4 pi x 0.05 (a mean convergence of 0.05);
    smoothing angles of 2-3 pixel sizes of nside (Sec. 3.2: a few
    inter-ray spacings).  Returns float64 theta, phi, weight, sigma [n]."""
    rng = np.random.default_rng(seed)
    nh = int(n * halo_fraction)
    nf = n - nh
    z = rng.uniform(-1.0, 1.0, nf)
    ph = rng.uniform(0.0, 2.0 * np.pi, nf)
    ncen = max(1, nh // 200)
    occ = rng.pareto(1.0, ncen) + 1.0
    host = rng.choice(ncen, nh, p=occ / occ.sum())
    cz = rng.uniform(-1.0, 1.0, ncen)
    cph = rng.uniform(0.0, 2.0 * np.pi, ncen)
    cs = np.sqrt((1.0 - cz) * (1.0 + cz))
    c = np.stack([cs * np.cos(cph), cs * np.sin(cph), cz], axis=1)[host]
    # a random tangent direction at the centre and a Rayleigh-distributed angle
    a = rng.standard_normal((nh, 3))
    a -= np.sum(a * c, axis=1)[:, None] * c
    a /= np.linalg.norm(a, axis=1)[:, None]
    r = halo_radius * np.sqrt(-2.0 * np.log(1.0 - rng.uniform(0.0, 1.0, nh)))
    v = np.cos(r)[:, None] * c + np.sin(r)[:, None] * a
    th = np.concatenate([np.arccos(z), np.arctan2(np.hypot(v[:, 0], v[:, 1]), v[:, 2])])
    phi = np.concatenate([ph, np.mod(np.arctan2(v[:, 1], v[:, 0]), 2.0 * np.pi)])
    w = np.full(n, 4.0 * np.pi * 0.05 / n)
    pix = np.sqrt(4.0 * np.pi / (12.0 * nside * nside))
    sigma = pix * rng.uniform(2.0, 3.0, n)
    return th, phi, w, sigma


def sky_order(theta, phi, ntheta):
    """Indices that order points by latitude-longitude tile (ntheta bands in
    theta, tiles of about equal width in each band, band after band): the
    input order of the deposition benchmarks, so that neighbouring threads
    handle neighbouring particles."""
    band = np.minimum((theta / np.pi * ntheta).astype(np.int64), ntheta - 1)
    width = np.maximum(1, np.round(2 * ntheta * np.sin((band + 0.5) * np.pi / ntheta)))
    tile = np.minimum((np.mod(phi, 2 * np.pi) / (2 * np.pi) * width).astype(np.int64),
                      width.astype(np.int64) - 1)
    return np.lexsort((tile, band))
