"""Full-sky convergence, shear E/B and rotation power spectra of a ray
state, for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Sec. 5 of the paper measures the angular power spectra of the convergence,
of the E- and B-modes of the shear and of the rotation, from HEALPix maps
of the final plane's inverse magnification matrices (eq. invmagmat), with a
full-sky E/B decomposition (no ambiguous modes on the whole sphere).

Readings (the paper names the HEALPix package, not its conventions):
* the maps sit on the ray grid: ray p, the NESTED pixel p of the image
  plane, gives the value at that pixel centre.  Its Jacobian is held in the
  basis at the ray's current position and is parallel transported to the
  pixel centre (App. B) first;
* from A = [[1 - kappa - gamma_1, -gamma_2 + omega],
            [-gamma_2 - omega, 1 - kappa + gamma_1]] (eq. invmagmat):
  kappa = 1 - (A11 + A22)/2, gamma_1 = (A22 - A11)/2,
  gamma_2 = -(A12 + A21)/2, omega = (A12 - A21)/2;
* E/B: the potential psi = Y_lm has the shear (half the trace-free part of
  the covariant Hessian of App. A) gamma_1 = X_lm(theta) e^{i m phi},
  gamma_2 = i Y_lm(theta) e^{i m phi} with (z = cos, s = sin theta,
  dlambda = d lambda_lm / d theta)
      X = (m^2/s^2 - l(l+1)/2) lambda - (z/s) dlambda,
      Y = (m/s) (dlambda - (z/s) lambda);
  the B basis field is that shear turned by 45 degrees (gamma -> i gamma).
  Both have squared norm N_l^2 / 4, N_l^2 = (l-1) l (l+1) (l+2), so
      E_lm = (2 / N_l) int [gamma_1 X_lm - i gamma_2 Y_lm] e^{-i m phi} dOmega,
      B_lm = (2 / N_l) int [gamma_2 X_lm + i gamma_1 Y_lm] e^{-i m phi} dOmega
  for l >= 2 (0 below), with the HEALPix quadrature weight 4 pi / N_pix.
  A pure-E field from psi then has E_lm = N_l psi_lm / 2, B = 0, and
  C_l^EE = (l-1)(l+2) / (l(l+1)) C_l^kappa;
* C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1).
"""
import numpy as np

from . import healpix as hp
from . import sht
from .rays import transport_matrix


def fields_from_rays(nside, theta, phi, A):
    """kappa, gamma_1, gamma_2, omega RING maps from a ray state in NESTED
    order (theta, phi [n], A [4][n] row-major 2 x 2 in the basis at the ray's
    position), each Jacobian transported to its pixel centre."""
    n = 12 * nside * nside
    ring = hp.nest2ring(nside, np.arange(n))
    zc, phc, sc = hp.pix2ang_ring(nside, ring)
    out = np.zeros((4, n))
    for p in range(n):
        n0 = hp.vec(np.cos(theta[p]), phi[p], np.sin(theta[p]))
        n1 = hp.vec(zc[p], phc[p], sc[p])
        M = transport_matrix(n0, n1)
        a = M @ np.array([[A[0, p], A[1, p]], [A[2, p], A[3, p]]]) @ M.T
        r = ring[p]
        out[0, r] = 1.0 - 0.5 * (a[0, 0] + a[1, 1])
        out[1, r] = 0.5 * (a[1, 1] - a[0, 0])
        out[2, r] = -0.5 * (a[0, 1] + a[1, 0])
        out[3, r] = 0.5 * (a[0, 1] - a[1, 0])
    return out


def spin2_map2alm(nside, lmax, g1, g2):
    """E_lm, B_lm (complex, a_lm order) of the RING shear maps g1, g2."""
    rt = hp.ring_table(nside)
    z, s = rt["z"], rt["sint"]
    F1 = sht.ring_forward(nside, lmax, g1)
    F2 = sht.ring_forward(nside, lmax, g2)
    w = 4.0 * np.pi / hp.npix(nside)
    E = np.zeros(sht.nalm(lmax), dtype=np.complex128)
    B = np.zeros(sht.nalm(lmax), dtype=np.complex128)
    prev = None
    for k, L in sht.lambda_diagonals(lmax, z, s):
        m = np.arange(lmax + 1 - k)
        l = (m + k).astype(np.float64)
        mf = m.astype(np.float64)
        lm1 = np.zeros_like(L) if k == 0 else prev[: m.size]
        c = np.sqrt(np.maximum((2 * l + 1) * (l * l - mf * mf), 0.0) /
                    np.maximum(2 * l - 1, 1.0))
        dlam = (l[:, None] * z[None, :] * L - c[:, None] * lm1) / s[None, :]
        X = (((mf * mf)[:, None] / (s * s)[None, :] - (0.5 * l * (l + 1))[:, None]) * L
             - (z / s)[None, :] * dlam)
        Y = (mf[:, None] / s[None, :]) * (dlam - (z / s)[None, :] * L)
        f1, f2 = F1[:, m].T, F2[:, m].T                   # [m, ring]
        nl = np.sqrt(np.maximum((l - 1) * l * (l + 1) * (l + 2), 0.0))
        norm = np.where(l >= 2, 2.0 / np.where(nl > 0, nl, 1.0), 0.0) * w
        idx = sht.alm_index(lmax, m + k, m)
        E[idx] = norm * np.sum(X * f1 - 1j * Y * f2, axis=1)
        B[idx] = norm * np.sum(X * f2 + 1j * Y * f1, axis=1)
        prev = L
    return E, B


def spectrum(lmax, alm):
    """C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1), l = 0..lmax."""
    l, m = sht.lm_arrays(lmax)
    p = np.abs(alm) ** 2 * np.where(m > 0, 2.0, 1.0)
    return np.bincount(l, weights=p, minlength=lmax + 1) / (2.0 * np.arange(lmax + 1) + 1.0)


def jacobian_spectra(nside, lmax, theta, phi, A):
    """Harmonic coefficients and spectra of kappa, E, B and omega of a ray
    state: dict with 'alm' [4][n_lm] complex and 'cl' [4][lmax+1] in the
    order kappa, E, B, omega."""
    f = fields_from_rays(nside, theta, phi, A)
    ak = sht.map2alm(nside, lmax, f[0])
    E, B = spin2_map2alm(nside, lmax, f[1], f[2])
    aw = sht.map2alm(nside, lmax, f[3])
    alm = np.stack([ak, E, B, aw])
    return dict(fields=f, alm=alm, cl=np.stack([spectrum(lmax, a) for a in alm]))
