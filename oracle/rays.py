"""Multiple-plane ray propagation on the sphere for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Sec. 2.2 of the paper: the propagation direction is rotated at every lens
plane about n x alpha by |alpha| (eq. betaprop), the Cartesian position moves
along it to the next plane's comoving radius (eq. posprop), the lensing
Jacobian follows the three-term recurrence (eq. Atraj) and is parallel
transported along the great circle joining consecutive angular positions
(App. B).  App. C shows the recurrence equals the direct sum (eq. Atrajold);
App. D gives the radial interpolation of the Jacobian to a galaxy's distance
(eq. gatraj).  Distances: r(chi) of Sec. 2.1 and chi(a) for flat LCDM.

Readings:
* the deflection that turns the ray is d = -grad psi (the ray bends toward
  mass, matching the sign of eq. disclighttraj in the small-angle limit);
* the first plane lenses: beta^(-1) = n^(0), chi_{-1} = 0;
* the K < 0 branch of r(chi) is the standard sinh((-K)^{1/2} chi)/(-K)^{1/2};
* both indices of A are transported; U^(m) is evaluated at x^(m)/|x^(m)|;
* pure-SHT planes give their gradient and Hessian at the pixel centres of
  the ray grid; at a ray they are the four-point HEALPix interpolation of
  those values, each transported from its pixel centre to the ray (App. B),
  as the Jacobians at galaxy images are (Sec. 3.3).  The paper does not say
  how its pure-SHT solver reaches rays that have left the pixel centres.
"""
import numpy as np

from . import healpix as hp
from .mg import basis


def r_of_chi(chi, K=0.0):
    """Comoving angular-diameter distance (Sec. 2.1)."""
    chi = np.asarray(chi, dtype=np.float64)
    if K > 0:
        return np.sin(np.sqrt(K) * chi) / np.sqrt(K)
    if K < 0:
        return np.sinh(np.sqrt(-K) * chi) / np.sqrt(-K)
    return chi


def chi_of_z(z, omega_m=0.3, c_over_h0=2997.92458, nstep=20000):
    """chi(a) = c int_a^1 da' / (a'^2 H(a')), flat LCDM (Sec. 2.1), in
    h^-1 Mpc; composite Simpson rule in a."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty_like(z)
    for k, zz in enumerate(z):
        a0 = 1.0 / (1.0 + zz)
        a = np.linspace(a0, 1.0, 2 * nstep + 1)
        f = 1.0 / (a * a * np.sqrt(omega_m / a ** 3 + 1.0 - omega_m))
        h = (1.0 - a0) / (2 * nstep)
        out[k] = c_over_h0 * h / 3.0 * (f[0] + f[-1] + 4 * f[1:-1:2].sum()
                                         + 2 * f[2:-1:2].sum())
    return out


def rodrigues(k, w, v):
    """Rotate v by angle w counter-clockwise about unit axis k."""
    return (v * np.cos(w) + np.cross(k, v) * np.sin(w)
            + k * np.dot(k, v) * (1.0 - np.cos(w)))


def transport_matrix(n_old, n_new):
    """M_kl = e_k(n_new) . R e_l(n_old), with R the rotation carrying n_old to
    n_new about n_old x n_new (App. B)."""
    th0, ph0 = hp.vec2ang(n_old)
    th1, ph1 = hp.vec2ang(n_new)
    et0, ep0 = basis(np.cos(th0), ph0)
    et1, ep1 = basis(np.cos(th1), ph1)
    ax = np.cross(n_old, n_new)
    sn = np.linalg.norm(ax)
    if sn > 0:
        k = ax / sn
        w = np.arctan2(sn, np.dot(n_old, n_new))
        et0, ep0 = rodrigues(k, w, et0), rodrigues(k, w, ep0)
    return np.array([[et1 @ et0, et1 @ ep0], [ep1 @ et0, ep1 @ ep0]])


def plane_coeffs(chi, m, K=0.0):
    """c_m and d_m of eq. Atraj with chi_{-1} = 0:
    c_m = D_m / D_{m+1} * D_{m-1,m+1} / D_{m-1,m};  d_m = D_{m,m+1} / D_{m+1}.
    chi holds chi_0 .. chi_N (N planes plus the final target)."""
    cm1 = 0.0 if m == 0 else chi[m - 1]
    D = lambda a, b: float(r_of_chi(b - a, K))
    c = (D(0, chi[m]) / D(0, chi[m + 1])) * (D(cm1, chi[m + 1]) / D(cm1, chi[m]))
    d = D(chi[m], chi[m + 1]) / D(0, chi[m + 1])
    return c, d


class Ray:
    """One ray: angular position, direction, A^(m), A^(m-1)."""

    def __init__(self, theta, phi):
        self.n = hp.vec(np.cos(theta), phi)
        self.beta = self.n.copy()
        self.A = np.eye(2)
        self.A_prev = np.eye(2)


def ray_step(ray, chi, m, g, U, K=0.0):
    """Advance one ray from plane m to plane m+1 given the gradient g and the
    covariant Hessian U of psi^(m) at the ray (global theta/phi basis)."""
    th, ph = hp.vec2ang(ray.n)
    et, ep = basis(np.cos(th), ph)
    d = -(g[0] * et + g[1] * ep)                       # bend toward mass
    dn = np.linalg.norm(d)
    if dn > 0:
        k = np.cross(ray.n, d / dn)
        ray.beta = rodrigues(k / np.linalg.norm(k), dn, ray.beta)
    x = chi[m] * ray.n
    b = x @ ray.beta
    q = chi[m + 1] ** 2 - chi[m] ** 2
    lam = q / (b + np.sqrt(b * b + q))                 # root of eq. posprop
    x = x + lam * ray.beta
    n_new = x / np.linalg.norm(x)
    c, dd = plane_coeffs(chi, m, K)
    A_next = (1 - c) * ray.A_prev + c * ray.A - dd * U @ ray.A
    M = transport_matrix(ray.n, n_new)
    ray.A_prev = M @ ray.A @ M.T
    ray.A = M @ A_next @ M.T
    ray.n = n_new


def jacobian_direct_sum(chi, Us, K=0.0):
    """A_k = I - sum_{i<k} D_ik / D_k U_i A_i (eq. Atrajold), no transport."""
    As = [np.eye(2)]
    for k in range(1, len(Us) + 1):
        acc = np.eye(2)
        for i in range(k):
            acc = acc - (r_of_chi(chi[k] - chi[i], K) / r_of_chi(chi[k], K)) * Us[i] @ As[i]
        As.append(acc)
    return As


def jacobian_recurrence(chi, Us, K=0.0):
    """eq. Atraj with A^(0) = A^(-1) = I, chi_{-1} = 0, no transport."""
    A_prev, A = np.eye(2), np.eye(2)
    out = [A]
    for m in range(len(Us)):
        c, d = plane_coeffs(chi, m, K)
        A_prev, A = A, (1 - c) * A_prev + c * A - d * Us[m] @ A
        out.append(A)
    return out


def shell_edges(chi_planes):
    """Comoving edges of the lens-plane shells: 0, then midpoints between
    consecutive planes, then the midpoint toward the final target."""
    chi = np.asarray(chi_planes, dtype=np.float64)
    return np.concatenate([[0.0], 0.5 * (chi[:-1] + chi[1:])])


def galaxy_weight(chi, k, chi_g, K=0.0):
    """w of eq. gatraj for a galaxy in shell k: A_g = (1-w) A^(k-1) + w A^(k),
    w = D_k D_{k-1,g} / (D_g D_{k-1,k})."""
    D = lambda a, b: float(r_of_chi(b - a, K))
    return (D(0, chi[k]) * D(chi[k - 1], chi_g)) / (D(0, chi_g) * D(chi[k - 1], chi[k]))


def pixel_field_at(nside, g_ring, U_ring, n):
    """Gradient and covariant Hessian of a pure-SHT plane at unit vector n
    from their values at the RING pixel centres (g_ring [2][npix]: g_t, g_p;
    U_ring [3][npix]: U_tt, U_pp, U_tp): four-point HEALPix interpolation of
    the values transported from each pixel centre to n (App. B).  Returns
    (g [2], U [2][2]) in the basis at n."""
    th, ph = hp.vec2ang(n)
    pix, wt = hp.interp_weights(nside, np.array([th]), np.array([ph]))
    zc, pc, sc = hp.pix2ang_ring(nside, pix[:, 0])
    g = np.zeros(2)
    U = np.zeros((2, 2))
    for c in range(4):
        p = pix[c, 0]
        M = transport_matrix(hp.vec(zc[c], pc[c], sc[c]), n)
        gq = np.array([g_ring[0, p], g_ring[1, p]])
        Uq = np.array([[U_ring[0, p], U_ring[2, p]], [U_ring[2, p], U_ring[1, p]]])
        g += wt[c, 0] * (M @ gq)
        U += wt[c, 0] * (M @ Uq @ M.T)
    return g, U
