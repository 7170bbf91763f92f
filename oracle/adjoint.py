"""Transpose (adjoint) of the kappa -> shear map of the SHT+MG solve, for the
FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

With the patch geometry, the readings and the number of V-cycles fixed, the
map from the fine convergence map to the gradient and covariant Hessian of
psi at a set of points is linear (the SHT boundary data are themselves
linear in kappa), so a least-squares loss such as the shear chi^2 has the
gradient F^T [dL/d(grad, hess)].  F^T is assembled here from the transposes
of the steps of `oracle.mg` and `oracle.sht`, applied in reverse order:
demean, degrade, ring transforms with the Legendre sums (analysis and
synthesis), the harmonic Poisson factor, HEALPix linear interpolation, the
ghost construction, the finite-volume operator, the red-black half sweeps,
restriction, prolongation, the coarsest solve, the finite differences and
the covariant terms of App. A with the rotation to the global basis.

Conventions.  Harmonic coefficients are real vectors of (Re, Im) pairs in
HEALPix order; the imaginary part of m = 0 is not an input of synthesis.
The correction du is carried as its interior (the ghosts are the reflected
interior, Sec. 3.2 face condition).  The patch potential u0 carries its
ghost ring.  Hessian adjoints come as (U_tt, U_pp, U_tp) with U_tp standing
for both off-diagonal entries.
"""
import numpy as np

from . import healpix as hp
from . import mg
from . import sht


# --------------------------------------------------------------------------
# SHT steps
# --------------------------------------------------------------------------
def _cm(lmax):
    _, m = sht.lm_arrays(lmax)
    return m


def alm2map_T(nside, lmax, ybar):
    """Transpose of synthesis: abar_lm = c_m sum_p lambda_lm e^{-i m phi_p}
    ybar_p (unweighted analysis, c_0 = 1, c_m = 2), Im of m = 0 zero."""
    w = 4.0 * np.pi / hp.npix(nside)
    a = sht.map2alm(nside, lmax, ybar) / w
    m = _cm(lmax)
    a = np.where(m == 0, a.real + 0j, 2.0 * a)
    return a


def map2alm_T(nside, lmax, abar):
    """Transpose of the (uniform-weight) analysis a = w sum lambda e^{-im phi}:
    ybar_p = w Re sum_lm abar_lm lambda_lm e^{i m phi_p} over m >= 0, i.e. the
    synthesis of abar with the m >= 1 terms halved (synthesis doubles them)."""
    w = 4.0 * np.pi / hp.npix(nside)
    m = _cm(lmax)
    b = np.where(m == 0, abar.real + 0j, 0.5 * abar)
    return w * sht.alm2map(nside, lmax, b)


def interp_T(nside, theta, phi, vals):
    """Transpose of HEALPix linear interpolation: scatter vals with the
    bilinear weights onto the RING map."""
    pix, w = hp.interp_weights(nside, theta, phi)
    out = np.zeros(hp.npix(nside))
    np.add.at(out, pix.ravel(), (w * np.asarray(vals)[None, :]).ravel())
    return out


def degrade_T(nside_f, nside_s, ybar_ring_s):
    """Transpose of (demeaned fine RING map) -> (RING map at nside_s, mean of
    the NESTED children): each fine pixel gets its parent's value / k."""
    k = (nside_f // nside_s) ** 2
    ybar_nest_s = ybar_ring_s[hp.nest2ring(nside_s, np.arange(hp.npix(nside_s)))]
    fine_nest = np.repeat(ybar_nest_s, k) / k
    out = np.empty(hp.npix(nside_f))
    out[hp.nest2ring(nside_f, np.arange(hp.npix(nside_f)))] = fine_nest
    return out


def demean_T(xbar):
    """Transpose of x -> x - mean(x) (a symmetric projection)."""
    return xbar - np.mean(xbar)


# --------------------------------------------------------------------------
# multigrid steps (interior representation of du)
# --------------------------------------------------------------------------
def full_diag(c):
    n = c["n"]
    sm, sp, sc = c["s_m"][:, None], c["s_p"][:, None], c["s_c"][:, None]
    D = (sm + sp + 2.0 / sc) * np.ones((n, n))
    D[0, :] += c["s_m"][0]
    D[-1, :] += c["s_p"][-1]
    D[:, 0] += 1.0 / c["s_c"]
    D[:, -1] += 1.0 / c["s_c"]
    return D


def L0(x, c):
    """The finite-volume operator on a correction field given by its
    interior (ghost = -interior)."""
    n = c["n"]
    u = np.zeros((n + 2, n + 2))
    u[1:-1, 1:-1] = x
    return mg.apply_L0(u, c)


def L0_T(y, c):
    """Transpose of L0: the row scaling 1/A, then each link scattered back."""
    n = c["n"]
    ya = y / c["area"][:, None]
    sm, sp, sc = c["s_m"][:, None], c["s_p"][:, None], c["s_c"][:, None]
    out = -full_diag(c) * ya
    out[:-1, :] += (sm * ya)[1:, :]           # cell i uses u_{i-1} with s_m(i)
    out[1:, :] += (sp * ya)[:-1, :]           # cell i uses u_{i+1} with s_p(i)
    out[:, :-1] += (ya / sc)[:, 1:]
    out[:, 1:] += (ya / sc)[:, :-1]
    return out


def half_sweep_T(ubar, c, color):
    """Transpose of one red-black half sweep u' = H_c(u, f): returns
    (ubar before the sweep, fbar contribution)."""
    n = c["n"]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = ((ii + jj) % 2) == color
    t = np.where(mask, ubar / full_diag(c), 0.0)
    fbar = -c["area"][:, None] * t
    out = np.where(mask, 0.0, ubar)
    sm, sp, sc = c["s_m"][:, None], c["s_p"][:, None], c["s_c"][:, None]
    out[:-1, :] += (sm * t)[1:, :]
    out[1:, :] += (sp * t)[:-1, :]
    out[:, :-1] += (t / sc)[:, 1:]
    out[:, 1:] += (t / sc)[:, :-1]
    return out, fbar


def smooth_T(ubar, c, sweeps):
    fbar = np.zeros_like(ubar)
    for _ in range(sweeps):
        for color in (1, 0):
            ubar, fb = half_sweep_T(ubar, c, color)
            fbar += fb
    return ubar, fbar


def restrict_T(ybar, c_fine):
    A = c_fine["area"]
    a0 = A[0::2][:, None]
    a1 = A[1::2][:, None]
    den = 2.0 * (a0 + a1)
    n = A.size
    out = np.empty((n, n))
    out[0::2, 0::2] = out[0::2, 1::2] = a0 / den * ybar
    out[1::2, 0::2] = out[1::2, 1::2] = a1 / den * ybar
    return out


def prolong_T(xbar, nH):
    """Transpose of mg.prolong (bilinear 9/3/3/1 with injection on the
    outermost fine ring) from a fine field to the coarse nH x nH level."""
    n = xbar.shape[0]
    eg = np.zeros((nH + 2, nH + 2))
    i = np.arange(n)
    I = i // 2
    di = np.where(i % 2 == 0, -1, 1)
    II, JJ = np.meshgrid(I, I, indexing="ij")
    DI, DJ = np.meshgrid(di, di, indexing="ij")
    edge = np.zeros((n, n), dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    inner = ~edge
    x = xbar[inner]
    np.add.at(eg, (II[inner] + 1, JJ[inner] + 1), 9.0 / 16.0 * x)
    np.add.at(eg, (II[inner] + 1 + DI[inner], JJ[inner] + 1), 3.0 / 16.0 * x)
    np.add.at(eg, (II[inner] + 1, JJ[inner] + 1 + DJ[inner]), 3.0 / 16.0 * x)
    np.add.at(eg, (II[inner] + 1 + DI[inner], JJ[inner] + 1 + DJ[inner]), 1.0 / 16.0 * x)
    np.add.at(eg, (II[edge] + 1, JJ[edge] + 1), xbar[edge])
    return eg[1:-1, 1:-1]


def coarsest_T(ubar, c):
    n = c["n"]
    M = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros((n, n))
        e.flat[k] = 1.0
        M[:, k] = L0(e, c).ravel()
    return np.linalg.solve(M.T, ubar.ravel()).reshape(n, n)


def vcycle_T(spec, ubar_out, level, coeffs):
    """Transpose of one FAS V-cycle (u_in, f) -> u_out on interior fields:
    returns (ubar_in, fbar)."""
    c = coeffs[level]
    if c["n"] <= 4:
        return np.zeros_like(ubar_out), coarsest_T(ubar_out, c)
    ub, fbar = smooth_T(ubar_out, c, spec.nu2)
    cH = coeffs[level + 1]
    e = prolong_T(ub, cH["n"])
    uHbar_in, fHbar = vcycle_T(spec, e, level + 1, coeffs)
    ubarbar = -e + uHbar_in + L0_T(fHbar, cH)
    rbarbar = fHbar
    ub = ub + restrict_T(ubarbar, c)
    rf = restrict_T(rbarbar, c)
    fbar = fbar + rf
    ub = ub - L0_T(rf, c)
    ub_in, fb = smooth_T(ub, c, spec.nu1)
    return ub_in, fbar + fb


def mg_solve_T(spec, dubar, vcycles=None):
    """Transpose of du = mg_solve(spec, f') on interiors: f'bar."""
    coeffs = mg.all_coeffs(spec)
    fbar = np.zeros_like(dubar)
    ub = dubar.copy()
    for _ in range(spec.vcycles if vcycles is None else vcycles):
        ub, fb = vcycle_T(spec, ub, 0, coeffs)
        fbar += fb
    return fbar


def ghosts_T(ufull):
    """Transpose of interior -> reflected ghost ring: every ghost adds minus
    its value to the interior cell it reflects (corners: the diagonal)."""
    g = ufull.copy()
    x = g[1:-1, 1:-1].copy()
    x[0, :] -= g[0, 1:-1]
    x[-1, :] -= g[-1, 1:-1]
    x[:, 0] -= g[1:-1, 0]
    x[:, -1] -= g[1:-1, -1]
    x[0, 0] -= g[0, 0]
    x[0, -1] -= g[0, -1]
    x[-1, 0] -= g[-1, 0]
    x[-1, -1] -= g[-1, -1]
    return x


def apply_L_T(y, c):
    """Transpose of mg.apply_L (interior values of a field with a stored
    ghost ring): returns the (n+2)^2 field."""
    n = c["n"]
    ya = y / c["area"][:, None]
    sm, sp, sc = c["s_m"][:, None], c["s_p"][:, None], c["s_c"][:, None]
    out = np.zeros((n + 2, n + 2))
    out[1:-1, 1:-1] -= (sm + sp + 2.0 / sc) * ya
    out[:-2, 1:-1] += sm * ya
    out[2:, 1:-1] += sp * ya
    out[1:-1, :-2] += ya / sc
    out[1:-1, 2:] += ya / sc
    return out


def patch_setup_T(spec, b, u0bar, fpbar):
    """Transpose of patch_setup in (kappa - mean, psi_SHT): returns
    (kappa'bar on the fine RING map, psi_SHT bar on the SHT RING map)."""
    n, L = spec.n, spec.L
    R = mg.patch_rotation(spec.nb, b)
    c = mg.level_coeffs(spec, n)
    ub = u0bar.copy() - apply_L_T(fpbar, c)     # f' = f - L u0
    fbar = fpbar                                # f' = f - ...
    th, ph = mg.patch_cell_dirs(spec, R)
    kbar = interp_T(spec.nf, th.ravel(), ph.ravel(), 2.0 * fbar.ravel())
    # ghosts: u0_g = 2 b - u0_adj
    tc, pc = mg.patch_angles(spec, n, ghosts=0)
    lo_t, hi_t = np.pi / 2 - L / 2, np.pi / 2 + L / 2
    lo_p, hi_p = -L / 2, L / 2
    psibar = np.zeros(hp.npix(spec.ns))
    faces = [((lo_t, pc), (0, slice(1, -1)), (1, slice(1, -1))),
             ((hi_t, pc), (-1, slice(1, -1)), (-2, slice(1, -1))),
             ((tc, lo_p), (slice(1, -1), 0), (slice(1, -1), 1)),
             ((tc, hi_p), (slice(1, -1), -1), (slice(1, -1), -2))]
    for (tt, pp), gidx, aidx in faces:
        g = ub[gidx].copy()
        ub[aidx] -= g
        t, p = mg.patch_dirs(spec, R, tt, pp)
        psibar += interp_T(spec.ns, np.ravel(t), np.ravel(p), 2.0 * np.ravel(g))
    corners = [((lo_t, lo_p), (0, 0), (1, 1)), ((lo_t, hi_p), (0, -1), (1, -2)),
               ((hi_t, lo_p), (-1, 0), (-2, 1)), ((hi_t, hi_p), (-1, -1), (-2, -2))]
    for (tt, pp), gidx, aidx in corners:
        g = ub[gidx]
        ub[aidx] -= g
        t, p = mg.patch_dirs(spec, R, np.array([tt]), np.array([pp]))
        psibar += interp_T(spec.ns, np.ravel(t), np.ravel(p), np.array([2.0 * g]))
    psibar += interp_T(spec.ns, th.ravel(), ph.ravel(), ub[1:-1, 1:-1].ravel())
    return kbar, psibar


# --------------------------------------------------------------------------
# evaluation at points
# --------------------------------------------------------------------------
def eval_point_T(spec, R, theta, phi, gbar, hbar):
    """Transpose of mg.eval_point in psi = u0 + du: returns the (n+2)^2 field
    bar (ghosts included).  gbar = (g_t, g_p) bar, hbar = (U_tt, U_pp, U_tp)
    bar."""
    v = hp.vec(np.cos(theta), phi)
    vp = R @ v
    thp, php = hp.vec2ang(vp)
    php = php - 2 * np.pi if php > np.pi else php
    n, d = spec.n, spec.delta
    fi = (thp - (np.pi / 2 - spec.L / 2)) / d - 0.5
    fj = (php + spec.L / 2) / d - 0.5
    i0, j0 = int(np.floor(fi)), int(np.floor(fj))
    if not (0 <= i0 <= n - 2 and 0 <= j0 <= n - 2):
        raise ValueError("point outside its patch")
    t, s = fi - i0, fj - j0
    etp, epp = mg.basis(np.cos(thp), php)
    etp, epp = R.T @ etp, R.T @ epp
    et, ep = mg.basis(np.cos(theta), phi)
    Q = np.array([[et @ etp, et @ epp], [ep @ etp, ep @ epp]])
    Ub = np.array([[hbar[0], 0.5 * hbar[2]], [0.5 * hbar[2], hbar[1]]])
    gpb = Q.T @ np.asarray(gbar, float)
    Upb = Q.T @ Ub @ Q
    st, ct = np.sin(thp), np.cos(thp)
    off = Upb[0, 1] + Upb[1, 0]
    pb = np.zeros(5)
    pb[0] = gpb[0] + (ct / st) * Upb[1, 1]
    pb[1] = gpb[1] / st - ct / st ** 2 * off
    pb[2] = Upb[0, 0]
    pb[3] = Upb[1, 1] / st ** 2
    pb[4] = off / st
    out = np.zeros((n + 2, n + 2))
    for (ii, jj), w in (((i0, j0), (1 - t) * (1 - s)), ((i0, j0 + 1), (1 - t) * s),
                        ((i0 + 1, j0), t * (1 - s)), ((i0 + 1, j0 + 1), t * s)):
        _raw_partials_T(out, d, ii, jj, w * pb)
    return out


def _raw_partials_T(out, delta, i, j, pbar):
    n = out.shape[0] - 2
    o1i, w1i = mg.stencil(i, n, 1)
    o2i, w2i = mg.stencil(i, n, 2)
    o1j, w1j = mg.stencil(j, n, 1)
    o2j, w2j = mg.stencil(j, n, 2)
    for o, w in zip(o1i, w1i):
        out[i + o + 1, j + 1] += w * pbar[0] / delta
    for o, w in zip(o1j, w1j):
        out[i + 1, j + o + 1] += w * pbar[1] / delta
    for o, w in zip(o2i, w2i):
        out[i + o + 1, j + 1] += w * pbar[2] / delta ** 2
    for o, w in zip(o2j, w2j):
        out[i + 1, j + o + 1] += w * pbar[3] / delta ** 2
    for oa, wa in zip(o1i, w1i):
        for ob, wb in zip(o1j, w1j):
            out[i + oa + 1, j + ob + 1] += wa * wb * pbar[4] / delta ** 2


# --------------------------------------------------------------------------
# the whole map and the shear chi^2 of the C5 workload
# --------------------------------------------------------------------------
def forward(spec, kappa, theta, phi):
    """(grad [2, npts], hess [3, npts]: U_tt, U_pp, U_tp) of the SHT+MG
    solution at the points."""
    bund = hp.ang2pix_nest(spec.nb, np.cos(theta), phi)
    sol = mg.solve_plane(spec, kappa, np.unique(bund))
    g = np.zeros((2, theta.size))
    h = np.zeros((3, theta.size))
    for k in range(theta.size):
        gg, U = mg.eval_point(spec, sol["patches"][int(bund[k])], theta[k], phi[k])
        g[:, k] = gg
        h[:, k] = (U[0, 0], U[1, 1], U[0, 1])
    return g, h


def adjoint(spec, theta, phi, gbar, hbar):
    """F^T (gbar, hbar): the fine-map gradient of sum(gbar * grad + hbar *
    hess)."""
    bund = hp.ang2pix_nest(spec.nb, np.cos(theta), phi)
    kbar = np.zeros(hp.npix(spec.nf))
    psibar = np.zeros(hp.npix(spec.ns))
    for b in np.unique(bund):
        R = mg.patch_rotation(spec.nb, b)
        ub = np.zeros((spec.n + 2, spec.n + 2))
        for k in np.nonzero(bund == b)[0]:
            ub += eval_point_T(spec, R, theta[k], phi[k], gbar[:, k], hbar[:, k])
        fpbar = mg_solve_T(spec, ghosts_T(ub))      # u = u0 + du
        kb, pb = patch_setup_T(spec, int(b), ub, fpbar)
        kbar += kb
        psibar += pb
    abar = alm2map_T(spec.ns, spec.lmax, psibar)
    abar = sht.poisson(spec.lmax, abar)             # a real diagonal
    ksbar = map2alm_T(spec.ns, spec.lmax, abar)
    if spec.ns == spec.nf:
        kbar += ksbar
    else:
        kbar += degrade_T(spec.nf, spec.ns, ksbar)
    return demean_T(kbar)


def shear_chi2(hess, g1obs, g2obs, sigma_e=0.26):
    """chi^2 = sum [(gamma1 - obs1)^2 + (gamma2 - obs2)^2] / sigma_e^2 with
    gamma1 = (U_tt - U_pp) / 2, gamma2 = U_tp; returns (chi2, hess bar)."""
    g1 = 0.5 * (hess[0] - hess[1])
    g2 = hess[2]
    r1, r2 = g1 - g1obs, g2 - g2obs
    chi2 = float(np.sum(r1 * r1 + r2 * r2) / sigma_e ** 2)
    hbar = np.stack([r1, -r1, 2.0 * r2]) / sigma_e ** 2
    return chi2, hbar
