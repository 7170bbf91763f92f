"""SHT+MG Poisson solve on rotated patches, finite-difference derivatives and
their evaluation at points, for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Follows Sec. 3.2 of the paper.  For every ray bundle (a NESTED HEALPix pixel,
Sec. 3.1) a patch is built in a rotated frame that puts the bundle centre at
(theta', phi') = (pi/2, 0), with equal spacing Delta theta' = Delta phi' and a
side four times the bundle size.  The SHT potential supplies the boundary
values (by HEALPix linear interpolation) and the starting guess; the fine
solution is relaxed with red-black Gauss-Seidel inside an FAS multigrid
V-cycle with strictly conservative restriction and bilinear prolongation
that switches to direct injection at the boundary.  Derivatives come from
4th-order finite differences (one-sided stencils from Fornberg's algorithm
where the centred one does not fit), are bilinearly interpolated to the
points, corrected with the Christoffel terms of App. A and rotated back to
the global (theta-hat, phi-hat) basis.

Readings (the paper is silent or refers to an absent reference):
* patch rows are (c, phi-hat_c, -theta-hat_c): no roll about the centre;
* cell-centred cells, one ghost ring; finite-volume 5-point Laplacian with
  exact cell areas; the Dirichlet data sit on the patch faces (the SHT
  potential interpolated at the face midpoints, ghost = 2 b - interior), so
  every level sees the same boundary; the unknown is du = u - u0 with zero
  face value on every level (equivalent to FAS on u for this linear problem);
* nu1 = nu2 = 2 red-black sweeps (red = (i+j) even first), levels down to
  4 x 4 solved exactly; injection on the outermost ring of fine cells;
* the MG source is 2 x the HEALPix interpolation of the demeaned fine map;
  with particles (Sec. 3.2: "a similar procedure is employed for the MG
  patches") it is 2 x (the Epanechnikov deposition onto the patch cells
  minus the mean), the deposition normalised over the cells of the patch's
  grid continued beyond its faces, so that a particle's mass splits
  between the patch and the outside exactly (patch_deposit);
* raw partials are interpolated, the metric is applied at the point.
"""
import numpy as np

from . import healpix as hp
from . import sht


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
class PatchSpec:
    """Sizes of the SHT+MG solve: fine (ray) grid, SHT grid, bundle grid,
    patch factor and finest cells per side."""

    def __init__(self, nside_fine, nside_sht, lmax, nside_bundle, factor=4,
                 ncell=None, nu1=2, nu2=2, vcycles=4):
        self.nf, self.ns, self.lmax, self.nb = nside_fine, nside_sht, lmax, nside_bundle
        self.factor = factor
        self.n = ncell if ncell else max(256, factor * nside_fine // nside_bundle)
        self.nu1, self.nu2, self.vcycles = nu1, nu2, vcycles
        self.side_b = np.sqrt(4.0 * np.pi / (12.0 * nside_bundle ** 2))
        self.L = factor * self.side_b
        self.delta = self.L / self.n
        self.nlev = int(np.log2(self.n)) - 1      # n -> 4

    def theta_edges(self, nk):
        """theta' of the nk+1 cell edges of a level with nk cells per side."""
        return np.pi / 2 - self.L / 2 + np.arange(nk + 1) * (self.L / nk)


def basis(z, phi, sint=None):
    """(theta-hat, phi-hat) at directions (z, phi); each (..., 3)."""
    z = np.asarray(z, dtype=np.float64)
    if sint is None:
        sint = np.sqrt((1 - z) * (1 + z))
    cp, sp = np.cos(phi), np.sin(phi)
    et = np.stack([z * cp, z * sp, -sint * np.ones_like(cp)], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(cp)], axis=-1)
    return et, ep


def patch_rotation(nside_bundle, b):
    """R_b with rows (c, phi-hat_c, -theta-hat_c): v' = R_b v puts the
    bundle centre c at (theta', phi') = (pi/2, 0)."""
    z, phi, s = hp.pix2ang_nest(nside_bundle, np.array([b]))
    c = hp.vec(z, phi, s)[0]
    et, ep = basis(z, phi, s)
    return np.stack([c, ep[0], -et[0]])


def patch_angles(spec, nk, ghosts=1):
    """Cell-centre theta', phi' (1-D each) of a level, ghosts included."""
    d = spec.L / nk
    idx = np.arange(-ghosts, nk + ghosts)
    th = np.pi / 2 - spec.L / 2 + (idx + 0.5) * d
    ph = -spec.L / 2 + (idx + 0.5) * d
    return th, ph


def patch_dirs(spec, R, thp, php):
    """Global (theta, phi) of patch-frame points (theta', phi'):
    v = R^T (sin th' cos ph', sin th' sin ph', cos th')."""
    thp, php = np.broadcast_arrays(np.asarray(thp, float), np.asarray(php, float))
    vp = np.stack([np.sin(thp) * np.cos(php), np.sin(thp) * np.sin(php),
                   np.cos(thp)], -1)
    return hp.vec2ang(vp @ R)


def patch_cell_dirs(spec, R):
    """Global (theta, phi) of the finest interior cell centres, [n, n]
    indexed [i (theta'), j (phi')]."""
    th, ph = patch_angles(spec, spec.n, ghosts=0)
    T, P = np.meshgrid(th, ph, indexing="ij")
    return patch_dirs(spec, R, T, P)


# --------------------------------------------------------------------------
# discrete operator
# --------------------------------------------------------------------------
def level_coeffs(spec, nk):
    """Row coefficients of the finite-volume Laplacian on a level:
    s_m = sin theta'_{i-1/2}, s_p = sin theta'_{i+1/2}, s_c = sin theta'_i,
    area_i = Delta (cos theta'_{i-1/2} - cos theta'_{i+1/2})
           = 2 Delta sin theta'_i sin(Delta/2)."""
    e = spec.theta_edges(nk)
    d = spec.L / nk
    tc = 0.5 * (e[:-1] + e[1:])
    return dict(s_m=np.sin(e[:-1]), s_p=np.sin(e[1:]), s_c=np.sin(tc),
                area=2.0 * d * np.sin(tc) * np.sin(0.5 * d), n=nk)


def reflect_ghosts(u):
    """Ghosts of a correction field under the face Dirichlet condition:
    the value on the patch boundary (the cell face) is zero, so each ghost
    is the negative of the interior cell it faces; a corner ghost is the
    negative of the diagonal interior cell."""
    u[0, 1:-1] = -u[1, 1:-1]
    u[-1, 1:-1] = -u[-2, 1:-1]
    u[1:-1, 0] = -u[1:-1, 1]
    u[1:-1, -1] = -u[1:-1, -2]
    u[0, 0], u[0, -1] = -u[1, 1], -u[1, -2]
    u[-1, 0], u[-1, -1] = -u[-2, 1], -u[-2, -2]
    return u


def apply_L(u, c):
    """(L u)_ij on interior cells, using the ghost ring of u as stored:
    (L u)_ij = [s_m (u_{i-1,j} - u_ij) + s_p (u_{i+1,j} - u_ij)
                + (u_{i,j-1} - 2 u_ij + u_{i,j+1}) / s_c] / area_i."""
    n = c["n"]
    uc = u[1:-1, 1:-1]
    up, dn = u[:-2, 1:-1], u[2:, 1:-1]
    lf, rt = u[1:-1, :-2], u[1:-1, 2:]
    sm, sp, sc, A = (c[k][:, None] for k in ("s_m", "s_p", "s_c", "area"))
    assert uc.shape == (n, n)
    return (sm * (up - uc) + sp * (dn - uc) + (lf - 2 * uc + rt) / sc) / A


def apply_L0(u, c):
    """L applied to a correction field (zero on the patch faces)."""
    return apply_L(reflect_ghosts(u), c)


def rb_half_sweep(u, f, c, color):
    """Gauss-Seidel solve of the cells with (i + j) % 2 == color for a
    correction field (face value zero):
      u_ij <- (s_m u_{i-1,j} + s_p u_{i+1,j} + (u_{i,j-1} + u_{i,j+1})/s_c
               - A_i f_ij) / (s_m + s_p + 2/s_c)
    where a neighbour across the patch boundary is the ghost -u_ij, i.e. it
    drops out of the numerator and its coefficient is added once more to the
    denominator."""
    n = c["n"]
    sm, sp, sc, A = (c[k][:, None] for k in ("s_m", "s_p", "s_c", "area"))
    g = u.copy()
    g[0, :] = g[-1, :] = g[:, 0] = g[:, -1] = 0.0
    diag = (sm + sp + 2.0 / sc) * np.ones((n, n))
    diag[0, :] += sm[0]
    diag[-1, :] += sp[-1]
    diag[:, 0] += 1.0 / sc[:, 0]
    diag[:, -1] += 1.0 / sc[:, 0]
    new = (sm * g[:-2, 1:-1] + sp * g[2:, 1:-1]
           + (g[1:-1, :-2] + g[1:-1, 2:]) / sc - A * f) / diag
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = ((ii + jj) % 2) == color
    u[1:-1, 1:-1][mask] = new[mask]
    reflect_ghosts(u)


def smooth(u, f, c, sweeps):
    for _ in range(sweeps):
        rb_half_sweep(u, f, c, 0)
        rb_half_sweep(u, f, c, 1)


def restrict(x, c_fine):
    """Area-weighted (strictly conservative) average of the 2x2 children."""
    A = c_fine["area"]
    a0 = A[0::2][:, None]
    a1 = A[1::2][:, None]
    top = x[0::2, 0::2] + x[0::2, 1::2]
    bot = x[1::2, 0::2] + x[1::2, 1::2]
    return (a0 * top + a1 * bot) / (2.0 * (a0 + a1))


def prolong(e, n_fine):
    """Bilinear cell-centred interpolation (9/16, 3/16, 3/16, 1/16) of the
    coarse correction e, with direct injection on the outermost fine ring."""
    nH = e.shape[0]
    eg = np.zeros((nH + 2, nH + 2))
    eg[1:-1, 1:-1] = e
    out = np.empty((n_fine, n_fine))
    i = np.arange(n_fine)
    I = i // 2
    di = np.where(i % 2 == 0, -1, 1)
    II, JJ = np.meshgrid(I, I, indexing="ij")
    DI, DJ = np.meshgrid(di, di, indexing="ij")
    out = (9.0 * eg[II + 1, JJ + 1] + 3.0 * eg[II + 1 + DI, JJ + 1]
           + 3.0 * eg[II + 1, JJ + 1 + DJ] + eg[II + 1 + DI, JJ + 1 + DJ]) / 16.0
    edge = np.zeros((n_fine, n_fine), dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    out[edge] = eg[II + 1, JJ + 1][edge]
    return out


def coarsest_solve(f, c):
    """Exact solve of L u = f on the coarsest level (zero ghosts)."""
    n = c["n"]
    M = np.zeros((n * n, n * n))
    for k in range(n * n):
        u = np.zeros((n + 2, n + 2))
        u[1 + k // n, 1 + k % n] = 1.0
        M[:, k] = apply_L0(u, c).ravel()
    return np.linalg.solve(M, f.ravel()).reshape(n, n)


def vcycle(spec, u, f, level, coeffs):
    """One FAS V-cycle on level `level` (0 = finest); u has ghosts (zero)."""
    c = coeffs[level]
    if c["n"] <= 4:
        u[1:-1, 1:-1] = coarsest_solve(f, c)
        reflect_ghosts(u)
        return
    smooth(u, f, c, spec.nu1)
    r = f - apply_L0(u, c)
    ubar = restrict(u[1:-1, 1:-1], c)
    rbar = restrict(r, c)
    cH = coeffs[level + 1]
    uH = np.zeros((cH["n"] + 2, cH["n"] + 2))
    uH[1:-1, 1:-1] = ubar
    fH = apply_L0(uH, cH) + rbar
    vcycle(spec, uH, fH, level + 1, coeffs)
    u[1:-1, 1:-1] += prolong(uH[1:-1, 1:-1] - ubar, c["n"])
    reflect_ghosts(u)
    smooth(u, f, c, spec.nu2)


def all_coeffs(spec):
    out, nk = [], spec.n
    while nk >= 4:
        out.append(level_coeffs(spec, nk))
        nk //= 2
    return out


def residual_norm(spec, du, fp):
    """Area-weighted RMS of f' - L du on the finest level."""
    c = level_coeffs(spec, spec.n)
    r = fp - apply_L0(du.copy(), c)
    A = c["area"][:, None] * np.ones_like(r)
    return np.sqrt(np.sum(A * r * r) / np.sum(A))


def area_rms(x, area_rows):
    """Area-weighted RMS of a cell field (rows weighted by their area)."""
    A = area_rows[:, None] * np.ones_like(x)
    return np.sqrt(np.sum(A * x * x) / np.sum(A))


def eps_ratio(spec, du, fp):
    """Stopping quantity of Sec. 3.2: epsilon = ||r_h|| / ||tau|| with the
    residual r_h = f' - L_h du on the finest level and the relative
    truncation error tau = L_H(R du) - R(L_h du) on the first coarse level,
    both area-weighted RMS; du given with or without its ghost ring."""
    c = level_coeffs(spec, spec.n)
    cH = level_coeffs(spec, spec.n // 2)
    x = du[1:-1, 1:-1] if du.shape[0] == spec.n + 2 else du

    def L0(v, cc):
        u = np.zeros((cc["n"] + 2, cc["n"] + 2))
        u[1:-1, 1:-1] = v
        return apply_L0(u, cc)

    r = fp - L0(x, c)
    tau = L0(restrict(x, c), cH) - restrict(L0(x, c), c)
    nr, nt = area_rms(r, c["area"]), area_rms(tau, cH["area"])
    if nt == 0.0:
        return 0.0 if nr == 0.0 else np.inf
    return nr / nt


def mg_solve_eps(spec, fp, eps=0.1, max_cycles=20):
    """V-cycles from du = 0 until eps_ratio < eps (Sec. 3.2), at most
    max_cycles.  Returns (du, cycles, [epsilon after each cycle])."""
    coeffs = all_coeffs(spec)
    du = np.zeros((spec.n + 2, spec.n + 2))
    hist = []
    for k in range(max_cycles):
        vcycle(spec, du, fp, 0, coeffs)
        hist.append(eps_ratio(spec, du, fp))
        if hist[-1] < eps:
            return du, k + 1, hist
    return du, max_cycles, hist


# --------------------------------------------------------------------------
# the plane solve
# --------------------------------------------------------------------------
def sht_stage(spec, kappa_fine_ring):
    """Demean, degrade to the SHT grid, analyse, Poisson, synthesise.
    Returns (mean, kappa_sht_ring, psi_alm, psi_sht_ring)."""
    mean = np.mean(kappa_fine_ring)
    kp = kappa_fine_ring - mean
    if spec.ns == spec.nf:
        ks = kp
    else:
        nest = kp[hp.nest2ring(spec.nf, np.arange(hp.npix(spec.nf)))]
        ks_nest = hp.degrade_nest_mean(spec.nf, spec.ns, nest)
        ks = np.empty_like(ks_nest)
        ks[hp.nest2ring(spec.ns, np.arange(hp.npix(spec.ns)))] = ks_nest
    alm = sht.map2alm(spec.ns, spec.lmax, ks)
    palm = sht.poisson(spec.lmax, alm)
    psi = sht.alm2map(spec.ns, spec.lmax, palm)
    return mean, ks, palm, psi


def patch_deposit(spec, b, theta, phi, weight, sigma):
    """Mass per unit area on the n x n cells of patch b from particles
    (Sec. 3.2): each particle's Epanechnikov kernel K(angle) times the cell
    area, over the cell centres of the patch grid (continued beyond the
    faces) closer than sigma, normalised to the particle's weight; the part
    on cells of the patch is kept.  A particle whose sigma reaches no cell
    centre puts its weight in the cell that contains it (if in the patch).
    Cell areas: Delta (cos theta'_{i-1/2} - cos theta'_{i+1/2})."""
    from .deposit import kernel
    n, d = spec.n, spec.delta
    th0, ph0 = np.pi / 2 - spec.L / 2, -spec.L / 2
    R = patch_rotation(spec.nb, b)
    rho = np.zeros((n, n))
    for t, p, w, sg in zip(theta, phi, weight, sigma):
        v = R @ hp.vec(np.cos(t), p, np.sin(t))
        tp = np.arctan2(np.hypot(v[0], v[1]), v[2])
        pp = np.arctan2(v[1], v[0])
        smin = max(np.sin(min(np.pi / 2 + spec.L / 2 + sg, np.pi - 1e-3)), 1e-3)
        di, dj = int(sg / d) + 2, int(sg / (d * smin)) + 2
        ic, jc = int(np.floor((tp - th0) / d)), int(np.floor((pp - ph0) / d))
        ii = np.arange(ic - di, ic + di + 1)
        jj = np.arange(jc - dj, jc + dj + 1)
        tc = th0 + (ii + 0.5) * d
        pc = ph0 + (jj + 0.5) * d
        T, P = np.meshgrid(tc, pc, indexing="ij")
        C = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
        ang = np.arctan2(np.linalg.norm(np.cross(C, v), axis=-1), C @ v)
        area = (d * (np.cos(tc - 0.5 * d) - np.cos(tc + 0.5 * d)))[:, None]
        k = kernel(ang, sg) if sg > 0 else np.zeros_like(ang)
        tot = np.sum(k * area)
        inside_i = (ii >= 0) & (ii < n)
        inside_j = (jj >= 0) & (jj < n)
        if tot > 0:
            dens = w * k / tot
            rho[np.ix_(ii[inside_i], jj[inside_j])] += dens[np.ix_(inside_i, inside_j)]
        elif 0 <= ic < n and 0 <= jc < n:
            a = d * (np.cos(th0 + ic * d) - np.cos(th0 + (ic + 1) * d))
            rho[ic, jc] += w / a
    return rho


def patch_setup(spec, b, kappa_fine_ring, mean, psi_sht_ring, source=None):
    """u0 = interp(psi_SHT) at the cell centres (the starting guess) and
    Dirichlet data b = interp(psi_SHT) at the midpoints of the boundary faces
    (corner ghosts: at the patch corners), ghost u0 = 2 b - u0(adjacent
    interior cell); f = 2 interp(kappa - mean) at the cell centres, or
    f = 2 (source - mean) for a source on the cells (particles);
    f' = f - L u0.  Returns (R, u0 [n+2, n+2], f' [n, n])."""
    n, L = spec.n, spec.L
    R = patch_rotation(spec.nb, b)
    interp_psi = lambda t, p: hp.interp(spec.ns, psi_sht_ring, t.ravel(),
                                        p.ravel()).reshape(t.shape)
    th, ph = patch_cell_dirs(spec, R)
    u0 = np.zeros((n + 2, n + 2))
    u0[1:-1, 1:-1] = interp_psi(th, ph)
    tc, pc = patch_angles(spec, n, ghosts=0)
    lo_t, hi_t = np.pi / 2 - L / 2, np.pi / 2 + L / 2
    lo_p, hi_p = -L / 2, L / 2
    top = interp_psi(*patch_dirs(spec, R, lo_t, pc))
    bot = interp_psi(*patch_dirs(spec, R, hi_t, pc))
    lft = interp_psi(*patch_dirs(spec, R, tc, lo_p))
    rgt = interp_psi(*patch_dirs(spec, R, tc, hi_p))
    u0[0, 1:-1] = 2 * top - u0[1, 1:-1]
    u0[-1, 1:-1] = 2 * bot - u0[-2, 1:-1]
    u0[1:-1, 0] = 2 * lft - u0[1:-1, 1]
    u0[1:-1, -1] = 2 * rgt - u0[1:-1, -2]
    corners = interp_psi(*patch_dirs(spec, R, np.array([lo_t, lo_t, hi_t, hi_t]),
                                     np.array([lo_p, hi_p, lo_p, hi_p])))
    u0[0, 0] = 2 * corners[0] - u0[1, 1]
    u0[0, -1] = 2 * corners[1] - u0[1, -2]
    u0[-1, 0] = 2 * corners[2] - u0[-2, 1]
    u0[-1, -1] = 2 * corners[3] - u0[-2, -2]
    if source is None:
        f = 2.0 * (hp.interp(spec.nf, kappa_fine_ring, th.ravel(), ph.ravel()) - mean)
        f = f.reshape(n, n)
    else:
        f = 2.0 * (source - mean)
    fp = f - apply_L(u0, level_coeffs(spec, n))
    return R, u0, fp


def mg_solve(spec, fp, vcycles=None):
    """du after a fixed number of V-cycles from du = 0 (face value 0)."""
    coeffs = all_coeffs(spec)
    du = np.zeros((spec.n + 2, spec.n + 2))
    for _ in range(spec.vcycles if vcycles is None else vcycles):
        vcycle(spec, du, fp, 0, coeffs)
    return du


def solve_plane(spec, kappa_fine_ring, bundles, particles=None):
    """The full SHT+MG solve for the listed bundles.  With particles
    (theta, phi, weight, sigma), kappa_fine_ring is their deposition on the
    fine grid (it feeds the SHT stage) and each patch's source is their
    deposition on its cells."""
    mean, ks, palm, psi = sht_stage(spec, kappa_fine_ring)
    patches = {}
    for b in bundles:
        src = None if particles is None else patch_deposit(spec, b, *particles)
        R, u0, fp = patch_setup(spec, b, kappa_fine_ring, mean, psi, source=src)
        du = mg_solve(spec, fp)
        patches[int(b)] = dict(R=R, u0=u0, du=du, fp=fp)
    return dict(mean=mean, kappa_sht=ks, psi_alm=palm, psi_sht=psi,
                patches=patches)


# --------------------------------------------------------------------------
# finite differences and evaluation
# --------------------------------------------------------------------------
def fornberg_weights(x0, xs, order):
    """Finite-difference weights for derivatives 0..order at x0 on nodes xs
    (Fornberg 1988, Math. Comp. 51, 699): returns c[k, j]."""
    xs = np.asarray(xs, dtype=np.float64)
    n = xs.size
    c = np.zeros((order + 1, n))
    c1, c4 = 1.0, xs[0] - x0
    c[0, 0] = 1.0
    for i in range(1, n):
        mn = min(i, order)
        c2, c5 = 1.0, c4
        c4 = xs[i] - x0
        for j in range(i):
            c3 = xs[i] - xs[j]
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k, i] = c1 * (k * c[k - 1, i - 1] - c5 * c[k, i - 1]) / c2
                c[0, i] = -c1 * c5 * c[0, i - 1] / c2
            for k in range(mn, 0, -1):
                c[k, j] = (c4 * c[k, j] - k * c[k - 1, j]) / c3
            c[0, j] = c4 * c[0, j] / c3
        c1 = c2
    return c


def stencil(i, n, deriv):
    """(offsets, weights in units of Delta^-deriv) of the 4th-order stencil
    for derivative `deriv` at cell i of n (ghosts at -1 and n)."""
    if 1 <= i <= n - 2:
        offs = np.arange(-2, 3)
    elif i == 0:
        offs = np.arange(-1, 4) if deriv == 1 else np.arange(-1, 5)
    else:
        offs = np.arange(-3, 2) if deriv == 1 else np.arange(-4, 2)
    w = fornberg_weights(0.0, offs.astype(np.float64), deriv)[deriv]
    return offs, w


def raw_partials(u, delta, i, j):
    """(psi_t, psi_p, psi_tt, psi_pp, psi_tp) in the patch frame at cell
    (i, j); u carries one ghost ring."""
    n = u.shape[0] - 2
    g = lambda a, b: u[a + 1, b + 1]
    o1i, w1i = stencil(i, n, 1)
    o2i, w2i = stencil(i, n, 2)
    o1j, w1j = stencil(j, n, 1)
    o2j, w2j = stencil(j, n, 2)
    pt = sum(w * g(i + o, j) for o, w in zip(o1i, w1i)) / delta
    pp = sum(w * g(i, j + o) for o, w in zip(o1j, w1j)) / delta
    ptt = sum(w * g(i + o, j) for o, w in zip(o2i, w2i)) / delta ** 2
    ppp = sum(w * g(i, j + o) for o, w in zip(o2j, w2j)) / delta ** 2
    ptp = sum(wa * wb * g(i + oa, j + ob) for oa, wa in zip(o1i, w1i)
              for ob, wb in zip(o1j, w1j)) / delta ** 2
    return np.array([pt, pp, ptt, ppp, ptp])


def covariant(p, st, ct):
    """Gradient and covariant Hessian (orthonormal theta/phi basis, App. A)
    from raw partials p = (t, p, tt, pp, tp) at sin/cos theta = st, ct."""
    g = np.array([p[0], p[1] / st])
    U = np.array([[p[2], p[4] / st - ct * p[1] / st ** 2],
                  [p[4] / st - ct * p[1] / st ** 2,
                   p[3] / st ** 2 + (ct / st) * p[0]]])
    return g, U


def eval_point(spec, patch, theta, phi):
    """Gradient g = (g_theta, g_phi) and covariant Hessian U (2x2) of
    psi = u0 + du at (theta, phi), global basis.  Raises ValueError when the
    bilinear footprint leaves the patch interior."""
    R, u = patch["R"], patch["u0"] + patch["du"]
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
    P = ((1 - t) * (1 - s) * raw_partials(u, d, i0, j0)
         + (1 - t) * s * raw_partials(u, d, i0, j0 + 1)
         + t * (1 - s) * raw_partials(u, d, i0 + 1, j0)
         + t * s * raw_partials(u, d, i0 + 1, j0 + 1))
    gp, Up = covariant(P, np.sin(thp), np.cos(thp))
    # patch basis at the point, in global coordinates
    etp, epp = basis(np.cos(thp), php)
    etp, epp = R.T @ etp, R.T @ epp
    et, ep = basis(np.cos(theta), phi)
    Q = np.array([[et @ etp, et @ epp], [ep @ etp, ep @ epp]])
    return Q @ gp, Q @ Up @ Q.T


def bundle_of(spec, theta, phi):
    return int(hp.ang2pix_nest(spec.nb, np.cos(np.atleast_1d(theta)),
                               np.atleast_1d(phi))[0])
