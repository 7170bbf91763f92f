"""Pins of the oracle's SHT+MG patch solver, finite differences and point
evaluation (Sec. 3.2, App. A) against analytic fields, convergence orders and
discrete invariants."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import healpix as hp
from oracle import mg
from oracle import sht


def _spec(n, nf=64, nb=4, ns=32, lmax=32):
    return mg.PatchSpec(nside_fine=nf, nside_sht=ns, lmax=lmax, nside_bundle=nb,
                        ncell=n)


def _ylm_real(l, m, th, ph):
    return np.real(sph_harm_y(l, m, th, ph))


def _cell_field(spec, R, n, fn, ghosts=1):
    thp, php = mg.patch_angles(spec, n, ghosts=ghosts)
    T, P = np.meshgrid(thp, php, indexing="ij")
    th, ph = mg.patch_dirs(spec, R, T, P)
    return fn(th, ph)


def test_area_telescopes_and_sums_to_patch():
    spec = _spec(64)
    c = mg.level_coeffs(spec, 64)
    cH = mg.level_coeffs(spec, 32)
    assert np.allclose(cH["area"], 2 * (c["area"][0::2] + c["area"][1::2]), rtol=1e-14)
    e = spec.theta_edges(64)
    total = np.sum(c["area"]) * 64
    assert np.isclose(total, spec.L * (np.cos(e[0]) - np.cos(e[-1])), rtol=1e-13)


def test_laplacian_second_order():
    """Finite-volume L on Y_lm sampled at cell centres approaches
    -l(l+1) Y_lm at O(Delta^2)."""
    R = mg.patch_rotation(4, 17)
    fn = lambda t, p: _ylm_real(9, 4, t, p)
    errs = []
    for n in (32, 64, 128):
        spec = _spec(n)
        u = _cell_field(spec, R, n, fn)
        Lu = mg.apply_L(u, mg.level_coeffs(spec, n))
        errs.append(np.abs(Lu + 90 * u[1:-1, 1:-1]).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2) < 0.1), order


def test_red_black_sweep_solves_its_cells():
    spec = _spec(32)
    c = mg.level_coeffs(spec, 32)
    rng = np.random.default_rng(0)
    f = rng.normal(size=(32, 32))
    u = mg.reflect_ghosts(rng.normal(size=(34, 34)))
    mg.rb_half_sweep(u, f, c, 0)
    r = f - mg.apply_L0(u.copy(), c)
    ii, jj = np.meshgrid(range(32), range(32), indexing="ij")
    assert np.abs(r[(ii + jj) % 2 == 0]).max() < 1e-10 * np.abs(f).max()
    assert np.abs(r[(ii + jj) % 2 == 1]).max() > 1e-3


def test_restriction_conserves_and_prolongation_preserves():
    spec = _spec(32)
    c = mg.level_coeffs(spec, 32)
    cH = mg.level_coeffs(spec, 16)
    rng = np.random.default_rng(1)
    r = rng.normal(size=(32, 32))
    rb = mg.restrict(r, c)
    assert np.isclose(np.sum(c["area"][:, None] * r), np.sum(cH["area"][:, None] * rb))
    assert np.allclose(mg.prolong(np.full((16, 16), 2.5), 32), 2.5)
    # linear in index space: reproduced away from the injected outer ring
    I = np.arange(16)
    e = 0.3 * I[:, None] - 0.7 * I[None, :]
    i = (np.arange(32) - 0.5) / 2
    ref = 0.3 * i[:, None] - 0.7 * i[None, :]
    p = mg.prolong(e, 32)
    assert np.allclose(p[1:-1, 1:-1], ref[1:-1, 1:-1])
    assert np.allclose(p[0, :], e[0, np.arange(32) // 2])


def test_vcycle_contraction_and_convergence():
    spec = _spec(128)
    co = mg.all_coeffs(spec)
    rng = np.random.default_rng(2)
    f = rng.normal(size=(128, 128))
    u = np.zeros((130, 130))
    res = [mg.residual_norm(spec, u, f)]
    for _ in range(14):
        mg.vcycle(spec, u, f, 0, co)
        res.append(mg.residual_norm(spec, u, f))
    res = np.array(res)
    assert np.all(res[2:] / res[1:-1] < 0.2)
    assert res[-1] < 1e-11 * res[0]


def test_mg_solution_converges_second_order():
    """With exact face data and source, the MG solution tends to the
    analytic potential at O(Delta^2)."""
    R = mg.patch_rotation(4, 40)
    fn = lambda t, p: _ylm_real(7, 2, t, p)
    errs = []
    for n in (32, 64, 128):
        spec = _spec(n)
        L = spec.L
        tc, pc = mg.patch_angles(spec, n, ghosts=0)
        exact = _cell_field(spec, R, n, fn, ghosts=0)
        u0 = np.zeros((n + 2, n + 2))
        lo, hi = np.pi / 2 - L / 2, np.pi / 2 + L / 2
        u0[0, 1:-1] = 2 * fn(*mg.patch_dirs(spec, R, lo, pc))
        u0[-1, 1:-1] = 2 * fn(*mg.patch_dirs(spec, R, hi, pc))
        u0[1:-1, 0] = 2 * fn(*mg.patch_dirs(spec, R, tc, -L / 2))
        u0[1:-1, -1] = 2 * fn(*mg.patch_dirs(spec, R, tc, L / 2))
        fp = -56.0 * exact - mg.apply_L(u0, mg.level_coeffs(spec, n))
        du = mg.mg_solve(spec, fp, vcycles=20)
        errs.append(np.abs(du[1:-1, 1:-1] - exact).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2) < 0.25), (errs, order)


def test_fornberg_weights():
    w1 = mg.fornberg_weights(0.0, np.arange(-2, 3).astype(float), 2)
    assert np.allclose(w1[1], np.array([1, -8, 0, 8, -1]) / 12)
    assert np.allclose(w1[2], np.array([-1, 16, -30, 16, -1]) / 12)
    for i in (0, 5, 9):
        for d, deg in ((1, 4), (2, 5)):
            offs, w = mg.stencil(i, 10, d)
            assert offs.min() >= -1 - i and offs.max() <= 10 - i
            for k in range(deg + 1):
                exact = 0.0 if k < d else (1.0 if k == d == 1 else (2.0 if (k == 2 and d == 2) else 0.0))
                assert abs(np.sum(w * offs.astype(float) ** k) - exact) < 1e-10


def test_fd_fourth_order():
    """Raw partials on f(theta', phi') converge at 4th order, in the interior
    and with the one-sided edge stencils."""
    f = lambda t, p: np.sin(3 * t) * np.cos(2 * p) + t * p * p
    ft = lambda t, p: 3 * np.cos(3 * t) * np.cos(2 * p) + p * p
    fp = lambda t, p: -2 * np.sin(3 * t) * np.sin(2 * p) + 2 * t * p
    ftt = lambda t, p: -9 * np.sin(3 * t) * np.cos(2 * p)
    fpp = lambda t, p: -4 * np.sin(3 * t) * np.cos(2 * p) + 2 * t
    ftp = lambda t, p: -6 * np.cos(3 * t) * np.sin(2 * p) + 2 * p
    for (ci, cj) in [(0.5, 0.5), (0.0, 0.5), (1.0, 1.0)]:
        errs = []
        for n in (32, 64):
            spec = _spec(n)
            th, ph = mg.patch_angles(spec, n)
            T, P = np.meshgrid(th, ph, indexing="ij")
            u = f(T, P)
            i = min(int(ci * n), n - 1)
            j = min(int(cj * n), n - 1)
            t0, p0 = th[i + 1], ph[j + 1]
            got = mg.raw_partials(u, spec.delta, i, j)
            ref = np.array([g(t0, p0) for g in (ft, fp, ftt, fpp, ftp)])
            errs.append(np.abs(got - ref))
        order = np.log2(errs[0] / errs[1])
        assert np.all(order > 3.5), (ci, cj, order)


def test_eval_point_matches_pure_sht_derivatives():
    """u = psi sampled exactly (no MG): gradient and covariant Hessian at the
    bundle's pixel centres agree with the pure-SHT derivatives, so the
    Christoffel terms and the basis rotation are right."""
    Nf, Nb, lmax = 64, 4, 16
    spec = _spec(256, nf=Nf, nb=Nb)
    a = np.zeros(sht.nalm(lmax), complex)
    a[sht.alm_index(lmax, 5, 2)] = 0.4 - 0.3j
    a[sht.alm_index(lmax, 9, 0)] = 0.2
    a[sht.alm_index(lmax, 11, 7)] = 0.1 + 0.25j
    psi = sht.poisson(lmax, a)
    d = sht.derivative_maps(Nf, lmax, psi)
    l, m = sht.lm_arrays(lmax)
    nz = np.nonzero(psi)[0]
    fn = lambda t, p: sum(((sph_harm_y(l[k], m[k], t, p) * psi[k]).real * (1 if m[k] == 0 else 2))
                          for k in nz)
    for b in (0, 21, 100):
        R = mg.patch_rotation(Nb, b)
        patch = dict(R=R, u0=_cell_field(spec, R, 256, fn), du=np.zeros((258, 258)))
        pix = hp.nest2ring(Nf, np.arange(b * 256, (b + 1) * 256, 9))
        z, ph, s = hp.pix2ang_ring(Nf, pix)
        th = np.arctan2(s, z)
        for k in range(pix.size):
            g, U = mg.eval_point(spec, patch, th[k], ph[k])
            p = pix[k]
            ge = np.array([d["g_t"][p], d["g_p"][p]])
            Ue = np.array([[d["U_tt"][p], d["U_tp"][p]], [d["U_tp"][p], d["U_pp"][p]]])
            assert np.abs(g - ge).max() < 2e-4 * np.abs(ge).max() + 1e-12
            assert np.abs(U - Ue).max() < 2e-3 * np.abs(Ue).max() + 1e-12
    with pytest.raises(ValueError):
        mg.eval_point(spec, patch, th[0], ph[0] + 1.0)


def test_sht_mg_band_limited_field():
    """Full SHT+MG solve of a band-limited field: gradient and shear at the
    bundle pixels within 1% of the exact pure-SHT values (the error is the
    boundary interpolation, Sec. 4.1)."""
    Nf, Ns, lmax, Nb = 64, 32, 32, 4
    spec = mg.PatchSpec(nside_fine=Nf, nside_sht=Ns, lmax=lmax, nside_bundle=Nb, vcycles=6)
    a = np.zeros(sht.nalm(lmax), complex)
    a[sht.alm_index(lmax, 5, 2)] = 0.3 + 0.2j
    a[sht.alm_index(lmax, 3, 0)] = 0.5
    a[sht.alm_index(lmax, 12, 7)] = 0.1 - 0.05j
    kap = sht.alm2map(Nf, lmax, a)
    exact = sht.derivative_maps(Nf, lmax, sht.poisson(lmax, a))
    for b in (17, 191):
        sol = mg.solve_plane(spec, kap, [b])
        patch = sol["patches"][b]
        pix = hp.nest2ring(Nf, np.arange(b * 256, (b + 1) * 256, 11))
        z, ph, s = hp.pix2ang_ring(Nf, pix)
        th = np.arctan2(s, z)
        for k in range(pix.size):
            g, U = mg.eval_point(spec, patch, th[k], ph[k])
            p = pix[k]
            ge = np.array([exact["g_t"][p], exact["g_p"][p]])
            Ue = np.array([[exact["U_tt"][p], exact["U_tp"][p]],
                           [exact["U_tp"][p], exact["U_pp"][p]]])
            assert np.abs(g - ge).max() < 0.01 * np.abs(ge).max()
            assert np.abs(U - Ue).max() < 0.01 * np.abs(Ue).max()


def test_eps_rule_truncation_order_and_stopping():
    """tau of a smooth field falls as Delta^2 (the truncation error of the
    5-point operator); the residual of the exact discrete solution is zero;
    the epsilon rule stops at the first cycle with epsilon < eps and then
    equals the fixed-cycle iterate."""
    R = mg.patch_rotation(4, 40)
    fn = lambda t, p: _ylm_real(7, 2, t, p)
    taus = []
    for n in (32, 64, 128):
        spec = _spec(n)
        x = _cell_field(spec, R, n, fn, ghosts=0)
        c, cH = mg.level_coeffs(spec, n), mg.level_coeffs(spec, n // 2)
        L0 = lambda v, cc: mg.apply_L0(np.pad(v, 1), cc)
        tau = L0(mg.restrict(x, c), cH) - mg.restrict(L0(x, c), c)
        # away from the faces (where the ghost reflection dominates)
        m = n // 8
        taus.append(np.sqrt(np.mean(tau[m:-m, m:-m] ** 2)))
    order = np.log2(np.array(taus[:-1]) / np.array(taus[1:]))
    assert np.all(np.abs(order - 2.0) < 0.25), order
    spec = _spec(64)
    rng = np.random.default_rng(5)
    f = rng.normal(size=(64, 64))
    du_e, k, hist = mg.mg_solve_eps(spec, f, eps=1e-3, max_cycles=30)
    assert hist[-1] < 1e-3 and all(h >= 1e-3 for h in hist[:-1])
    assert np.all(np.diff(hist) < 0)
    du_f = mg.mg_solve(spec, f, vcycles=k)
    assert np.array_equal(du_e, du_f)
    # exact discrete solution: zero residual, so epsilon -> 0
    co = mg.all_coeffs(spec)
    u = np.zeros((66, 66))
    for _ in range(40):
        mg.vcycle(spec, u, f, 0, co)
    assert mg.eps_ratio(spec, u, f) < 1e-9
