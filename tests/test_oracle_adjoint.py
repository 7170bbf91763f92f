"""Pins of the oracle's transpose of the kappa -> shear map (C5): every
transposed step passes the dot-product test <A x, y> = <x, A^T y> against the
oracle's own forward step (a dropped term, a wrong coefficient or a swapped
neighbour in either breaks it), the whole chain passes it too, and the
gradient of the shear chi^2, which is exactly quadratic in kappa, matches
central finite differences up to rounding."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import healpix as hp
from oracle import mg
from oracle import sht
from paper_1210_3069_amd import inputs


def rel_dot(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.fixture(scope="module")
def spec():
    return mg.PatchSpec(16, 4, 8, 4, ncell=16, vcycles=2)


def _full(x):
    n = x.shape[0]
    u = np.zeros((n + 2, n + 2))
    u[1:-1, 1:-1] = x
    return u


def test_operator_and_sweep_transposes(spec):
    rng = np.random.default_rng(1)
    c = mg.level_coeffs(spec, 16)
    x, y = rng.standard_normal((16, 16)), rng.standard_normal((16, 16))
    assert rel_dot(np.sum(adj.L0(x, c) * y), np.sum(x * adj.L0_T(y, c))) < 1e-13
    for color in (0, 1):
        u, f, yb = (rng.standard_normal((16, 16)) for _ in range(3))
        uf = _full(u)
        mg.rb_half_sweep(uf, f, c, color)
        ub, fb = adj.half_sweep_T(yb, c, color)
        assert rel_dot(np.sum(uf[1:-1, 1:-1] * yb), np.sum(u * ub) + np.sum(f * fb)) < 1e-13
    # restriction, prolongation, apply_L with a stored ghost ring
    yc = rng.standard_normal((8, 8))
    assert rel_dot(np.sum(mg.restrict(x, c) * yc), np.sum(x * adj.restrict_T(yc, c))) < 1e-13
    e = rng.standard_normal((8, 8))
    assert rel_dot(np.sum(mg.prolong(e, 16) * y), np.sum(e * adj.prolong_T(y, 8))) < 1e-13
    uf = rng.standard_normal((18, 18))
    assert rel_dot(np.sum(mg.apply_L(uf, c) * y), np.sum(uf * adj.apply_L_T(y, c))) < 1e-13
    g = rng.standard_normal((18, 18))
    assert rel_dot(np.sum(mg.reflect_ghosts(_full(x)) * g), np.sum(x * adj.ghosts_T(g))) < 1e-13


def test_vcycle_and_solve_transposes(spec):
    rng = np.random.default_rng(2)
    coeffs = mg.all_coeffs(spec)
    u, f, yb = (rng.standard_normal((16, 16)) for _ in range(3))
    uf = _full(u)
    mg.reflect_ghosts(uf)
    mg.vcycle(spec, uf, f, 0, coeffs)
    ub, fb = adj.vcycle_T(spec, yb, 0, coeffs)
    assert rel_dot(np.sum(uf[1:-1, 1:-1] * yb), np.sum(u * ub) + np.sum(f * fb)) < 1e-12
    du = mg.mg_solve(spec, f)
    assert rel_dot(np.sum(du[1:-1, 1:-1] * yb), np.sum(f * adj.mg_solve_T(spec, yb))) < 1e-12


def test_sht_transposes():
    rng = np.random.default_rng(3)
    N, lmax = 4, 8
    m = rng.standard_normal(hp.npix(N))
    a = inputs.gaussian_alm(lmax, seed=5, amplitude=1.0)
    _, mm = sht.lm_arrays(lmax)
    a = np.where(mm == 0, a.real + 0j, a)
    ybar = rng.standard_normal(hp.npix(N))
    dot = lambda p, q: float(np.sum(p.real * q.real + p.imag * q.imag))
    assert rel_dot(np.sum(sht.alm2map(N, lmax, a) * ybar), dot(a, adj.alm2map_T(N, lmax, ybar))) < 1e-12
    abar = inputs.gaussian_alm(lmax, seed=6, amplitude=1.0)
    assert rel_dot(dot(sht.map2alm(N, lmax, m), abar), np.sum(m * adj.map2alm_T(N, lmax, abar))) < 1e-12
    k = rng.standard_normal(hp.npix(16))
    kn = k[hp.nest2ring(16, np.arange(hp.npix(16)))]
    ks = np.empty(hp.npix(4))
    ks[hp.nest2ring(4, np.arange(hp.npix(4)))] = hp.degrade_nest_mean(16, 4, kn)
    yb = rng.standard_normal(hp.npix(4))
    assert rel_dot(np.sum(ks * yb), np.sum(k * adj.degrade_T(16, 4, yb))) < 1e-13


def test_setup_and_eval_transposes(spec):
    rng = np.random.default_rng(4)
    b = 37
    kap = rng.standard_normal(hp.npix(spec.nf))
    psi = rng.standard_normal(hp.npix(spec.ns))
    R, u0, fp = mg.patch_setup(spec, b, kap, 0.0, psi)
    u0b, fpb = rng.standard_normal(u0.shape), rng.standard_normal(fp.shape)
    kb, pb = adj.patch_setup_T(spec, b, u0b, fpb)
    assert rel_dot(np.sum(u0 * u0b) + np.sum(fp * fpb), np.sum(kap * kb) + np.sum(psi * pb)) < 1e-12
    # evaluation at points of bundle b, linear in u
    z, ph, _ = hp.pix2ang_nest(spec.nb, np.array([b]))
    th0 = np.arccos(z[0])
    u = rng.standard_normal(u0.shape)
    patch = dict(R=R, u0=u, du=np.zeros_like(u))
    for k in range(5):
        th, p = th0 + 0.05 * rng.uniform(-1, 1), ph[0] + 0.05 * rng.uniform(-1, 1)
        g, U = mg.eval_point(spec, patch, th, p)
        gb, hb = rng.standard_normal(2), rng.standard_normal(3)
        ub = adj.eval_point_T(spec, R, th, p, gb, hb)
        lhs = g @ gb + U[0, 0] * hb[0] + U[1, 1] * hb[1] + U[0, 1] * hb[2]
        assert rel_dot(lhs, np.sum(u * ub)) < 1e-12


@pytest.fixture(scope="module")
def chain(spec):
    rng = np.random.default_rng(7)
    g = sht.alm2map(16, 32, inputs.gaussian_alm(32, seed=8, sigma=0.5))
    kap = 0.01 * (np.exp(g) - np.mean(np.exp(g)))
    th, ph = inputs.uniform_sphere(40, seed=9)
    return kap, th, ph, rng


def test_whole_chain_dot_product(spec, chain):
    kap, th, ph, rng = chain
    g, h = adj.forward(spec, kap, th, ph)
    gb, hb = rng.standard_normal(g.shape), rng.standard_normal(h.shape)
    kb = adj.adjoint(spec, th, ph, gb, hb)
    assert rel_dot(np.sum(g * gb) + np.sum(h * hb), np.sum(kap * kb)) < 1e-11


def test_chi2_gradient_matches_central_differences(spec, chain):
    kap, th, ph, rng = chain
    g1o, g2o = 0.26 * rng.standard_normal(th.size), 0.26 * rng.standard_normal(th.size)
    _, h = adj.forward(spec, kap, th, ph)
    chi2, hb = adj.shear_chi2(h, g1o, g2o)
    grad = adj.adjoint(spec, th, ph, np.zeros((2, th.size)), hb)
    step = 1e-3 * np.sqrt(np.mean(kap ** 2))
    for p in rng.choice(hp.npix(16), 4, replace=False):
        e = np.zeros_like(kap)
        e[p] = step
        cp, _ = adj.shear_chi2(adj.forward(spec, kap + e, th, ph)[1], g1o, g2o)
        cm, _ = adj.shear_chi2(adj.forward(spec, kap - e, th, ph)[1], g1o, g2o)
        fd = (cp - cm) / (2 * step)
        assert abs(fd - grad[p]) <= 1e-7 * (abs(grad[p]) + 1e-3 * np.abs(grad).max()), (p, fd, grad[p])
