"""Partial sky (Sec. 3.4; clm_plan_set_domain): the SHT over the whole sky,
the multigrid step, the shear evaluation and the rays over a domain of
bundles only.

Every patch is an independent solve whose boundary values come from the
full-sky SHT, so a patch of the domain must come out exactly as in the
whole-sky run: the checks compare the two runs bit for bit (fixed cycle
count and the epsilon rule, both multigrid precisions), check what lies
outside the domain (untouched outputs, NaN and the latched status at
points, 0 cycles and NaN epsilon), and compare two patches of the domain
with the oracle's patch solve (oracle/mg.py, which solves any list of
bundles)."""
import numpy as np
import pytest
import torch

from oracle import healpix as hp
from oracle import mg as omg
from oracle import sht as osht
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu

NF, NS, LMAX, NB = 64, 16, 32, 4


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


@pytest.fixture(scope="module")
def kap():
    g = osht.alm2map(NF, LMAX, inputs.gaussian_alm(LMAX, seed=11, sigma=0.5))
    s = inputs.deflection_scale(LMAX, 0.5, alpha_rms=10 * inputs.ARCMIN)
    return s * (np.exp(g) - np.mean(np.exp(g)))


def domain(theta0, phi0, radius):
    """The bundles whose centres lie within `radius` of (theta0, phi0)."""
    z, ph, s = hp.pix2ang_nest(NB, np.arange(12 * NB * NB))
    c = hp.vec(np.cos(theta0), phi0)
    return np.nonzero(hp.vec(z, ph, s) @ c > np.cos(radius))[0]


def plans(clm, n, prec, vcyc, dom):
    kw = dict(nside_sht=NS, lmax=LMAX, nside_bundle=NB, patch_cells=n, mg_prec=prec,
              mg_vcycles=vcyc, mg_eps=0.1, mg_max_vcycles=12)
    full = clm.Plan(NF, **kw)
    part = clm.Plan(NF, **kw)
    part.set_domain(dom)
    return full, part


@pytest.mark.parametrize("n,prec,vcyc", [(64, "fp64", 3), (256, "fp32", 3), (256, "fp64", 0),
                                         (128, "fp32", 0)])
def test_domain_patches_equal_whole_sky(clm, kap, n, prec, vcyc):
    # a cap of about 1/6 of the sky that reaches the north pole
    dom = domain(0.35, 1.0, 0.8)
    assert 10 < dom.size < 60 and 15 in dom       # bundle 15 holds the north pole
    full, part = plans(clm, n, prec, vcyc, dom)
    k = torch.from_numpy(kap).cuda()
    full.poisson_solve(k)
    part.poisson_solve(k)
    for b in dom:
        assert torch.equal(part.patch_potential(int(b), 1), full.patch_potential(int(b), 1)), b
    ef, cf = (t.cpu().numpy() for t in full.mg_convergence())
    ep, cp = (t.cpu().numpy() for t in part.mg_convergence())
    out = np.setdiff1d(np.arange(12 * NB * NB), dom)
    np.testing.assert_array_equal(cp[dom], cf[dom])
    assert (cp[out] == 0).all() and np.isnan(ep[out]).all()
    if vcyc == 0:
        np.testing.assert_array_equal(ep[dom], ef[dom])
        assert (cp[dom] >= 1).all()
    # shear at every pixel: the domain's pixels as in the whole-sky run, the
    # others untouched
    npix = 12 * NF * NF
    for order in ("nested", "ring"):
        gf, hf = full.shear_at_pixels(order=order)
        g = torch.full((2, npix), 1234.5, dtype=torch.float64, device="cuda")
        h = torch.full((3, npix), 1234.5, dtype=torch.float64, device="cuda")
        part.shear_at_pixels(order=order, out=(g, h))
        nest = np.concatenate([b * (NF // NB) ** 2 + np.arange((NF // NB) ** 2) for b in dom])
        idx = nest if order == "nested" else hp.nest2ring(NF, nest)
        inside = np.zeros(npix, bool)
        inside[idx] = True
        g, h, gf, hf = (t.cpu().numpy() for t in (g, h, gf, hf))
        np.testing.assert_array_equal(g[:, inside], gf[:, inside])
        np.testing.assert_array_equal(h[:, inside], hf[:, inside])
        assert (g[:, ~inside] == 1234.5).all() and (h[:, ~inside] == 1234.5).all()
    full.sync_status()
    part.sync_status()
    full.close()
    part.close()


def test_domain_points_and_rays(clm, kap):
    dom = domain(2.2, 4.0, 0.9)
    full, part = plans(clm, 64, "fp64", 3, dom)
    k = torch.from_numpy(np.stack([kap, 0.7 * kap[::-1].copy()])).cuda()
    full.poisson_solve(k[:1])
    part.poisson_solve(k[:1])
    # points: inside the domain as in the whole-sky run; outside NaN, and the
    # plan latches CLM_ERAY_LEFT_PATCH
    rng = np.random.default_rng(4)
    th = np.arccos(rng.uniform(-1, 1, 400))
    ph = rng.uniform(0, 2 * np.pi, 400)
    b = hp.ang2pix_nest(NB, np.cos(th), ph)
    ins = np.isin(b, dom)
    assert 10 < ins.sum() < 390
    tt, pt = torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()
    gf, hf = (t.cpu().numpy() for t in full.shear_from_potential(tt, pt))
    gp, hp_ = (t.cpu().numpy() for t in part.shear_from_potential(tt, pt))
    np.testing.assert_array_equal(gp[:, ins], gf[:, ins])
    np.testing.assert_array_equal(hp_[:, ins], hf[:, ins])
    assert np.isnan(gp[:, ~ins]).all() and np.isnan(hp_[:, ~ins]).all()
    with pytest.raises(clm.ClmError) as ei:
        part.sync_status()
    assert ei.value.status == clm.CLM_ERAY_LEFT_PATCH
    full.sync_status()
    # rays through two planes: the domain's rays as in the whole-sky run,
    # the others still at their pixel centres
    chi = np.array([100.0, 200.0, 300.0])
    rf, rp = full.new_rays(), part.new_rays()
    r0 = part.new_rays()
    full.raytrace_planes(k, chi, 0, rf)
    part.raytrace_planes(k, chi, 0, rp)
    full.sync_status()
    part.sync_status()
    shift = 2 * int(np.log2(NF // NB))
    inb = np.isin(np.arange(12 * NF * NF) >> shift, dom)
    for key in ("theta", "phi", "beta", "A", "A_prev"):
        a, f, z = (x[key].cpu().numpy() for x in (rp, rf, r0))
        np.testing.assert_array_equal(a[..., inb], f[..., inb])
        np.testing.assert_array_equal(a[..., ~inb], z[..., ~inb])
    assert not np.array_equal(rp["theta"].cpu().numpy()[inb], r0["theta"].cpu().numpy()[inb])
    # the whole sky again
    part.set_domain(None)
    part.poisson_solve(k[:1])
    _, cp = part.mg_convergence()
    assert (cp.cpu().numpy() == 3).all()
    full.close()
    part.close()


def test_domain_patches_against_oracle(clm, kap):
    """Two patches of a domain (one of them the polar patch) against the
    oracle's patch solve."""
    dom = domain(0.35, 1.0, 0.8)
    spec = omg.PatchSpec(NF, NS, LMAX, NB, ncell=64, vcycles=3)
    sol = omg.solve_plane(spec, kap, [15, int(dom[-1])])
    _, part = plans(clm, 64, "fp64", 3, dom)
    part.poisson_solve(torch.from_numpy(kap).cuda())
    for b in (15, int(dom[-1])):
        pt = sol["patches"][b]
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = part.patch_potential(b, 1)[0].cpu().numpy()
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), b
    part.sync_status()
    part.close()


def test_domain_errors(clm):
    mg = clm.Plan(NF, nside_sht=NS, lmax=LMAX, nside_bundle=NB, patch_cells=64, adjoint=1,
                  mg_vcycles=2)
    for bad in ([192], [-1], [3, 500]):
        with pytest.raises(clm.ClmError) as ei:
            mg.set_domain(bad)
        assert ei.value.status == clm.CLM_EINVAL
    mg.set_domain([1, 2, 3])
    with pytest.raises(clm.ClmError) as ei:
        mg.poisson_adjoint()
    assert ei.value.status == clm.CLM_EUNSUPPORTED
    mg.set_domain([])
    mg.close()
    sht = clm.Plan(16, nside_sht=16, lmax=32, solver="sht")
    with pytest.raises(clm.ClmError) as ei:
        sht.set_domain([0])
    assert ei.value.status == clm.CLM_EUNSUPPORTED
    sht.close()
