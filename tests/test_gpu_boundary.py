"""GPU checks of the C ABI's error path and of its thinner entry points:
the non-finite latch, clm_galaxies_reduced against clm_galaxies_shell, the
timing filter and clm_plan_timings, and the autograd wrapper's gradient
shape.
Every kernel exits normally in these tests: the non-finite input is a host
tensor value, not a device fault."""
import numpy as np
import pytest
import torch

from oracle import sht as osht
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


def _kappa(N, lmax, seed=2, sigma=0.05):
    return osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=seed, sigma=sigma))


@pytest.mark.parametrize("mg_vcycles", [2, 0])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nan_pixel_latches_nonfinite(clm, mg_vcycles, dtype):
    """One NaN convergence pixel: the solve (fixed cycles, or the epsilon
    rule) runs to its end and the plan reports CLM_ENONFINITE; the latch is
    cleared by the report, and a clean solve afterwards reports nothing."""
    N = 64
    print("case: NaN pixel, vcycles %d, %s" % (mg_vcycles, dtype), flush=True)
    plan = clm.Plan(N, nside_sht=16, lmax=32, nside_bundle=4, patch_cells=64,
                    mg_vcycles=mg_vcycles, mg_max_vcycles=6, mg_prec="fp64")
    kap = torch.from_numpy(_kappa(N, 32)).to(dtype).cuda()
    bad = kap.clone()
    bad[1234] = float("nan")
    plan.poisson_solve(bad)
    g, h = plan.shear_at_pixels(order="ring")
    with pytest.raises(clm.ClmError) as ei:
        plan.sync_status()
    assert ei.value.status == clm.CLM_ENONFINITE
    assert not torch.isfinite(g).all()
    plan.sync_status()                 # the report cleared the latch
    plan.poisson_solve(kap)
    g, h = plan.shear_at_pixels(order="ring")
    plan.sync_status()
    assert torch.isfinite(g).all() and torch.isfinite(h).all()
    plan.close()


def test_infinite_pixel_latches_nonfinite(clm):
    N = 32
    plan = clm.Plan(N, nside_sht=N, lmax=2 * N, solver="sht")
    kap = torch.from_numpy(_kappa(N, 2 * N)).cuda()
    kap[7] = float("inf")
    plan.poisson_solve(kap)
    with pytest.raises(clm.ClmError) as ei:
        plan.sync_status()
    assert ei.value.status == clm.CLM_ENONFINITE
    plan.close()


def test_galaxies_entry_matches_shell_call(clm):
    """clm_galaxies_reduced (distances of the latest ray update kept by the
    plan) gives bit-identical A_g to clm_galaxies_shell with the shell passed
    explicitly, plane after plane; before any ray update it is rejected."""
    Nf, lmax = 64, 32
    chi = np.array([(m + 0.5) * 100.0 for m in range(3)] + [350.0])
    plan = clm.Plan(Nf, nside_sht=16, lmax=lmax, nside_bundle=4, patch_cells=64,
                    mg_vcycles=2, mg_prec="fp64")
    rays = plan.new_rays()
    th, ph = (torch.from_numpy(a).cuda() for a in inputs.uniform_sphere(4000, seed=31))
    gchi = torch.from_numpy(np.random.default_rng(32).uniform(1.0, 349.0, 4000)).cuda()
    gal1 = dict(theta=th, phi=ph, chi=gchi,
                A=torch.full((4, 4000), np.nan, dtype=torch.float32, device="cuda"))
    gal2 = dict(gal1, A=gal1["A"].clone())
    with pytest.raises(clm.ClmError) as ei:
        plan.galaxies(rays, gal1)
    assert ei.value.status == clm.CLM_EINVAL
    for m in range(3):
        k = torch.from_numpy(_kappa(Nf, lmax, seed=40 + m, sigma=0.02)).cuda()
        plan.poisson_solve(k)
        plan.ray_update(chi, m, rays)
        plan.galaxies(rays, gal1)
        plan.galaxies_shell(chi, m + 1, rays, gal2)
    plan.sync_status()
    # bitwise equal, the untouched shell-0 galaxies NaN in both
    assert torch.allclose(gal1["A"], gal2["A"], rtol=0.0, atol=0.0, equal_nan=True)
    # every galaxy beyond shell 0 got its Jacobian
    done = torch.isfinite(gal1["A"]).all(0)
    assert done.sum().item() == (gchi >= 100.0).sum().item()
    plan.close()


def test_timing_filter_and_plan_timings(clm):
    N = 64
    plan = clm.Plan(N, nside_sht=16, lmax=32, nside_bundle=4, patch_cells=64, mg_vcycles=2)
    kap = torch.from_numpy(_kappa(N, 32)).cuda()
    plan.set_timing(True)
    plan.get_timing()
    plan.poisson_solve(kap)
    every = plan.get_timing()
    assert "patch_setup" in every and "mean" in every
    plan.set_timing(True, stages=["patch_setup"])
    plan.poisson_solve(kap)
    only = plan.get_timing()
    assert only["patch_setup"][1] == every["patch_setup"][1]
    assert all(v[1] == 0 for k, v in only.items() if k != "patch_setup")
    plan.set_timing(True)
    plan.poisson_solve(kap)
    t = plan.timings()
    assert set(t) >= set(every) and all(v >= 0.0 for v in t.values())
    assert t["patch_setup"] > 0.0
    plan.set_timing(False)
    plan.close()


def test_autograd_two_dimensional_kappa(clm):
    """A [1, npix] convergence gets a gradient of its own shape."""
    N = 32
    plan = clm.Plan(N, nside_sht=8, lmax=16, nside_bundle=4, patch_cells=64, mg_vcycles=2,
                    mg_prec="fp64", adjoint=1)
    rng = np.random.default_rng(5)
    kap = torch.from_numpy(0.01 * rng.standard_normal((1, 12 * N * N))).cuda()
    kap.requires_grad_(True)
    th, ph = (torch.from_numpy(a).cuda() for a in inputs.uniform_sphere(200, seed=6))
    g, h = clm.PoissonShearFn.apply(kap, th, ph, plan)
    (h[0] - h[1]).pow(2).sum().backward()
    assert kap.grad.shape == kap.shape
    # the same gradient as for the flat map
    kap1 = kap.detach().reshape(-1).clone().requires_grad_(True)
    g1, h1 = clm.PoissonShearFn.apply(kap1, th, ph, plan)
    (h1[0] - h1[1]).pow(2).sum().backward()
    # the transposed scatter adds with atomics, so the order of its sums
    # (and the last bits) may differ between calls
    gmax = float(kap1.grad.abs().max())
    assert gmax > 0.0
    assert float((kap.grad.reshape(-1) - kap1.grad).abs().max()) <= 1e-12 * gmax
    plan.sync_status()
    plan.close()
