"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU
oracle on the same seeded inputs, element by element.

Tolerances: float64 paths agree to 1e-10 relative (the target for the FP64
form); the float32 multigrid form agrees to 1e-6 relative on the potential
u0 + du; float32 ray Jacobians (stored in float32 after every plane) to
2e-6 absolute after a few planes."""
import numpy as np
import pytest
import torch

from oracle import healpix as hp
from oracle import mg as omg
from oracle import rays as orays
from oracle import sht as osht
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def report(tag, value):
    print("PARITY %s %.3e" % (tag, value), flush=True)
    return value


# ---------------------------------------------------------------- pure SHT
@pytest.fixture(scope="module")
def c1_case():
    N, lmax = 64, 128
    alm = inputs.gaussian_alm(lmax, seed=1, amplitude=1.0)
    kap = osht.alm2map(N, lmax, alm)
    # the solve demeans the map first (the l = 0 term is set to zero, and
    # HEALPix quadrature of a constant is not exactly l = 0)
    palm = osht.poisson(lmax, osht.map2alm(N, lmax, kap - kap.mean()))
    return dict(N=N, lmax=lmax, alm=alm, kap=kap, palm=palm,
                psi=osht.alm2map(N, lmax, palm), der=osht.derivative_maps(N, lmax, palm))


def test_alm2map_parity(clm, c1_case):
    c = c1_case
    a = torch.from_numpy(c["alm"]).cuda()
    m = clm.alm2map(a, c["lmax"], c["N"]).cpu().numpy()
    assert rel(m, c["kap"]) < 1e-12


def test_alm2map_ragged_lmax(clm):
    # lmax not tied to nside, above and below 2 N, and ring lengths shorter
    # than lmax + 1 (aliasing)
    for N, lmax in [(4, 37), (16, 7), (8, 16)]:
        alm = inputs.gaussian_alm(lmax, seed=N + lmax, amplitude=1.0)
        ref = osht.alm2map(N, lmax, alm)
        got = clm.alm2map(torch.from_numpy(alm).cuda(), lmax, N).cpu().numpy()
        assert rel(got, ref) < 1e-12, (N, lmax)


@pytest.mark.parametrize("N,lmax", [(256, 300), (512, 200), (1024, 48)])
def test_ring_transforms_long_odd_rings(clm, N, lmax):
    """Polar-cap rings of 4i samples whose odd factor exceeds the direct-DFT
    limit go through the chirp (Bluestein) transform: synthesis (inverse
    ring transforms) and analysis + Poisson (forward) against the oracle,
    whose ring DFTs are plain FFTs of each ring."""
    alm = inputs.gaussian_alm(lmax, seed=N + lmax, amplitude=1.0)
    ref = osht.alm2map(N, lmax, alm)
    got = clm.alm2map(torch.from_numpy(alm).cuda(), lmax, N).cpu().numpy()
    assert report("ring_inverse N=%d lmax=%d" % (N, lmax), rel(got, ref)) < 1e-12
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht")
    plan.poisson_solve(torch.from_numpy(ref).cuda())
    palm = osht.poisson(lmax, osht.map2alm(N, lmax, ref - ref.mean()))
    assert report("ring_forward N=%d lmax=%d" % (N, lmax),
                  rel(plan.psi_alm().cpu().numpy(), palm)) < 1e-10
    plan.sync_status()
    plan.close()


def test_sht_poisson_parity(clm, c1_case):
    c = c1_case
    plan = clm.Plan(c["N"], nside_sht=c["N"], lmax=c["lmax"], solver="sht")
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    assert rel(plan.psi_alm().cpu().numpy(), c["palm"]) < 1e-10
    assert rel(plan.psi_map().cpu().numpy(), c["psi"]) < 1e-10
    g, h = plan.shear_at_pixels(order="ring")
    g, h = g.cpu().numpy(), h.cpu().numpy()
    d = c["der"]
    assert rel(g[0], d["g_t"]) < 1e-10 and rel(g[1], d["g_p"]) < 1e-10
    assert rel(h[0], d["U_tt"]) < 1e-10 and rel(h[1], d["U_pp"]) < 1e-10
    assert rel(h[2], d["U_tp"]) < 1e-10
    gn, hn = plan.shear_at_pixels(order="nested", fp64=False)
    r = hp.nest2ring(c["N"], np.arange(12 * c["N"] ** 2))
    assert rel(hn.cpu().numpy()[0], d["U_tt"][r]) < 1e-6
    plan.sync_status()
    plan.close()


def test_sht_analysis_refinement(clm):
    """Jacobi refinement of the analysis (a <- a + A(f - S a)) against the
    oracle's map2alm with the same number of iterations; on a band-limited
    map (lmax <= Nside) it drives the quadrature error down."""
    N, lmax = 16, 16
    alm = inputs.gaussian_alm(lmax, seed=7, amplitude=1.0)
    m = osht.alm2map(N, lmax, alm)
    m = m - m.mean()
    for iters in (0, 3):
        plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", analysis_iters=iters)
        plan.poisson_solve(torch.from_numpy(m).cuda())
        ref = osht.poisson(lmax, osht.map2alm(N, lmax, m, iters=iters))
        got = plan.psi_alm().cpu().numpy()
        assert report("sht_refine iters=%d" % iters, rel(got, ref)) < 1e-10
        exact = osht.poisson(lmax, osht.map2alm(N, lmax, m, iters=12))
        if iters == 0:
            e0 = rel(got, exact)
        else:
            assert rel(got, exact) < e0 / 100, (rel(got, exact), e0)
        plan.sync_status()
        plan.close()


def test_sht_float32_input_and_batch(clm):
    N, lmax = 16, 32
    maps = [osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=40 + i, amplitude=1.0))
            for i in range(3)]
    k = torch.from_numpy(np.stack(maps)).float().cuda()
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=3)
    plan.poisson_solve(k)
    for i in range(3):
        m32 = maps[i].astype(np.float32).astype(np.float64)
        ref = osht.poisson(lmax, osht.map2alm(N, lmax, m32 - m32.mean()))
        assert rel(plan.psi_alm(i).cpu().numpy(), ref) < 1e-10
    plan.close()


@pytest.mark.parametrize("form,tol", [("fp32", 5e-6), ("bf16x3", 1e-4), ("bf16x6", 5e-6)])
def test_sht_batched_matrix_core_forms(clm, form, tol):
    """Planes batched as GEMM columns (ragged: 5 planes), Legendre transforms
    on the matrix cores, against the FP64 oracle plane by plane."""
    N, lmax, P = 16, 40, 5
    maps = [osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=60 + i, amplitude=1.0))
            for i in range(P)]
    k = torch.from_numpy(np.stack(maps)).cuda()
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P, legendre_prec=form)
    plan.poisson_solve(k)
    for i in range(P):
        ref = osht.poisson(lmax, osht.map2alm(N, lmax, maps[i] - maps[i].mean()))
        e_alm = rel(plan.psi_alm(i).cpu().numpy(), ref)
        e_map = rel(plan.psi_map(i).cpu().numpy(), osht.alm2map(N, lmax, ref))
        print("PARITY sht_%s plane %d alm %.3e map %.3e" % (form, i, e_alm, e_map), flush=True)
        assert e_alm < tol and e_map < tol, (form, i, e_alm, e_map)
    plan.sync_status()
    plan.close()


def test_sht_matrix_core_several_batches(clm):
    """18 planes: one full GEMM batch of 16 and a ragged batch of 2, each
    plane against the FP64 oracle (the kappa offset and slot of the second
    batch)."""
    N, lmax, P = 16, 40, 18
    maps = [osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=90 + i, amplitude=1.0))
            for i in range(P)]
    k = torch.from_numpy(np.stack(maps)).cuda()
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P, legendre_prec="fp32")
    plan.poisson_solve(k)
    worst = 0.0
    for i in range(P):
        ref = osht.poisson(lmax, osht.map2alm(N, lmax, maps[i] - maps[i].mean()))
        e = rel(plan.psi_alm(i).cpu().numpy(), ref)
        worst = max(worst, e)
        assert e < 5e-6, (i, e)
    report("sht_fp32 18 planes", worst)
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("N", [512, 1024])
def test_sht_matrix_core_large_against_fp64(clm, N):
    """Full-size ring counts (one ring block at Nside 512; two blocks whose
    partial sums are reduced at Nside 1024): the matrix-core forms against
    the FP64 GPU form, 3 planes, max-norm relative error of the psi map
    (the oracle comparison at Nside 512 is in the full-size tests)."""
    lmax, P = 2 * N, 3
    alm = [torch.from_numpy(inputs.gaussian_alm(lmax, seed=70 + i, amplitude=1.0)).cuda()
           for i in range(P)]
    k = torch.stack([clm.alm2map(a, lmax, N) for a in alm])
    ref = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P)
    ref.poisson_solve(k)
    for form, tol in (("fp32", 2e-5), ("bf16x3", 1e-3), ("bf16x6", 2e-5)):
        plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P,
                        legendre_prec=form)
        plan.poisson_solve(k)
        for i in range(P):
            e = rel(plan.psi_map(i).cpu().numpy(), ref.psi_map(i).cpu().numpy())
            print("PARITY sht_%s N=%d plane %d map %.3e" % (form, N, i, e), flush=True)
            assert e < tol, (form, N, i, e)
        plan.sync_status()
        plan.close()
    ref.close()


# ---------------------------------------------------------------- SHT + MG
# 15 and 128 hold the north and south poles (their patches contain them)
MG_BUNDLES = [0, 15, 37, 100, 128, 191]


@pytest.fixture(scope="module")
def mg_case():
    Nf, Ns, lmax, Nb = 64, 16, 32, 4
    g = osht.alm2map(Nf, lmax, inputs.gaussian_alm(lmax, seed=3, sigma=0.5))
    kap = np.exp(g) - np.mean(np.exp(g))
    out = dict(Nf=Nf, Ns=Ns, lmax=lmax, Nb=Nb, kap=kap)
    for n in (64, 256):
        spec = omg.PatchSpec(Nf, Ns, lmax, Nb, ncell=n, vcycles=3)
        out[n] = (spec, omg.solve_plane(spec, kap, MG_BUNDLES))
    return out


@pytest.mark.parametrize("n", [64, 256])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mg_patch_potential_parity(clm, mg_case, n, prec):
    c = mg_case
    spec, sol = c[n]
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    assert rel(plan.psi_alm().cpu().numpy(), sol["psi_alm"]) < 1e-10
    assert rel(plan.psi_map().cpu().numpy(), sol["psi_sht"]) < 1e-10
    tol_u = 1e-10 if prec == "fp64" else 1e-6
    for b in MG_BUNDLES:
        pt = sol["patches"][b]
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("mg_u n=%d %s b=%d" % (n, prec, b), rel(got, ref)) < tol_u, b
        # the correction itself (u - u0) to float32 rounding in the fp32 form
        dref = pt["du"][1:-1, 1:-1]
        dgot = got - pt["u0"][1:-1, 1:-1]
        assert report("mg_du n=%d %s b=%d" % (n, prec, b), rel(dgot, dref)) < \
            (1e-8 if prec == "fp64" else 2e-4), b
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mg_wide_patch_global_ring_tables(clm, prec):
    """Setup tiles whose region spans more rings than a block's LDS ring
    stores hold (256 of the fine grid) interpolate from the global ring
    tables.  Patches of about 1 rad (bundles at Nside 2, patch factor 2) on
    a Nside 512 fine grid span some 700 fine rings each."""
    Nf, Ns, lmax, Nb, n = 512, 32, 64, 2, 64
    g = osht.alm2map(Nf, lmax, inputs.gaussian_alm(lmax, seed=5, sigma=0.5))
    kap = np.exp(g) - np.mean(np.exp(g))
    spec = omg.PatchSpec(Nf, Ns, lmax, Nb, factor=2, ncell=n, vcycles=2)
    bl = [5, 20]
    sol = omg.solve_plane(spec, kap, bl)
    rt = hp.ring_table(Nf)
    for b in bl:
        th, _ = omg.patch_cell_dirs(spec, sol["patches"][b]["R"])
        z = np.cos(th)
        assert np.sum((rt["z"] >= z.min()) & (rt["z"] <= z.max())) > 256
    plan = clm.Plan(Nf, nside_sht=Ns, lmax=lmax, nside_bundle=Nb, patch_factor=2,
                    patch_cells=n, mg_vcycles=2, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(kap).cuda())
    tol_u = 1e-10 if prec == "fp64" else 1e-6
    for b in bl:
        pt = sol["patches"][b]
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("wide patch %s b=%d" % (prec, b), rel(got, ref)) < tol_u, b
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("kdtype", [np.float64, np.float32])
def test_mg_setup_azimuth_wrap(clm, mg_case, kdtype):
    """Patches across the azimuth phi = 0 of the RING order (bundles 64 to
    67): the setup's interpolation reads both maps across the end of every
    ring, in both map precisions."""
    c = mg_case
    n, bl = 64, [64, 65, 66, 67]
    kap = c["kap"].astype(kdtype)
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], ncell=n, vcycles=3)
    sol = omg.solve_plane(spec, kap.astype(np.float64), bl)
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec="fp64")
    plan.poisson_solve(torch.from_numpy(kap).cuda())
    for b in bl:
        pt = sol["patches"][b]
        _, ph = omg.patch_cell_dirs(spec, pt["R"])
        assert ph.min() < 0.05 and ph.max() > 2 * np.pi - 0.05, b
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("azimuth wrap %s b=%d" % (np.dtype(kdtype).name, b), rel(got, ref)) < \
            1e-10, b
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mg_float32_kappa_input(clm, mg_case, prec):
    """A float32 convergence map (the input type of the Nside 2048 workload):
    the mean, the degrade to the SHT grid and the setup's fine-map gathers
    read float32; the oracle takes the same values widened to float64."""
    c = mg_case
    n = 64
    k32 = c["kap"].astype(np.float32)
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], ncell=n, vcycles=3)
    sol = omg.solve_plane(spec, k32.astype(np.float64), MG_BUNDLES[:3])
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(k32).cuda())
    assert rel(plan.psi_alm().cpu().numpy(), sol["psi_alm"]) < 1e-10
    tol_u = 1e-10 if prec == "fp64" else 1e-6
    for b in MG_BUNDLES[:3]:
        pt = sol["patches"][b]
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("mg_u float32 kappa %s b=%d" % (prec, b), rel(got, ref)) < tol_u, b
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("nu", [(1, 3), (3, 1), (1, 1), (4, 4)])
def test_mg_sweep_counts(clm, mg_case, nu):
    """Other (nu_pre, nu_post) than (2, 2) on a tiled finest level (n = 128):
    fused post + pre smoothing when nu_pre + nu_post <= 4 (halo 2 (nu_pre +
    nu_post) + 2), separate pre and post tiles otherwise; FP64 against the
    oracle."""
    c = mg_case
    n = 128
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], ncell=n, nu1=nu[0], nu2=nu[1],
                         vcycles=3)
    bl = MG_BUNDLES[1:4]
    sol = omg.solve_plane(spec, c["kap"], bl)
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec="fp64", nu_pre=nu[0], nu_post=nu[1])
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    for b in bl:
        pt = sol["patches"][b]
        dref = pt["du"][1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        e = rel(got - pt["u0"][1:-1, 1:-1], dref)
        assert report("mg_du nu=%s b=%d" % (nu, b), e) < 1e-8, b
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mg_three_tile_levels(clm, mg_case, prec):
    """n = 512: levels 512, 256 and 128 streamed as tiles (level 2 keeps its
    own source and second iterate), 64 and below in LDS."""
    c = mg_case
    n = 512
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], ncell=n, vcycles=2)
    bl = [37, 100]
    sol = omg.solve_plane(spec, c["kap"], bl)
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=2, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    for b in bl:
        pt = sol["patches"][b]
        ref = (pt["u0"] + pt["du"])[1:-1, 1:-1]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("mg_u n=512 %s b=%d" % (prec, b), rel(got, ref)) < \
            (1e-10 if prec == "fp64" else 1e-6), b
        e = rel(got - pt["u0"][1:-1, 1:-1], pt["du"][1:-1, 1:-1])
        assert report("mg_du n=512 %s b=%d" % (prec, b), e) < (1e-8 if prec == "fp64" else 2e-4)
    plan.sync_status()
    plan.close()


def test_mg_fp32_form_tracks_fp64_form(clm, mg_case):
    """The float32 multigrid form at 4 V-cycles of (2, 2) sweeps, where the
    finest level's post- and pre-smoothing run fused, against the float64
    form on the same plane.  u0 is float64 in both forms, so they differ
    only through the float32 correction du = u - u0 (u0 from the oracle):
    float32 rounding, well below the bound, which exposes kernel-level errors
    that the looser oracle tolerance of the float32 form would let through."""
    c = mg_case
    spec, sol = c[256]
    kap = torch.from_numpy(c["kap"]).cuda()
    du = {}
    for prec in ("fp32", "fp64"):
        plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                        patch_cells=256, mg_vcycles=4, mg_prec=prec)
        plan.poisson_solve(kap)
        du[prec] = np.stack([plan.patch_potential(b, 1)[0].cpu().numpy() -
                             sol["patches"][b]["u0"][1:-1, 1:-1] for b in MG_BUNDLES])
        plan.sync_status()
        plan.close()
    e = report("mg_du fp32 form vs fp64 form (4 cycles, fused)", rel(du["fp32"], du["fp64"]))
    assert e < 1e-5


@pytest.mark.parametrize("n,prec,eps", [(64, "fp64", 1e-3), (256, "fp64", 5e-4),
                                         (64, "fp32", 1e-2), (256, "fp32", 1e-2)])
def test_mg_eps_rule_parity(clm, mg_case, n, prec, eps):
    """The Sec. 3.2 stopping rule per patch: the number of V-cycles each
    patch runs and its final epsilon match the oracle's mg_solve_eps (the
    thresholds sit between the oracle's per-cycle values, at least a factor
    1.3 from each), and the correction matches the oracle's after that many
    cycles."""
    c = mg_case
    spec, sol = c[n]
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=0, mg_eps=eps, mg_max_vcycles=20,
                    mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    plan.sync_status()
    e_gpu, k_gpu = (t.cpu().numpy() for t in plan.mg_convergence())
    assert np.all((k_gpu >= 1) & (k_gpu <= 20)) and np.all(e_gpu < eps)
    tol_e = 1e-9 if prec == "fp64" else 2e-2
    for b in MG_BUNDLES:
        pt = sol["patches"][b]
        du, k, hist = omg.mg_solve_eps(spec, pt["fp"], eps, 20)
        assert all(h > 1.3 * eps or h < eps / 1.3 for h in hist), hist
        report("mg_eps n=%d %s b=%d cycles %d/%d eps" % (n, prec, b, k_gpu[b], k),
               abs(e_gpu[b] - hist[-1]) / hist[-1])
        assert k_gpu[b] == k, (b, k_gpu[b], k)
        assert abs(e_gpu[b] - hist[-1]) <= tol_e * hist[-1], (b, e_gpu[b], hist[-1])
        got = plan.patch_potential(b, 1)[0].cpu().numpy() - pt["u0"][1:-1, 1:-1]
        assert report("mg_eps_du n=%d %s b=%d" % (n, prec, b), rel(got, du[1:-1, 1:-1])) < \
            (1e-8 if prec == "fp64" else 2e-4), b
    plan.close()


def test_mg_eps_rule_not_converged_and_fixed_count(clm, mg_case):
    """A patch still above mg_eps after mg_max_vcycles latches ENOTCONV,
    with the epsilon of its last cycle reported; a fixed cycle count reports
    that count and leaves epsilon unmeasured (NaN)."""
    c = mg_case
    spec, sol = c[256]
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=256, mg_vcycles=0, mg_eps=1e-6, mg_max_vcycles=2,
                    mg_prec="fp64")
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    with pytest.raises(clm.ClmError) as ei:
        plan.sync_status()
    assert ei.value.status == clm.CLM_ENOTCONV
    e_gpu, k_gpu = (t.cpu().numpy() for t in plan.mg_convergence())
    assert np.all(k_gpu == 2)
    for b in MG_BUNDLES:
        _, _, hist = omg.mg_solve_eps(spec, sol["patches"][b]["fp"], 1e-6, 2)
        assert abs(e_gpu[b] - hist[-1]) <= 1e-9 * hist[-1], (b, e_gpu[b], hist)
    plan.sync_status()  # the latched condition was cleared
    plan.close()
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=256, mg_vcycles=3)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    plan.sync_status()
    e_gpu, k_gpu = (t.cpu().numpy() for t in plan.mg_convergence())
    assert np.all(k_gpu == 3) and np.all(np.isnan(e_gpu))
    plan.close()


@pytest.mark.parametrize("n", [8, 16])
def test_mg_smallest_patches(clm, mg_case, n):
    """The smallest patches (8^2 and 16^2: two and three levels, all in LDS)
    against the oracle, polar bundles included."""
    c = mg_case
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], ncell=n, vcycles=3)
    sol = omg.solve_plane(spec, c["kap"], MG_BUNDLES)
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec="fp64")
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    for b in MG_BUNDLES:
        pt = sol["patches"][b]
        got = plan.patch_potential(b, 1)[0].cpu().numpy()
        assert report("mg_small n=%d b=%d" % (n, b), rel(got, (pt["u0"] + pt["du"])[1:-1, 1:-1])) < 1e-10
    plan.sync_status()
    plan.close()


def test_degenerate_inputs(clm):
    """A constant convergence has no potential and no shear: the SHT side is
    exactly zero (the monopole is removed exactly), the patch side is zero
    up to the rounding of the interpolation weights' sum; empty point and
    galaxy sets are valid no-ops."""
    N = 64
    plan = clm.Plan(N, nside_sht=16, lmax=32, nside_bundle=4, patch_cells=64, mg_vcycles=2)
    k = torch.full((12 * N * N,), 0.37, dtype=torch.float32, device="cuda")
    plan.poisson_solve(k)
    assert torch.count_nonzero(plan.psi_alm()).item() == 0
    assert torch.count_nonzero(plan.psi_map()).item() == 0
    assert plan.patch_potential(0, 192).abs().max().item() < 1e-15
    g, h = plan.shear_at_pixels(order="ring")
    assert g.abs().max().item() < 1e-10 and h.abs().max().item() < 1e-10
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    g0, h0 = plan.shear_from_potential(e, e)
    assert g0.shape == (2, 0) and h0.shape == (3, 0)
    rays = plan.new_rays()
    gal = dict(theta=e, phi=e, chi=e, A=torch.empty(4, 0, dtype=torch.float32, device="cuda"))
    plan.galaxies_shell(np.array([100.0, 200.0]), 0, rays, gal)
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mg_shear_parity(clm, mg_case, prec):
    c = mg_case
    n = 256
    spec, sol = c[n]
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=n, mg_vcycles=3, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    gN, hN = plan.shear_at_pixels(order="nested")
    gR, hR = plan.shear_at_pixels(order="ring", fp64=False)
    rng = np.random.default_rng(9)
    th, ph = [], []
    for b in MG_BUNDLES:
        # random points well inside the bundle: perturb pixel centres
        pix = b * 256 + rng.integers(0, 256, 8)
        z, p, s = hp.pix2ang_nest(c["Nf"], pix)
        t = np.arctan2(s, z) + rng.uniform(-2e-3, 2e-3, 8)
        pp = p + rng.uniform(-2e-3, 2e-3, 8)
        keep = hp.ang2pix_nest(c["Nb"], np.cos(t), pp) == b
        th.append(t[keep])
        ph.append(pp[keep])
    th, ph = np.concatenate(th), np.concatenate(ph)
    gP, hP = plan.shear_from_potential(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda())
    plan.sync_status()
    gN, hN, gR, hR = (x.cpu().numpy() for x in (gN, hN, gR, hR))
    gP, hP = gP.cpu().numpy(), hP.cpu().numpy()
    tol = 1e-9 if prec == "fp64" else 2e-4
    r2n = hp.ring2nest(c["Nf"], np.arange(12 * c["Nf"] ** 2))
    for b in MG_BUNDLES:
        pt = sol["patches"][b]
        for p in range(b * 256, (b + 1) * 256, 13):
            z, phh, s = hp.pix2ang_nest(c["Nf"], np.array([p]))
            gr, Ur = omg.eval_point(spec, pt, np.arctan2(s[0], z[0]), phh[0])
            ur = np.array([Ur[0, 0], Ur[1, 1], Ur[0, 1]])
            scale_g, scale_u = np.abs(gr).max(), np.abs(ur).max()
            assert np.abs(gN[:, p] - gr).max() < tol * scale_g, (b, p)
            assert np.abs(hN[:, p] - ur).max() < tol * scale_u, (b, p)
            rp = hp.nest2ring(c["Nf"], np.array([p]))[0]
            assert r2n[rp] == p
            assert np.abs(hR[:, rp] - ur).max() < max(tol, 2e-6) * scale_u
    for k in range(th.size):
        b = omg.bundle_of(spec, th[k], ph[k])
        gr, Ur = omg.eval_point(spec, sol["patches"][b], th[k], ph[k])
        ur = np.array([Ur[0, 0], Ur[1, 1], Ur[0, 1]])
        assert np.abs(gP[:, k] - gr).max() < tol * np.abs(gr).max()
        assert np.abs(hP[:, k] - ur).max() < tol * np.abs(ur).max()
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shear_edge_stencils(clm, mg_case, prec):
    """Points in the outer two cell rows / columns of a patch take the
    one-sided stencils (Sec. 3.2).  With patch factor 1 (patch = bundle) the
    bundle's corners reach the patch faces, so points along the patch axes
    close to a face still belong to the bundle whose patch holds them."""
    c = mg_case
    n, bl = 64, [37, 100]
    spec = omg.PatchSpec(c["Nf"], c["Ns"], c["lmax"], c["Nb"], factor=1, ncell=n, vcycles=2)
    sol = omg.solve_plane(spec, c["kap"], bl)
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_factor=1, patch_cells=n, mg_vcycles=2, mg_prec=prec)
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    mid = n / 2 - 0.5
    # fractional cell coordinates (fi, fj): first / last two cells of each
    # axis, the other coordinate near the middle
    near = [0.2, 0.7, 1.4, 2.6]
    fij = [(f, mid + 0.3) for f in near] + [(n - 2 - f, mid - 0.4) for f in near] + \
          [(mid + 0.2, f) for f in near] + [(mid - 0.3, n - 2 - f) for f in near]
    th, ph, owner, cells = [], [], [], []
    for b in bl:
        R = sol["patches"][b]["R"]
        for fi, fj in fij:
            thp = np.pi / 2 - spec.L / 2 + (fi + 0.5) * spec.delta
            php = -spec.L / 2 + (fj + 0.5) * spec.delta
            t, p = omg.patch_dirs(spec, R, thp, php)
            t, p = float(t), float(p) % (2 * np.pi)
            if omg.bundle_of(spec, t, p) != b:
                continue
            th.append(t)
            ph.append(p)
            owner.append(b)
            cells.append((int(np.floor(fi)), int(np.floor(fj))))
    # the set must reach the one-sided stencils on every face
    i0s, j0s = [cc[0] for cc in cells], [cc[1] for cc in cells]
    assert min(i0s) <= 1 and max(i0s) >= n - 3 and min(j0s) <= 1 and max(j0s) >= n - 3
    gP, hP = plan.shear_from_potential(torch.tensor(th, dtype=torch.float64, device="cuda"),
                                       torch.tensor(ph, dtype=torch.float64, device="cuda"))
    plan.sync_status()
    gP, hP = gP.cpu().numpy(), hP.cpu().numpy()
    tol = 1e-9 if prec == "fp64" else 2e-4
    worst = 0.0
    for k, b in enumerate(owner):
        gr, Ur = omg.eval_point(spec, sol["patches"][b], th[k], ph[k])
        ur = np.array([Ur[0, 0], Ur[1, 1], Ur[0, 1]])
        eg = np.abs(gP[:, k] - gr).max() / np.abs(gr).max()
        eu = np.abs(hP[:, k] - ur).max() / np.abs(ur).max()
        worst = max(worst, eg, eu)
        assert eg < tol and eu < tol, (b, cells[k], eg, eu)
    report("shear_edge %s" % prec, worst)
    plan.close()


def test_points_outside_patch_are_flagged(clm, mg_case):
    c = mg_case
    plan = clm.Plan(c["Nf"], nside_sht=c["Ns"], lmax=c["lmax"], nside_bundle=c["Nb"],
                    patch_cells=64, mg_vcycles=1, mg_prec="fp64")
    plan.poisson_solve(torch.from_numpy(c["kap"]).cuda())
    # empty request is fine
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    plan.shear_from_potential(e, e)
    plan.sync_status()
    # rays pushed far from their bundle leave the patch: NaN and a latched status
    rays = plan.new_rays()
    rays["phi"] += 1.0
    chi = np.array([100.0, 200.0])
    plan.ray_update(chi, 0, rays)
    with pytest.raises(clm.ClmError) as ei:
        plan.sync_status()
    assert ei.value.status == clm.CLM_ERAY_LEFT_PATCH
    assert torch.isnan(rays["A"]).any()
    plan.sync_status()   # cleared
    plan.close()


# ---------------------------------------------------------------- rays
def test_raytrace_parity(clm):
    """Five planes; sample rays of four bundles, two of them the bundles at
    the poles (15 and 128), against the oracle's ray steps; galaxies of
    those bundles against eq. gatraj with the oracle's ray Jacobians."""
    Nf, Ns, lmax, Nb, n = 64, 16, 32, 4, 64
    nplanes = 5
    chi = np.array([(m + 0.5) * 100.0 for m in range(nplanes)] + [nplanes * 100.0 + 50.0])
    kaps = []
    for m in range(nplanes):
        sig = 0.2 + 0.2 * m
        g = osht.alm2map(Nf, lmax, inputs.gaussian_alm(lmax, seed=100 + m, sigma=sig))
        s = inputs.deflection_scale(lmax, sig, alpha_rms=20 * inputs.ARCMIN)
        kaps.append(s * (np.exp(g) - np.mean(np.exp(g))))
    kaps = np.stack(kaps)
    bundles = [5, 15, 77, 128]
    spec = omg.PatchSpec(Nf, Ns, lmax, Nb, ncell=n, vcycles=4)
    sols = [omg.solve_plane(spec, kaps[m], bundles) for m in range(nplanes)]

    # galaxies inside the two bundles, spread over the shells
    rng = np.random.default_rng(200)
    gth, gph, gchi = [], [], []
    for b in bundles:
        pix = b * 256 + rng.integers(0, 256, 6)
        z, p, s = hp.pix2ang_nest(Nf, pix)
        gth.append(np.arctan2(s, z) + rng.uniform(-3e-3, 3e-3, 6))
        gph.append(p + rng.uniform(-3e-3, 3e-3, 6))
        gchi.append(rng.uniform(10.0, chi[-1] + 40.0, 6))
    gth, gph, gchi = map(np.concatenate, (gth, gph, gchi))
    # keep galaxies whose four interpolation pixels lie in the two bundles
    gpix, gw = hp.interp_weights(Nf, gth, gph)
    r2n = hp.ring2nest(Nf, np.arange(12 * Nf * Nf))
    inside = np.all(np.isin(r2n[gpix] >> 8, bundles), axis=0)
    gth, gph, gchi, gpix, gw = gth[inside], gph[inside], gchi[inside], gpix[:, inside], gw[:, inside]
    assert gth.size >= 6
    # rays the oracle must follow: sample rays of the bundles plus each
    # galaxy's four interpolation pixels
    need = set(int(r2n[q]) for q in gpix.ravel())
    need |= set(int(b * 256 + k) for b in bundles for k in range(0, 256, 29))
    need = sorted(q for q in need if (q >> 8) in bundles)
    ref = {}
    for q in need:
        z, p, s = hp.pix2ang_nest(Nf, np.array([q]))
        r = orays.Ray(np.arctan2(s[0], z[0]), p[0])
        hist = []
        for m in range(nplanes):
            th, ph = hp.vec2ang(r.n)
            gr, Ur = omg.eval_point(spec, sols[m]["patches"][q >> 8], th, ph)
            orays.ray_step(r, chi, m, gr, Ur)
            hist.append((r.A.copy(), r.A_prev.copy()))
        ref[q] = (r, hist)

    plan = clm.Plan(Nf, nside_sht=Ns, lmax=lmax, nside_bundle=Nb, patch_cells=n,
                    mg_vcycles=4, mg_prec="fp64")
    rays = plan.new_rays()
    gal = dict(theta=torch.from_numpy(gth).cuda(), phi=torch.from_numpy(gph).cuda(),
               chi=torch.from_numpy(gchi).cuda(),
               A=torch.full((4, gth.size), np.nan, dtype=torch.float32, device="cuda"))
    plan.raytrace_planes(torch.from_numpy(kaps).cuda(), chi, 0, rays, galaxies=gal)
    plan.sync_status()
    th, ph = rays["theta"].cpu().numpy(), rays["phi"].cpu().numpy()
    beta, A, Ap = (rays[k].cpu().numpy() for k in ("beta", "A", "A_prev"))
    moved = 0.0
    for q in need:
        r, hist = ref[q]
        t, p = hp.vec2ang(r.n)
        assert abs(th[q] - t) < 1e-12
        assert abs(np.angle(np.exp(1j * (ph[q] - p)))) < 1e-12
        assert np.abs(beta[:, q] - r.beta).max() < 1e-12
        assert np.abs(A[:, q] - r.A.ravel()).max() < 2e-6
        assert np.abs(Ap[:, q] - r.A_prev.ravel()).max() < 2e-6
        z0, p0, s0 = hp.pix2ang_nest(Nf, np.array([q]))
        moved = max(moved, np.arccos(np.clip(hp.vec(z0, p0, s0)[0] @ r.n, -1, 1)))
    assert moved > 1e-4        # the rays were really deflected
    # galaxies: eq. gatraj with Jacobians interpolated on the image grid
    Ag = gal["A"].cpu().numpy()
    edges = orays.shell_edges(chi)
    for i in range(gth.size):
        k = int(np.searchsorted(edges, gchi[i], side="right") - 1)
        if k == 0:
            expect = np.eye(2).ravel()
        else:
            Ai = sum(gw[j, i] * ref[int(r2n[gpix[j, i]])][1][k - 1][0] for j in range(4))
            Api = sum(gw[j, i] * ref[int(r2n[gpix[j, i]])][1][k - 1][1] for j in range(4))
            w = orays.galaxy_weight(chi, k, gchi[i])
            expect = ((1 - w) * Api + w * Ai).ravel()
        assert np.abs(Ag[:, i] - expect).max() < 3e-6, (i, k)
    # the same run driven plane by plane through clm_poisson_solve,
    # clm_ray_update and clm_galaxies_shell gives identical results
    rays2 = plan.new_rays()
    gal2 = dict(gal, A=torch.full_like(gal["A"], np.nan))
    plan.galaxies_shell(chi, 0, rays2, gal2)
    for m in range(nplanes):
        plan.poisson_solve(torch.from_numpy(kaps[m]).cuda())
        plan.ray_update(chi, m, rays2)
        plan.galaxies_shell(chi, m + 1, rays2, gal2)
    plan.sync_status()
    for key in ("theta", "phi", "beta", "A", "A_prev"):
        assert torch.equal(rays2[key], rays[key]), key
    assert torch.equal(gal2["A"], gal["A"])
    plan.close()


def _capture(fn):
    """fn's launches captured into a graph on a side stream (after one eager
    warm-up call there), as torch.cuda.graph does."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


@pytest.mark.parametrize("kind", ["sht_mg_fp32", "sht_batched_fp32"])
def test_graph_capture_replays_match_eager(clm, kind):
    """The fixed-cycle solve path makes no allocation, memset or host wait,
    so it can be captured in a HIP graph: every replay (with eager work and
    synchronisation between replays) reproduces the eager outputs bit for
    bit."""
    if kind == "sht_mg_fp32":
        N, lmax = 64, 32
        g0 = osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=3, sigma=0.5))
        k = torch.from_numpy(np.exp(g0) - np.mean(np.exp(g0))).cuda()
        plan = clm.Plan(N, nside_sht=16, lmax=lmax, nside_bundle=4, patch_cells=256,
                        mg_vcycles=3, mg_prec="fp32")
        outs = (torch.empty(2, plan.npix_fine, dtype=torch.float32, device="cuda"),
                torch.empty(3, plan.npix_fine, dtype=torch.float32, device="cuda"))

        def run():
            plan.poisson_solve(k)
            plan.shear_at_pixels(order="nested", fp64=False, out=outs)
    else:
        N, lmax, P = 128, 256, 5
        k = torch.stack([clm.alm2map(torch.from_numpy(
            inputs.gaussian_alm(lmax, seed=90 + i, amplitude=1.0)).cuda(), lmax, N)
            for i in range(P)])
        plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P,
                        legendre_prec="fp32")
        outs = (torch.empty(P, plan.npix_sht, dtype=torch.float64, device="cuda"),)

        def run():
            plan.poisson_solve(k)
            for i in range(P):
                outs[0][i].copy_(plan.psi_map(i))
    run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    g = _capture(run)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), (kind, rep)
        plan.sync_status()
    plan.close()


# ---------------------------------------------------------------- adjoint (C5)
@pytest.fixture(scope="module")
def adj_case():
    from oracle import adjoint as oadj
    spec = omg.PatchSpec(16, 4, 8, 4, ncell=16, vcycles=2)
    g = osht.alm2map(16, 32, inputs.gaussian_alm(32, seed=8, sigma=0.5))
    kap = 0.01 * (np.exp(g) - np.mean(np.exp(g)))
    th, ph = inputs.uniform_sphere(300, seed=9)
    rng = np.random.default_rng(10)
    g1o, g2o = 0.26 * rng.standard_normal(th.size), 0.26 * rng.standard_normal(th.size)
    _, h = oadj.forward(spec, kap, th, ph)
    chi2, hbar = oadj.shear_chi2(h, g1o, g2o)
    grad = oadj.adjoint(spec, th, ph, np.zeros((2, th.size)), hbar)
    return dict(spec=spec, kap=kap, th=th, ph=ph, g1o=g1o, g2o=g2o, chi2=chi2, grad=grad)


def _adj_plan(clm, N, Ns, lmax, Nb, n, cyc, nu_pre=2, nu_post=2):
    return clm.Plan(N, nside_sht=Ns, lmax=lmax, nside_bundle=Nb, patch_cells=n,
                    mg_vcycles=cyc, mg_prec="fp64", adjoint=1, nu_pre=nu_pre, nu_post=nu_post)


def test_adjoint_gradient_matches_oracle(clm, adj_case):
    c = adj_case
    plan = _adj_plan(clm, 16, 4, 8, 4, 16, 2)
    th, ph = torch.from_numpy(c["th"]).cuda(), torch.from_numpy(c["ph"]).cuda()
    kap = torch.from_numpy(c["kap"]).cuda()
    plan.poisson_solve(kap)
    _, h = plan.shear_from_potential(th, ph)
    hn = h.cpu().numpy()
    r1 = 0.5 * (hn[0] - hn[1]) - c["g1o"]
    r2 = hn[2] - c["g2o"]
    hbar = torch.from_numpy(np.stack([r1, -r1, 2.0 * r2]) / 0.26 ** 2).cuda()
    plan.shear_adjoint(th, ph, torch.zeros(2, th.numel(), dtype=torch.float64, device="cuda"), hbar)
    grad = plan.poisson_adjoint().cpu().numpy()
    e = rel(grad, c["grad"])
    print("PARITY adjoint grad vs oracle %.3e" % e, flush=True)
    assert e < 1e-10
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("nu", [(2, 2), (3, 1), (1, 4)])
def test_adjoint_dot_product_tile_levels(clm, nu):
    """<F kappa, y> = <kappa, F^T y> with the tile-level forward (patches of
    256^2) and the adjoint on the GPU, FP64; sweep counts whose transposed
    smoothing spans one launch, a 4 + 2 split and a 4 + 4 split."""
    N, Ns, lmax, Nb = 64, 16, 32, 4
    plan = _adj_plan(clm, N, Ns, lmax, Nb, 256, 3, *nu)
    rng = np.random.default_rng(11)
    kap = torch.from_numpy(0.01 * rng.standard_normal(12 * N * N)).cuda()
    th, ph = (torch.from_numpy(a).cuda() for a in inputs.uniform_sphere(2000, seed=12))
    plan.poisson_solve(kap)
    g, h = plan.shear_from_potential(th, ph)
    gb = torch.from_numpy(rng.standard_normal((2, th.numel()))).cuda()
    hb = torch.from_numpy(rng.standard_normal((3, th.numel()))).cuda()
    plan.shear_adjoint(th, ph, gb, hb)
    kb = plan.poisson_adjoint()
    lhs = float((g * gb).sum() + (h * hb).sum())
    rhs = float((kap * kb).sum())
    e = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    print("PARITY adjoint dot product %.3e (%.6e, %.6e)" % (e, lhs, rhs), flush=True)
    assert e < 1e-10
    plan.sync_status()
    plan.close()


def test_autograd_chi2_central_differences(clm):
    """PoissonShearFn gradient of the shear chi^2 (exactly quadratic) against
    central differences of the GPU forward."""
    N = 32
    plan = _adj_plan(clm, N, 8, 16, 4, 64, 2)
    rng = np.random.default_rng(13)
    kap0 = torch.from_numpy(0.01 * rng.standard_normal(12 * N * N)).cuda()
    th, ph = (torch.from_numpy(a).cuda() for a in inputs.uniform_sphere(500, seed=14))
    o1 = torch.from_numpy(0.26 * rng.standard_normal(th.numel())).cuda()
    o2 = torch.from_numpy(0.26 * rng.standard_normal(th.numel())).cuda()

    def chi2(k):
        _, h = clm.PoissonShearFn.apply(k, th, ph, plan)
        return (((0.5 * (h[0] - h[1]) - o1) ** 2 + (h[2] - o2) ** 2) / 0.26 ** 2).sum()

    kap = kap0.clone().requires_grad_(True)
    (grad,) = torch.autograd.grad(chi2(kap), kap)
    step = 1e-3 * float(kap0.abs().mean())
    for p in rng.choice(12 * N * N, 4, replace=False):
        e = torch.zeros_like(kap0)
        e[p] = step
        fd = (float(chi2(kap0 + e)) - float(chi2(kap0 - e))) / (2 * step)
        g = float(grad[p])
        print("PARITY autograd pixel %d fd %.9e grad %.9e" % (p, fd, g), flush=True)
        assert abs(fd - g) <= 1e-6 * (abs(g) + 1e-3 * float(grad.abs().max()))
    plan.sync_status()
    plan.close()
