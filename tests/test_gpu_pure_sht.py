"""The pure-SHT solver's derivative fields on the matrix cores (Sec. 3.2,
last paragraph): several planes per launch, against the FP64 oracle
(`derivative_maps` of the oracle's own solve), element by element.

The comparison is end to end: the float32 matrix-core analysis of the solve
and the float32 derivative synthesis both contribute.  Bar: max-norm error
of each field below 2e-6 of the field's largest magnitude.  The float32
rounding of the Legendre functions and of psi_lm is 6e-8 relative per
product, and the sums run over at most lmax + 1 terms in float32 partial
sums, so each stage stays well under 1e-6 of the field scale (measured:
2e-7 to 5e-7 at Nside 64 and 256)."""
import numpy as np
import pytest
import torch

from oracle import healpix as hp
from oracle import sht as osht
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS_G = ("g_t", "g_p")
FIELDS_H = ("U_tt", "U_pp", "U_tp")


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


def case(N, lmax, P, seed):
    kaps, ders = [], []
    for i in range(P):
        kap = osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=seed + i, amplitude=1.0))
        palm = osht.poisson(lmax, osht.map2alm(N, lmax, kap - kap.mean()))
        kaps.append(kap)
        ders.append(osht.derivative_maps(N, lmax, palm))
    return np.stack(kaps), ders


def field_errors(g, h, der):
    out = {}
    for k, name in enumerate(FIELDS_G):
        ref = der[name]
        out[name] = np.abs(g[k] - ref).max() / np.abs(ref).max()
    for k, name in enumerate(FIELDS_H):
        ref = der[name]
        out[name] = np.abs(h[k] - ref).max() / np.abs(ref).max()
    return out


@pytest.mark.parametrize("N,lmax,P,waves", [(64, 128, 10, 4), (64, 128, 10, 8),
                                            (256, 300, 1, 4)])
def test_pure_sht_matrix_core_derivatives(clm, N, lmax, P, waves):
    """10 planes = one launch of 8 and a ragged launch of 2 (Nside 64, both
    workgroup shapes); Nside 256 with lmax 300 (two ring blocks of 256 rings,
    a ragged last step of l); RING and NESTED order, float64 and float32
    outputs, a sub-range of slots, and the single-plane entry point."""
    kaps, ders = case(N, lmax, P, seed=500 + N)
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P,
                    legendre_prec="fp32", mfma_der_waves=waves)
    assert plan.desc["mfma_der_waves"] == waves
    plan.poisson_solve(torch.from_numpy(kaps).cuda())
    g, h = plan.shear_at_pixels_batch(0, P, order="ring")
    g, h = g.cpu().numpy(), h.cpu().numpy()
    worst = 0.0
    for i in range(P):
        e = field_errors(g[i], h[i], ders[i])
        print("PARITY pure_sht N=%d plane %d %s" % (N, i, " ".join(
            "%s %.2e" % kv for kv in e.items())), flush=True)
        worst = max(worst, max(e.values()))
        assert max(e.values()) < 2e-6, (i, e)
    # NESTED order, float32 output, a sub-range of slots (one plane, through
    # both entry points)
    r = hp.nest2ring(N, np.arange(12 * N * N))
    first = max(0, P - 2)
    gn, hn = plan.shear_at_pixels_batch(first, P - first, order="nested", fp64=False)
    for k in range(P - first):
        der = ders[first + k]
        e = field_errors(gn[k].cpu().numpy(), hn[k].cpu().numpy(),
                         {n: der[n][r] for n in FIELDS_G + FIELDS_H})
        assert max(e.values()) < 2e-6, (k, e)
    g1, h1 = plan.shear_at_pixels(slot=P - 1, order="ring")
    assert torch.equal(g1.cpu(), torch.from_numpy(g[P - 1]))
    assert torch.equal(h1.cpu(), torch.from_numpy(h[P - 1]))
    plan.sync_status()
    plan.close()


def test_pure_sht_derivative_errors(clm):
    sht = clm.Plan(16, nside_sht=16, lmax=32, solver="sht", max_planes=2,
                   legendre_prec="fp32")
    g = torch.empty(3, 2, 12 * 16 * 16, dtype=torch.float64, device="cuda")
    h = torch.empty(3, 3, 12 * 16 * 16, dtype=torch.float64, device="cuda")
    for first, n in ((0, 3), (1, 2), (-1, 1), (0, 0)):
        with pytest.raises(clm.ClmError) as ei:
            sht.shear_at_pixels_batch(first, n, out=(g, h))
        assert ei.value.status == clm.CLM_EINVAL
    sht.close()
    mg = clm.Plan(64, nside_sht=16, lmax=32, nside_bundle=4, patch_cells=64)
    with pytest.raises(clm.ClmError) as ei:
        mg.shear_at_pixels_batch(0, 1)
    assert ei.value.status == clm.CLM_EUNSUPPORTED
    mg.close()


def test_pure_sht_fp64_batch(clm):
    """An FP64 plan runs the FP64 synthesis plane by plane under the batch
    entry point."""
    N, lmax, P = 16, 32, 3
    kaps, ders = case(N, lmax, P, seed=640)
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P)
    plan.poisson_solve(torch.from_numpy(kaps).cuda())
    g, h = plan.shear_at_pixels_batch(0, P, order="ring")
    for i in range(P):
        e = field_errors(g[i].cpu().numpy(), h[i].cpu().numpy(), ders[i])
        assert max(e.values()) < 1e-10, (i, e)
    plan.sync_status()
    plan.close()


@pytest.mark.parametrize("form,tol_a", [("fp64", 2e-6), ("fp32", 3e-6)])
def test_raytrace_pure_sht_parity(clm, form, tol_a):
    """Rays through three pure-SHT planes (Nside 32, lmax 64) against the
    oracle's ray steps, which take g and U at each ray by the transported
    four-point interpolation of its own derivative fields; every 13th ray
    and the rays of the polar rings.  Positions (unit vectors) and
    directions to 1e-12 (FP64 form) or 5e-8 (float32 fields: 5e-7 of the
    0.015 rad the rays move), Jacobians to the float32 level.  The batched call (one derivative synthesis of the three planes)
    and the plane-by-plane calls give the same rays bit for bit."""
    from oracle import rays as orays
    N, lmax, nplanes = 32, 64, 3
    chi = np.array([(m + 0.5) * 100.0 for m in range(nplanes)] + [nplanes * 100.0 + 50.0])
    kaps = []
    for m in range(nplanes):
        sig = 0.3 + 0.1 * m
        g = osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=800 + m, sigma=sig))
        s = inputs.deflection_scale(lmax, sig, alpha_rms=20 * inputs.ARCMIN)
        kaps.append(s * (np.exp(g) - np.mean(np.exp(g))))
    kaps = np.stack(kaps)
    fields = []
    for m in range(nplanes):
        palm = osht.poisson(lmax, osht.map2alm(N, lmax, kaps[m] - kaps[m].mean()))
        d = osht.derivative_maps(N, lmax, palm)
        fields.append((np.stack([d["g_t"], d["g_p"]]), np.stack([d["U_tt"], d["U_pp"], d["U_tp"]])))
    n = 12 * N * N
    polar = set(hp.ring2nest(N, np.arange(8)).tolist()) | set(hp.ring2nest(N, n - 1 - np.arange(8)).tolist())
    need = sorted(set(range(0, n, 13)) | polar)
    ref = {}
    for q in need:
        z, p, s = hp.pix2ang_nest(N, np.array([q]))
        r = orays.Ray(np.arctan2(s[0], z[0]), p[0])
        for m in range(nplanes):
            gr, Ur = orays.pixel_field_at(N, fields[m][0], fields[m][1], r.n)
            orays.ray_step(r, chi, m, gr, Ur)
        ref[q] = r
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=nplanes,
                    legendre_prec=form)
    kt = torch.from_numpy(kaps).cuda()
    rays = plan.new_rays()
    plan.raytrace_planes(kt, chi, 0, rays)
    plan.sync_status()
    # plane by plane: solve, then one ray update per slot
    rays2 = plan.new_rays()
    plan.poisson_solve(kt)
    for m in range(nplanes):
        plan.ray_update(chi, m, rays2, slot=m)
    plan.sync_status()
    for k in ("theta", "phi", "beta", "A", "A_prev"):
        assert torch.equal(rays[k], rays2[k]), k
    th, ph = rays["theta"].cpu().numpy(), rays["phi"].cpu().numpy()
    beta, A, Ap = (rays[k].cpu().numpy() for k in ("beta", "A", "A_prev"))
    tol_x = 1e-12 if form == "fp64" else 5e-8
    moved, worst = 0.0, 0.0
    for q in need:
        r = ref[q]
        nq = hp.vec(np.cos(th[q]), ph[q], np.sin(th[q]))
        assert np.abs(nq - r.n).max() < tol_x
        assert np.abs(beta[:, q] - r.beta).max() < tol_x
        ea = max(np.abs(A[:, q] - r.A.ravel()).max(), np.abs(Ap[:, q] - r.A_prev.ravel()).max())
        worst = max(worst, ea)
        assert ea < tol_a, (q, ea)
        z0, p0, s0 = hp.pix2ang_nest(N, np.array([q]))
        moved = max(moved, np.arccos(np.clip(hp.vec(z0, p0, s0)[0] @ r.n, -1, 1)))
    print("PARITY pure_sht rays %s A %.2e moved %.2e" % (form, worst, moved), flush=True)
    assert moved > 1e-3        # rays left their pixel centres (pixel ~ 0.03 rad)
    plan.close()
