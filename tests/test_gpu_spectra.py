"""GPU parity of the full-sky spectra of a ray state (clm_jacobian_spectra,
Sec. 5) with the oracle (oracle/spectra.py).

The ray state is synthetic and seeded: rays at their pixel centres turned by
a smooth random rotation (a fraction of a pixel) and Jacobians
A = [[1 - k - g1, -g2 + w], [-g2 - w, 1 - k + g1]] whose four fields are
band-limited random fields (C_l ~ l^-2), stored in float32 as the ray state
stores them.  The same state goes to the library and to the oracle.  Both
work in FP64 from there (transport, spin-0 and spin-2 analyses), so the
coefficients and spectra agree to 1e-10 of the largest."""
import numpy as np
import pytest
import torch

from oracle import healpix as hp
from oracle import sht as osht
from oracle import spectra as osp
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


def synthetic_state(N, seed, shift):
    """Positions: pixel centres turned about a random axis by `shift` rad
    times a smooth factor; Jacobians from four fields of rms 0.02
    band-limited at l = Nside (NESTED order, float32)."""
    n = 12 * N * N
    rng = np.random.default_rng(seed)
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    c = rng.standard_normal(3)
    z, ph, s = hp.pix2ang_nest(N, np.arange(n))
    v = hp.vec(z, ph, s)
    pos = v + shift * (1.0 + 0.5 * (v @ c))[:, None] * np.cross(ax, v)
    pos /= np.linalg.norm(pos, axis=1)[:, None]
    th, phi = hp.vec2ang(pos)
    lmax = N
    ring = hp.nest2ring(N, np.arange(n))
    f = [osht.alm2map(N, lmax, inputs.gaussian_alm(lmax, seed=seed + 1 + k, sigma=0.02))[ring]
         for k in range(4)]
    k_, g1, g2, w = f
    A = np.stack([1 - k_ - g1, -g2 + w, -g2 - w, 1 - k_ + g1]).astype(np.float32)
    return th, phi, A


@pytest.mark.parametrize("N,lmax", [(32, 64), (64, 100)])
def test_jacobian_spectra_match_oracle(clm, N, lmax):
    th, phi, A = synthetic_state(N, seed=31 + N, shift=0.3 * np.sqrt(4 * np.pi / (12 * N * N)))
    ref = osp.jacobian_spectra(N, lmax, th, phi, A.astype(np.float64))
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht")
    n = 12 * N * N
    rays = dict(theta=torch.from_numpy(th).cuda(), phi=torch.from_numpy(phi).cuda(),
                beta=torch.zeros(3, n, dtype=torch.float64, device="cuda"),
                A=torch.from_numpy(A).cuda(), A_prev=torch.from_numpy(A).cuda())
    alm, cl = plan.jacobian_spectra(rays)
    plan.sync_status()
    alm, cl = alm.cpu().numpy(), cl.cpu().numpy()
    for k, name in enumerate(("kappa", "E", "B", "omega")):
        ea = np.abs(alm[k] - ref["alm"][k]).max() / np.abs(ref["alm"][k]).max()
        ec = np.abs(cl[k] - ref["cl"][k]).max() / np.abs(ref["cl"][k]).max()
        print("PARITY spectra N=%d %s alm %.2e cl %.2e" % (N, name, ea, ec), flush=True)
        assert ea < 1e-10 and ec < 1e-10, (name, ea, ec)
    # the sums of the spectra are the maps' variances (Parseval, up to the
    # quadrature error of the analysis), a check independent of the oracle
    f = ref["fields"]
    for k in (0, 3):
        var = np.sum((2 * np.arange(lmax + 1) + 1) * cl[k]) / (4 * np.pi)
        assert abs(var - np.mean(f[k] ** 2)) < 2e-2 * np.mean(f[k] ** 2)
    plan.close()


def test_jacobian_spectra_errors(clm):
    N = 16
    n = 12 * N * N
    rays = dict(theta=torch.zeros(n, dtype=torch.float64, device="cuda"),
                phi=torch.zeros(n, dtype=torch.float64, device="cuda"),
                beta=torch.zeros(3, n, dtype=torch.float64, device="cuda"),
                A=torch.zeros(4, n, dtype=torch.float32, device="cuda"),
                A_prev=torch.zeros(4, n, dtype=torch.float32, device="cuda"))
    other = clm.Plan(32, nside_sht=32, lmax=32, solver="sht")
    with pytest.raises(clm.ClmError) as ei:
        other.jacobian_spectra(rays)
    assert ei.value.status == clm.CLM_EINVAL
    other.close()
    # an SHT+MG plan whose SHT grid matches the rays
    mg = clm.Plan(64, nside_sht=16, lmax=32, nside_bundle=4, patch_cells=64)
    with pytest.raises(clm.ClmError) as ei:
        mg.jacobian_spectra(rays)
    assert ei.value.status == clm.CLM_EUNSUPPORTED
    mg.close()
