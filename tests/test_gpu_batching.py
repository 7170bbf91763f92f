"""GPU checks of the batched matrix-core form: planes of several grids
(uneven nside and lmax) in one persistent Legendre launch per round
(clm_poisson_solve_multi), against the same planes solved plan by plan and
against the FP64 oracle; its capture in a HIP graph; the autotuner's
choice of workgroup shapes."""
import numpy as np
import pytest
import torch

from oracle import sht as osht
from paper_1210_3069_amd import inputs

pytestmark = pytest.mark.gpu

# (nside, planes): ragged batches, one grid with more planes than a round
GRIDS = [(16, 5), (32, 3), (64, 18)]


@pytest.fixture(scope="module")
def clm():
    from paper_1210_3069_amd import clm as c
    c.lib()
    assert torch.cuda.is_available()
    return c


@pytest.fixture(scope="module")
def maps():
    out = {}
    for N, P in GRIDS:
        out[N] = [osht.alm2map(N, 2 * N, inputs.gaussian_alm(2 * N, seed=1000 + 10 * N + i,
                                                             amplitude=1.0))
                  for i in range(P)]
    return out


def _plans(clm, form, ana=8, syn=16):
    return [clm.Plan(N, nside_sht=N, lmax=2 * N, solver="sht", max_planes=P,
                     legendre_prec=form, mfma_ana_waves=ana, mfma_syn_waves=syn)
            for N, P in GRIDS]


@pytest.mark.parametrize("form,tol", [("fp32", 5e-6), ("bf16x6", 5e-6), ("bf16x3", 1e-4)])
def test_multi_matches_single_and_oracle(clm, maps, form, tol):
    """With the same workgroup shapes, one persistent launch over three
    grids gives the same bits as the plans solved one by one; every plane
    against the oracle (max-norm relative error of psi_lm)."""
    print("case: multi-grid solve, %s" % form, flush=True)
    multi = _plans(clm, form)
    single = _plans(clm, form)
    ks = [torch.from_numpy(np.stack(maps[N])).cuda() for N, _ in GRIDS]
    clm.poisson_solve_multi(multi, ks)
    for pl, k in zip(single, ks):
        pl.poisson_solve(k)
    for (N, P), pm, ps in zip(GRIDS, multi, single):
        for i in range(P):
            assert torch.equal(pm.psi_alm(i), ps.psi_alm(i)), (N, i)
            assert torch.equal(pm.psi_map(i), ps.psi_map(i)), (N, i)
            m = maps[N][i]
            ref = osht.poisson(2 * N, osht.map2alm(N, 2 * N, m - m.mean()))
            got = pm.psi_alm(i).cpu().numpy()
            e = np.abs(got - ref).max() / np.abs(ref).max()
            assert e < tol, (form, N, i, e)
    for pl in multi + single:
        pl.sync_status()
        pl.close()


def test_multi_graph_replays(clm, maps):
    """The multi-grid solve captured in a graph and replayed three times,
    with eager solves of other planes between the replays: each replay
    equals the eager result."""
    plans = _plans(clm, "fp32")
    ks = [torch.from_numpy(np.stack(maps[N])).cuda() for N, _ in GRIDS]
    clm.poisson_solve_multi(plans, ks)
    torch.cuda.synchronize()
    eager = [[pl.psi_alm(i).clone() for i in range(P)] for pl, (N, P) in zip(plans, GRIDS)]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            clm.poisson_solve_multi(plans, ks)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    other = [k.flip(0).contiguous() for k in ks]
    for rep in range(3):
        clm.poisson_solve_multi(plans, other)        # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for pl, (N, P), ref in zip(plans, GRIDS, eager):
            for i in range(P):
                assert torch.equal(pl.psi_alm(i), ref[i]), (rep, N, i)
    for pl in plans:
        pl.sync_status()
        pl.close()


def test_autotuner_choice(clm, tmp_path, monkeypatch):
    """Shapes left at 0 are chosen at plan creation among the built ones and
    kept in the JSON cache, which the next plan of that grid and form reads;
    given shapes are kept; an unknown shape is rejected."""
    import json
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("CALCLENS_MI_TUNE_CACHE", str(cache))
    pl = clm.Plan(64, nside_sht=64, lmax=128, solver="sht", max_planes=4,
                  legendre_prec="bf16x6")
    names = ("mfma_ana_waves", "mfma_syn_waves", "mfma_der_waves")
    pick = tuple(pl.desc[n] for n in names)
    assert pick[0] in (8, 16) and pick[1] in (8, 12, 16) and pick[2] in (4, 8)
    pl.close()
    table = json.loads(cache.read_text())
    assert list(table.values()) == [list(pick)]
    # a planted entry is what the next plan of the same key uses
    key = list(table)[0]
    other = (16, 12, 8) if pick != (16, 12, 8) else (8, 8, 4)
    cache.write_text(json.dumps({key: list(other)}))
    pl = clm.Plan(64, nside_sht=64, lmax=128, solver="sht", max_planes=4,
                  legendre_prec="bf16x6")
    assert tuple(pl.desc[n] for n in names) == other
    pl.close()
    pl = clm.Plan(64, nside_sht=64, lmax=128, solver="sht", max_planes=4,
                  legendre_prec="fp32", mfma_ana_waves=16, mfma_syn_waves=12)
    assert (pl.desc["mfma_ana_waves"], pl.desc["mfma_syn_waves"]) == (16, 12)
    pl.close()
    with pytest.raises(clm.ClmError):
        clm.Plan(64, nside_sht=64, lmax=128, solver="sht", legendre_prec="fp32",
                 mfma_syn_waves=10)


def test_multi_rejects_mixed_forms(clm):
    a = clm.Plan(16, nside_sht=16, lmax=32, solver="sht", legendre_prec="fp32")
    b = clm.Plan(32, nside_sht=32, lmax=64, solver="sht", legendre_prec="bf16x6")
    ka = torch.zeros(12 * 16 * 16, dtype=torch.float64, device="cuda")
    kb = torch.zeros(12 * 32 * 32, dtype=torch.float64, device="cuda")
    with pytest.raises(clm.ClmError) as ei:
        clm.poisson_solve_multi([a, b], [ka, kb])
    assert ei.value.status == clm.CLM_EINVAL
    a.close()
    b.close()
