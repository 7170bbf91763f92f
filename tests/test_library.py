"""The C-ABI library loads and exports every entry point the header
declares; argument validation that needs no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1210_3069_amd import clm
    if not os.path.exists(clm.LIB_PATH):
        from paper_1210_3069_amd import build
        build.build()
    return clm.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "calclens_mi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(clm_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "clm_plan_create" in names and "clm_raytrace_planes" in names
    for n in names:
        assert hasattr(L, n), n


def test_default_description(L):
    from paper_1210_3069_amd import clm
    d = clm.PlanDesc()
    assert L.clm_plan_desc_default(ctypes.byref(d), 2048) == clm.CLM_OK
    assert (d.nside_sht, d.lmax, d.nside_bundle, d.patch_cells) == (256, 512, 32, 256)
    assert (d.mg_vcycles, d.nu_pre, d.nu_post, d.patch_factor) == (4, 2, 2, 4)
    assert (d.mg_max_vcycles, d.mg_eps, d.adjoint) == (20, 0.1, 0)
    assert d.analysis_iters == 0
    assert (d.mfma_ana_waves, d.mfma_syn_waves, d.mfma_der_waves) == (0, 0, 0)
    assert ctypes.sizeof(d) == 88  # 14 int32, a double, five int32, padding


@pytest.mark.parametrize("fields", [
    dict(nside_fine=100), dict(nside_sht=4096), dict(patch_cells=96), dict(nu_pre=0),
    dict(mg_vcycles=-1), dict(max_planes=0), dict(solver=7), dict(mg_prec=9),
    dict(nside_bundle=1), dict(legendre_prec=4), dict(legendre_prec=-1),
    dict(mfma_ana_waves=4), dict(mfma_syn_waves=10), dict(mfma_der_waves=16),
    dict(lmax=(1 << 20) + 1),
    # the epsilon rule needs a positive threshold and cycle limit, and the
    # adjoint a fixed cycle count
    dict(mg_vcycles=0, mg_eps=0.0), dict(mg_vcycles=0, mg_max_vcycles=0),
    dict(mg_eps=-1.0), dict(mg_eps=float("nan")), dict(mg_vcycles=0, adjoint=1),
    # analysis refinement: 0..16, FP64 Legendre transforms, no adjoint
    dict(analysis_iters=17), dict(analysis_iters=-1), dict(analysis_iters=1, legendre_prec=1),
    dict(analysis_iters=2, adjoint=1)])
def test_invalid_descriptions_rejected(L, fields):
    from paper_1210_3069_amd import clm
    d = clm.PlanDesc()
    L.clm_plan_desc_default(ctypes.byref(d), 2048)
    for field, value in fields.items():
        setattr(d, field, value)
    h = ctypes.c_void_p()
    assert L.clm_plan_create(ctypes.byref(d), 0, ctypes.byref(h)) == clm.CLM_EINVAL
    assert not h.value


def test_null_arguments_rejected(L):
    from paper_1210_3069_amd import clm
    assert L.clm_plan_create(None, 0, None) == clm.CLM_EINVAL
    assert L.clm_poisson_solve(None, None, 1, 0, 1, None) == clm.CLM_EINVAL
    assert L.clm_plan_destroy(None) == clm.CLM_EINVAL
    assert L.clm_status_string(5) == b"a point left its bundle's patch"


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    """The autotuner's JSON cache: stored choices are read back; a missing or
    unreadable file reads as empty."""
    from paper_1210_3069_amd import clm
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("CALCLENS_MI_TUNE_CACHE", str(path))
    assert clm.tune_cache_path() == str(path)
    assert clm._tune_load() == {}
    clm._tune_store("gpu|nside 512|lmax 1024|form 1|batch 6|solver 1", 8, 16, 0)
    clm._tune_store("gpu|nside 2048|lmax 4096|form 3|batch 15|solver 0", 16, 12, 4)
    assert clm._tune_load() == {"gpu|nside 512|lmax 1024|form 1|batch 6|solver 1": [8, 16, 0],
                                "gpu|nside 2048|lmax 4096|form 3|batch 15|solver 0": [16, 12, 4]}
    path.write_text("not json")
    assert clm._tune_load() == {}
