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


@pytest.mark.parametrize("field,value", [
    ("nside_fine", 100), ("nside_sht", 4096), ("patch_cells", 96), ("nu_pre", 0),
    ("mg_vcycles", 0), ("max_planes", 0), ("solver", 7), ("mg_prec", 9),
    ("nside_bundle", 1), ("legendre_prec", 3), ("legendre_prec", -1)])
def test_invalid_descriptions_rejected(L, field, value):
    from paper_1210_3069_amd import clm
    d = clm.PlanDesc()
    L.clm_plan_desc_default(ctypes.byref(d), 2048)
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
