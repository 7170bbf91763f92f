"""clm_alm2map_noalloc (the synthesis with its tables and intermediates in
the library's file-scope device array) against clm_alm2map, which builds a
plan: two calls in a row, the second smaller; its size limits; and replays
of a captured graph with other calls of it in between."""
import ctypes

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


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _alm(lmax, seed):
    return torch.from_numpy(inputs.gaussian_alm(lmax, seed=seed, sigma=0.5)).cuda()


def test_noalloc_matches_alm2map_two_calls(clm):
    """Largest size first, then a smaller one: each equals clm_alm2map to the
    FP64 bar (1e-10 relative, max norm), and the smaller one equals the
    oracle's synthesis too."""
    for N, lmax, seed in [(256, 512, 11), (64, 128, 12)]:
        print("case: noalloc nside %d lmax %d" % (N, lmax), flush=True)
        a = _alm(lmax, seed)
        ref = clm.alm2map(a, lmax, N)
        out = torch.full((12 * N * N,), np.nan, dtype=torch.float64, device="cuda")
        clm.alm2map_noalloc(a, lmax, N, out)
        torch.cuda.synchronize()
        err = rel(out, ref)
        print("PARITY noalloc vs alm2map nside %d lmax %d %.3e" % (N, lmax, err), flush=True)
        assert err < 1e-10
        if N == 64:
            o = osht.alm2map(N, lmax, a.cpu().numpy())
            assert rel(out.cpu(), torch.from_numpy(o)) < 1e-10


def test_noalloc_limits(clm):
    a = _alm(16, 3)
    out = torch.empty(12 * 512 * 512, dtype=torch.float64, device="cuda")
    L = clm.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ap = ctypes.c_void_p(a.data_ptr())
    op = ctypes.c_void_p(out.data_ptr())
    assert L.clm_alm2map_noalloc(ap, 16, 512, op, s) == clm.CLM_EUNSUPPORTED
    assert L.clm_alm2map_noalloc(ap, 513, 256, op, s) == clm.CLM_EUNSUPPORTED
    assert L.clm_alm2map_noalloc(ap, 0, 16, op, s) == clm.CLM_EINVAL
    assert L.clm_alm2map_noalloc(ap, 16, 48, op, s) == clm.CLM_EINVAL
    assert L.clm_alm2map_noalloc(None, 16, 16, op, s) == clm.CLM_EINVAL
    with pytest.raises(clm.ClmError, match="limits"):
        clm.alm2map_noalloc(a, 16, 512, out)


def test_noalloc_graph_replays(clm):
    """A captured call (tables rebuilt inside the graph) replayed three
    times, with eager calls of other sizes overwriting the shared array in
    between: every replay equals the eager result."""
    N, lmax = 128, 256
    a = _alm(lmax, 21)
    out = torch.empty(12 * N * N, dtype=torch.float64, device="cuda")
    clm.alm2map_noalloc(a, lmax, N, out)
    torch.cuda.synchronize()
    eager = out.clone()
    other = _alm(40, 22)
    o2 = torch.empty(12 * 32 * 32, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            clm.alm2map_noalloc(a, lmax, N, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in range(3):
        out.fill_(np.nan)
        clm.alm2map_noalloc(other, 40, 32, o2)     # scribbles over the scratch
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
