"""Python binding of libcalclens_mi.so (ctypes).  Argument marshalling only:
tensors are passed by device pointer together with the current HIP stream;
every step of the computation runs in the library's kernels.  Raises when
the library is missing or a call fails; there is no fallback path."""
import ctypes
import json
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcalclens_mi.so")

CLM_OK, CLM_EINVAL, CLM_ENOMEM, CLM_EHIP = 0, 1, 2, 3
CLM_ENOTCONV, CLM_ERAY_LEFT_PATCH, CLM_ENONFINITE, CLM_EUNSUPPORTED = 4, 5, 6, 7
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
SOLVER_SHT, SOLVER_SHT_MG = 0, 1
ORDER_RING, ORDER_NESTED = 0, 1


class PlanDesc(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "nside_fine", "nside_sht", "lmax", "nside_bundle", "patch_factor", "patch_cells",
        "mg_vcycles", "nu_pre", "nu_post", "solver", "mg_prec", "max_planes",
        "legendre_prec", "mg_max_vcycles")] + [("mg_eps", ctypes.c_double),
                                               ("adjoint", ctypes.c_int32),
                                               ("analysis_iters", ctypes.c_int32),
                                               ("mfma_ana_waves", ctypes.c_int32),
                                               ("mfma_syn_waves", ctypes.c_int32),
                                               ("mfma_der_waves", ctypes.c_int32)]


class Rays(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("A_prev", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Particles(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Galaxies(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("chi", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("n", ctypes.c_int64)]


class ClmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "clm_plan_desc_default": (ctypes.POINTER(PlanDesc), _I32),
    "clm_plan_create": (ctypes.POINTER(PlanDesc), ctypes.c_int, ctypes.POINTER(_P)),
    "clm_plan_destroy": (_P,),
    "clm_status_string": (_I32,),
    "clm_plan_last_error": (_P, ctypes.c_char_p, ctypes.c_size_t),
    "clm_plan_sync_status": (_P, _P),
    "clm_plan_workspace_bytes": (_P,),
    "clm_plan_get_desc": (_P, ctypes.POINTER(PlanDesc)),
    "clm_alm2map": (_P, _I32, _I32, _P, _P),
    "clm_alm2map_noalloc": (_P, _I32, _I32, _P, _P),
    "clm_poisson_solve": (_P, _P, _I32, _I32, _I32, _P),
    "clm_poisson_solve_multi": (ctypes.POINTER(_P), _I32, ctypes.POINTER(_P),
                                ctypes.POINTER(_I32), ctypes.POINTER(_I32), _P),
    "clm_get_psi_alm": (_P, _I32, _P, _P),
    "clm_get_psi_map": (_P, _I32, _P, _P),
    "clm_get_patch_potential": (_P, _I32, _I64, _I64, _P, _P),
    "clm_shear_from_potential": (_P, _I32, _P, _P, _I64, _I32, _P, _P, _P),
    "clm_shear_at_pixels": (_P, _I32, _I32, _I32, _P, _P, _P),
    "clm_shear_at_pixels_batch": (_P, _I32, _I32, _I32, _I32, _P, _P, _P),
    "clm_rays_init": (_P, ctypes.POINTER(Rays), _P),
    "clm_jacobian_spectra": (_P, ctypes.POINTER(Rays), _P, _P, _P),
    "clm_plan_set_domain": (_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64),
    "clm_deposit_epanechnikov": (_P, _P, _P, _P, ctypes.c_int64, _I32, _P, _P),
    "clm_poisson_solve_particles": (_P, ctypes.POINTER(Particles), _I32, _P),
    "clm_raytrace_planes": (_P, _P, _I32, ctypes.POINTER(_D), _I32, _I32, _I32, _D,
                            ctypes.POINTER(Rays), ctypes.POINTER(Galaxies), _P),
    "clm_ray_update": (_P, _I32, ctypes.POINTER(_D), _I32, _I32, _D, ctypes.POINTER(Rays), _P),
    "clm_galaxies_shell": (_P, ctypes.POINTER(_D), _I32, _I32, _D, ctypes.POINTER(Rays),
                           ctypes.POINTER(Galaxies), _P),
    "clm_shear_adjoint": (_P, _I32, _P, _P, _I64, _P, _P, _P),
    "clm_poisson_adjoint": (_P, _I32, _P, _P),
    "clm_get_mg_convergence": (_P, _P, _P, _P),
    "clm_plan_set_timing": (_P, _I32),
    "clm_plan_set_timing_stages": (_P, ctypes.c_char_p),
    "clm_plan_timings": (_P, ctypes.POINTER(_D), _I32),
    "clm_plan_stage_name": (_P, _I32),
    "clm_galaxies_reduced": (_P, ctypes.POINTER(Rays), _P, _P, _P, _I64, _P, _P),
    "clm_galaxy_images": (_P, ctypes.POINTER(_D), _I32, _I32, _D, ctypes.POINTER(Rays),
                          ctypes.POINTER(Galaxies), _D, _P, _P, _P, _P),
    "clm_plan_get_timing": (_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_D),
                            ctypes.POINTER(_I64), _I32, ctypes.POINTER(_I32)),
}


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcalclens_mi.so is not built: run python -m paper_1210_3069_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = list(args)
            f.restype = ctypes.c_int32
        L.clm_status_string.restype = ctypes.c_char_p
        L.clm_plan_workspace_bytes.restype = ctypes.c_size_t
        L.clm_plan_stage_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous %s tensor on the GPU" % dtype)
    return t


def _out(t, dtype, numel, name):
    """A caller's output tensor: contiguous, of the dtype the call writes and
    with room for the values it writes (the library checks the rest)."""
    _dev(t, dtype)
    if t.numel() < numel:
        raise ValueError("%s has %d values, the call writes %d" % (name, t.numel(), numel))
    return t


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def alm2map(alm, lmax, nside):
    """Real map (RING, float64) of complex a_lm (HEALPix order) on the GPU."""
    a = torch.view_as_real(_dev(alm, torch.complex128)).contiguous()
    out = torch.empty(12 * nside * nside, dtype=torch.float64, device=alm.device)
    st = lib().clm_alm2map(_ptr(a), lmax, nside, _ptr(out), _stream())
    if st != CLM_OK:
        raise ClmError(st, "clm_alm2map failed: %s" % lib().clm_status_string(st).decode())
    return out


def deposit_epanechnikov(theta, phi, weight, sigma, nside, out=None):
    """Epanechnikov deposition of particles (float64 tensors on the GPU) onto
    a RING map of nside, added into `out` (zeros when None); returns the map."""
    for t in (theta, phi, weight, sigma):
        _dev(t, torch.float64)
    n = theta.numel()
    if not (phi.numel() == weight.numel() == sigma.numel() == n):
        raise ValueError("theta, phi, weight and sigma must have one value per particle")
    if out is None:
        out = torch.zeros(12 * nside * nside, dtype=torch.float64, device=theta.device)
    _dev(out, torch.float64)
    if out.numel() != 12 * nside * nside:
        raise ValueError("out has %d values, expected %d" % (out.numel(), 12 * nside * nside))
    st = lib().clm_deposit_epanechnikov(_ptr(theta), _ptr(phi), _ptr(weight), _ptr(sigma), n,
                                        nside, _ptr(out), _stream())
    if st != CLM_OK:
        raise ClmError(st, "clm_deposit_epanechnikov failed: %s"
                       % lib().clm_status_string(st).decode())
    return out


NOALLOC_MAX_NSIDE, NOALLOC_MAX_LMAX = 256, 512


def alm2map_noalloc(alm, lmax, nside, out):
    """alm2map into the caller's `out` (float64 [12 nside^2] on the GPU)
    through clm_alm2map_noalloc: the library allocates nothing and the call
    may be captured in a graph (nside <= 256, lmax <= 512)."""
    a = torch.view_as_real(_dev(alm, torch.complex128))
    _dev(out, torch.float64)
    if out.numel() != 12 * nside * nside:
        raise ValueError("out has %d values, expected %d" % (out.numel(), 12 * nside * nside))
    st = lib().clm_alm2map_noalloc(_ptr(a), lmax, nside, _ptr(out), _stream())
    if st == CLM_EUNSUPPORTED:
        raise ClmError(st, "clm_alm2map_noalloc: nside %d / lmax %d beyond its limits "
                           "(nside <= %d, lmax <= %d)" % (nside, lmax, NOALLOC_MAX_NSIDE,
                                                          NOALLOC_MAX_LMAX))
    if st != CLM_OK:
        raise ClmError(st, "clm_alm2map_noalloc failed: %s" % lib().clm_status_string(st).decode())
    return out


def poisson_solve_multi(plans, kappas):
    """clm_poisson_solve_multi: the planes kappas[i] ([P_i, npix_i] or
    [npix_i], float64 or float32, on the GPU) of plans[i] (matrix-core forms,
    up to 4 plans) solved with one persistent Legendre launch per round of
    up to 16 planes per plan."""
    n = len(plans)
    if n != len(kappas) or not 1 <= n <= 4:
        raise ValueError("1 to 4 plans, one convergence batch each")
    ks = []
    for pl, k in zip(plans, kappas):
        k = k if k.dim() == 2 else k.reshape(1, -1)
        if k.dtype not in (torch.float64, torch.float32):
            raise ValueError("kappa must be float64 or float32")
        _dev(k, k.dtype)
        if k.shape[1] != pl.npix_fine:
            raise ValueError("kappa has %d pixels, plan expects %d" % (k.shape[1], pl.npix_fine))
        ks.append(k)
    hs = (ctypes.c_void_p * n)(*[pl.h.value for pl in plans])
    kp = (ctypes.c_void_p * n)(*[k.data_ptr() for k in ks])
    f64 = (ctypes.c_int32 * n)(*[int(k.dtype == torch.float64) for k in ks])
    npl = (ctypes.c_int32 * n)(*[k.shape[0] for k in ks])
    plans[0]._check(lib().clm_poisson_solve_multi(hs, n, kp, f64, npl, _stream()),
                    "poisson_solve_multi")


def tune_cache_path():
    """JSON file of the autotuner's choices: $CALCLENS_MI_TUNE_CACHE, else
    ~/.cache/calclens_mi/autotune.json."""
    return os.environ.get("CALCLENS_MI_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "calclens_mi", "autotune.json")


def _tune_key(dev, d):
    batch = min(d.max_planes, 16)
    return "%s|nside %d|lmax %d|form %d|batch %d|solver %d" % (
        torch.cuda.get_device_name(dev), d.nside_sht, d.lmax, d.legendre_prec, batch, d.solver)


def _tune_load():
    try:
        with open(tune_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _tune_store(key, ana, syn, der):
    path = tune_cache_path()
    table = _tune_load()
    table[key] = [int(ana), int(syn), int(der)]
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home keeps the in-process choice only


class Plan:
    """A solver plan (workspace on the current device).  Matrix-core plans
    whose workgroup shapes are not given take them from the autotuner's JSON
    cache (tune_cache_path()) or, on a miss, from the library's autotuner,
    whose choice is then added to the cache."""

    def __init__(self, nside_fine, device=None, **kw):
        L = lib()
        d = PlanDesc()
        self._check(L.clm_plan_desc_default(ctypes.byref(d), nside_fine), "desc_default", None)
        for k, v in kw.items():
            if k == "solver" and isinstance(v, str):
                v = {"sht": SOLVER_SHT, "sht_mg": SOLVER_SHT_MG}[v]
            if k in ("mg_prec", "legendre_prec") and isinstance(v, str):
                v = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}[v]
            setattr(d, k, float(v) if k == "mg_eps" else int(v))
        dev = torch.cuda.current_device() if device is None else int(device)
        tune_key = None
        sht_only = d.solver == SOLVER_SHT
        if d.legendre_prec != FP64 and (d.mfma_ana_waves == 0 or d.mfma_syn_waves == 0 or
                                        (sht_only and d.mfma_der_waves == 0)):
            tune_key = _tune_key(dev, d)
            hit = _tune_load().get(tune_key)
            if hit and len(hit) == 3:
                d.mfma_ana_waves = d.mfma_ana_waves or int(hit[0])
                d.mfma_syn_waves = d.mfma_syn_waves or int(hit[1])
                if sht_only:
                    d.mfma_der_waves = d.mfma_der_waves or int(hit[2])
                tune_key = None
        h = ctypes.c_void_p()
        st = L.clm_plan_create(ctypes.byref(d), dev, ctypes.byref(h))
        if st != CLM_OK:
            raise ClmError(st, "clm_plan_create failed: %s" % L.clm_status_string(st).decode())
        self.h = h
        self.device = torch.device("cuda", dev)
        out = PlanDesc()
        L.clm_plan_get_desc(self.h, ctypes.byref(out))
        self.desc = {f: getattr(out, f) for f, _ in PlanDesc._fields_}
        nf = self.desc["nside_fine"]
        self.npix_fine = 12 * nf * nf
        self.npix_sht = 12 * self.desc["nside_sht"] ** 2
        self.lmax = self.desc["lmax"]
        if tune_key is not None:
            _tune_store(tune_key, self.desc["mfma_ana_waves"], self.desc["mfma_syn_waves"],
                        self.desc["mfma_der_waves"])

    def _check(self, st, what, h="self"):
        if st == CLM_OK:
            return
        L = lib()
        msg = "%s: %s" % (what, L.clm_status_string(st).decode())
        if h == "self" and getattr(self, "h", None):
            buf = ctypes.create_string_buffer(512)
            L.clm_plan_last_error(self.h, buf, 512)
            if buf.value:
                msg += " (" + buf.value.decode() + ")"
        raise ClmError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().clm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return lib().clm_plan_workspace_bytes(self.h)

    def set_timing(self, enable=True, stages=None):
        """Bracket the kernel launches of this plan with HIP events: every
        stage, or only those named in `stages` (an iterable of names)."""
        sel = None if not stages else ",".join(stages).encode()
        self._check(lib().clm_plan_set_timing_stages(self.h, sel), "set_timing_stages")
        self._check(lib().clm_plan_set_timing(self.h, int(enable)), "set_timing")

    def timings(self, nstages=64):
        """{stage: total ms} since the last reset, through clm_plan_timings
        and clm_plan_stage_name (synchronises, resets)."""
        ms = (ctypes.c_double * nstages)()
        self._check(lib().clm_plan_timings(self.h, ms, nstages), "timings")
        out = {}
        for i in range(nstages):
            nm = lib().clm_plan_stage_name(self.h, i)
            if nm is None:
                break
            out[nm.decode()] = ms[i]
        return out

    def get_timing(self):
        """{stage: (total ms, launches)} since the last call (synchronises)."""
        names = ctypes.create_string_buffer(4096)
        ms = (ctypes.c_double * 64)()
        cnt = (ctypes.c_int64 * 64)()
        ns = ctypes.c_int32()
        self._check(lib().clm_plan_get_timing(self.h, names, 4096, ms, cnt, 64,
                                              ctypes.byref(ns)), "get_timing")
        keys = names.value.decode().split(",") if names.value else []
        return {k: (ms[i], cnt[i]) for i, k in enumerate(keys[: ns.value])}

    def sync_status(self):
        """Synchronise and raise if a kernel latched an error."""
        self._check(lib().clm_plan_sync_status(self.h, _stream()), "device status")

    # ---------------------------------------------------------------- solve
    def poisson_solve(self, kappa, first_slot=0):
        k = kappa if kappa.dim() == 2 else kappa.reshape(1, -1)
        if k.dtype not in (torch.float64, torch.float32):
            raise ValueError("kappa must be float64 or float32")
        _dev(k, k.dtype)
        if k.shape[1] != self.npix_fine:
            raise ValueError("kappa has %d pixels, plan expects %d" % (k.shape[1], self.npix_fine))
        self._check(lib().clm_poisson_solve(self.h, _ptr(k), int(k.dtype == torch.float64),
                                            first_slot, k.shape[0], _stream()), "poisson_solve")

    def poisson_solve_particles(self, theta, phi, weight, sigma, slot=0):
        """The plane solve from particles (float64 tensors on the GPU):
        Epanechnikov deposition on the fine grid for the SHT step and, in
        SHT+MG plans, on the patch cells for the multigrid source."""
        for t in (theta, phi, weight, sigma):
            _dev(t, torch.float64)
        n = theta.numel()
        if not (phi.numel() == weight.numel() == sigma.numel() == n):
            raise ValueError("theta, phi, weight and sigma must have one value per particle")
        pr = Particles(theta.data_ptr(), phi.data_ptr(), weight.data_ptr(), sigma.data_ptr(), n)
        self._check(lib().clm_poisson_solve_particles(self.h, ctypes.byref(pr), slot, _stream()),
                    "poisson_solve_particles")

    def mg_convergence(self):
        """(epsilon [nbundle] float64, V-cycles [nbundle] int32) of the latest
        multigrid solve, per patch in bundle order."""
        nb = 12 * self.desc["nside_bundle"] ** 2
        eps = torch.empty(nb, dtype=torch.float64, device=self.device)
        cyc = torch.empty(nb, dtype=torch.int32, device=self.device)
        self._check(lib().clm_get_mg_convergence(self.h, _ptr(eps), _ptr(cyc), _stream()),
                    "get_mg_convergence")
        return eps, cyc

    def psi_alm(self, slot=0):
        out = torch.empty(nalm(self.lmax), 2, dtype=torch.float64, device=self.device)
        self._check(lib().clm_get_psi_alm(self.h, slot, _ptr(out), _stream()), "get_psi_alm")
        return torch.view_as_complex(out)

    def psi_map(self, slot=0):
        out = torch.empty(self.npix_sht, dtype=torch.float64, device=self.device)
        self._check(lib().clm_get_psi_map(self.h, slot, _ptr(out), _stream()), "get_psi_map")
        return out

    def patch_potential(self, first, npatch, slot=0):
        n = self.desc["patch_cells"]
        out = torch.empty(npatch, n, n, dtype=torch.float64, device=self.device)
        self._check(lib().clm_get_patch_potential(self.h, slot, first, npatch, _ptr(out),
                                                  _stream()), "get_patch_potential")
        return out

    def shear_from_potential(self, theta, phi, slot=0, fp64=True):
        _dev(theta, torch.float64)
        _dev(phi, torch.float64)
        n = theta.numel()
        dt = torch.float64 if fp64 else torch.float32
        g = torch.empty(2, n, dtype=dt, device=self.device)
        h = torch.empty(3, n, dtype=dt, device=self.device)
        self._check(lib().clm_shear_from_potential(self.h, slot, _ptr(theta), _ptr(phi), n,
                                                   int(fp64), _ptr(g), _ptr(h), _stream()),
                    "shear_from_potential")
        return g, h

    def shear_adjoint(self, theta, phi, dgrad, dhess, slot=0):
        """Accumulate the transpose of the point evaluation for dL/dgrad
        [2, n] and dL/dhess [3, n] (float64 device tensors)."""
        for t in (theta, phi, dgrad, dhess):
            _dev(t, torch.float64)
        n = theta.numel()
        self._check(lib().clm_shear_adjoint(self.h, slot, _ptr(theta), _ptr(phi), n,
                                            _ptr(dgrad), _ptr(dhess), _stream()),
                    "shear_adjoint")

    def poisson_adjoint(self, slot=0):
        """dL/dkappa (fine RING map, float64) from the accumulated adjoints."""
        out = torch.empty(self.npix_fine, dtype=torch.float64, device=self.device)
        self._check(lib().clm_poisson_adjoint(self.h, slot, _ptr(out), _stream()),
                    "poisson_adjoint")
        return out

    def shear_at_pixels(self, slot=0, order="ring", fp64=True, out=None):
        o = ORDER_RING if order == "ring" else ORDER_NESTED
        dt = torch.float64 if fp64 else torch.float32
        if out is None:
            g = torch.empty(2, self.npix_fine, dtype=dt, device=self.device)
            h = torch.empty(3, self.npix_fine, dtype=dt, device=self.device)
        else:
            g = _out(out[0], dt, 2 * self.npix_fine, "the gradient output")
            h = _out(out[1], dt, 3 * self.npix_fine, "the Hessian output")
        self._check(lib().clm_shear_at_pixels(self.h, slot, o, int(fp64), _ptr(g), _ptr(h),
                                              _stream()), "shear_at_pixels")
        return g, h

    def shear_at_pixels_batch(self, first_slot=0, nplanes=1, order="ring", fp64=True,
                              out=None):
        """Pure-SHT plans: gradient [nplanes][2][npix] and Hessian
        [nplanes][3][npix] of slots first_slot .. first_slot + nplanes - 1."""
        o = ORDER_RING if order == "ring" else ORDER_NESTED
        dt = torch.float64 if fp64 else torch.float32
        if out is None:
            g = torch.empty(nplanes, 2, self.npix_fine, dtype=dt, device=self.device)
            h = torch.empty(nplanes, 3, self.npix_fine, dtype=dt, device=self.device)
        else:
            g = _out(out[0], dt, nplanes * 2 * self.npix_fine, "the gradient output")
            h = _out(out[1], dt, nplanes * 3 * self.npix_fine, "the Hessian output")
        self._check(lib().clm_shear_at_pixels_batch(self.h, first_slot, nplanes, o, int(fp64),
                                                    _ptr(g), _ptr(h), _stream()),
                    "shear_at_pixels_batch")
        return g, h

    # ---------------------------------------------------------------- rays
    def new_rays(self):
        n = self.npix_fine
        f64 = dict(dtype=torch.float64, device=self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        r = dict(theta=torch.empty(n, **f64), phi=torch.empty(n, **f64),
                 beta=torch.empty(3, n, **f64), A=torch.empty(4, n, **f32),
                 A_prev=torch.empty(4, n, **f32))
        self.rays_init(r)
        return r

    @staticmethod
    def _rays_struct(r):
        return Rays(r["theta"].data_ptr(), r["phi"].data_ptr(), r["beta"].data_ptr(),
                    r["A"].data_ptr(), r["A_prev"].data_ptr(), r["theta"].numel())

    def rays_init(self, r):
        s = self._rays_struct(r)
        self._check(lib().clm_rays_init(self.h, ctypes.byref(s), _stream()), "rays_init")

    def set_domain(self, bundles=None):
        """Partial sky: the multigrid step, shear and rays over these NESTED
        bundles only (None or empty: the whole sky)."""
        b = np.ascontiguousarray([] if bundles is None else bundles, dtype=np.int32)
        ptr = b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if b.size else None
        self._check(lib().clm_plan_set_domain(self.h, ptr, b.size), "set_domain")

    def jacobian_spectra(self, rays):
        """SHT-only plans on the rays' grid: (alm [4][n_lm] complex128,
        cl [4][lmax+1] float64) of kappa, E, B and omega of the rays' A."""
        nlm = (self.lmax + 1) * (self.lmax + 2) // 2
        alm = torch.empty(4, nlm, dtype=torch.complex128, device=self.device)
        cl = torch.empty(4, self.lmax + 1, dtype=torch.float64, device=self.device)
        s = self._rays_struct(rays)
        self._check(lib().clm_jacobian_spectra(self.h, ctypes.byref(s), _ptr(alm), _ptr(cl),
                                               _stream()), "jacobian_spectra")
        return alm, cl

    def raytrace_planes(self, kappa, chi, first_plane, rays, K=0.0, galaxies=None):
        k = kappa if kappa.dim() == 2 else kappa.reshape(1, -1)
        _dev(k, k.dtype)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        s = self._rays_struct(rays)
        gp = None
        if galaxies is not None:
            g = Galaxies(galaxies["theta"].data_ptr(), galaxies["phi"].data_ptr(),
                         galaxies["chi"].data_ptr(), galaxies["A"].data_ptr(),
                         galaxies["theta"].numel())
            gp = ctypes.byref(g)
        self._check(lib().clm_raytrace_planes(
            self.h, _ptr(k), int(k.dtype == torch.float64),
            chi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), chi.size, first_plane,
            k.shape[0], K, ctypes.byref(s), gp, _stream()), "raytrace_planes")

    def galaxies_shell(self, chi, k, rays, galaxies, K=0.0):
        """eq. gatraj for the galaxies of shell k from the rays' current
        A (= A^(k)) and A_prev (= A^(k-1))."""
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        s = self._rays_struct(rays)
        g = Galaxies(galaxies["theta"].data_ptr(), galaxies["phi"].data_ptr(),
                     galaxies["chi"].data_ptr(), galaxies["A"].data_ptr(),
                     galaxies["theta"].numel())
        cp = chi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._check(lib().clm_galaxies_shell(self.h, cp, chi.size, k, K, ctypes.byref(s),
                                             ctypes.byref(g), _stream()), "galaxies_shell")

    def galaxies(self, rays, galaxies):
        """eq. gatraj for the galaxies of the shell the rays have just
        reached (distances of the latest ray update), through
        clm_galaxies_reduced."""
        s = self._rays_struct(rays)
        for k in ("theta", "phi", "chi"):
            _dev(galaxies[k], torch.float64)
        _dev(galaxies["A"], torch.float32)
        self._check(lib().clm_galaxies_reduced(self.h, ctypes.byref(s), _ptr(galaxies["theta"]),
                                       _ptr(galaxies["phi"]), _ptr(galaxies["chi"]),
                                       galaxies["theta"].numel(), _ptr(galaxies["A"]),
                                       _stream()), "galaxies")

    def galaxy_images(self, chi, k, rays, galaxies, radius=0.0, K=0.0):
        """The grid search for the images of the galaxies of shell k (after the
        ray update through plane k - 1): returns (theta_img, phi_img, found)
        device tensors [ngal] and writes galaxies["A"] (the Jacobian at the
        image) for the shell's galaxies."""
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        s = self._rays_struct(rays)
        n = galaxies["theta"].numel()
        g = Galaxies(galaxies["theta"].data_ptr(), galaxies["phi"].data_ptr(),
                     galaxies["chi"].data_ptr(), galaxies["A"].data_ptr(), n)
        th = torch.full((n,), float("nan"), dtype=torch.float64, device=self.device)
        ph = torch.full((n,), float("nan"), dtype=torch.float64, device=self.device)
        fd = torch.zeros(n, dtype=torch.int32, device=self.device)
        self._check(lib().clm_galaxy_images(self.h, chi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            chi.size, k, K, ctypes.byref(s), ctypes.byref(g),
                                            float(radius), _ptr(th), _ptr(ph), _ptr(fd),
                                            _stream()), "galaxy_images")
        return th, ph, fd

    def ray_update(self, chi, m, rays, slot=0, K=0.0):
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        s = self._rays_struct(rays)
        self._check(lib().clm_ray_update(self.h, slot,
                                         chi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         chi.size, m, K, ctypes.byref(s), _stream()),
                    "ray_update")


class PoissonShearFn(torch.autograd.Function):
    """kappa (fine RING map, float64) -> (grad [2, n], hess [3, n]) of psi at
    the points (theta, phi), differentiable in kappa: the forward pass is
    clm_poisson_solve + clm_shear_from_potential, the backward pass
    clm_shear_adjoint + clm_poisson_adjoint.  The plan must be SHT+MG with
    adjoint = 1."""

    @staticmethod
    def forward(ctx, kappa, theta, phi, plan, slot=0):
        plan.poisson_solve(kappa.detach().contiguous(), first_slot=slot)
        g, h = plan.shear_from_potential(theta, phi, slot=slot, fp64=True)
        ctx.plan, ctx.slot = plan, slot
        ctx.kappa_shape = kappa.shape
        ctx.save_for_backward(theta, phi)
        return g, h

    @staticmethod
    def backward(ctx, dg, dh):
        theta, phi = ctx.saved_tensors
        dg = torch.zeros(2, theta.numel(), dtype=torch.float64, device=theta.device) \
            if dg is None else dg.contiguous().double()
        dh = torch.zeros(3, theta.numel(), dtype=torch.float64, device=theta.device) \
            if dh is None else dh.contiguous().double()
        ctx.plan.shear_adjoint(theta, phi, dg, dh, slot=ctx.slot)
        grad = ctx.plan.poisson_adjoint(slot=ctx.slot)
        return grad.view(ctx.kappa_shape), None, None, None, None
