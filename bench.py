"""Benchmark: SHT+MG lens-plane steps per second at HEALPix Nside 2048 on one
MI355X.

One step is one pass of the whole hot path over one lens plane:
  kappa (device, float32, Nside 2048) -> demean + degrade to Nside 256 ->
  SHT analysis (lmax 512) -> psi_lm -> synthesis -> 12,288 patches of 256^2
  cells (bundles at Nside 32), 4 FAS V-cycles of red-black Gauss-Seidel ->
  gradient and shear at all 50,331,648 pixel centres -> update of 50,331,648
  rays (direction, position, Jacobian, transport) -> galaxies of the shell.
Input: lognormal convergence (sigma_g 0.5, C_l ~ l^-2 up to lmax 512, seed 3)
scaled to a 1 arcmin rms deflection; planes equally spaced in comoving
distance to z = 1.5 (20 planes of 152.735 h^-1 Mpc); 1e6 galaxies uniform on
the sphere with z ~ U[0.3, 1.5].  Inputs are resident in HBM before timing.

Prints one JSON line (see the keys below)."""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NF, NS, LMAX, NB, NCELL, VCYC = 2048, 256, 512, 32, 256, 4
EPS_RULE = 0.1  # the typical convergence parameter of Sec. 3.2
CHI_Z15 = 3054.70          # comoving distance to z = 1.5, h^-1 Mpc (flat, Omega_m 0.3)
PLANES_TO_Z15 = 20
DCHI = CHI_Z15 / PLANES_TO_Z15
NGAL = 1_000_000
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c2.txt")


def source_digest():
    """sha256 over the HIP sources; counter figures taken from other sources
    are stale."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1210_3069_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def stage_kernels(nbundle, ncell):
    """rocprof kernel name fragment and grid size (work-items) of each timed
    stage's kernel at this workload (float32 form)."""
    t0 = (ncell // 64) ** 2
    t1 = (ncell // 128) ** 2
    return {
        "patch_setup": ("k_patch_setup<float, 64>", nbundle * t0 * 512),
        "mg_pre_l0": ("k_mg_pre<float", nbundle * t0 * 512),
        "mg_post_l0": ("k_mg_post<float", nbundle * t0 * 512),
        "mg_postpre_l0": ("k_mg_postpre<float", nbundle * t0 * 1024),
        "mg_pre_l1+": ("k_mg_pre<float", nbundle * t1 * 512),
        "mg_post_l1+": ("k_mg_post<float", nbundle * t1 * 512),
        "mg_lds": ("k_mg_lds<float", None),
        "eval_pixels": ("k_eval<float", None),
        "ray_update": ("k_ray_update<float", None),
    }


def read_traffic(stage):
    """HBM bytes per launch of a stage from the committed counter summary, or
    None if absent or taken from other sources."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        parts = ln.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes_per_launch":
            kv[parts[1]] = float(parts[2])
        elif len(parts) == 2 and parts[0] == "source_sha256":
            kv["_sha"] = parts[1]
    if kv.get("_sha") != source_digest():
        return None
    return kv.get(stage)


def short_name(k):
    """Kernel name without namespaces, return type and parameter list."""
    k = k.replace("(anonymous namespace)::", "").replace("clm::", "")
    k = k[5:] if k.startswith("void ") else k
    depth = 0
    for i, ch in enumerate(k):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return k[:i]
    return k


def read_pmc(path, counter):
    """{(kernel, grid): [mean value per dispatch, dispatches]} of one counter."""
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], int(r["Grid_Size"]))
        v = acc.setdefault(key, [0.0, 0])
        v[0] += float(r["Counter_Value"])
        v[1] += 1
    return {k: [v[0] / v[1], v[1]] for k, v in acc.items()}


def summarize_pmc(fetch_csv, write_csv, fetch_cmd, write_cmd):
    """Counter summary text: FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per
    kernel, calibrated by the plain copy kernel of COPY_BYTES each way."""
    fe, wr = read_pmc(fetch_csv, "FETCH_SIZE"), read_pmc(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if "neg_kernel" in k[0]]
    if not copy:
        raise SystemExit("no copy-calibration dispatch in " + fetch_csv)
    cf = COPY_BYTES / (fe[copy[0]][0] * 1024.0)
    cw = COPY_BYTES / (wr[copy[0]][0] * 1024.0)
    out = ["# HBM traffic per dispatch, C2 workload (float32 form)",
           "# fetch pass: " + fetch_cmd, "# write pass: " + write_cmd,
           "# calibration: a copy kernel (torch.neg, float32) reading and writing "
           "%d bytes reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB"
           % (COPY_BYTES, fe[copy[0]][0], wr[copy[0]][0]),
           "calibration_fetch %.6f" % cf, "calibration_write %.6f" % cw,
           "source_sha256 " + source_digest(),
           "# kernel | grid | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated GB"]
    for k in sorted(fe, key=lambda k: -fe[k][0]):
        w = wr.get(k, [0.0, 0])[0]
        gb = (fe[k][0] * cf + w * cw) * 1024.0 / 1e9
        out.append("# %s | %d | %d | %.1f | %.1f | %.4f" % (short_name(k[0])[:90], k[1], fe[k][1],
                                                           fe[k][0], w, gb))
    nb = 12 * NB * NB
    for st, (frag, grid) in stage_kernels(nb, NCELL).items():
        ks = [k for k in fe if frag in k[0] and (grid is None or k[1] == grid)]
        if len(ks) == 1:
            k = ks[0]
            b = (fe[k][0] * cf + wr.get(k, [0.0])[0] * cw) * 1024.0
            out.append("traffic_bytes_per_launch %s %.0f" % (st, b))
    return "\n".join(out) + "\n"


def summarize_counters(pmc_csv, cmd, title):
    """Counter summary text: per kernel and grid, the mean of each counter
    per dispatch, with VALU and MFMA busy fractions where their inputs were
    collected (256 CUs, 1024 SIMDs)."""
    acc = {}
    for r in csv.DictReader(open(pmc_csv)):
        key = (short_name(r["Kernel_Name"])[:90], int(r["Grid_Size"]))
        d = acc.setdefault(key, {})
        v = d.setdefault(r["Counter_Name"], [0.0, 0])
        v[0] += float(r["Counter_Value"])
        v[1] += 1
    names = sorted({c for d in acc.values() for c in d})
    out = ["# " + title, "# command: " + cmd,
           "# kernel | grid | dispatches | " + " | ".join(names)]
    for key, d in sorted(acc.items(), key=lambda kv: -max(v[0] / v[1] for v in kv[1].values())):
        n = max(v[1] for v in d.values())
        vals = " | ".join("%.4g" % (d[c][0] / d[c][1]) if c in d else "-" for c in names)
        out.append("%s | %d | %d | %s" % (key[0], key[1], n, vals))
    return "\n".join(out) + "\n"


def summarize_stats(stats_csv, cmd, title="rocprofv3 kernel statistics, C2 workload"):
    """Kernel-trace summary text: per kernel calls and average duration, then
    per kernel and grid size (the levels of one kernel differ in grid) from the
    trace beside the statistics file."""
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["# " + title, "# command: " + cmd,
           "# kernel | calls | average us | total ms | percent"]
    for r in rows:
        out.append("%s | %s | %.1f | %.3f | %.2f" % (
            short_name(r["Name"])[:90], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    trace = stats_csv.replace("kernel_stats", "kernel_trace")
    if os.path.exists(trace):
        acc = {}
        for r in csv.DictReader(open(trace)):
            key = (short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]))
            v = acc.setdefault(key, [0, 0.0])
            v[0] += 1
            v[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        out.append("# per kernel and grid (work-items) from the trace: "
                   "kernel | grid | calls | average us")
        for k, v in sorted(acc.items(), key=lambda kv: -kv[1][1]):
            if v[1] > 100.0:
                out.append("%s | %d | %d | %.1f" % (k[0][:90], k[1], v[0], v[1] / v[0]))
    return "\n".join(out) + "\n"


def bytes_model(stage, plan_n, nbundle, npix, ncyc, launches=None):
    """Algorithmic HBM bytes of one launch of a stage (float32 multigrid):
    every array the step must read or write once, no halo re-reads.
    `launches` (per step) tells the finest level's pre-smoothing of the
    first cycle only (fused smoothing) from one per cycle."""
    cells = nbundle * plan_n * plan_n
    c1 = cells / 4
    first_only = launches is not None and launches <= 1
    return {
        # f' and du read, du written, ubar/rbar of the next level written; the
        # first cycle starts from du = 0 and skips its read
        "mg_pre_l0": cells * (4 + 4 + 2) if first_only
        else cells * (4 + 4 + 4 + 2) - cells * 4 / ncyc,
        # post-smoothing of a cycle fused with the next pre-smoothing: du, f'
        # and the coarse u_H, ubar read; du, ubar, rbar written
        "mg_postpre_l0": cells * (4 + 4 + 2 + 4 + 2),
        # du, f' and the coarse u_H, ubar read, du written
        "mg_post_l0": cells * (4 + 4 + 2 + 4),
        "mg_pre_l1+": c1 * (4 + 4 + 4 + 4 + 2),
        "mg_post_l1+": c1 * (4 + 4 + 2 + 4),
        # ubar, rbar of the 64^2 level read, u written
        "mg_lds": cells / 16 * 12,
        # u0 (float64, with ghosts) and f' written, fine kappa read once
        "patch_setup": nbundle * (plan_n + 2) ** 2 * 8 + cells * 4 + npix * 4,
        # five float32 outputs per pixel, u0 + du over the bundle cores read once
        "eval_pixels": npix * (20 + 12),
        # theta, phi, beta, A, A_prev read and written, patch cores read once
        "ray_update": npix * (2 * (8 + 8 + 24 + 16 + 16) + 12),
    }.get(stage)


def make_inputs(clm, torch, inputs, cosmo):
    alm = torch.from_numpy(inputs.gaussian_alm(LMAX, seed=3, sigma=0.5)).cuda()
    g = clm.alm2map(alm, LMAX, NF)
    e = torch.exp(g)
    s = inputs.deflection_scale(LMAX, 0.5)
    kappa = (s * (e - e.mean())).float().contiguous()
    del g, e
    th, ph, z = inputs.galaxy_redshifts(NGAL, seed=200)
    gal = dict(theta=torch.from_numpy(th).cuda(), phi=torch.from_numpy(ph).cuda(),
               chi=torch.from_numpy(cosmo.chi_of_z(z)).cuda(),
               A=torch.zeros(4, NGAL, dtype=torch.float32, device="cuda"))
    return kappa, gal


def plane_distances(nplanes):
    """Comoving distances of a run of lens planes equally spaced to z = 1.5,
    chi_m = (m + 1/2) dchi for m = 0 .. N - 1, followed by the target
    chi_N = (N + 1/2) dchi: N = 20 planes (dchi = 152.735 h^-1 Mpc), or more,
    with a finer spacing, when more steps are timed."""
    n = max(PLANES_TO_Z15, int(nplanes))
    return (np.arange(n + 1) + 0.5) * (CHI_Z15 / n)


def run_form(clm, torch, kappa, gal, prec, steps, warmup, vcycles=VCYC, eps=0.1,
             stage_steps=0, timed_stages=None, domain=None):
    """Times `steps` lens-plane steps (solve, shear at all pixels, ray update,
    galaxies of the shell) of one form on a fresh light cone.

    The warmup runs first, on planes 0, 1, ... of its own pass (the rays are
    reset when a pass reaches the last plane).  With stage_steps > 0 a second
    pass of that many steps, every launch bracketed by HIP events, gives the
    per-stage breakdown.  The timed pass then starts from reset rays and
    galaxies; only the stages in `timed_stages` (a list, or a function of
    the stage pass's events that returns one) carry events in it.
    Returns (plan, rays, ms per step, wall s, events of the timed pass,
    events of the stage pass)."""
    plan = clm.Plan(NF, nside_sht=NS, lmax=LMAX, nside_bundle=NB, patch_cells=NCELL,
                    mg_vcycles=vcycles, mg_eps=eps, mg_max_vcycles=20, mg_prec=prec)
    if domain is not None:
        plan.set_domain(domain)
    rays = plan.new_rays()
    chi = plane_distances(steps)
    last = len(chi) - 2                       # index of the last plane
    gout = (torch.empty(2, plan.npix_fine, dtype=torch.float32, device="cuda"),
            torch.empty(3, plan.npix_fine, dtype=torch.float32, device="cuda"))

    def step(m):
        plan.raytrace_planes(kappa, chi, m, rays, galaxies=gal)
        plan.shear_at_pixels(order="nested", fp64=False, out=gout)

    def fresh():
        plan.rays_init(rays)
        gal["A"].zero_()

    m = 0
    for _ in range(warmup):
        if m > last:
            fresh()
            m = 0
        step(m)
        m += 1
    torch.cuda.synchronize()
    plan.sync_status()
    stage_pass = {}
    if stage_steps > 0:
        fresh()
        plan.set_timing(True)
        plan.get_timing()
        for k in range(stage_steps):
            step(k)
        stage_pass = plan.get_timing()
        plan.set_timing(False)
        plan.sync_status()
    fresh()
    if callable(timed_stages):
        timed_stages = timed_stages(stage_pass)
    if timed_stages:
        plan.set_timing(True, stages=timed_stages)
        plan.get_timing()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    t0.record(stream)
    for k in range(steps):
        step(k)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms = t0.elapsed_time(t1) / steps
    timed = {}
    if timed_stages:
        timed = plan.get_timing()
        plan.set_timing(False)
    plan.sync_status()
    return plan, rays, ms, wall, timed, stage_pass


_ORACLE = {}


def _oracle_patch(b):
    """One patch of the oracle (in a worker process, one thread): setup,
    V-cycles, shear and one ray step at the bundle's pixels.  Returns the
    bundle, the patch potential u0 + du and the seconds it took."""
    from threadpoolctl import threadpool_limits
    from oracle import healpix as hp
    from oracle import mg as omg
    from oracle import rays as orays
    o = _ORACLE
    with threadpool_limits(1):
        t = time.perf_counter()
        R, u0, fp = omg.patch_setup(o["spec"], b, o["kap"], o["mean"], o["psi"])
        du = omg.mg_solve(o["spec"], fp)
        patch = dict(R=R, u0=u0, du=du)
        per = (NF // NB) ** 2
        pix = np.arange(b * per, (b + 1) * per)
        z, ph, s = hp.pix2ang_nest(NF, pix)
        th = np.arctan2(s, z)
        for k in range(per):
            g, U = omg.eval_point(o["spec"], patch, th[k], ph[k])
            orays.ray_step(orays.Ray(th[k], ph[k]), o["chi"], 0, g, U)
        return int(b), (u0 + du)[1:-1, 1:-1], time.perf_counter() - t


def host_cpu():
    """(usable cores, CPU model) of this host; the cores are the process's
    CPU affinity, capped at the 16 host cores that go with one GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(n, 16), n, model


def cpu_baseline(torch, kappa, plan64, nsample):
    """The FP64 oracle, as it stands, on a bounded sample of the same plane:
    the full SHT stage (numpy, one thread), then `nsample` patches evenly
    spread over the sphere (setup, 4 V-cycles, shear and one ray step at the
    bundle's pixels), spread over a pool of one-thread worker processes, one
    per usable core; scaled to one plane.  The per-patch worker times also
    give the one-core figure.  The GPU FP64 form's patch potentials are
    compared with the oracle's on the same patches."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import mg as omg
    cores, visible, model = host_cpu()
    kap = kappa.double().cpu().numpy()
    spec = omg.PatchSpec(NF, NS, LMAX, NB, ncell=NCELL, vcycles=VCYC)
    with threadpool_limits(1):
        t = time.perf_counter()
        mean, _, palm, psi = omg.sht_stage(spec, kap)
        t_sht = time.perf_counter() - t
    nb = 12 * NB * NB
    sample = sorted({int(round(i * (nb - 1) / max(1, nsample - 1))) for i in range(nsample)})
    _ORACLE.update(spec=spec, kap=kap, mean=mean, psi=psi,
                   chi=np.array([0.5 * DCHI, 1.5 * DCHI]))
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map_async(_oracle_patch, sample, chunksize=1).get(timeout=600)
    t_pool = time.perf_counter() - t
    _ORACLE.clear()
    worst = 0.0
    for b, ur, _ in res:
        ug = plan64.patch_potential(b, 1)[0].cpu().numpy()
        worst = max(worst, float(np.abs(ug - ur).max() / np.abs(ur).max()))
    t_patch = float(np.mean([r[2] for r in res]))
    t_plane = t_sht + t_pool / len(sample) * nb
    t_plane_1 = t_sht + t_patch * nb
    per = (NF // NB) ** 2
    return dict(value=1.0 / t_plane, unit="plane solves/s", cores=cores, kind="oracle",
                cpu_model=model, cpus_visible=visible,
                value_one_core=1.0 / t_plane_1,
                sample="full SHT stage on one thread (%.1f s) + %d of %d patches (setup, "
                       "4 V-cycles, shear and one ray step at their %d pixels; %.2f s each "
                       "on one core) over %d one-thread worker processes (%.1f s wall), "
                       "scaled to one plane"
                       % (t_sht, len(sample), nb, per, t_patch, cores, t_pool),
                sampled_patches=sample[:8] + (["..."] if len(sample) > 8 else []),
                gpu_fp64_vs_oracle_rel_err_u=worst)


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}
MFMA_PRODUCTS = {"fp32": 1, "bf16x3": 3, "bf16x6": 6}


def jacobian_spectra_summary(clm, torch, rays, nside, lmax):
    """Sec. 5 on the final plane of a ray tracing run: full-sky spectra of
    kappa, the shear E- and B-modes and the rotation omega of the rays'
    Jacobians (an FP64 SHT plan on the ray grid), the time of the call, and
    band averages of C_EE / C_kk (divided by (l-1)(l+2)/(l(l+1)), 1 for a
    Born-level shear), C_BB / C_EE, C_ww / C_EE and C_BB / C_ww."""
    sp = clm.Plan(nside, nside_sht=nside, lmax=lmax, solver="sht")
    sp.jacobian_spectra(rays)                      # first call: kernel set-up
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    _, cl = sp.jacobian_spectra(rays)
    t1.record()
    torch.cuda.synchronize()
    sp.sync_status()
    sp.close()
    cl = cl.cpu().numpy()
    l = np.arange(lmax + 1, dtype=np.float64)
    ee_kk = np.zeros_like(l)
    ok = l >= 2
    ee_kk[ok] = cl[1, ok] / cl[0, ok] * l[ok] * (l[ok] + 1) / ((l[ok] - 1) * (l[ok] + 2))
    bands = {}
    for lo, hi in ((10, 100), (100, 300), (300, 1000), (1000, lmax + 1)):
        b = slice(lo, min(hi, lmax + 1))
        bands["%d-%d" % (lo, min(hi, lmax + 1) - 1)] = dict(
            ee_over_kk_born=float(np.mean(ee_kk[b])),
            bb_over_ee=float(np.mean(cl[2, b] / cl[1, b])),
            ww_over_ee=float(np.mean(cl[3, b] / cl[1, b])),
            bb_over_ww=float(np.mean(cl[2, b] / cl[3, b])))
    return dict(ms=t0.elapsed_time(t1), lmax=lmax, bands=bands,
                note="kappa, E, B, omega of eq. invmagmat on the Nside %d ray grid, Jacobians "
                     "transported to the pixel centres, FP64 analyses" % nside)


def cap_bundles(nside_bundle, theta0, phi0, radius):
    """NESTED bundles whose centres lie within `radius` of (theta0, phi0)
    (host geometry of the benchmark's domain, through the library's own
    pixel centres)."""
    import torch
    from paper_1210_3069_amd import clm
    pl = clm.Plan(nside_bundle, nside_sht=nside_bundle, lmax=2, solver="sht")
    r = pl.new_rays()
    torch.cuda.synchronize()
    th, ph = r["theta"].cpu().numpy(), r["phi"].cpu().numpy()
    pl.close()
    v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    c = np.array([np.sin(theta0) * np.cos(phi0), np.sin(theta0) * np.sin(phi0), np.cos(theta0)])
    return np.nonzero(v @ c > np.cos(radius))[0]


def partial_sky_run(clm, torch, kappa, gal, steps, warmup, full_ms):
    """Sec. 3.4: the headline step with the multigrid, shear and rays
    restricted to a domain of about 1/8 of the sky (the bundles whose
    centres lie in a cap of half-angle 41.4 degrees about theta = 120 deg,
    phi = 0), the SHT still over the whole sky; the galaxies are those whose
    bundle lies in the cap shrunk by one bundle size.  Timed like the
    headline (stage pass, then the timed steps)."""
    theta0, radius = np.radians(120.0), np.arccos(0.75)
    dom = cap_bundles(NB, theta0, 0.0, radius)
    inner = cap_bundles(NB, theta0, 0.0, radius - 2.0 * np.sqrt(4 * np.pi / (12 * NB * NB)))
    th, ph = gal["theta"].cpu().numpy(), gal["phi"].cpu().numpy()
    v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    c = np.array([np.sin(theta0), 0.0, np.cos(theta0)])
    keep = np.nonzero(v @ c > np.cos(radius - 2.0 * np.sqrt(4 * np.pi / (12 * NB * NB))))[0]
    keep_t = torch.from_numpy(keep).cuda()
    g2 = {k: (gal[k][..., keep_t].contiguous()) for k in ("theta", "phi", "chi", "A")}
    S = 2
    plan, rays, ms, _, _, stages = run_form(clm, torch, kappa, g2, "fp32", steps, warmup,
                                            stage_steps=S, domain=dom)
    plan.close()
    del plan, rays
    torch.cuda.empty_cache()
    return dict(bundles=int(dom.size), sky_fraction=dom.size / (12.0 * NB * NB),
                inner_bundles=int(inner.size), galaxies=int(keep.size),
                ms_per_step=ms, value=1000.0 / ms, speedup_vs_whole_sky=full_ms / ms,
                stage_ms_per_step={k: v[0] / S for k, v in stages.items() if v[1]},
                workload="the headline step (Nside 2048, SHT Nside 256 / lmax 512 over the "
                         "whole sky) with multigrid, shear and rays over a cap of 1/8 of the "
                         "sky (theta0 120 deg, half-angle 41.4 deg)")


def particles_run(clm, torch, inputs, npart=4_000_000):
    """Sec. 3.2's input path: one lens plane from particles at the headline
    geometry (fine grid Nside 2048, SHT Nside 256 / lmax 512, 12,288
    patches of 256^2, 4 V-cycles, float32 multigrid).  A synthetic particle
    light cone (half field, half in halos; smoothing angles of 2-3 fine
    pixels), ordered by latitude-longitude tile of about 0.7 degrees (part
    of the input recipe) so that neighbouring threads deposit into
    neighbouring cells.  Timed: the Epanechnikov deposition on the fine
    grid, the SHT, the patch setup, the deposition on the patch cells and
    the V-cycles."""
    th, ph, w, sg = inputs.particle_cone(npart, seed=5, nside=NF)
    key = inputs.sky_order(th, ph, 256)
    args = [torch.from_numpy(np.ascontiguousarray(x[key])).cuda() for x in (th, ph, w, sg)]
    plan = clm.Plan(NF, nside_sht=NS, lmax=LMAX, nside_bundle=NB, patch_cells=NCELL,
                    mg_vcycles=VCYC, mg_prec="fp32")
    plan.poisson_solve_particles(*args)                 # kernel set-up
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    t0.record()
    for _ in range(reps):
        plan.poisson_solve_particles(*args)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    plan.set_timing(True)
    plan.get_timing()
    plan.poisson_solve_particles(*args)
    st = plan.get_timing()
    plan.set_timing(False)
    plan.sync_status()
    plan.close()
    m = torch.zeros(12 * NF * NF, dtype=torch.float64, device="cuda")
    clm.deposit_epanechnikov(*args, NF, out=m)
    torch.cuda.synchronize()
    t0.record()
    clm.deposit_epanechnikov(*args, NF, out=m)
    t1.record()
    torch.cuda.synchronize()
    map_ms = t0.elapsed_time(t1)
    mass = float(m.sum()) * 4 * np.pi / (12 * NF * NF) / 2.0   # two depositions
    pd = st.get("patch_deposit", (0.0, 1))[0]
    del m, args
    torch.cuda.empty_cache()
    return dict(particles=npart, ms_per_plane=ms, planes_per_s=1000.0 / ms,
                stage_ms={k: v[0] for k, v in st.items() if v[1]},
                fine_map_deposit_ms=map_ms, fine_map_particles_per_s=npart / (map_ms * 1e-3),
                patch_deposit_particles_per_s=npart / (pd * 1e-3) if pd else None,
                mass_conservation_rel=abs(mass - float(w.sum())) / float(w.sum()),
                workload="one plane from %d particles at the headline geometry (Nside 2048 "
                         "fine grid, SHT Nside 256 / lmax 512, 12,288 patches of 256^2, "
                         "4 V-cycles)" % npart)


def c3_run(clm, torch, inputs, cosmo, gal):
    """Multiplane ray tracing: 20 lens planes at chi_m = (m + 1/2) dchi to
    z = 1.5, each an Nside 2048 lognormal kappa (sigma_g 0.1 -> 0.6 with the
    plane index, C_l ~ l^-2 to lmax 2048, seeds 100 + m, scaled to a 1 arcmin
    rms deflection), solved by SHT at Nside 1024 / lmax 2048 + MG (12,288
    patches of 256^2, 4 V-cycles, float32 correction), 50.3M rays and the
    1e6 galaxies.  Inputs are generated on the GPU before timing; the 20
    plane steps (solve, shear, ray update, galaxies) are timed together."""
    nplanes, ns3, l3 = 20, 1024, 2048
    sig = inputs.multiplane_sigmas(nplanes)
    kap = torch.empty(nplanes, 12 * NF * NF, dtype=torch.float32, device="cuda")
    for m in range(nplanes):
        alm = torch.from_numpy(inputs.gaussian_alm(l3, seed=100 + m, sigma=sig[m])).cuda()
        e = torch.exp(clm.alm2map(alm, l3, NF))
        kap[m] = (inputs.deflection_scale(l3, sig[m]) * (e - e.mean())).float()
        del e
    plan = clm.Plan(NF, nside_sht=ns3, lmax=l3, nside_bundle=NB, patch_cells=NCELL,
                    mg_vcycles=VCYC, mg_prec="fp32")
    rays = plan.new_rays()
    chi = (np.arange(nplanes + 1) + 0.5) * DCHI
    # untimed pass over the first planes (kernel set-up), then the timed
    # pass from reset rays with events around the ray update only; a third
    # pass over 3 planes with every launch timed gives the stage breakdown
    for m in range(2):
        plan.raytrace_planes(kap[m], chi, m, rays, galaxies=gal)
    plan.rays_init(rays)
    gal["A"].zero_()
    torch.cuda.synchronize()
    plan.sync_status()
    plan.set_timing(True, stages=["ray_update"])
    plan.get_timing()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for m in range(nplanes):
        plan.raytrace_planes(kap[m], chi, m, rays, galaxies=gal)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ru = plan.get_timing().get("ray_update", (0.0, 1))
    plan.set_timing(False)
    plan.sync_status()
    npix = plan.npix_fine
    A = gal["A"].double()
    spectra = jacobian_spectra_summary(clm, torch, rays, NF, 2048)
    # a second pass over all planes with every launch timed: the stage
    # breakdown, and after each plane the grid search for the images of the
    # galaxies of the shell the rays have just reached (Sec. 3.3)
    rays2 = plan.new_rays()
    ng = gal["theta"].numel()
    gimg = dict(theta=gal["theta"], phi=gal["phi"], chi=gal["chi"], A=torch.zeros_like(gal["A"]))
    found = torch.zeros(ng, dtype=torch.int32, device="cuda")
    plan.set_timing(True)
    plan.get_timing()
    found += plan.galaxy_images(chi, 0, rays2, gimg)[2]
    for m in range(nplanes):
        plan.raytrace_planes(kap[m], chi, m, rays2)
        found += plan.galaxy_images(chi, m + 1, rays2, gimg)[2]
    tm = plan.get_timing()
    stages = {k: (v[0] / nplanes, v[1] / nplanes) for k, v in tm.items() if k != "galaxy_images"}
    img_ms = tm.get("galaxy_images", (0.0, 0))[0]
    plan.set_timing(False)
    plan.sync_status()
    # the Jacobian at the found image against the reduced step's (taken at
    # the galaxy's own position): they differ by the image-source offset
    Ai = gimg["A"].double()
    ok = found > 0
    dA = (Ai[:, ok] - A[:, ok]).abs().amax(0)
    images = dict(galaxies=ng, found=int(ok.sum()), ms_all_shells=img_ms,
                  galaxies_per_s=ng / max(img_ms * 1e-3, 1e-12),
                  jacobian_vs_reduced=dict(median=float(dA.median()) if dA.numel() else None,
                                           max=float(dA.max()) if dA.numel() else None))
    del rays2, gimg
    plan.close()
    del plan, rays
    torch.cuda.empty_cache()
    pure = c3_pure_sht(clm, torch, kap, chi, gal)
    out = dict(
        planes=nplanes, nside_sht=ns3, lmax=l3, ms_all_planes=ms, ms_per_plane=ms / nplanes,
        ray_plane_updates_per_s=dict(end_to_end=npix * nplanes / (ms * 1e-3),
                                     kernel_only=npix / (ru[0] / ru[1] * 1e-3)),
        stage_ms_per_plane={k: v[0] for k, v in stages.items()},
        stage_note="per plane, from a second pass with every launch timed",
        galaxy_images=images,
        final_plane_spectra=spectra,
        pure_sht_solver=pure,
        galaxies=int(gal["theta"].numel()),
        galaxies_with_A=int((A.abs().sum(0) > 0).sum()),
        galaxy_A_finite=bool(torch.isfinite(A).all()))
    del kap
    torch.cuda.empty_cache()
    return out


def c3_pure_sht(clm, torch, kap, chi, gal):
    """The same 20 planes and galaxies through the pure-SHT solver (Sec.
    3.2, last paragraph) at the ray grid: Nside 2048, lmax 4096, float32
    matrix-core form, 8 planes per derivative synthesis, g and U at the rays
    by transported four-point interpolation; timed over all planes (solve,
    fields, rays, galaxies), then the final-plane spectra as for SHT+MG."""
    nplanes = kap.shape[0]
    plan = clm.Plan(NF, nside_sht=NF, lmax=2 * NF, solver="sht", max_planes=8,
                    legendre_prec="fp32")
    rays = plan.new_rays()
    g2 = dict(gal, A=torch.zeros_like(gal["A"]))
    plan.raytrace_planes(kap[:1], chi, 0, rays, galaxies=g2)      # kernel set-up
    plan.rays_init(rays)
    g2["A"].zero_()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    plan.raytrace_planes(kap, chi, 0, rays, galaxies=g2)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    plan.sync_status()
    # a second pass with every launch timed: the stage breakdown
    rays2 = plan.new_rays()
    plan.set_timing(True)
    plan.get_timing()
    plan.raytrace_planes(kap, chi, 0, rays2)
    tm = plan.get_timing()
    plan.set_timing(False)
    plan.sync_status()
    del rays2
    plan.close()
    del plan
    torch.cuda.empty_cache()
    spectra = jacobian_spectra_summary(clm, torch, rays, NF, 2048)
    A = g2["A"]
    out = dict(ms_all_planes=ms, ms_per_plane=ms / nplanes,
               ray_plane_updates_per_s=12 * NF * NF * nplanes / (ms * 1e-3),
               stage_ms_per_plane={k: v[0] / nplanes for k, v in tm.items() if v[1]},
               galaxies_with_A=int((A.abs().sum(0) > 0).sum()),
               final_plane_spectra=spectra,
               workload="the C3 planes, rays and galaxies; pure-SHT solver at Nside 2048, lmax "
                        "4096 (float32 matrix-core form)")
    del rays, g2
    torch.cuda.empty_cache()
    return out


def _oracle_sht_plane(arg):
    """(convergence map, psi map) of one batched-precision plane from the
    oracle: Gaussian kappa synthesised at Nside n (lmax 2n, sigma 0.5), then
    demean, analysis, Poisson and synthesis (in a worker process)."""
    from threadpoolctl import threadpool_limits
    from oracle import sht as osht
    from paper_1210_3069_amd import inputs
    n, seed = arg
    with threadpool_limits(1):
        kap = osht.alm2map(n, 2 * n, inputs.gaussian_alm(2 * n, seed=seed, sigma=0.5))
        palm = osht.poisson(2 * n, osht.map2alm(n, 2 * n, kap - kap.mean()))
        return kap, osht.alm2map(n, 2 * n, palm)


def c4_run(clm, torch, inputs):
    """Batched precision forms: 32 pure-SHT Poisson solves at Nside drawn
    from {512, 1024, 2048} (lmax = 2 Nside, Gaussian kappa with sigma 0.5,
    C_l ~ l^-2, seeds 400 + i), grouped by Nside as GEMM columns.  Each form
    is timed over all planes; its psi maps are compared with the FP64 form's
    (relative L2 per plane) and, on the Nside 512 planes, with the oracle's;
    the matrix-core kernels' algorithmic flops
    (4 H n_lm per transform per plane, analysis and synthesis) over their
    HIP-event time give the MFMA throughput."""
    import multiprocessing as mp
    ns = inputs.c4_nsides()
    groups = {}
    for i, n in enumerate(ns):
        groups.setdefault(n, []).append(i)
    # the Nside 512 planes: convergence and psi map from the oracle (in worker
    # processes), so the forms' errors are measured against it on the same input
    n_or = min(groups)
    cores = host_cpu()[0]
    t = time.perf_counter()
    with mp.get_context("fork").Pool(min(cores, len(groups[n_or]))) as pool:
        orc = pool.map_async(_oracle_sht_plane, [(n_or, 400 + i) for i in groups[n_or]],
                             chunksize=1).get(timeout=900)
    t_or = time.perf_counter() - t
    kap = {}
    for n, idx in groups.items():
        if n == n_or:
            kap[n] = torch.from_numpy(np.stack([o[0] for o in orc])).cuda()
        else:
            kap[n] = torch.stack([clm.alm2map(torch.from_numpy(
                inputs.gaussian_alm(2 * n, seed=400 + i, sigma=0.5)).cuda(), 2 * n, n)
                for i in idx])
    psi_or = {i: torch.from_numpy(o[1]) for i, o in zip(groups[n_or], orc)}
    torch.cuda.synchronize()
    out, ref = {}, {}
    oracle_err = {}
    order = sorted(groups, reverse=True)          # largest grid first
    for form in ("fp64", "fp32", "bf16x3", "bf16x6"):
        ms_total, mfma_ms, flops, errs, stage_ms = 0.0, 0.0, 0.0, [], {}
        extra = {}
        if form == "fp64":
            # the FP64 form: vector Legendre transforms, one plan per grid
            for n in order:
                idx = groups[n]
                plan = clm.Plan(n, nside_sht=n, lmax=2 * n, solver="sht", max_planes=len(idx),
                                legendre_prec=form)
                plan.poisson_solve(kap[n][:1])          # first call: lazy set-up
                torch.cuda.synchronize()
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0.record()
                plan.poisson_solve(kap[n])
                t1.record()
                torch.cuda.synchronize()
                ms_total += t0.elapsed_time(t1)
                plan.sync_status()
                for k, i in enumerate(idx):
                    psi = plan.psi_map(k)
                    if i in psi_or:
                        oracle_err.setdefault(form, []).append(
                            float((psi.cpu() - psi_or[i]).norm() / psi_or[i].norm()))
                    ref[i] = psi
                plan.close()
                del plan
                torch.cuda.empty_cache()
        else:
            # the matrix-core forms: all grids in one clm_poisson_solve_multi
            # call (one persistent analysis and one synthesis launch), shapes
            # from the autotuner at plan creation
            t = time.perf_counter()
            plans = [clm.Plan(n, nside_sht=n, lmax=2 * n, solver="sht",
                              max_planes=len(groups[n]), legendre_prec=form) for n in order]
            t_create = time.perf_counter() - t
            ks = [kap[n] for n in order]
            clm.poisson_solve_multi(plans, ks)       # warm
            torch.cuda.synchronize()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            clm.poisson_solve_multi(plans, ks)
            t1.record()
            torch.cuda.synchronize()
            ms_total = t0.elapsed_time(t1)
            # a second pass with events around the two persistent launches
            plans[0].set_timing(True, stages=["sht_analysis_mfma", "sht_synthesis_mfma"])
            plans[0].get_timing()
            clm.poisson_solve_multi(plans, ks)
            st = plans[0].get_timing()
            plans[0].set_timing(False)
            mfma_ms = sum(st.get(k, (0.0, 0))[0] for k in ("sht_analysis_mfma",
                                                          "sht_synthesis_mfma"))
            stage_ms = {k: v[0] for k, v in st.items() if v[1]}
            # the same call captured in a HIP graph and replayed
            graph = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                with torch.cuda.graph(graph, stream=cs):
                    clm.poisson_solve_multi(plans, ks)
            torch.cuda.current_stream().wait_stream(cs)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            t0.record()
            for _ in range(3):
                graph.replay()
            t1.record()
            torch.cuda.synchronize()
            ms_graph = t0.elapsed_time(t1) / 3
            for pl in plans:
                pl.sync_status()
            extra = dict(graph_ms_all_planes=ms_graph, graph_planes_per_s=len(ns) * 1000.0 / ms_graph,
                         plan_create_s=t_create,
                         autotuned_waves={str(n): [pl.desc["mfma_ana_waves"], pl.desc["mfma_syn_waves"]]
                                          for n, pl in zip(order, plans)},
                         launches="one persistent analysis and one persistent synthesis launch "
                                  "over the three grids (waves per workgroup of the Nside %d "
                                  "plan)" % order[0])
            for n, pl in zip(order, plans):
                H = 2 * n
                nlm = (2 * n + 1) * (2 * n + 2) // 2
                flops += len(groups[n]) * 2 * 4.0 * H * nlm
                for k, i in enumerate(groups[n]):
                    psi = pl.psi_map(k)
                    if i in psi_or:
                        oracle_err.setdefault(form, []).append(
                            float((psi.cpu() - psi_or[i]).norm() / psi_or[i].norm()))
                    errs.append(float((psi - ref[i]).norm() / ref[i].norm()))
            del graph
            for pl in plans:
                pl.close()
            del plans
            torch.cuda.empty_cache()
        oe = oracle_err.get(form, [])
        tol = 1e-10 if form == "fp64" else 1e-6
        rec = dict(planes_per_s=len(ns) * 1000.0 / ms_total, ms_all_planes=ms_total,
                   stage_ms=stage_ms, **extra,
                   vs_oracle=dict(planes=len(oe), nside=n_or, max_rel_l2_psi=max(oe),
                                  median_rel_l2_psi=float(np.median(oe)), tolerance=tol,
                                  within_tolerance=bool(max(oe) <= tol)))
        if form != "fp64":
            tf = flops / (mfma_ms * 1e-3) / 1e12
            rec.update(legendre_ms=mfma_ms, legendre_alg_tflops=tf,
                       mfma_peak_tflops=MFMA_PEAK_TFLOPS[form],
                       mfma_frac=tf * MFMA_PRODUCTS[form] / MFMA_PEAK_TFLOPS[form],
                       max_rel_l2_psi_vs_fp64_form=max(errs),
                       median_rel_l2_psi_vs_fp64_form=float(np.median(errs)),
                       within_tolerance_1e6=bool(max(oe) <= 1e-6 and max(errs) <= 1e-6))
        out[form] = rec
    out["planes"] = {str(n): len(idx) for n, idx in sorted(groups.items())}
    out["oracle"] = ("FP64 oracle (numpy) psi maps of the %d Nside %d planes, computed in %d "
                     "worker processes in %.1f s; those planes' convergence maps are the "
                     "oracle's own synthesis" % (len(groups[n_or]), n_or,
                                                 min(cores, len(groups[n_or])), t_or))
    out["workload"] = ("32 planes, Nside from {512, 1024, 2048} (seed 4), lmax = 2 Nside, pure-SHT "
                       "Poisson; matrix-core forms: planes of one Nside are the GEMM columns, "
                       "the three grids share one persistent launch per Legendre stage")
    return out


def next2_run(clm, torch, inputs):
    """The pure-SHT solver as a production path at Nside 2048 (Sec. 3.2,
    last paragraph): 8 planes of Gaussian kappa (lmax 4096, sigma 0.5,
    C_l ~ l^-2, seeds 700 + i) solved as one GEMM batch on the matrix cores
    (float32 form), then the gradient and covariant Hessian at all 50.3M
    pixels of every plane by the matrix-core derivative synthesis (NESTED,
    float32 outputs).  Timed end to end; a second pass with events around
    the matrix-core launches gives their algorithmic rates (derivative
    synthesis: 2 flops x 10 real columns x H x n_lm per plane).  One plane
    of the FP64 form (vector Legendre sums) is timed beside it and its
    fields compared with the float32 form's."""
    N, lmax, P = 2048, 4096, 8
    npix = 12 * N * N
    kap = torch.stack([clm.alm2map(torch.from_numpy(
        inputs.gaussian_alm(lmax, seed=700 + i, sigma=0.5)).cuda(), lmax, N) for i in range(P)])
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=P, legendre_prec="fp32")
    t_create = time.perf_counter() - t
    g = torch.empty(P, 2, npix, dtype=torch.float32, device="cuda")
    h = torch.empty(P, 3, npix, dtype=torch.float32, device="cuda")

    def step():
        plan.poisson_solve(kap)
        plan.shear_at_pixels_batch(0, P, order="nested", fp64=False, out=(g, h))

    step()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 2
    t0.record()
    for _ in range(reps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    plan.set_timing(True)
    plan.get_timing()
    step()
    st = plan.get_timing()
    plan.set_timing(False)
    plan.sync_status()
    H = 2 * N
    nlm = (lmax + 1) * (lmax + 2) // 2
    mfma = {}
    for k, cols in (("sht_analysis_mfma", 2), ("sht_synthesis_mfma", 2), ("sht_deriv_mfma", 10)):
        tot, cnt = st.get(k, (0.0, 0))
        if cnt:
            tf = P * 2.0 * cols * H * nlm / (tot * 1e-3) / 1e12
            mfma[k] = dict(ms=tot, launches=int(cnt), alg_tflops=tf,
                           mfma_frac=tf / MFMA_PEAK_TFLOPS["fp32"])
    # one plane of the FP64 form beside it
    p64 = clm.Plan(N, nside_sht=N, lmax=lmax, solver="sht", max_planes=1)
    p64.poisson_solve(kap[:1])
    torch.cuda.synchronize()
    t0.record()
    g64, h64 = p64.shear_at_pixels(0, order="nested", fp64=True)
    t1.record()
    torch.cuda.synchronize()
    ms64 = t0.elapsed_time(t1)
    p64.sync_status()
    err = {}
    for k, name in enumerate(("g_t", "g_p")):
        d = g[0, k].double() - g64[k]
        err[name] = float(d.norm() / g64[k].norm())
    for k, name in enumerate(("U_tt", "U_pp", "U_tp")):
        d = h[0, k].double() - h64[k]
        err[name] = float(d.norm() / h64[k].norm())
    p64.close()
    plan.close()
    del plan, p64, g, h, g64, h64, kap
    torch.cuda.empty_cache()
    return dict(
        planes_per_s=P * 1000.0 / ms, ms_per_plane=ms / P, ms_all_planes=ms,
        stage_ms_per_plane={k: v[0] / P for k, v in st.items() if v[1]},
        matrix_core=mfma, plan_create_s=t_create,
        fp64_form=dict(deriv_ms_one_plane=ms64,
                       rel_l2_fp32_vs_fp64_form=err),
        workload="8 planes at Nside 2048, lmax 4096, pure-SHT Poisson solve (float32 "
                 "matrix-core analysis) + gradient and covariant Hessian at all 50.3M pixels "
                 "(matrix-core derivative synthesis, 8 planes per launch, 5 ring inverses "
                 "per plane)")


def c5_run(clm, torch, inputs):
    """Differentiation workload: 8 planes at Nside_fine (256, 512, 1024, 2048)
    x 2 (Nside_sht = Nside / 8, lmax = 2 Nside_sht, bundles Nside / 64,
    patches of 256^2, 4 V-cycles, FP64); lognormal kappa_true (sigma_g 0.5,
    seeds 500 + i), 1e5 uniform positions per plane (700 + i), observed shear
    = shear of kappa_true + N(0, 0.26^2) per component (600 + i); the chi^2
    gradient is taken at another draw kappa_eval (900 + i).  Timed: forward
    solve + shear at the points + transpose, per plane.  Checks: the dot
    product <F x, y> = <x, F^T y> per plane and central differences of the
    (exactly quadratic) chi^2 at random fine pixels (64 on the two smallest
    planes, 8 on the others)."""
    nsides = [256, 512, 1024, 2048] * 2
    plans = {}
    out = dict(planes=[], workload="8 planes Nside_fine 256..2048, 1e5 shear points each, "
                                   "chi^2 gradient through SHT+MG (FP64)")
    total_ms = 0.0
    for i, N in enumerate(nsides):
        if N not in plans:
            plans[N] = clm.Plan(N, nside_sht=N // 8, lmax=N // 4, nside_bundle=N // 64,
                                patch_cells=256, mg_vcycles=4, mg_prec="fp64", adjoint=1)
        plan = plans[N]
        lmax = N // 4

        def lognormal(seed):
            g = clm.alm2map(torch.from_numpy(inputs.gaussian_alm(lmax, seed=seed, sigma=0.5)).cuda(),
                            lmax, N)
            e = torch.exp(g)
            return (inputs.deflection_scale(lmax, 0.5) * (e - e.mean())).contiguous()
        k_true, k_eval = lognormal(500 + i), lognormal(900 + i)
        th, ph = (torch.from_numpy(a).cuda() for a in inputs.uniform_sphere(100000, seed=700 + i))
        rng = np.random.default_rng(600 + i)
        plan.poisson_solve(k_true)
        _, h = plan.shear_from_potential(th, ph)
        o1 = 0.5 * (h[0] - h[1]) + torch.from_numpy(0.26 * rng.standard_normal(th.numel())).cuda()
        o2 = h[2] + torch.from_numpy(0.26 * rng.standard_normal(th.numel())).cuda()

        def chi2_of(k):
            plan.poisson_solve(k)
            _, hh = plan.shear_from_potential(th, ph)
            r1, r2 = 0.5 * (hh[0] - hh[1]) - o1, hh[2] - o2
            return float(((r1 * r1 + r2 * r2) / 0.26 ** 2).sum()), r1, r2

        zero = torch.zeros(2, th.numel(), dtype=torch.float64, device="cuda")
        _, r1, r2 = chi2_of(k_eval)           # warm: forward and transpose
        plan.shear_adjoint(th, ph, zero, torch.stack([r1, -r1, 2.0 * r2]) / 0.26 ** 2)
        plan.poisson_adjoint()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c2, r1, r2 = chi2_of(k_eval)
        hb = torch.stack([r1, -r1, 2.0 * r2]) / 0.26 ** 2
        plan.shear_adjoint(th, ph, zero, hb)
        grad = plan.poisson_adjoint()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        total_ms += ms
        # dot-product test with random (x, y)
        x = torch.from_numpy(rng.standard_normal(plan.npix_fine) * float(k_eval.std())).cuda()
        plan.poisson_solve(x)
        g, hh = plan.shear_from_potential(th, ph)
        gy = torch.from_numpy(rng.standard_normal((2, th.numel()))).cuda()
        hy = torch.from_numpy(rng.standard_normal((3, th.numel()))).cuda()
        plan.shear_adjoint(th, ph, gy, hy)
        xt = plan.poisson_adjoint()
        lhs, rhs = float((g * gy).sum() + (hh * hy).sum()), float((x * xt).sum())
        # central differences
        npx = 64 if N <= 512 else 8
        step = 1e-3 * float(k_eval.pow(2).mean().sqrt())
        worst = 0.0
        gmax = float(grad.abs().max())
        for p in rng.choice(plan.npix_fine, npx, replace=False):
            e = torch.zeros_like(k_eval)
            e[p] = step
            fd = (chi2_of(k_eval + e)[0] - chi2_of(k_eval - e)[0]) / (2 * step)
            worst = max(worst, abs(fd - float(grad[p])) / (abs(float(grad[p])) + 1e-3 * gmax))
        # the loss is exactly quadratic: a large step removes the rounding of
        # the chi^2 sums from the comparison
        big = 10.0 * float(k_eval.pow(2).mean().sqrt())
        worst_big = 0.0
        for p in rng.choice(plan.npix_fine, 8, replace=False):
            e = torch.zeros_like(k_eval)
            e[p] = big
            fd = (chi2_of(k_eval + e)[0] - chi2_of(k_eval - e)[0]) / (2 * big)
            worst_big = max(worst_big, abs(fd - float(grad[p])) / (abs(float(grad[p])) + 1e-3 * gmax))
        plan.sync_status()
        out["planes"].append(dict(nside=N, ms_gradient=ms, chi2=c2,
                                  dot_product_rel=abs(lhs - rhs) / max(abs(lhs), abs(rhs)),
                                  fd_pixels=npx, fd_step=step, fd_max_rel=worst,
                                  fd_max_rel_step_10rms=worst_big))
    for pl in plans.values():
        pl.close()
    out["gradients_per_s"] = len(nsides) * 1000.0 / total_ms
    return out


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--stage-steps", type=int, default=5,
                    help="steps of the separate pass with every launch timed (per-stage table)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32,
                    help="patches of the oracle's timed sample")
    ap.add_argument("--no-eps", action="store_true",
                    help="skip the run under the epsilon stopping rule")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 20-plane ray tracing run")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the batched-precision workload (32 uneven pure-SHT planes)")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the differentiation workload (8 planes, chi^2 gradient)")
    ap.add_argument("--no-pure-sht", action="store_true",
                    help="skip the pure-SHT production path (8 planes at Nside 2048)")
    ap.add_argument("--no-particles", action="store_true",
                    help="skip the plane from particles (Epanechnikov deposition)")
    ap.add_argument("--no-partial-sky", action="store_true",
                    help="skip the partial-sky run (the headline step over 1/8 of the sky)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with a plain copy kernel of known size (counter calibration)")
    ap.add_argument("--summarize-stats", nargs="+", metavar="ARG",
                    help="CSV CMD [TITLE]: print a rocprofv3 --stats summary (no GPU)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("CSV", "CMD", "TITLE"),
                    help="print a per-kernel summary of a rocprofv3 --pmc run (no GPU)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "FCMD", "WCMD"),
                    help="print the HBM traffic summary of two --pmc passes (no GPU)")
    return ap.parse_args(argv)


def check_args(args):
    """(exit status, message) for a request this benchmark cannot run, else
    (0, None).  Any step and warmup counts are accepted: the timed steps are
    the planes of one light cone (20 planes to z = 1.5, or a finer spacing
    for more steps) and the warmup runs on its own passes."""
    if args.gpus != 1:
        return 2, ("bench.py runs on one GPU only: this build has no multi-GPU path "
                   "(--gpus %d requested)" % args.gpus)
    if args.steps < 1 or args.warmup < 0 or args.stage_steps < 0:
        return 2, "--steps must be >= 1 and --warmup, --stage-steps >= 0"
    return 0, None


def ranked_stages(stage_pass, nsteps, nbundle, npix):
    """The stages with a byte model, most time per step first."""
    ks = [k for k, (tot, cnt) in stage_pass.items()
          if bytes_model(k, NCELL, nbundle, npix, VCYC, cnt / nsteps) is not None]
    return sorted(ks, key=lambda k: -stage_pass[k][0])


def copy_rate(torch, nbytes=2 << 30, reps=5):
    """GB/s (bytes read + written) of a plain device-to-device copy."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def main():
    args = parse_args()
    if args.summarize_stats:
        sys.stdout.write(summarize_stats(*args.summarize_stats))
        return
    if args.summarize_counters:
        sys.stdout.write(summarize_counters(*args.summarize_counters))
        return
    if args.summarize_pmc:
        sys.stdout.write(summarize_pmc(*args.summarize_pmc))
        return
    rc, msg = check_args(args)
    if rc:
        print(msg, file=sys.stderr)
        sys.exit(rc)
    import torch
    from paper_1210_3069_amd import clm, cosmo, inputs
    clm.lib()
    torch.cuda.set_device(0)
    print("bench: generating inputs", file=sys.stderr, flush=True)
    kappa, gal = make_inputs(clm, torch, inputs, cosmo)
    torch.cuda.synchronize()
    npix = 12 * NF * NF
    nbundle = 12 * NB * NB
    S = max(1, min(args.stage_steps, args.steps)) if args.stage_steps else 1
    # stage pass first (every launch timed), then the timed pass with events
    # around the dominant kernel's launches only
    print("bench: fp32 form (stage pass %d steps, then %d timed steps)" % (S, args.steps),
          file=sys.stderr, flush=True)
    picked = {}

    def pick(stage_pass):
        ranked = ranked_stages(stage_pass, S, nbundle, npix)
        picked["dom"] = ranked[0]
        picked["next"] = ranked[1] if len(ranked) > 1 else None
        return ranked[:2]

    plan, rays, ms, wall, timed, stages = run_form(clm, torch, kappa, gal, "fp32", args.steps,
                                                   args.warmup, stage_steps=S,
                                                   timed_stages=pick)
    sample = list(range(0, nbundle, 64))
    u32 = torch.stack([plan.patch_potential(b, 1)[0] for b in sample]).cpu()
    plan.close()
    del plan, rays
    torch.cuda.empty_cache()
    print("bench: fp32 form %.3f ms/step" % ms, file=sys.stderr, flush=True)

    per_stage = {}
    for k, (tot, cnt) in stages.items():
        per_stage[k] = dict(ms_per_step=tot / S, launches_per_step=cnt / S,
                            ms_per_launch=tot / max(cnt, 1))
        b = bytes_model(k, NCELL, nbundle, npix, VCYC, cnt / S)
        if b is not None:
            per_stage[k]["alg_GBps"] = b / (tot / cnt * 1e-3) / 1e9
        t = read_traffic(k)
        if t is not None:
            per_stage[k]["hbm_GB_per_launch"] = t / 1e9
            per_stage[k]["hbm_GBps"] = t / (per_stage[k]["ms_per_launch"] * 1e-3) / 1e9
    copy_gbs = copy_rate(torch)

    def stage_roofline(st):
        tot, cnt = timed[st]
        b_st = bytes_model(st, NCELL, nbundle, npix, VCYC, cnt / args.steps)
        ms_launch = tot / cnt
        achieved = b_st / (ms_launch * 1e-3) / 1e9
        traffic = read_traffic(st)
        return dict(bound="hbm", kernel=st, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS,
                    copy_GBps=copy_gbs, frac_of_copy=achieved / copy_gbs,
                    copy_note="a plain device-to-device copy of 2 GiB (read + write bytes), "
                              "timed in this run: the streaming rate the HBM reaches in practice",
                    traffic=None if traffic is None else traffic / 1e9,
                    traffic_unit="GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                    alg_bytes_per_launch=b_st, ms_per_launch=ms_launch,
                    ms_per_step=tot / args.steps, launches_timed=int(cnt),
                    timing="HIP events around each launch of this kernel, on its stream, "
                           "over the timed steps")

    roofline = stage_roofline(picked["dom"])
    # the kernel second in time per step, measured the same way (the fused
    # smoother and the patch setup take nearly equal time per step)
    runner_up = stage_roofline(picked["next"]) if picked.get("next") in timed else None
    ru = stages.get("ray_update", (0.0, 1))

    out = {
        "metric": "SHT+MG plane solves/s @Nside 2048",
        "value": 1000.0 / ms,
        "unit": "plane solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_s_timed": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "multigrid correction float32; SHT, u0, f', geometry and rays float64; "
                        "ray Jacobians stored float32",
        "data": "synthetic",
        "config": {"workload": "one lens plane per step at Nside 2048: SHT Nside 256 lmax 512 "
                               "+ MG 12288 patches 256^2, 4 V-cycles (2,2) + shear at "
                               "50.3M pixels + 50.3M-ray update + 1e6 galaxies",
                   "nside_fine": NF, "nside_sht": NS, "lmax": LMAX, "nside_bundle": NB,
                   "patch_cells": NCELL, "vcycles": VCYC, "rays": npix, "galaxies": NGAL,
                   "planes_in_light_cone": len(plane_distances(args.steps)) - 1},
        "ray_plane_updates_per_s": {
            "end_to_end": npix * 1000.0 / ms,
            "kernel_only": npix / (ru[0] / max(ru[1], 1) * 1e-3)},
        "stages": per_stage,
        "stage_pass": {"steps": S, "note": "separate pass with HIP events around every launch",
                       "ms_per_step_sum_of_stages": sum(v["ms_per_step"] for v in per_stage.values())},
        "roofline": roofline,
        "roofline_runner_up": runner_up,
    }
    if not args.no_fp64:
        print("bench: fp64 form", file=sys.stderr, flush=True)
        plan64, rays64, ms64, _, _, _ = run_form(clm, torch, kappa, gal, "fp64", args.steps,
                                                 args.warmup)
        u64 = torch.stack([plan64.patch_potential(b, 1)[0] for b in sample]).cpu()
        d = (u32 - u64).double()
        out["fp64_form"] = dict(ms_per_step=ms64, value=1000.0 / ms64,
                                fp32_vs_fp64_rel_l2_u=float(d.norm() / u64.norm()),
                                sampled_patches=len(sample))
        del rays64
        if not args.no_cpu_baseline:
            print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(torch, kappa, plan64, max(1, args.cpu_sample))
        plan64.close()
        del plan64
        torch.cuda.empty_cache()
    if not args.no_eps:
        # the stopping rule of Sec. 3.2 in place of the fixed cycle count
        print("bench: epsilon rule", file=sys.stderr, flush=True)
        pe, re_, mse, _, st_e, _ = run_form(clm, torch, kappa, gal, "fp32", args.steps,
                                            args.warmup, vcycles=0, eps=EPS_RULE,
                                            timed_stages=["mg_eps"])
        e, k = (t.cpu().numpy() for t in pe.mg_convergence())
        ue = torch.stack([pe.patch_potential(b, 1)[0] for b in sample]).cpu()
        d = (ue - u32).double()
        out["eps_rule"] = dict(
            mg_eps=EPS_RULE, ms_per_step=mse, value=1000.0 / mse,
            vcycles_histogram={int(c): int((k == c).sum()) for c in np.unique(k)},
            eps_max=float(e.max()), eps_median=float(np.median(e)),
            mg_eps_ms_per_step=st_e.get("mg_eps", (0.0, 0))[0] / args.steps,
            rel_l2_u_vs_fixed=float(d.norm() / u32.double().norm()),
            note="convergence figures are the last plane's")
        pe.close()
        del pe, re_
        torch.cuda.empty_cache()
    if not args.no_partial_sky:
        print("bench: partial sky", file=sys.stderr, flush=True)
        out["partial_sky"] = partial_sky_run(clm, torch, kappa, gal, args.steps, args.warmup, ms)
    if not args.no_particles:
        print("bench: plane from particles", file=sys.stderr, flush=True)
        out["particles_plane"] = particles_run(clm, torch, inputs)
    if not args.no_c3:
        print("bench: multiplane ray tracing", file=sys.stderr, flush=True)
        out["c3_multiplane"] = c3_run(clm, torch, inputs, cosmo, gal)
    if not args.no_c4:
        print("bench: batched precision forms", file=sys.stderr, flush=True)
        out["c4_precision_forms"] = c4_run(clm, torch, inputs)
    if not args.no_c5:
        print("bench: differentiation", file=sys.stderr, flush=True)
        out["c5_gradient"] = c5_run(clm, torch, inputs)
    if not args.no_pure_sht:
        print("bench: pure-SHT solver", file=sys.stderr, flush=True)
        out["pure_sht_nside2048"] = next2_run(clm, torch, inputs)
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
