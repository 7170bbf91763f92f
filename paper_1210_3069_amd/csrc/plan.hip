// Plan creation, workspace, geometry tables and the small C-ABI entry points
// (status, getters, dispatch to the stage launchers).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "clm_internal.h"
#include "healpix_dev.h"

namespace clm {

int Plan::stage_id(const char* name) {
  for (size_t i = 0; i < stage_names.size(); ++i)
    if (stage_names[i] == name) return int(i);
  stage_names.push_back(name);
  return int(stage_names.size()) - 1;
}

hipEvent_t Plan::take_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

Plan::~Plan() {
  for (auto& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : pool) (void)hipEventDestroy(e);
  auto f = [](void* q) { if (q) (void)hipFree(q); };
  f(ring_s); f(ringi_s); f(ringx_s); f(ring_f); f(ringi_f); f(ringx_f); f(lam_mant);
  f(lam_scale); f(blu_off); f(blu);
  f(r2n_s); f(r2n_f); f(rot); f(coef); f(rowt); f(cinv); f(kap_s); f(F); f(G); f(red);
  f(rcoef); f(dcoef); f(Fb); f(Gb); f(apart); f(psib); f(mfma_ctr);
  f(deriv); f(fprime); f(dutmp); f(status_dev); f(iter_map); f(iter_alm);
  for (auto* q : ubar) f(q);
  f(ubar1b);
  f(setup_meta); f(spad); f(kpad);
  for (auto* q : rbar) f(q);
  for (auto* q : flev) f(q);
  for (auto* q : ulev) f(q);
  for (auto* q : ulev2) f(q);
  for (auto& s : slots) { f(s.alm); f(s.psi_s); f(s.u0); f(s.du); }
  f(adj_ubar); f(adj_psi); f(adj_ks); f(adj_alm); f(adj_psi_priv); f(adj_rrows);
  f(mg_eps_dev); f(mg_cycles_dev); f(mg_done_dev); f(mg_eps_part); f(mg_active_dev);
  f(dom_map); f(dom_flag);
  if (mg_active_host) (void)hipHostFree(mg_active_host);
  for (auto* q : adj_u) f(q);
  for (auto* q : adj_v) f(q);
  for (auto* q : adj_f) f(q);
  for (auto* q : adj_w) f(q);
}

namespace {

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Host ring tables of a HEALPix grid (rings 1..4N-1 stored 0-based).
void host_rings(int N, std::vector<double>& rt, std::vector<int>& ri, std::vector<double>& rx) {
  const int nr = 4 * N - 1;
  rt.assign(4 * nr, 0.0);
  ri.assign(2 * nr, 0);
  const double pi = 3.14159265358979323846;
  for (int q = 0; q < nr; ++q) {
    const int64_t i = q + 1;
    double z, st;
    int64_t n, first;
    bool shifted = true;
    if (i < N) {
      const double omz = double(i) * double(i) / (3.0 * N * N);
      z = 1.0 - omz;
      st = std::sqrt(omz * (1.0 + z));
      n = 4 * i;
      first = 2 * i * (i - 1);
    } else if (i <= 3 * N) {
      z = (4.0 * N - 2.0 * i) / (3.0 * N);
      st = std::sqrt((1.0 - z) * (1.0 + z));
      n = 4 * N;
      first = 2 * int64_t(N) * (N - 1) + 4 * int64_t(N) * (i - N);
      shifted = ((i - N) % 2) == 0;
    } else {
      const int64_t ip = 4 * N - i;
      const double opz = double(ip) * double(ip) / (3.0 * N * N);
      z = opz - 1.0;
      st = std::sqrt(opz * (2.0 - opz));
      n = 4 * ip;
      first = 12 * int64_t(N) * N - 2 * ip * (ip + 1);
    }
    rt[4 * q + 0] = z;
    rt[4 * q + 1] = st;
    rt[4 * q + 2] = std::atan2(st, z);
    rt[4 * q + 3] = shifted ? pi / double(n) : 0.0;
    ri[2 * q + 0] = int(n);
    ri[2 * q + 1] = int(first);
  }
  // interpolation helpers: n/(2 pi) per ring, reciprocal theta gaps
  rx.assign(2 * (nr + 1), 0.0);
  for (int q = 0; q < nr; ++q) {
    rx[2 * q] = double(ri[2 * q]) / (2.0 * pi);
    rx[2 * q + 1] = 1.0 / (rt[4 * q + 2] - (q ? rt[4 * (q - 1) + 2] : 0.0));
  }
  rx[2 * nr + 1] = 1.0 / (pi - rt[4 * (nr - 1) + 2]);
}

__global__ void k_ring2nest(int64_t N, int* table) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= 12 * N * N) return;
  table[hpx::nest2ring(N, p)] = int(p);
}

// R_b rows (c, phi-hat_c, -theta-hat_c) for every bundle (NESTED index).
__global__ void k_rotations(int64_t Nb, int64_t nb, double* rot) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double z, st, phi;
  hpx::pix2ang_ring(Nb, hpx::nest2ring(Nb, b), z, st, phi);
  const double cp = cos(phi), sp = sin(phi);
  double* R = rot + 9 * b;
  R[0] = st * cp; R[1] = st * sp; R[2] = z;        // c
  R[3] = -sp;     R[4] = cp;      R[5] = 0.0;      // phi-hat
  R[6] = -z * cp; R[7] = -z * sp; R[8] = st;       // -theta-hat
}

template <typename T>
clm_status alloc(Plan* p, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return CLM_OK;
  hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    p->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed";
    return CLM_ENOMEM;
  }
  p->bytes += count * sizeof(T);
  return CLM_OK;
}

clm_status adjoint_alloc(Plan* p) {
  if (!p->mg) return CLM_OK;
  const size_t G = size_t(p->n + 2) * (p->n + 2);
  clm_status s;
  if ((s = alloc(p, &p->adj_ubar, size_t(p->nbundle) * G)) != CLM_OK) return s;
  p->adj_u.assign(p->nlev, nullptr);
  p->adj_v.assign(p->nlev, nullptr);
  p->adj_f.assign(p->nlev, nullptr);
  p->adj_w.assign(p->nlev, nullptr);
  for (int l = 0; l < p->nlev; ++l) {
    const size_t c = size_t(p->nbundle) * (p->n >> l) * (p->n >> l);
    if ((s = alloc(p, &p->adj_u[l], c)) != CLM_OK) return s;
    if ((s = alloc(p, &p->adj_v[l], c)) != CLM_OK) return s;
    if ((s = alloc(p, &p->adj_f[l], c)) != CLM_OK) return s;
    if ((s = alloc(p, &p->adj_w[l], c)) != CLM_OK) return s;
  }
  if ((s = alloc(p, &p->adj_psi, size_t(p->npix_s))) != CLM_OK) return s;
  // private copies of the SHT-grid accumulator (at most 256 MB, 64 copies)
  p->adj_ncopy = int(std::max<int64_t>(1, std::min<int64_t>(64, (int64_t(1) << 28) /
                                                                    (p->npix_s * 8))));
  if ((s = alloc(p, &p->adj_psi_priv, size_t(p->adj_ncopy) * p->npix_s)) != CLM_OK) return s;
  if ((s = alloc(p, &p->adj_ks, size_t(p->npix_s))) != CLM_OK) return s;
  if ((s = alloc(p, &p->adj_alm, size_t(p->nalm) * 2)) != CLM_OK) return s;
  if (hipMemset(p->adj_ubar, 0, size_t(p->nbundle) * G * 8) != hipSuccess) return CLM_EHIP;
  size_t nrows = 0;
  for (int l = 0; l < p->nlev; ++l) nrows += size_t(p->n >> l);
  if ((s = alloc(p, &p->adj_rrows, 4 * nrows)) != CLM_OK) return s;
  return adjoint_tables(p);
}


#define CLM_TRY(x)                   \
  do {                               \
    clm_status s_ = (x);             \
    if (s_ != CLM_OK) return s_;     \
  } while (0)

// Dense inverse (Gauss-Jordan, partial pivoting) of an n x n matrix.
bool invert(std::vector<double>& a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(a[c * n + k], a[piv * n + k]);
      std::swap(inv[c * n + k], inv[piv * n + k]);
    }
    const double d = a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] /= d; inv[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        inv[r * n + k] -= f * inv[c * n + k];
      }
    }
  }
  a = inv;
  return true;
}

}  // namespace

clm_status build_tables(Plan* p) {
  const clm_plan_desc& d = p->d;
  std::vector<double> rt, rx;
  std::vector<int> ri;
  host_rings(d.nside_sht, rt, ri, rx);
  CLM_TRY(alloc(p, &p->ring_s, rt.size()));
  CLM_TRY(alloc(p, &p->ringi_s, ri.size()));
  CLM_TRY(alloc(p, &p->ringx_s, rx.size()));
  CLM_HIP(hipMemcpy(p->ring_s, rt.data(), rt.size() * 8, hipMemcpyHostToDevice));
  CLM_HIP(hipMemcpy(p->ringi_s, ri.data(), ri.size() * 4, hipMemcpyHostToDevice));
  CLM_HIP(hipMemcpy(p->ringx_s, rx.data(), rx.size() * 8, hipMemcpyHostToDevice));
  host_rings(d.nside_fine, rt, ri, rx);
  CLM_TRY(alloc(p, &p->ring_f, rt.size()));
  CLM_TRY(alloc(p, &p->ringi_f, ri.size()));
  CLM_TRY(alloc(p, &p->ringx_f, rx.size()));
  CLM_HIP(hipMemcpy(p->ring_f, rt.data(), rt.size() * 8, hipMemcpyHostToDevice));
  CLM_HIP(hipMemcpy(p->ringi_f, ri.data(), ri.size() * 4, hipMemcpyHostToDevice));
  CLM_HIP(hipMemcpy(p->ringx_f, rx.data(), rx.size() * 8, hipMemcpyHostToDevice));

  CLM_TRY(ring_plan(p));

  // Legendre starting values on the north rings of the SHT grid
  CLM_TRY(alloc(p, &p->lam_mant, size_t(d.lmax + 1) * p->H));
  CLM_TRY(alloc(p, &p->lam_scale, size_t(d.lmax + 1) * p->H));
  hipLaunchKernelGGL(k_lambda_mm, dim3((p->H + 127) / 128), dim3(128), 0, 0, p->ring_s, p->H,
                     d.lmax, p->lam_mant, p->lam_scale);
  CLM_LAUNCH_CHECK();

  CLM_TRY(alloc(p, &p->r2n_s, size_t(p->npix_s)));
  hipLaunchKernelGGL(k_ring2nest, dim3((p->npix_s + 255) / 256), dim3(256), 0, 0,
                     int64_t(d.nside_sht), p->r2n_s);
  CLM_LAUNCH_CHECK();
  CLM_TRY(alloc(p, &p->r2n_f, size_t(p->npix_f)));
  hipLaunchKernelGGL(k_ring2nest, dim3((p->npix_f + 255) / 256), dim3(256), 0, 0,
                     int64_t(d.nside_fine), p->r2n_f);
  CLM_LAUNCH_CHECK();

  if (!p->mg) return CLM_OK;

  CLM_TRY(alloc(p, &p->rot, size_t(p->nbundle) * 9));
  hipLaunchKernelGGL(k_rotations, dim3((p->nbundle + 127) / 128), dim3(128), 0, 0,
                     int64_t(d.nside_bundle), p->nbundle, p->rot);
  CLM_LAUNCH_CHECK();

  // finite-volume Laplacian row coefficients per level:
  // s_m = sin theta'_{i-1/2}, s_p = sin theta'_{i+1/2}, s_c = sin theta'_i,
  // area = 2 Delta_k sin theta'_i sin(Delta_k / 2)
  const double pi = 3.14159265358979323846;
  std::vector<double> cf;
  for (int l = 0; l < p->nlev; ++l) {
    const int nk = p->n >> l;
    p->lev.push_back({nk, cf.size()});
    const double dk = p->L / nk;
    for (int i = 0; i < nk; ++i) {
      const double e0 = pi / 2 - p->L / 2 + i * dk;
      const double e1 = pi / 2 - p->L / 2 + (i + 1) * dk;
      const double tc = 0.5 * (e0 + e1);
      cf.push_back(std::sin(e0));
      cf.push_back(std::sin(e1));
      cf.push_back(std::sin(tc));
      cf.push_back(2.0 * dk * std::sin(tc) * std::sin(0.5 * dk));
    }
  }
  CLM_TRY(alloc(p, &p->coef, cf.size()));
  CLM_HIP(hipMemcpy(p->coef, cf.data(), cf.size() * 8, hipMemcpyHostToDevice));

  // the tile kernels' row table (same row order as cf, 8 values per row):
  // a patch face above or below the row adds its missing neighbour's
  // coefficient to the diagonal (ghost = -u); a side face adds 1 / s_c
  {
    std::vector<double> rt(2 * cf.size(), 0.0);
    for (const LevelGeom& lg : p->lev)
      for (int i = 0; i < lg.n; ++i) {
        const double* c = cf.data() + lg.crow + 4 * i;
        double* r = rt.data() + 2 * (lg.crow + 4 * i);
        const double ic = 1.0 / c[2];
        const double e = (i == 0 ? c[0] : 0.0) + (i == lg.n - 1 ? c[1] : 0.0);
        const double dg = c[0] + c[1] + 2.0 * ic + e;
        r[0] = c[0]; r[1] = c[1]; r[2] = ic; r[3] = c[3]; r[4] = e;
        r[5] = 1.0 / dg;
        r[6] = 1.0 / (dg + ic);
        r[7] = (i % 2 == 0 && i + 1 < lg.n) ? 1.0 / (2.0 * (c[3] + c[7])) : 0.25;
      }
    if (p->fp64mg) {
      double* q = nullptr;
      CLM_TRY(alloc(p, &q, rt.size()));
      p->rowt = q;
      CLM_HIP(hipMemcpy(q, rt.data(), rt.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> r32(rt.begin(), rt.end());
      float* q = nullptr;
      CLM_TRY(alloc(p, &q, r32.size()));
      p->rowt = q;
      CLM_HIP(hipMemcpy(q, r32.data(), r32.size() * 4, hipMemcpyHostToDevice));
    }
  }

  // coarsest level (4 x 4): dense operator with zero face values, inverted
  {
    const int nc = 4;
    const double* c = cf.data() + p->lev.back().crow;
    std::vector<double> M(16 * 16, 0.0);
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) {
        const double sm = c[4 * i], sp = c[4 * i + 1], sc = c[4 * i + 2], A = c[4 * i + 3];
        const int row = i * nc + j;
        double diag = sm + sp + 2.0 / sc;
        if (i > 0) M[row * 16 + (i - 1) * nc + j] += sm / A; else diag += sm;
        if (i < nc - 1) M[row * 16 + (i + 1) * nc + j] += sp / A; else diag += sp;
        if (j > 0) M[row * 16 + i * nc + j - 1] += 1.0 / (sc * A); else diag += 1.0 / sc;
        if (j < nc - 1) M[row * 16 + i * nc + j + 1] += 1.0 / (sc * A); else diag += 1.0 / sc;
        M[row * 16 + row] -= diag / A;
      }
    if (!invert(M, 16)) return fail(p, CLM_EINVAL, "singular coarsest operator");
    CLM_TRY(alloc(p, &p->cinv, 256));
    CLM_HIP(hipMemcpy(p->cinv, M.data(), 256 * 8, hipMemcpyHostToDevice));
  }
  return CLM_OK;
}

}  // namespace clm

using namespace clm;

namespace clm {
__global__ void k_zero_f64(int64_t n, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = 0.0;
}
}  // namespace clm

extern "C" {

const char* clm_status_string(clm_status s) {
  switch (s) {
    case CLM_OK: return "ok";
    case CLM_EINVAL: return "invalid argument";
    case CLM_ENOMEM: return "out of device memory";
    case CLM_EHIP: return "HIP runtime error";
    case CLM_ENOTCONV: return "multigrid did not converge";
    case CLM_ERAY_LEFT_PATCH: return "a point left its bundle's patch";
    case CLM_ENONFINITE: return "non-finite value";
    case CLM_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

clm_status clm_plan_desc_default(clm_plan_desc* d, int32_t nside_fine) {
  if (!d || nside_fine < 1) return CLM_EINVAL;
  std::memset(d, 0, sizeof(*d));
  d->nside_fine = nside_fine;
  d->nside_sht = nside_fine >= 8 ? nside_fine / 8 : 1;
  d->lmax = 2 * d->nside_sht;
  d->nside_bundle = nside_fine >= 64 ? nside_fine / 64 : 1;
  d->patch_factor = 4;
  const int64_t c = int64_t(4) * nside_fine / d->nside_bundle;
  d->patch_cells = int32_t(c > 256 ? c : 256);
  d->mg_vcycles = 4;
  d->mg_max_vcycles = 20;
  d->mg_eps = 0.1;
  d->nu_pre = 2;
  d->nu_post = 2;
  d->solver = CLM_SOLVER_SHT_MG;
  d->mg_prec = CLM_FP32;
  d->max_planes = 1;
  return CLM_OK;
}

clm_status clm_plan_create(const clm_plan_desc* desc, int device, clm_plan* out) {
  if (!out) return CLM_EINVAL;
  *out = nullptr;
  if (!desc) return CLM_EINVAL;
  const clm_plan_desc& d = *desc;
  if (!pow2(d.nside_fine) || !pow2(d.nside_sht) || d.nside_sht > d.nside_fine ||
      d.nside_fine > 8192 || d.lmax < 1 || d.lmax > (1 << 20) || d.max_planes < 1 ||
      (d.solver != CLM_SOLVER_SHT && d.solver != CLM_SOLVER_SHT_MG) ||
      (d.legendre_prec != CLM_FP64 && d.legendre_prec != CLM_FP32 &&
       d.legendre_prec != CLM_BF16X3 && d.legendre_prec != CLM_BF16X6) ||
      (d.adjoint != 0 && d.adjoint != 1) || d.analysis_iters < 0 || d.analysis_iters > 16 ||
      (d.analysis_iters > 0 && (d.legendre_prec != CLM_FP64 || d.adjoint)) ||
      (d.mfma_ana_waves != 0 && d.mfma_ana_waves != 8 && d.mfma_ana_waves != 16) ||
      (d.mfma_syn_waves != 0 && d.mfma_syn_waves != 8 && d.mfma_syn_waves != 12 &&
       d.mfma_syn_waves != 16) ||
      (d.mfma_der_waves != 0 && d.mfma_der_waves != 4 && d.mfma_der_waves != 8))
    return CLM_EINVAL;
  if (d.solver == CLM_SOLVER_SHT && d.nside_sht != d.nside_fine) return CLM_EINVAL;
  if (d.solver == CLM_SOLVER_SHT_MG) {
    if (!pow2(d.nside_bundle) || d.nside_bundle > d.nside_fine || d.patch_factor < 1 ||
        !pow2(d.patch_cells) || d.patch_cells < 8 || d.patch_cells > 4096 ||
        d.mg_vcycles < 0 || (d.mg_vcycles == 0 && (d.mg_max_vcycles < 1 || !(d.mg_eps > 0))) ||
        !(d.mg_eps >= 0) || d.nu_pre < 1 || d.nu_pre > 4 || d.nu_post < 1 ||
        d.nu_post > 4 || (d.mg_prec != CLM_FP32 && d.mg_prec != CLM_FP64) ||
        (d.adjoint && d.mg_vcycles == 0))
      return CLM_EINVAL;
    // the patch must stay far from the poles of its rotated frame
    const double side = std::sqrt(4.0 * 3.14159265358979323846 /
                                  (12.0 * double(d.nside_bundle) * d.nside_bundle));
    if (d.patch_factor * side > 2.0) return CLM_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return CLM_EINVAL;

  clm_plan P = new clm_plan_s();
  Plan* p = P;
  p->d = d;
  p->device = device;
  p->mg = d.solver == CLM_SOLVER_SHT_MG;
  p->fp64mg = d.mg_prec == CLM_FP64;
  p->npix_f = 12 * int64_t(d.nside_fine) * d.nside_fine;
  p->npix_s = 12 * int64_t(d.nside_sht) * d.nside_sht;
  p->nalm = int64_t(d.lmax + 1) * (d.lmax + 2) / 2;
  p->nring_s = 4 * d.nside_sht - 1;
  p->nring_f = 4 * d.nside_fine - 1;
  p->H = 2 * d.nside_sht;
  auto bail = [&](clm_status s) {
    delete P;
    return s;
  };
  if (p->mg) {
    p->nbundle = 12 * int64_t(d.nside_bundle) * d.nside_bundle;
    p->bundle_shift = 2 * ilog2(d.nside_fine / d.nside_bundle);
    p->n = d.patch_cells;
    p->nlev = ilog2(p->n) - 1;  // n .. 4
    p->side_b = std::sqrt(4.0 * 3.14159265358979323846 /
                          (12.0 * double(d.nside_bundle) * d.nside_bundle));
    p->L = d.patch_factor * p->side_b;
    p->delta = p->L / p->n;
    int k = 0;
    while ((p->n >> k) > kLdsLevelMax) ++k;
    p->ktile = k;
  }

  clm_status s;
  if ((s = build_tables(p)) != CLM_OK) return bail(s);

  const int64_t nF = int64_t(p->nring_s) * (d.lmax + 1) * 2;
  if ((s = alloc(p, &p->kap_s, size_t(p->npix_s))) != CLM_OK) return bail(s);
  if (d.analysis_iters > 0) {
    if ((s = alloc(p, &p->iter_map, size_t(p->npix_s))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->iter_alm, size_t(p->nalm) * 2)) != CLM_OK) return bail(s);
  }
  if ((s = alloc(p, &p->F, size_t(nF))) != CLM_OK) return bail(s);
  if ((s = alloc(p, &p->G, size_t(nF) * (p->mg ? 1 : 5))) != CLM_OK) return bail(s);
  if ((s = alloc(p, &p->red, 1024)) != CLM_OK) return bail(s);
  if ((s = alloc(p, &p->status_dev, 1)) != CLM_OK) return bail(s);
  if (hipMemset(p->status_dev, 0, sizeof(int)) != hipSuccess) return bail(CLM_EHIP);
  if (d.adjoint && (s = adjoint_alloc(p)) != CLM_OK) return bail(s);
  if (d.legendre_prec != CLM_FP64) {
    p->batch = d.max_planes < 16 ? d.max_planes : 16;
    if (hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, device) !=
        hipSuccess)
      return bail(CLM_EHIP);
    if ((s = alloc(p, &p->mfma_ctr, 4)) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->rcoef, size_t(p->nalm) * 2)) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->Fb, size_t(nF) * p->batch)) != CLM_OK) return bail(s);
    // pure-SHT plans: the derivative synthesis writes five fields per plane
    const int gfields = p->mg ? p->batch
                              : std::max(p->batch, 5 * std::min(p->batch, mfma_deriv_planes()));
    if ((s = alloc(p, &p->Gb, size_t(nF) * gfields)) != CLM_OK) return bail(s);
    if (!p->mg && (s = alloc(p, &p->dcoef, size_t(p->nalm))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->psib, size_t(p->nalm) * 32)) != CLM_OK) return bail(s);
    const int R = mfma_ring_blocks(p->H);
    if (R > 1 && (s = alloc(p, &p->apart, size_t(R) * p->nalm * 32)) != CLM_OK) return bail(s);
    if ((s = mfma_tables(p, nullptr)) != CLM_OK) return bail(s);
    if (hipDeviceSynchronize() != hipSuccess) return bail(CLM_EHIP);
  }

  const size_t esz = p->fp64mg ? 8 : 4;
  p->slots.resize(d.max_planes);
  for (auto& sl : p->slots) {
    if ((s = alloc(p, &sl.alm, size_t(p->nalm) * 2)) != CLM_OK) return bail(s);
    if ((s = alloc(p, &sl.psi_s, size_t(p->npix_s))) != CLM_OK) return bail(s);
    if (p->mg) {
      const size_t cells = size_t(p->nbundle) * p->n * p->n;
      const size_t gcells = size_t(p->nbundle) * (p->n + 2) * (p->n + 2);
      if ((s = alloc(p, &sl.u0, gcells)) != CLM_OK) return bail(s);
      char* du = nullptr;
      if ((s = alloc(p, &du, cells * esz)) != CLM_OK) return bail(s);
      sl.du = du;
    }
  }
  if (d.legendre_prec != CLM_FP64) {
    if ((s = mfma_autotune(p)) != CLM_OK) return bail(s);
    if (hipDeviceSynchronize() != hipSuccess) return bail(CLM_EHIP);
  }
  if (p->mg) {
    if ((s = alloc(p, &p->mg_eps_dev, size_t(p->nbundle))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->mg_cycles_dev, size_t(p->nbundle))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->mg_done_dev, size_t(p->nbundle))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->dom_map, size_t(p->nbundle))) != CLM_OK) return bail(s);
    if ((s = alloc(p, &p->dom_flag, size_t(p->nbundle))) != CLM_OK) return bail(s);
    p->nactive = p->nbundle;
    if (d.mg_vcycles == 0) {
      // epsilon rule: per-tile partial sums
      const size_t nc = size_t(p->n / 2), tc = std::min<size_t>(kEpsTile, nc);
      const size_t tiles = (nc / tc) * (nc / tc);
      if ((s = alloc(p, &p->mg_eps_part, size_t(p->nbundle) * tiles * 4)) != CLM_OK)
        return bail(s);
      if ((s = alloc(p, &p->mg_active_dev, 1)) != CLM_OK) return bail(s);
      if (hipHostMalloc(reinterpret_cast<void**>(&p->mg_active_host), sizeof(int)) !=
          hipSuccess)
        return bail(CLM_EHIP);
    }
  }
  if (p->mg) {
    const size_t cells = size_t(p->nbundle) * p->n * p->n;
    char* q = nullptr;
    if ((s = alloc(p, &q, cells * esz)) != CLM_OK) return bail(s);
    p->fprime = q;
    if ((s = alloc(p, &q, cells * esz)) != CLM_OK) return bail(s);
    p->dutmp = q;
    // levels 1 .. ktile: restricted u and residual; tile levels also keep
    // their source and two iterates
    p->ubar.assign(p->nlev, nullptr);
    p->rbar.assign(p->nlev, nullptr);
    p->flev.assign(p->nlev, nullptr);
    p->ulev.assign(p->nlev, nullptr);
    p->ulev2.assign(p->nlev, nullptr);
    for (int l = 1; l <= p->ktile && l < p->nlev; ++l) {
      const size_t c = size_t(p->nbundle) * (p->n >> l) * (p->n >> l);
      if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
      p->ubar[l] = q;
      if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
      p->rbar[l] = q;
      if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
      p->ulev[l] = q;
      if (l < p->ktile) {
        if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
        p->flev[l] = q;
        if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
        p->ulev2[l] = q;
      }
      if (l == 1 && d.mg_vcycles > 0) {
        if ((s = alloc(p, &q, c * esz)) != CLM_OK) return bail(s);
        p->ubar1b = q;
      }
    }
    if ((s = alloc(p, &p->setup_meta, size_t(setup_tiles(p)) * kSetupMetaBytes)) != CLM_OK)
      return bail(s);
    p->pad_s = setup_ring_pad(d.nside_sht);
    p->pad_f = setup_ring_pad(d.nside_fine);
    if ((s = alloc(p, &p->spad, size_t(p->npix_s) + 2 * size_t(p->pad_s) * p->nring_s)) !=
        CLM_OK)
      return bail(s);
    double* kp = nullptr;  // sized for float64 maps; float32 maps use half of it
    if ((s = alloc(p, &kp, size_t(p->npix_f) + 2 * size_t(p->pad_f) * p->nring_f)) != CLM_OK)
      return bail(s);
    p->kpad = kp;
    if ((s = setup_tables(p, nullptr)) != CLM_OK) return bail(s);
  } else {
    if ((s = alloc(p, &p->deriv, size_t(p->npix_s) * 5)) != CLM_OK) return bail(s);
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    p->err = "device synchronisation after table construction failed";
    return bail(CLM_EHIP);
  }
  *out = P;
  return CLM_OK;
}

clm_status clm_plan_destroy(clm_plan plan) {
  if (!plan) return CLM_EINVAL;
  (void)hipSetDevice(plan->device);
  delete plan;
  return CLM_OK;
}

clm_status clm_plan_last_error(clm_plan plan, char* buf, size_t len) {
  if (!plan || !buf || len == 0) return CLM_EINVAL;
  std::snprintf(buf, len, "%s", plan->err.c_str());
  return CLM_OK;
}

size_t clm_plan_workspace_bytes(clm_plan plan) { return plan ? plan->bytes : 0; }

clm_status clm_plan_get_desc(clm_plan plan, clm_plan_desc* out) {
  if (!plan || !out) return CLM_EINVAL;
  *out = plan->d;
  return CLM_OK;
}

clm_status clm_plan_set_timing(clm_plan plan, int32_t enable) {
  if (!plan) return CLM_EINVAL;
  plan->timing = enable != 0;
  return CLM_OK;
}

clm_status clm_plan_set_timing_stages(clm_plan plan, const char* stages) {
  if (!plan) return CLM_EINVAL;
  plan->timing_only.clear();
  if (!stages) return CLM_OK;
  std::string cur;
  for (const char* c = stages;; ++c) {
    if (*c == ',' || *c == '\0') {
      if (!cur.empty()) plan->timing_only.push_back(cur);
      cur.clear();
      if (*c == '\0') break;
    } else {
      cur += *c;
    }
  }
  return CLM_OK;
}

clm_status clm_plan_timings(clm_plan plan, double* ms_per_stage, int32_t nstages) {
  if (!plan || !ms_per_stage || nstages < 0) return CLM_EINVAL;
  // the per-stage totals in the order of clm_plan_stage_name, then reset
  std::vector<double> ms(64, 0.0);
  std::vector<int64_t> cnt(64, 0);
  char names[4096];
  int32_t got = 0;
  const clm_status st = clm_plan_get_timing(plan, names, sizeof names, ms.data(), cnt.data(),
                                            64, &got);
  for (int i = 0; i < nstages; ++i) ms_per_stage[i] = i < got ? ms[i] : 0.0;
  return st;
}

const char* clm_plan_stage_name(clm_plan plan, int32_t i) {
  if (!plan || i < 0 || i >= int32_t(plan->stage_names.size())) return nullptr;
  return plan->stage_names[size_t(i)].c_str();
}

clm_status clm_plan_get_timing(clm_plan plan, char* names, size_t len, double* ms,
                               int64_t* count, int32_t max_stages, int32_t* nstages) {
  if (!plan || !names || len == 0 || !ms || !count || !nstages || max_stages < 1)
    return CLM_EINVAL;
  Plan* p = plan;
  const int ns = int(p->stage_names.size());
  std::vector<double> acc(ns, 0.0);
  std::vector<int64_t> cnt(ns, 0);
  clm_status st = CLM_OK;
  for (auto& r : p->recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      st = CLM_EHIP;
    acc[r.stage] += t;
    cnt[r.stage] += 1;
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->recs.clear();
  std::string all;
  for (int i = 0; i < ns; ++i) {
    if (i) all += ",";
    all += p->stage_names[i];
  }
  std::snprintf(names, len, "%s", all.c_str());
  const int k = ns < max_stages ? ns : max_stages;
  for (int i = 0; i < k; ++i) {
    ms[i] = acc[i];
    count[i] = cnt[i];
  }
  *nstages = k;
  return st;
}

clm_status clm_plan_sync_status(clm_plan plan, hipStream_t stream) {
  if (!plan) return CLM_EINVAL;
  Plan* p = plan;
  int st = 0;
  CLM_HIP(hipMemcpyAsync(&st, p->status_dev, sizeof(int), hipMemcpyDeviceToHost, stream));
  CLM_HIP(hipStreamSynchronize(stream));
  CLM_HIP(hipMemsetAsync(p->status_dev, 0, sizeof(int), stream));
  CLM_HIP(hipStreamSynchronize(stream));
  if (st & ST_LEFT_PATCH) return fail(p, CLM_ERAY_LEFT_PATCH, "a point left its bundle's patch");
  if (st & ST_NONFINITE) return fail(p, CLM_ENONFINITE, "non-finite value produced");
  if (st & ST_NOTCONV)
    return fail(p, CLM_ENOTCONV, "a patch did not meet mg_eps within mg_max_vcycles");
  return CLM_OK;
}

clm_status clm_get_mg_convergence(clm_plan plan, double* eps_dev, int32_t* cycles_dev,
                                  hipStream_t stream) {
  if (!plan || !eps_dev || !cycles_dev) return CLM_EINVAL;
  Plan* p = plan;
  if (!p->mg) return fail(p, CLM_EUNSUPPORTED, "no multigrid in an SHT-only plan");
  CLM_HIP(hipMemcpyAsync(eps_dev, p->mg_eps_dev, size_t(p->nbundle) * 8,
                         hipMemcpyDeviceToDevice, stream));
  CLM_HIP(hipMemcpyAsync(cycles_dev, p->mg_cycles_dev, size_t(p->nbundle) * 4,
                         hipMemcpyDeviceToDevice, stream));
  return CLM_OK;
}

clm_status clm_poisson_solve(clm_plan plan, const void* kappa, int32_t kappa_is_fp64,
                             int32_t first_slot, int32_t nplanes, hipStream_t stream) {
  if (!plan || !kappa || nplanes < 1 || first_slot < 0 ||
      first_slot + nplanes > plan->d.max_planes)
    return CLM_EINVAL;
  Plan* p = plan;
  CLM_HIP(hipSetDevice(p->device));
  const size_t esz = kappa_is_fp64 ? 8 : 4;
  if (p->batch > 0) {
    // matrix-core Legendre transforms: planes batched as GEMM columns; the
    // multigrid then runs per plane, after that plane's mean is taken again
    for (int k0 = 0; k0 < nplanes; k0 += p->batch) {
      const int nb = nplanes - k0 < p->batch ? nplanes - k0 : p->batch;
      const char* kp = static_cast<const char*>(kappa) + size_t(k0) * p->npix_f * esz;
      clm_status s = sht_solve_batch(p, kp, kappa_is_fp64, first_slot + k0, nb, stream);
      if (s != CLM_OK) return s;
      for (int k = 0; p->mg && k < nb; ++k) {
        const char* kk = kp + size_t(k) * p->npix_f * esz;
        if ((s = plane_mean(p, kk, kappa_is_fp64, stream)) != CLM_OK) return s;
        if ((s = mg_solve(p, kk, kappa_is_fp64, first_slot + k0 + k, stream)) != CLM_OK)
          return s;
      }
    }
    return CLM_OK;
  }
  for (int k = 0; k < nplanes; ++k) {
    const char* kp = static_cast<const char*>(kappa) + size_t(k) * p->npix_f * esz;
    clm_status s = sht_solve(p, kp, kappa_is_fp64, first_slot + k, stream);
    if (s != CLM_OK) return s;
    if (p->mg) {
      s = mg_solve(p, kp, kappa_is_fp64, first_slot + k, stream);
      if (s != CLM_OK) return s;
    }
  }
  return CLM_OK;
}

clm_status clm_poisson_solve_particles(clm_plan plan, const clm_particles* parts, int32_t slot,
                                       hipStream_t stream) {
  if (!plan || !parts || parts->n < 0 || slot < 0 || slot >= plan->d.max_planes ||
      (parts->n > 0 && (!parts->theta || !parts->phi || !parts->weight || !parts->sigma)))
    return CLM_EINVAL;
  Plan* p = plan;
  CLM_HIP(hipSetDevice(p->device));
  double* map = nullptr;
  if (p->mg) {
    const size_t ws = size_t(p->nbundle) * p->n * p->n * (p->fp64mg ? 8 : 4);
    if (ws < size_t(p->npix_f) * 8)
      return fail(p, CLM_EUNSUPPORTED, "particles: patches too coarse to hold the fine map");
    map = static_cast<double*>(p->dutmp);
  } else {
    map = p->deriv;
  }
  hipLaunchKernelGGL(clm::k_zero_f64, dim3(unsigned((p->npix_f + 255) / 256)), dim3(256), 0,
                     stream, p->npix_f, map);
  CLM_LAUNCH_CHECK();
  clm_status s = deposit_map(parts, p->d.nside_fine, map, stream);
  if (s != CLM_OK) return s;
  if (p->batch > 0)
    s = sht_solve_batch(p, map, 1, slot, 1, stream);
  else
    s = sht_solve(p, map, 1, slot, stream);
  if (s != CLM_OK || !p->mg) return s;
  if (p->batch > 0 && (s = plane_mean(p, map, 1, stream)) != CLM_OK) return s;
  return mg_solve(p, nullptr, 1, slot, stream, parts);
}

clm_status clm_poisson_solve_multi(const clm_plan* plans, int32_t nplans,
                                   const void* const* kappa, const int32_t* kappa_is_fp64,
                                   const int32_t* nplanes, hipStream_t stream) {
  if (!plans || !kappa || !kappa_is_fp64 || !nplanes || nplans < 1 || nplans > 4)
    return CLM_EINVAL;
  Plan* ps[4];
  for (int i = 0; i < nplans; ++i) {
    ps[i] = plans[i];
    if (!ps[i] || !kappa[i] || nplanes[i] < 1 || nplanes[i] > ps[i]->d.max_planes)
      return CLM_EINVAL;
    if (ps[i]->batch == 0 || ps[i]->d.legendre_prec != ps[0]->d.legendre_prec ||
        ps[i]->device != ps[0]->device)
      return fail(ps[0], CLM_EINVAL,
                  "clm_poisson_solve_multi: one device and one matrix-core form for all plans");
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) return fail(ps[0], CLM_EINVAL, "a plan appears twice");
  }
  CLM_HIP_P(ps[0], hipSetDevice(ps[0]->device));
  return sht_solve_multi(ps, nplans, kappa, kappa_is_fp64, nplanes, stream);
}

clm_status clm_get_psi_alm(clm_plan plan, int32_t slot, double* out, hipStream_t stream) {
  if (!plan || !out || slot < 0 || slot >= plan->d.max_planes) return CLM_EINVAL;
  Plan* p = plan;
  CLM_HIP(hipMemcpyAsync(out, p->slots[slot].alm, size_t(p->nalm) * 16,
                         hipMemcpyDeviceToDevice, stream));
  return CLM_OK;
}

clm_status clm_get_psi_map(clm_plan plan, int32_t slot, double* out, hipStream_t stream) {
  if (!plan || !out || slot < 0 || slot >= plan->d.max_planes) return CLM_EINVAL;
  Plan* p = plan;
  CLM_HIP(hipMemcpyAsync(out, p->slots[slot].psi_s, size_t(p->npix_s) * 8,
                         hipMemcpyDeviceToDevice, stream));
  return CLM_OK;
}

clm_status clm_get_patch_potential(clm_plan plan, int32_t slot, int64_t first, int64_t np,
                                   double* out, hipStream_t stream) {
  if (!plan || !out || slot < 0 || slot >= plan->d.max_planes) return CLM_EINVAL;
  if (!plan->mg) return CLM_EUNSUPPORTED;
  if (first < 0 || np < 1 || first + np > plan->nbundle) return CLM_EINVAL;
  return mg_patch_potential(plan, slot, first, np, out, stream);
}

clm_status clm_shear_from_potential(clm_plan plan, int32_t slot, const double* th,
                                    const double* ph, int64_t npts, int32_t out_fp64,
                                    void* grad, void* hess, hipStream_t stream) {
  if (!plan || npts < 0 || slot < 0 || slot >= plan->d.max_planes) return CLM_EINVAL;
  if (!plan->mg) return CLM_EUNSUPPORTED;
  if (npts == 0) return CLM_OK;
  if (!th || !ph || !grad || !hess) return CLM_EINVAL;
  return eval_points(plan, slot, th, ph, npts, -1, out_fp64, grad, hess, stream);
}

clm_status clm_shear_at_pixels(clm_plan plan, int32_t slot, int32_t order, int32_t out_fp64,
                               void* grad, void* hess, hipStream_t stream) {
  if (!plan || !grad || !hess || slot < 0 || slot >= plan->d.max_planes ||
      (order != CLM_ORDER_RING && order != CLM_ORDER_NESTED))
    return CLM_EINVAL;
  if (!plan->mg) return sht_pixel_derivs_batch(plan, slot, 1, order, out_fp64, grad, hess, stream);
  return eval_points(plan, slot, nullptr, nullptr, plan->npix_f, order, out_fp64, grad, hess,
                     stream);
}

clm_status clm_plan_set_domain(clm_plan plan, const int32_t* bundles, int64_t nb) {
  if (!plan || nb < 0 || (nb > 0 && !bundles)) return CLM_EINVAL;
  Plan* p = plan;
  if (!p->mg) return fail(p, CLM_EUNSUPPORTED, "a domain restricts the multigrid step only");
  std::vector<int> flag(size_t(p->nbundle), nb > 0 ? 0 : 1);
  for (int64_t k = 0; k < nb; ++k) {
    if (bundles[k] < 0 || bundles[k] >= p->nbundle)
      return fail(p, CLM_EINVAL, "domain: bundle index outside 0 .. nbundle - 1");
    flag[size_t(bundles[k])] = 1;
  }
  std::vector<int> list;
  for (int64_t b = 0; b < p->nbundle; ++b)
    if (flag[size_t(b)]) list.push_back(int(b));
  CLM_HIP_P(p, hipSetDevice(p->device));
  // the device may be running the plan's kernels: wait for them first
  CLM_HIP_P(p, hipDeviceSynchronize());
  CLM_HIP_P(p, hipMemcpy(p->dom_map, list.data(), list.size() * sizeof(int),
                         hipMemcpyHostToDevice));
  CLM_HIP_P(p, hipMemcpy(p->dom_flag, flag.data(), flag.size() * sizeof(int),
                         hipMemcpyHostToDevice));
  p->nactive = int64_t(list.size());
  p->domain = p->nactive < p->nbundle;
  return CLM_OK;
}

clm_status clm_shear_at_pixels_batch(clm_plan plan, int32_t first_slot, int32_t nplanes,
                                     int32_t order, int32_t out_fp64, void* grad, void* hess,
                                     hipStream_t stream) {
  if (!plan || !grad || !hess || first_slot < 0 || nplanes < 1 ||
      nplanes > plan->d.max_planes - first_slot ||
      (order != CLM_ORDER_RING && order != CLM_ORDER_NESTED))
    return CLM_EINVAL;
  if (plan->mg) return CLM_EUNSUPPORTED;
  return sht_pixel_derivs_batch(plan, first_slot, nplanes, order, out_fp64, grad, hess, stream);
}

clm_status clm_jacobian_spectra(clm_plan plan, const clm_rays* rays, double* alm,
                                double* cl, hipStream_t stream) {
  if (!plan || !rays || !alm || !cl || !rays->theta || !rays->phi || !rays->A ||
      rays->n != plan->npix_s)
    return CLM_EINVAL;
  if (plan->mg) return CLM_EUNSUPPORTED;
  return sht_jacobian_spectra(plan, rays, alm, cl, stream);
}

clm_status clm_rays_init(clm_plan plan, const clm_rays* rays, hipStream_t stream) {
  if (!plan || !rays || rays->n != plan->npix_f || !rays->theta || !rays->phi || !rays->beta ||
      !rays->A || !rays->A_prev)
    return CLM_EINVAL;
  plan->ray_plane = -1;
  return rays_init(plan, rays, stream);
}

clm_status clm_ray_update(clm_plan plan, int32_t slot, const double* chi, int32_t nchi,
                          int32_t m, double K, const clm_rays* rays, hipStream_t stream) {
  if (!plan || !rays || !chi || rays->n != plan->npix_f || slot < 0 ||
      slot >= plan->d.max_planes || m < 0 || m + 1 >= nchi)
    return CLM_EINVAL;
  clm_status s = CLM_OK;
  if (!plan->mg && (s = sht_plane_fields(plan, slot, stream)) != CLM_OK) return s;
  s = ray_update(plan, slot, chi, nchi, m, K, rays, stream);
  if (s == CLM_OK) {
    plan->ray_chi.assign(chi, chi + nchi);
    plan->ray_K = K;
    plan->ray_plane = m;
  }
  return s;
}

clm_status clm_galaxies_reduced(clm_plan plan, const clm_rays* rays, const double* theta,
                                const double* phi, const double* chi_g, int64_t ngal,
                                float* A_g, hipStream_t stream) {
  if (!plan || !rays || rays->n != plan->npix_f || ngal < 0 ||
      (ngal > 0 && (!theta || !phi || !chi_g || !A_g)))
    return CLM_EINVAL;
  Plan* p = plan;
  if (p->ray_plane < 0)
    return fail(p, CLM_EINVAL, "clm_galaxies_reduced needs a prior ray update (its distances)");
  if (ngal == 0) return CLM_OK;
  CLM_HIP(hipSetDevice(p->device));
  clm_galaxies g{theta, phi, chi_g, A_g, ngal};
  return galaxies_shell(p, p->ray_chi.data(), int(p->ray_chi.size()), p->ray_plane + 1,
                        p->ray_K, rays, &g, stream);
}

clm_status clm_galaxies_shell(clm_plan plan, const double* chi, int32_t nchi, int32_t k,
                              double K, const clm_rays* rays, const clm_galaxies* gal,
                              hipStream_t stream) {
  if (!plan || !chi || !rays || !gal || rays->n != plan->npix_f || k < 0 || k >= nchi ||
      gal->n < 0 || (gal->n > 0 && (!gal->theta || !gal->phi || !gal->chi || !gal->A)))
    return CLM_EINVAL;
  for (int q = 1; q < nchi; ++q)
    if (!(chi[q] > chi[q - 1]) || !(chi[0] > 0)) return CLM_EINVAL;
  if (gal->n == 0) return CLM_OK;
  Plan* p = plan;
  CLM_HIP(hipSetDevice(p->device));
  return galaxies_shell(p, chi, nchi, k, K, rays, gal, stream);
}

clm_status clm_galaxy_images(clm_plan plan, const double* chi, int32_t nchi, int32_t k,
                             double K, const clm_rays* rays, const clm_galaxies* gal,
                             double search_radius, double* theta_img, double* phi_img,
                             int32_t* found, hipStream_t stream) {
  if (!plan || !chi || !rays || !gal || rays->n != plan->npix_f || k < 0 || k >= nchi ||
      gal->n < 0 || !(search_radius >= 0) || search_radius > 0.02 ||
      (gal->n > 0 && (!gal->theta || !gal->phi || !gal->chi || !gal->A || !theta_img ||
                      !phi_img || !found)))
    return CLM_EINVAL;
  for (int q = 1; q < nchi; ++q)
    if (!(chi[q] > chi[q - 1]) || !(chi[0] > 0)) return CLM_EINVAL;
  if (gal->n == 0) return CLM_OK;
  Plan* p = plan;
  CLM_HIP(hipSetDevice(p->device));
  return galaxy_images(p, chi, nchi, k, K, rays, gal, search_radius, theta_img, phi_img, found,
                       stream);
}

clm_status clm_raytrace_planes(clm_plan plan, const void* kappa, int32_t kappa_is_fp64,
                               const double* chi, int32_t nchi, int32_t first_plane,
                               int32_t nplanes, double K, const clm_rays* rays,
                               const clm_galaxies* gal, hipStream_t stream) {
  if (!plan || !kappa || !chi || !rays || rays->n != plan->npix_f || first_plane < 0 ||
      nplanes < 1 || first_plane + nplanes + 1 > nchi)
    return CLM_EINVAL;
  if (gal && (gal->n < 0 || (gal->n > 0 && (!gal->theta || !gal->phi || !gal->chi || !gal->A))))
    return CLM_EINVAL;
  for (int k = 1; k < nchi; ++k)
    if (!(chi[k] > chi[k - 1]) || !(chi[0] > 0)) return CLM_EINVAL;
  Plan* p = plan;
  CLM_HIP(hipSetDevice(p->device));
  const size_t esz = kappa_is_fp64 ? 8 : 4;
  clm_status s;
  if (gal && gal->n > 0 && first_plane == 0) {
    s = galaxies_shell(p, chi, nchi, 0, K, rays, gal, stream);
    if (s != CLM_OK) return s;
  }
  // one plane after the other: its rays, then the galaxies of the shell
  // the rays have just reached
  auto advance = [&](int slot, int m) -> clm_status {
    clm_status e = ray_update(p, slot, chi, nchi, m, K, rays, stream);
    if (e != CLM_OK) return e;
    p->ray_chi.assign(chi, chi + nchi);
    p->ray_K = K;
    p->ray_plane = m;
    if (gal && gal->n > 0) return galaxies_shell(p, chi, nchi, m + 1, K, rays, gal, stream);
    return CLM_OK;
  };
  if (p->mg) {
    for (int k = 0; k < nplanes; ++k) {
      const char* kp = static_cast<const char*>(kappa) + size_t(k) * p->npix_f * esz;
      if ((s = sht_solve(p, kp, kappa_is_fp64, 0, stream)) != CLM_OK) return s;
      if ((s = mg_solve(p, kp, kappa_is_fp64, 0, stream)) != CLM_OK) return s;
      if ((s = advance(0, first_plane + k)) != CLM_OK) return s;
    }
    return CLM_OK;
  }
  // pure-SHT planes: psi_lm of a batch of planes (slots 0 ..), no psi maps;
  // the derivative fields of the batch in one matrix-core launch (FP64
  // plans: plane by plane); per plane the fields at the pixel centres, then
  // its rays
  const int dp = p->batch > 0 ? std::min(p->batch, mfma_deriv_planes()) : 1;
  for (int k0 = 0; k0 < nplanes; k0 += dp) {
    const int nb = std::min(dp, nplanes - k0);
    const char* kp = static_cast<const char*>(kappa) + size_t(k0) * p->npix_f * esz;
    if (p->batch > 0) {
      if ((s = sht_solve_batch(p, kp, kappa_is_fp64, 0, nb, stream, false)) != CLM_OK) return s;
      if ((s = mfma_deriv_synthesis(p, 0, nb, stream)) != CLM_OK) return s;
      for (int k = 0; k < nb; ++k) {
        if ((s = sht_batch_fields(p, k, stream)) != CLM_OK) return s;
        if ((s = advance(k, first_plane + k0 + k)) != CLM_OK) return s;
      }
    } else {
      if ((s = sht_solve(p, kp, kappa_is_fp64, 0, stream, false)) != CLM_OK) return s;
      if ((s = sht_plane_fields(p, 0, stream)) != CLM_OK) return s;
      if ((s = advance(0, first_plane + k0)) != CLM_OK) return s;
    }
  }
  return CLM_OK;
}

}  // extern "C"

clm_status clm_shear_adjoint(clm_plan plan, int32_t slot, const double* theta, const double* phi,
                             int64_t npts, const double* dgrad, const double* dhess,
                             hipStream_t stream) {
  if (!plan || slot < 0 || slot >= plan->d.max_planes || npts < 0) return CLM_EINVAL;
  Plan* p = plan;
  if (!p->mg || !p->d.adjoint)
    return fail(p, CLM_EUNSUPPORTED, "the adjoint needs an SHT+MG plan created with adjoint = 1");
  if (p->domain) return fail(p, CLM_EUNSUPPORTED, "the adjoint covers the whole sky only");
  if (npts == 0) return CLM_OK;
  if (!theta || !phi || !dgrad || !dhess) return CLM_EINVAL;
  CLM_HIP(hipSetDevice(p->device));
  return shear_adjoint(p, theta, phi, npts, dgrad, dhess, stream);
}

clm_status clm_poisson_adjoint(clm_plan plan, int32_t slot, double* dkappa, hipStream_t stream) {
  if (!plan || !dkappa || slot < 0 || slot >= plan->d.max_planes) return CLM_EINVAL;
  Plan* p = plan;
  if (!p->mg || !p->d.adjoint)
    return fail(p, CLM_EUNSUPPORTED, "the adjoint needs an SHT+MG plan created with adjoint = 1");
  if (p->domain) return fail(p, CLM_EUNSUPPORTED, "the adjoint covers the whole sky only");
  CLM_HIP(hipSetDevice(p->device));
  return poisson_adjoint(p, dkappa, stream);
}
