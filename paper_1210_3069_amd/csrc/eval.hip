// Deflection and shear at points or at every pixel centre from the solved
// patch potentials (Sec. 3.2): one thread per point, gather of the 6 x 6
// cell window around the point from u0 (float64) and du.
#include <cmath>

#include "clm_internal.h"
#include "eval_dev.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlock = 256;

struct EvalArgs {
  PatchField P;
  const double* th;    // nullptr: all pixel centres of the fine grid
  const double* ph;
  int64_t npts;
  int order;           // pixel mode: CLM_ORDER_RING or CLM_ORDER_NESTED
  const int* r2n_f;
  int64_t Nf, Nb;
  int shift;
  void* grad;
  void* hess;
  int* status;
  const int* pmap;     // partial sky: the domain's bundles (pixel mode), or nullptr
  const int* dflag;    // partial sky: 1 for a bundle of the domain (point mode), or nullptr
};

template <typename T, typename TO>
__global__ __launch_bounds__(kBlock) void k_eval(EvalArgs a) {
  // consecutive points (a NESTED range: one region of one patch) stay on
  // one XCD, so the L2 of one XCD holds their cell window
  const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
  int64_t i = c;  // output index
  double vx, vy, vz;
  int64_t b;
  bool inside = true;
  if (a.th) {
    if (c >= a.npts) return;
    double st, ct, sp, cp;
    sincos(a.th[i], &st, &ct);
    sincos(a.ph[i], &sp, &cp);
    vx = st * cp; vy = st * sp; vz = ct;
    b = hpx::ang2nest(a.Nb, ct, a.ph[i]);
    inside = !a.dflag || a.dflag[b];
  } else {
    int64_t pring, pnest;
    if (a.pmap) {
      // the pixels of the domain's bundles, NESTED ranges one after the other
      if ((c >> a.shift) >= a.npts) return;
      pnest = (int64_t(a.pmap[c >> a.shift]) << a.shift) | (c & ((int64_t(1) << a.shift) - 1));
      pring = hpx::nest2ring(a.Nf, pnest);
      i = a.order == CLM_ORDER_NESTED ? pnest : pring;
    } else if (c >= a.npts) {
      return;
    } else if (a.order == CLM_ORDER_NESTED) {
      pnest = i;
      pring = hpx::nest2ring(a.Nf, i);
    } else {
      pring = i;
      pnest = a.r2n_f[i];
    }
    double z, st, phi;
    hpx::pix2ang_ring(a.Nf, pring, z, st, phi);
    double sp, cp;
    sincos(phi, &sp, &cp);
    vx = st * cp; vy = st * sp; vz = z;
    b = pnest >> a.shift;
  }
  const int64_t nout = a.pmap ? a.Nf * a.Nf * 12 : a.npts;  // output stride
  double g[2], U[3];
  TO* gr = static_cast<TO*>(a.grad);
  TO* hs = static_cast<TO*>(a.hess);
  if (!inside || !eval_patch<T>(a.P, b, vx, vy, vz, g, U)) {
    atomicOr(a.status, ST_LEFT_PATCH);
    const TO nan = TO(NAN);
    gr[i] = nan; gr[nout + i] = nan;
    hs[i] = nan; hs[nout + i] = nan; hs[2 * nout + i] = nan;
    return;
  }
  gr[i] = TO(g[0]);
  gr[nout + i] = TO(g[1]);
  hs[i] = TO(U[0]);
  hs[nout + i] = TO(U[1]);
  hs[2 * nout + i] = TO(U[2]);
}

}  // namespace

clm_status eval_points(Plan* p, int slot, const double* th, const double* ph, int64_t npts,
                       int order, int out_fp64, void* grad, void* hess, hipStream_t s) {
  EvalArgs a;
  a.P = PatchField{p->rot, p->slots[slot].u0, p->slots[slot].du, p->n, p->L, p->delta};
  a.th = th;
  a.ph = ph;
  a.npts = npts;
  a.order = order;
  a.r2n_f = p->r2n_f;
  a.Nf = p->d.nside_fine;
  a.Nb = p->d.nside_bundle;
  a.shift = p->bundle_shift;
  a.grad = grad;
  a.hess = hess;
  a.status = p->status_dev;
  a.pmap = nullptr;
  a.dflag = nullptr;
  int64_t nthreads = npts;
  if (p->domain) {
    if (th) {
      a.dflag = p->dom_flag;
    } else {
      // pixel mode: threads over the domain's pixels; a.npts counts its bundles
      a.pmap = p->dom_map;
      a.npts = p->nactive;
      nthreads = p->nactive << p->bundle_shift;
    }
  }
  const dim3 g(unsigned((nthreads + kBlock - 1) / kBlock));
  CLM_TIMED(p, s, th ? "eval_points" : "eval_pixels");
  if (p->fp64mg) {
    if (out_fp64) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eval<double, double>), g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eval<double, float>), g, dim3(kBlock), 0, s, a);
  } else {
    if (out_fp64) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eval<float, double>), g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eval<float, float>), g, dim3(kBlock), 0, s, a);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace clm
