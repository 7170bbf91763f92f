// Epanechnikov deposition of particles onto a HEALPix map (Sec. 3.2): each
// particle's mass is smoothed with the kernel 1 - (theta / sigma)^2 inside
// its smoothing angle sigma and binned over the pixel centres, normalised
// so that its weights add up to one (exact mass conservation).  The
// kernel's normalisation on the sphere cancels in that ratio.  A particle
// whose sigma reaches no pixel centre puts all its mass in its own pixel.
// The map receives mass per unit area, w W(p) / Omega_pix.
//
// One thread per particle: the rings that its disc can touch, and on each
// the azimuth window of the disc widened by a pixel either side; the exact
// separation (atan2 of |a x b| and a . b) decides.  The first pass sums the
// kernel, the second adds the normalised weights with float64 atomics, so
// the summation order over particles, and the last bits, vary from run to
// run.
#include <cmath>

#include "clm_internal.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlock = 256;
constexpr double kPiD = 3.14159265358979323846;

// Ring i (1-based, 1 .. 4N - 1) of resolution N.
struct RingG {
  double z, s, phi0, dphi;
  int64_t n, first;
};

__device__ __forceinline__ RingG ring_geom(int64_t N, int64_t i) {
  RingG g;
  const int64_t npix = 12 * N * N;
  if (i < N || i > 3 * N) {
    const bool north = i < N;
    const int64_t k = north ? i : 4 * N - i;
    const double omz = double(k) * double(k) / (3.0 * double(N) * double(N));
    g.z = north ? 1.0 - omz : omz - 1.0;
    g.s = sqrt(omz * (2.0 - omz));
    g.n = 4 * k;
    g.first = north ? 2 * k * (k - 1) : npix - 2 * k * (k + 1);
    g.phi0 = kPiD / (4.0 * double(k));
  } else {
    g.z = (4.0 * double(N) - 2.0 * double(i)) / (3.0 * double(N));
    g.s = sqrt((1.0 - g.z) * (1.0 + g.z));
    g.n = 4 * N;
    g.first = 2 * N * (N - 1) + 4 * N * (i - N);
    g.phi0 = ((i - N) & 1) == 0 ? kPiD / (4.0 * double(N)) : 0.0;
  }
  g.dphi = 2.0 * kPiD / double(g.n);
  return g;
}

// The (fractional) ring index at colatitude theta: the inverse of the ring
// latitudes, monotone in theta.
__device__ __forceinline__ double ring_of(int64_t N, double theta) {
  const double z = cos(theta);
  if (z > 2.0 / 3.0) {
    const double h = sin(0.5 * theta);  // 1 - z = 2 sin^2(theta / 2)
    return double(N) * sqrt(6.0) * h;
  }
  if (z < -2.0 / 3.0) {
    const double h = cos(0.5 * theta);  // 1 + z = 2 cos^2(theta / 2)
    return 4.0 * double(N) - double(N) * sqrt(6.0) * h;
  }
  return double(N) * (2.0 - 1.5 * z);
}

// Runs f(pixel, kernel value) over the pixel centres within sigma of the
// unit vector p (colatitude th, azimuth ph in [0, 2 pi)).
template <typename F>
__device__ __forceinline__ void disc_pixels(int64_t N, const double p[3], double th, double ph,
                                            double sigma, F&& f) {
  const double lo = fmax(0.0, th - sigma), hi = fmin(kPiD, th + sigma);
  const int64_t i_lo = max(int64_t(1), int64_t(floor(ring_of(N, lo))) - 1);
  const int64_t i_hi = min(4 * N - 1, int64_t(ceil(ring_of(N, hi))) + 1);
  const double cs = cos(sigma), sp = sqrt(p[0] * p[0] + p[1] * p[1]);
  const double is2 = 1.0 / (sigma * sigma);
  for (int64_t i = i_lo; i <= i_hi; ++i) {
    const RingG g = ring_geom(N, i);
    // azimuths within sigma: cos dphi >= (cos sigma - z_p z_r) / (s_p s_r)
    int64_t j0 = 0, j1 = g.n - 1;
    const double den = sp * g.s;
    if (den > 1e-300) {
      const double c = (cs - p[2] * g.z) / den;
      if (c > -1.0) {
        const double dmax = c >= 1.0 ? 0.0 : acos(c);
        const int64_t a = int64_t(floor((ph - dmax - g.phi0) / g.dphi)) - 1;
        const int64_t b = int64_t(ceil((ph + dmax - g.phi0) / g.dphi)) + 1;
        if (b - a + 1 < g.n) {
          j0 = a;
          j1 = b;
        }
      }
    }
    for (int64_t j = j0; j <= j1; ++j) {
      const int64_t jj = ((j % g.n) + g.n) % g.n;
      double sf, cf;
      sincos(g.phi0 + double(jj) * g.dphi, &sf, &cf);
      const double v[3] = {g.s * cf, g.s * sf, g.z};
      const double cx = v[1] * p[2] - v[2] * p[1], cy = v[2] * p[0] - v[0] * p[2],
                   cz = v[0] * p[1] - v[1] * p[0];
      const double ang = atan2(sqrt(cx * cx + cy * cy + cz * cz),
                               v[0] * p[0] + v[1] * p[1] + v[2] * p[2]);
      if (ang < sigma) f(g.first + jj, 1.0 - ang * ang * is2);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_deposit(int64_t N, int64_t npart, const double* th,
                                                    const double* ph, const double* w,
                                                    const double* sg, double* map) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= npart) return;
  if (!isfinite(th[t]) || !isfinite(ph[t])) return;
  double st, ct, sp, cp;
  sincos(th[t], &st, &ct);
  sincos(ph[t], &sp, &cp);
  const double p[3] = {st * cp, st * sp, ct};
  // the direction's own colatitude and azimuth (any input angles)
  const double theta = atan2(sqrt(p[0] * p[0] + p[1] * p[1]), p[2]);
  double phi = atan2(p[1], p[0]);
  if (phi < 0.0) phi += 2.0 * kPiD;
  if (phi >= 2.0 * kPiD) phi = 0.0;
  const double omega = 4.0 * kPiD / double(12 * N * N);
  const double sigma = isfinite(sg[t]) && sg[t] > 0.0 ? fmin(sg[t], kPiD) : 0.0;
  double sum = 0.0;
  if (sigma > 0.0) disc_pixels(N, p, theta, phi, sigma, [&](int64_t, double k) { sum += k; });
  if (sum > 0.0) {
    const double f = w[t] / (sum * omega);
    disc_pixels(N, p, theta, phi, sigma,
                [&](int64_t q, double k) { unsafeAtomicAdd(map + q, f * k); });
  } else {
    const int64_t own = hpx::nest2ring(N, hpx::ang2nest(N, p[2], phi));
    unsafeAtomicAdd(map + own, w[t] / omega);
  }
}

// ------------------------------------------------------------- patches
// Sec. 3.2: the same smoothing binned over the multigrid patches' cells.
// A particle's kernel times the cell area is taken over the cell centres of
// the patch grid, continued past its faces, within sigma, and normalised
// to its weight there; the cells of the patch get their share, so a
// particle's mass splits exactly between a patch and its outside.  A
// particle whose sigma reaches no cell centre puts its weight in the cell
// that holds it.  The result enters the source as 2 x mass per area, added
// into f' (the setup wrote -2 mean - L u0).
struct PatchDep {
  const double* th;
  const double* ph;
  const double* w;
  const double* sg;
  int64_t npart;
  const double* rot;   // [nbundle][9] patch rotations
  int64_t Nb;          // bundle grid
  int n;               // cells per side
  double L, delta;
  const int* dflag;    // partial sky: 1 for a patch of the domain, or nullptr
  void* fp;            // f' [patch][n][n] of T
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_patch_deposit(PatchDep a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.npart) return;
  if (!isfinite(a.th[t]) || !isfinite(a.ph[t])) return;
  double st, ct, sp, cp;
  sincos(a.th[t], &st, &ct);
  sincos(a.ph[t], &sp, &cp);
  const double p[3] = {st * cp, st * sp, ct};
  const double theta = atan2(sqrt(p[0] * p[0] + p[1] * p[1]), p[2]);
  double phi = atan2(p[1], p[0]);
  if (phi < 0.0) phi += 2.0 * kPiD;
  if (phi >= 2.0 * kPiD) phi = 0.0;
  const double sigma = isfinite(a.sg[t]) && a.sg[t] > 0.0 ? fmin(a.sg[t], kPiD) : 0.0;
  const double w2 = 2.0 * a.w[t];
  const int n = a.n;
  const double d = a.delta, th0 = 0.5 * kPiD - 0.5 * a.L, ph0 = -0.5 * a.L;
  const double is2 = sigma > 0.0 ? 1.0 / (sigma * sigma) : 0.0;
  const double hs = sin(0.5 * sigma), hs2 = hs * hs;  // hav(sigma)
  double sh, ch, sd, cd;                             // sin, cos of half a cell, a cell
  sincos(0.5 * a.delta, &sh, &ch);
  sincos(a.delta, &sd, &cd);
  const double smin = fmax(sin(fmin(0.5 * kPiD + 0.5 * a.L + sigma, kPiD - 1e-3)), 1e-3);
  // cells within sigma lie within sigma / d + 1/2 cells of the particle's
  // fractional cell coordinate, so this window (from the cell holding it)
  // contains them all
  const int di = int(sigma / d + 0.5) + 1, dj = int(sigma / (d * smin) + 0.5) + 1;
  T* fp = static_cast<T*>(a.fp);
  const int64_t Nb = a.Nb;
  const double reach = 0.75 * a.L + sigma + 2.0 * d;
  // the patches whose square the disc can reach: bundle centres within
  // 0.75 L + sigma (a patch's corners are L / sqrt 2 from its centre).
  // Candidates: the bundle pixels of the rings within reach in colatitude,
  // in each ring those within the azimuth range of the reach (a superset of
  // the disc; the window test below drops the patches it misses).
  const double rlo = fmax(0.0, theta - reach), rhi = fmin(kPiD, theta + reach);
  const int64_t q_lo = max(int64_t(1), int64_t(floor(ring_of(Nb, rlo))) - 1);
  const int64_t q_hi = min(4 * Nb - 1, int64_t(ceil(ring_of(Nb, rhi))) + 1);
  const double creach = cos(fmin(reach, kPiD)), sp0 = sqrt(p[0] * p[0] + p[1] * p[1]);
  for (int64_t q = q_lo; q <= q_hi; ++q) {
    const RingG g = ring_geom(Nb, q);
    int64_t c0 = 0, c1 = g.n - 1;
    const double den = sp0 * g.s;
    if (den > 1e-300) {
      // azimuths within reach: cos dphi >= (cos reach - z_p z_r) / (s_p s_r)
      const double c = (creach - p[2] * g.z) / den;
      if (c >= 1.0) continue;
      if (c > -1.0) {
        const double dmax = acos(c);
        const int64_t ca = int64_t(floor((phi - dmax - g.phi0) / g.dphi)) - 1;
        const int64_t cb = int64_t(ceil((phi + dmax - g.phi0) / g.dphi)) + 1;
        if (cb - ca + 1 < g.n) {
          c0 = ca;
          c1 = cb;
        }
      }
    }
    for (int64_t cj = c0; cj <= c1; ++cj) {
      const int64_t rb = g.first + ((cj % g.n) + g.n) % g.n;
      double zb, sb, pb;
      hpx::pix2ang_ring(a.Nb, rb, zb, sb, pb);
      const int64_t b = hpx::ang2nest(a.Nb, zb, pb);
      if (a.dflag && !a.dflag[b]) continue;
      const double* R = a.rot + 9 * b;
      const double v0 = R[0] * p[0] + R[1] * p[1] + R[2] * p[2];
      const double v1 = R[3] * p[0] + R[4] * p[1] + R[5] * p[2];
      const double v2 = R[6] * p[0] + R[7] * p[1] + R[8] * p[2];
      const double rho = sqrt(v0 * v0 + v1 * v1);  // sin theta'_p (|v| = 1)
      const double tp = hpx::atan2_r(rho, v2), pp = hpx::atan2_r(v1, v0);
      const int ic = int(floor((tp - th0) / d)), jc = int(floor((pp - ph0) / d));
      if (ic + di < 0 || ic - di >= n || jc + dj < 0 || jc - dj >= n) continue;
      const double stp = rho;
      T* fb = fp + size_t(b) * n * n;
      // angle to a cell centre by the haversine (accurate at small angles):
      // hav = sin^2(dtheta / 2) + sin theta'_i sin theta'_p sin^2(dphi / 2),
      // inside sigma when hav < sin^2(sigma / 2).  The cell area is
      // 2 d sin(theta'_i) sin(d / 2).  Row i holds cells of the disc only
      // where sin^2(dphi / 2) < (hav(sigma) - sin^2(dtheta / 2)) /
      // (sin theta'_i sin theta'_p): its window is cut to that azimuth
      // range, widened by a cell (the float32 bound is far inside it).  The
      // sines along the rows (steps d and d / 2) and along a row (steps
      // d / 2) come from angle-addition recurrences, the start of each
      // row's azimuth run from the window's first column by a short sine
      // series of the offset; the squared angle from a series in hav.
      const int i0 = ic - di, j0 = jc - dj;
      double st0, ct0, hs0, hc0, sj0, cj0;
      sincos(th0 + (i0 + 0.5) * d, &st0, &ct0);
      sincos(0.5 * (th0 + (i0 + 0.5) * d - tp), &hs0, &hc0);
      sincos(0.5 * (ph0 + (j0 + 0.5) * d - pp), &sj0, &cj0);
      auto visit = [&](auto&& f) {
        double sti = st0, cti = ct0, hti = hs0, hci = hc0;
        for (int i = i0; i <= ic + di; ++i) {
          const double h2 = hti * hti, ss = sti * stp;
          if (h2 < hs2) {
            const double area = 2.0 * d * sti * sh;
            const double q = ss > 0.0 ? (hs2 - h2) / ss : 2.0;
            const double dph = q >= 1.0 ? 2.0 * kPiD : 2.0 * double(asinf(sqrtf(float(q))));
            const int jlo = max(jc - dj, int(floor((pp - dph - ph0) / d - 0.5)) - 1);
            const int jhi = min(jc + dj, int(ceil((pp + dph - ph0) / d - 0.5)) + 1);
            // sin, cos of half the azimuth offset of column jlo from j0
            const double x = 0.5 * d * double(jlo - j0);
            double sx, cx;
            if (x < 0.05) {
              const double x2 = x * x;
              sx = x * fma(x2, fma(x2, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
              cx = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
            } else {
              sincos(x, &sx, &cx);
            }
            double sa = fma(sj0, cx, cj0 * sx), ca = fma(cj0, cx, -sj0 * sx);
            for (int j = jlo; j <= jhi; ++j) {
              const double hv = fmin(fma(ss * sa, sa, h2), 1.0);
              if (hv < hs2) {
                // (2 asin sqrt(hv))^2 = 4 (hv + hv^2 / 3 + 8 hv^3 / 45 + ...)
                double a2;
                if (hv < 1e-3) {
                  a2 = 4.0 * hv *
                       fma(hv,
                           fma(hv, fma(hv, fma(hv, 128.0 / 1575.0, 4.0 / 35.0), 8.0 / 45.0),
                               1.0 / 3.0),
                           1.0);
                } else {
                  const double ang = 2.0 * hpx::asin_small(sqrt(hv));
                  a2 = ang * ang;
                }
                f(i, j, 1.0 - a2 * is2, area);
              }
              const double sn = fma(sa, ch, ca * sh);
              ca = fma(ca, ch, -sa * sh);
              sa = sn;
            }
          }
          // next row: theta'_i by d, the half offset by d / 2
          const double s1 = fma(sti, cd, cti * sd);
          cti = fma(cti, cd, -sti * sd);
          sti = s1;
          const double h1 = fma(hti, ch, hci * sh);
          hci = fma(hci, ch, -hti * sh);
          hti = h1;
        }
      };
      double tot = 0.0;
      if (sigma > 0.0) visit([&](int, int, double k, double area) { tot += k * area; });
      if (tot > 0.0) {
        const double f = w2 / tot;
        visit([&](int i, int j, double k, double) {
          if (i >= 0 && i < n && j >= 0 && j < n)
            unsafeAtomicAdd(fb + size_t(i) * n + j, T(f * k));
        });
      } else if (ic >= 0 && ic < n && jc >= 0 && jc < n) {
        const double ti = th0 + (ic + 0.5) * d;
        unsafeAtomicAdd(fb + size_t(ic) * n + jc, T(w2 / (2.0 * d * sin(ti) * sin(0.5 * d))));
      }
    }
  }
}

}  // namespace

clm_status patch_deposit(Plan* p, const clm_particles* parts, hipStream_t s) {
  if (parts->n == 0) return CLM_OK;
  PatchDep a;
  a.th = parts->theta;
  a.ph = parts->phi;
  a.w = parts->weight;
  a.sg = parts->sigma;
  a.npart = parts->n;
  a.rot = p->rot;
  a.Nb = p->d.nside_bundle;
  a.n = p->n;
  a.L = p->L;
  a.delta = p->delta;
  a.dflag = p->domain ? p->dom_flag : nullptr;
  a.fp = p->fprime;
  const dim3 g(unsigned((parts->n + kBlock - 1) / kBlock));
  CLM_TIMED(p, s, "patch_deposit");
  if (p->fp64mg)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_deposit<double>), g, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_deposit<float>), g, dim3(kBlock), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status deposit_map(const clm_particles* parts, int64_t nside, double* map, hipStream_t s) {
  if (parts->n == 0) return CLM_OK;
  const dim3 g(unsigned((parts->n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_deposit, g, dim3(kBlock), 0, s, nside, parts->n, parts->theta,
                     parts->phi, parts->weight, parts->sigma, map);
  return hipGetLastError() == hipSuccess ? CLM_OK : CLM_EHIP;
}

}  // namespace clm

extern "C" clm_status clm_deposit_epanechnikov(const double* theta, const double* phi,
                                               const double* weight, const double* sigma,
                                               int64_t npart, int32_t nside, double* map,
                                               hipStream_t stream) {
  if (npart < 0 || nside < 1 || (nside & (nside - 1)) || nside > 8192 || !map ||
      (npart > 0 && (!theta || !phi || !weight || !sigma)))
    return CLM_EINVAL;
  if (npart == 0) return CLM_OK;
  const int64_t blocks = (npart + clm::kBlock - 1) / clm::kBlock;
  hipLaunchKernelGGL(clm::k_deposit, dim3(unsigned(blocks)), dim3(clm::kBlock), 0, stream,
                     int64_t(nside), npart, theta, phi, weight, sigma, map);
  return hipGetLastError() == hipSuccess ? CLM_OK : CLM_EHIP;
}
