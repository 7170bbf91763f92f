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

}  // namespace
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
