// HEALPix pixelization on the device (Gorski et al. 2005): NESTED <-> RING
// numbering, direction -> NESTED pixel, and the public package's bilinear
// interpolation on a RING map, which Sec. 3.2 uses to carry the SHT
// potential onto the multigrid patches.  Ring tables (z, sin theta, theta,
// phi0; n, first pixel) are built on the host at plan creation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace clm {
namespace hpx {

// Base-face ring offset (units of N) and longitude offset of faces 0..11.
__device__ __constant__ static const int kJrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
__device__ __constant__ static const int kJpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

__device__ __forceinline__ int64_t spread(int64_t v) {
  // bit k -> bit 2k for the low 32 bits
  v &= 0xffffffffLL;
  v = (v | (v << 16)) & 0x0000ffff0000ffffLL;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffLL;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fLL;
  v = (v | (v << 2)) & 0x3333333333333333LL;
  v = (v | (v << 1)) & 0x5555555555555555LL;
  return v;
}

__device__ __forceinline__ int64_t compact(int64_t v) {
  v &= 0x5555555555555555LL;
  v = (v | (v >> 1)) & 0x3333333333333333LL;
  v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0fLL;
  v = (v | (v >> 4)) & 0x00ff00ff00ff00ffLL;
  v = (v | (v >> 8)) & 0x0000ffff0000ffffLL;
  v = (v | (v >> 16)) & 0x00000000ffffffffLL;
  return v;
}

// NESTED -> RING at resolution N.
__device__ __forceinline__ int64_t nest2ring(int64_t N, int64_t p) {
  const int64_t npface = N * N;
  const int face = int(p / npface);
  const int64_t q = p - face * npface;
  const int64_t ix = compact(q), iy = compact(q >> 1);
  const int64_t jr = int64_t(kJrll[face]) * N - ix - iy - 1;  // 1-based ring
  int64_t nr, first, kshift;
  if (jr < N) {
    nr = jr;
    first = 2 * jr * (jr - 1);
    kshift = 0;
  } else if (jr > 3 * N) {
    nr = 4 * N - jr;
    first = 12 * N * N - 2 * nr * (nr + 1);
    kshift = 0;
  } else {
    nr = N;
    first = 2 * N * (N - 1) + 4 * N * (jr - N);
    kshift = (jr - N) & 1;
  }
  int64_t jp = (int64_t(kJpll[face]) * nr + ix - iy + 1 + kshift) / 2;
  if (jp > 4 * N) jp -= 4 * N;
  if (jp < 1) jp += 4 * nr;
  return first + jp - 1;
}

// Direction (z = cos theta, phi) -> NESTED pixel at resolution N.
__device__ __forceinline__ int64_t ang2nest(int64_t N, double z, double phi) {
  const double twopi = 6.283185307179586476925286766559;
  double za = fabs(z);
  double tt = fmod(phi, twopi);
  if (tt < 0) tt += twopi;
  tt *= 0.63661977236758134307553505349006;  // 2/pi
  if (tt >= 4.0) tt -= 4.0;
  int face;
  int64_t ix, iy;
  if (za <= 2.0 / 3.0) {
    const double t1 = double(N) * (0.5 + tt);
    const double t2 = double(N) * (z * 0.75);
    const int64_t jp = int64_t(floor(t1 - t2));
    const int64_t jm = int64_t(floor(t1 + t2));
    const int64_t ifp = jp / N, ifm = jm / N;
    face = (ifp == ifm) ? int(ifp | 4) : (ifp < ifm ? int(ifp) : int(ifm + 8));
    ix = jm & (N - 1);
    iy = N - (jp & (N - 1)) - 1;
  } else {
    int ntt = int(floor(tt));
    if (ntt > 3) ntt = 3;
    const double tp = tt - ntt;
    const double tmp = double(N) * sqrt(3.0 * (1.0 - za));
    int64_t jp = int64_t(floor(tp * tmp));
    int64_t jm = int64_t(floor((1.0 - tp) * tmp));
    if (jp > N - 1) jp = N - 1;
    if (jm > N - 1) jm = N - 1;
    if (z >= 0) {
      face = ntt;
      ix = N - jm - 1;
      iy = N - jp - 1;
    } else {
      face = ntt + 8;
      ix = jp;
      iy = jm;
    }
  }
  return int64_t(face) * N * N + spread(ix) + (spread(iy) << 1);
}

// Centre of RING pixel p at resolution N: z = cos theta, sin theta, phi.
__device__ __forceinline__ void pix2ang_ring(int64_t N, int64_t p, double& z, double& st,
                                             double& phi) {
  const double pi = 3.14159265358979323846;
  const int64_t ncap = 2 * N * (N - 1), npix = 12 * N * N;
  if (p < ncap || p >= npix - ncap) {
    const bool north = p < ncap;
    const int64_t q = north ? p : npix - 1 - p;
    int64_t i = int64_t((1.0 + sqrt(1.0 + 2.0 * double(q))) * 0.5);
    while (2 * i * (i - 1) > q) --i;
    while (2 * (i + 1) * i <= q) ++i;
    const int64_t j = north ? p - 2 * i * (i - 1) : p - (npix - 2 * i * (i + 1));
    const double omz = double(i) * double(i) / (3.0 * double(N) * double(N));
    z = north ? 1.0 - omz : omz - 1.0;
    st = sqrt(omz * (2.0 - omz));
    phi = (double(j) + 0.5) * pi / (2.0 * double(i));
  } else {
    const int64_t q = p - ncap;
    const int64_t i = q / (4 * N) + N;
    const int64_t j = q % (4 * N);
    z = (4.0 * N - 2.0 * i) / (3.0 * N);
    st = sqrt((1.0 - z) * (1.0 + z));
    const bool shifted = ((i - N) & 1) == 0;
    phi = (double(j) + (shifted ? 0.5 : 0.0)) * pi / (2.0 * double(N));
  }
}

// Ring tables on the device: rt[4*q + {0,1,2,3}] = z, sin, theta, phi0 and
// ri[2*q + {0,1}] = pixels in ring, first pixel, for 0-based ring q.
// rx[2 q] = n_q / (2 pi); rx[2 q + 1] = 1 / (theta_q - theta_{q-1}) with
// theta_{-1} = 0, and rx[2 nring + 1] = 1 / (pi - theta_{nring-1}).
struct Rings {
  const double* rt;
  const int* ri;
  const double* rx;
  int nring;
  int N;
};

// atan(u), float64, for |u| <= 0.07: odd Taylor series to u^15 (remainder
// below 2e-22 relative).
__device__ __forceinline__ double atan_series(double u) {
  const double u2 = u * u;
  double s = -1.0 / 15.0;
  s = fma(s, u2, 1.0 / 13.0);
  s = fma(s, u2, -1.0 / 11.0);
  s = fma(s, u2, 1.0 / 9.0);
  s = fma(s, u2, -1.0 / 7.0);
  s = fma(s, u2, 1.0 / 5.0);
  s = fma(s, u2, -1.0 / 3.0);
  return fma(s * u2, u, u);
}

// atan(k / 8), k = 0 .. 8, rounded to float64.
static __constant__ double kAtanEighth[9] = {
    0.0,
    0.12435499454676144,
    0.24497866312686414,
    0.35877067027057225,
    0.4636476090008061,
    0.5585993153435624,
    0.6435011087932844,
    0.7188299996216245,
    0.7853981633974483};

// num / den, float64, for den > 0 of moderate size: hardware reciprocal,
// two Newton steps and a residual correction of the quotient.
__device__ __forceinline__ double div_pos(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  const double q = num * r;
  return fma(r, fma(-den, q, num), q);
}

// atan2(y, x), float64, branch-free: reduce to u = min/max of |x|, |y| in
// [0, 1]; with c = k/8 the nearest eighth, atan u = atan c + atan r,
// r = (u - c) / (1 + u c), |r| <= 1/16; then undo the octant.  (0, 0) -> 0.
__device__ __forceinline__ double atan2_r(double y, double x) {
  const double ax = fabs(x), ay = fabs(y);
  const double mx = fmax(ax, ay), mn = fmin(ax, ay);
  const float ef = mx > 0.0 ? float(mn) / float(mx) : 0.0f;
  const int k = min(int(fmaf(8.0f, ef, 0.5f)), 8);
  const double c = 0.125 * k;
  const double num = fma(-c, mx, mn), den = fma(c, mn, mx);
  const double r = den > 0.0 ? div_pos(num, den) : 0.0;
  double a = kAtanEighth[k] + atan_series(r);
  if (ay > ax) a = 1.5707963267948966 - a;
  if (x < 0.0) a = 3.141592653589793 - a;
  return y < 0.0 ? -a : a;
}

// asin(s), float64, for |s| < 0.05: Taylor series (2k)!/(4^k (k!)^2 (2k+1))
// s^(2k+1) to s^13 (remainder < 1e-21); asin_small adds atan2(s, sqrt(1 -
// s^2)) for larger |s|.
__device__ __forceinline__ double asin_series(double s) {
  const double s2 = s * s;
  double p = 231.0 / 13312.0;
  p = fma(p, s2, 63.0 / 2816.0);
  p = fma(p, s2, 35.0 / 1152.0);
  p = fma(p, s2, 5.0 / 112.0);
  p = fma(p, s2, 3.0 / 40.0);
  p = fma(p, s2, 1.0 / 6.0);
  return fma(p * s2, s, s);
}

__device__ __forceinline__ double asin_small(double s) {
  if (fabs(s) >= 0.05) return atan2_r(s, sqrt((1.0 - s) * (1.0 + s)));
  return asin_series(s);
}

// asin(s) for |s| < 0.004: s + s^3/6 + 3 s^5/40 (remainder below 1e-18).
__device__ __forceinline__ double asin_short(double s) {
  const double s2 = s * s;
  return fma(fma(3.0 / 40.0, s2, 1.0 / 6.0) * s2, s, s);
}

// Azimuth of (vx, vy) measured from a reference azimuth with cosine c and
// sine s, in [-pi, pi]: the series atan of the quotient of the rotated
// components when the offset is below 0.05 rad, atan2_r otherwise.
__device__ __forceinline__ double dphi_of(double vx, double vy, double c, double s) {
  const double cs = vx * c + vy * s, sn = vy * c - vx * s;
  if (cs > 20.0 * fabs(sn)) return atan_series(div_pos(sn, cs));
  return atan2_r(sn, cs);
}

// Ring-table accessors used by the interpolation.  A point is given by
// z = cos theta, rho = sin theta and its azimuth as an offset dphi from the
// table's reference azimuth phi_ref; t(q, dphi) is the point's coordinate
// along ring q in pixel units, (phi - phi0_q) n_q / (2 pi).
struct GlobalRingTab {
  Rings R;
  double phi_ref;
  __device__ __forceinline__ int nring() const { return R.nring; }
  __device__ __forceinline__ int N() const { return R.N; }
  __device__ __forceinline__ double z(int q) const { return R.rt[4 * q]; }
  __device__ __forceinline__ double s(int q) const { return R.rt[4 * q + 1]; }
  __device__ __forceinline__ double t(int q, double dphi) const {
    return (phi_ref - R.rt[4 * q + 3] + dphi) * R.rx[2 * q];
  }
  __device__ __forceinline__ double igap(int q) const { return R.rx[2 * q + 1]; }
  __device__ __forceinline__ int n(int q) const { return R.ri[2 * q]; }
  __device__ __forceinline__ int first(int q) const { return R.ri[2 * q + 1]; }
  // rings held, and the range of the bracketing index (ring g and g + 1,
  // or the pole gap, must be held)
  __device__ __forceinline__ int qmin() const { return 0; }
  __device__ __forceinline__ int qmax() const { return R.nring - 1; }
  __device__ __forceinline__ int lo() const { return -1; }
  __device__ __forceinline__ int hi() const { return R.nring - 1; }
};

// A contiguous range of rings base .. top copied to LDS (ring q at slot
// q - base) for one reference azimuth.
struct LdsRingTab {
  double* zq;     // [cap] z
  double* sq;     // [cap] sin theta
  double* tq;     // [cap] (phi_ref - phi0) n / (2 pi)
  double* kq;     // [cap] n / (2 pi)
  double* gq;     // [cap + 1] 1 / theta gap above ring (last: south pole gap)
  int* nq;        // [cap]
  int* fq;        // [cap]
  int base, top, nr, NN;
  __device__ __forceinline__ int nring() const { return nr; }
  __device__ __forceinline__ int N() const { return NN; }
  __device__ __forceinline__ double z(int q) const { return zq[q - base]; }
  __device__ __forceinline__ double s(int q) const { return sq[q - base]; }
  __device__ __forceinline__ double t(int q, double dphi) const {
    return fma(dphi, kq[q - base], tq[q - base]);
  }
  __device__ __forceinline__ double igap(int q) const { return gq[q - base]; }
  __device__ __forceinline__ int n(int q) const { return nq[q - base]; }
  __device__ __forceinline__ int first(int q) const { return fq[q - base]; }
  __device__ __forceinline__ int qmin() const { return base; }
  __device__ __forceinline__ int qmax() const { return top; }
  __device__ __forceinline__ int lo() const { return base > 0 ? base : -1; }
  __device__ __forceinline__ int hi() const { return top == nr - 1 ? top : top - 1; }
  // all threads of the block: copy rings [b, t] of R (gap entries b .. t+1)
  __device__ void fill(const Rings& R, int b, int t, double phi_ref) {
    base = b; top = t; nr = R.nring; NN = R.N;
    for (int k = threadIdx.x; k <= t - b + 1; k += blockDim.x) {
      const int q = b + k;
      if (q <= t) {
        zq[k] = R.rt[4 * q]; sq[k] = R.rt[4 * q + 1];
        kq[k] = R.rx[2 * q];
        tq[k] = (phi_ref - R.rt[4 * q + 3]) * R.rx[2 * q];
        nq[k] = R.ri[2 * q]; fq[k] = R.ri[2 * q + 1];
      }
      if (q <= R.nring) gq[k] = R.rx[2 * q + 1];
    }
  }
};

// Index of the last ring with z_q >= z (-1 above the first ring), kept in
// [lo, hi] of the table.  The ring formulas of the HEALPix construction
// (Sec. 2) give the continuous ring coordinate (ring i at i); its float32
// value is off by less than one ring, and one exact comparison each way
// settles the index.
template <typename Tab>
__device__ __forceinline__ int ring_above(const Tab& R, double z) {
  const float N = float(R.N());
  const float za = float(fabs(z));
  float fr;
  if (za > 2.0f / 3.0f) {
    const float fp = N * __builtin_amdgcn_sqrtf(fmaxf(float(3.0 * (1.0 - fabs(z))), 0.0f));
    fr = z > 0 ? fp : 4.0f * N - fp;
  } else {
    fr = N * (2.0f - 1.5f * float(z));
  }
  const int lo = R.lo(), hi = R.hi();
  int c = int(floorf(fr)) - 1;
  c = min(max(c, lo), hi);
  const double zb = R.z(min(c + 1, R.qmax()));  // ring below the guess
  const double za0 = R.z(max(c, R.qmin()));     // the guess
  if (c < hi && zb >= z)
    ++c;
  else if (c > lo && za0 < z)
    --c;
  return c;
}

// Four RING pixels and weights for bilinear interpolation at the point
// (z, rho, dphi) whose ring index from ring_above is g: rings bracketing
// theta, pixels bracketing phi in each,
// linear weights; above the first ring (below the last) the pole value is
// the mean of that ring's four pixels.  The theta offset from the upper ring
// is asin(rho z_q - z sin theta_q).
template <typename Tab>
__device__ __forceinline__ void interp_weights_g(const Tab& R, int g, double z, double rho,
                                                 double dphi, int pix[4], double w[4]) {
  const int nring = R.nring();

  auto pair = [&](int q, int& a, int& b, double& wp) {
    const int n = R.n(q);
    const int first = R.first(q);
    const double t = R.t(q, dphi);
    const double fl = floor(t);
    wp = t - fl;
    int i1 = int(fl);
    i1 += i1 < 0 ? n : 0;
    i1 -= i1 >= n ? n : 0;
    i1 = min(max(i1, 0), n - 1);  // azimuths outside (-pi, 3 pi) only
    const int i2 = i1 + 1 == n ? 0 : i1 + 1;
    a = first + i1;
    b = first + i2;
  };
  // theta - theta_q for the ring above (theta_{-1} = 0 at the north pole)
  auto dtheta = [&](int q) {
    const double z1 = q >= 0 ? R.z(q) : 1.0, s1 = q >= 0 ? R.s(q) : 0.0;
    return asin_small(fma(rho, z1, -z * s1));
  };

  if (g >= 0 && g < nring - 1) {
    int a1, a2, b1, b2;
    double wa, wb;
    pair(g, a1, a2, wa);
    pair(g + 1, b1, b2, wb);
    const double wt = dtheta(g) * R.igap(g + 1);
    pix[0] = a1; pix[1] = a2; pix[2] = b1; pix[3] = b2;
    w[0] = (1 - wt) * (1 - wa);
    w[1] = (1 - wt) * wa;
    w[2] = wt * (1 - wb);
    w[3] = wt * wb;
  } else if (g < 0) {
    int b1, b2;
    double wb;
    pair(0, b1, b2, wb);
    const double wt = dtheta(-1) * R.igap(0);
    const double fac = (1.0 - wt) * 0.25;
    pix[0] = b1; pix[1] = b2; pix[2] = (b1 + 2) & 3; pix[3] = (b2 + 2) & 3;
    w[0] = wt * (1 - wb) + fac;
    w[1] = wt * wb + fac;
    w[2] = fac;
    w[3] = fac;
  } else {
    const int q = nring - 1;
    int a1, a2;
    double wa;
    pair(q, a1, a2, wa);
    const double wt = dtheta(q) * R.igap(nring);
    const int base = R.first(q);
    const double fac = wt * 0.25;
    pix[0] = a1; pix[1] = a2;
    pix[2] = base + ((a1 - base + 2) & 3);
    pix[3] = base + ((a2 - base + 2) & 3);
    w[0] = (1 - wt) * (1 - wa) + fac;
    w[1] = (1 - wt) * wa + fac;
    w[2] = fac;
    w[3] = fac;
  }
}

template <typename Tab>
__device__ __forceinline__ void interp_weights_t(const Tab& R, double z, double rho, double dphi,
                                                 int pix[4], double w[4]) {
  interp_weights_g(R, ring_above(R, z), z, rho, dphi, pix, w);
}

// Interpolation at (z, rho, phi) from the global tables, phi in [0, 2 pi).
__device__ __forceinline__ void interp_weights(const Rings& R, double z, double rho, double phi,
                                               int pix[4], double w[4]) {
  interp_weights_t(GlobalRingTab{R, phi}, z, rho, 0.0, pix, w);
}

template <typename T, typename Tab>
__device__ __forceinline__ double interp_t(const Tab& R, const T* map, double z, double rho,
                                           double dphi) {
  int pix[4];
  double w[4];
  interp_weights_t(R, z, rho, dphi, pix, w);
  return w[0] * double(map[pix[0]]) + w[1] * double(map[pix[1]]) +
         w[2] * double(map[pix[2]]) + w[3] * double(map[pix[3]]);
}

template <typename T>
__device__ __forceinline__ double interp(const Rings& R, const T* map, double z, double rho,
                                         double phi) {
  return interp_t(GlobalRingTab{R, phi}, map, z, rho, 0.0);
}

}  // namespace hpx
}  // namespace clm
