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

// Four RING pixels and weights for bilinear interpolation at (theta, phi):
// rings bracketing theta, pixels bracketing phi in each, linear weights;
// above the first ring (below the last) the pole value is the mean of that
// ring's four pixels.
__device__ __forceinline__ void interp_weights(const Rings& R, double theta, double z,
                                               double phi, int64_t pix[4], double w[4]) {
  const double twopi = 6.283185307179586476925286766559;
  const int N = R.N;
  // first guess from the ring formulas (z = cos theta), then exact
  // bracketing on theta
  double fr;
  if (z > 2.0 / 3.0)
    fr = N * sqrt(3.0 * (1.0 - z));
  else if (z < -2.0 / 3.0)
    fr = 4.0 * N - N * sqrt(3.0 * (1.0 + z));
  else
    fr = N * (2.0 - 1.5 * z);
  int g = int(floor(fr)) - 1;  // 0-based candidate
  if (g < -1) g = -1;
  if (g > R.nring - 1) g = R.nring - 1;
  while (g + 1 < R.nring && R.rt[4 * (g + 1) + 2] <= theta) ++g;
  while (g >= 0 && R.rt[4 * g + 2] > theta) --g;

  auto pair = [&](int q, int64_t& a, int64_t& b, double& wp) {
    const int n = R.ri[2 * q];
    const int64_t first = R.ri[2 * q + 1];
    const double t = (phi - R.rt[4 * q + 3]) * R.rx[2 * q];
    const double fl = floor(t);
    wp = t - fl;
    int i1 = int(fl);
    while (i1 < 0) i1 += n;
    while (i1 >= n) i1 -= n;
    const int i2 = i1 + 1 == n ? 0 : i1 + 1;
    a = first + i1;
    b = first + i2;
  };

  if (g >= 0 && g < R.nring - 1) {
    int64_t a1, a2, b1, b2;
    double wa, wb;
    pair(g, a1, a2, wa);
    pair(g + 1, b1, b2, wb);
    const double wt = (theta - R.rt[4 * g + 2]) * R.rx[2 * (g + 1) + 1];
    pix[0] = a1; pix[1] = a2; pix[2] = b1; pix[3] = b2;
    w[0] = (1 - wt) * (1 - wa);
    w[1] = (1 - wt) * wa;
    w[2] = wt * (1 - wb);
    w[3] = wt * wb;
  } else if (g < 0) {
    int64_t b1, b2;
    double wb;
    pair(0, b1, b2, wb);
    const double wt = theta * R.rx[1];
    const double fac = (1.0 - wt) * 0.25;
    pix[0] = b1; pix[1] = b2; pix[2] = (b1 + 2) & 3; pix[3] = (b2 + 2) & 3;
    w[0] = wt * (1 - wb) + fac;
    w[1] = wt * wb + fac;
    w[2] = fac;
    w[3] = fac;
  } else {
    const int q = R.nring - 1;
    int64_t a1, a2;
    double wa;
    pair(q, a1, a2, wa);
    const double wt = (theta - R.rt[4 * q + 2]) * R.rx[2 * R.nring + 1];
    const int64_t base = R.ri[2 * q + 1];
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

template <typename T>
__device__ __forceinline__ double interp(const Rings& R, const T* map, double theta, double z,
                                         double phi) {
  int64_t pix[4];
  double w[4];
  interp_weights(R, theta, z, phi, pix, w);
  return w[0] * double(map[pix[0]]) + w[1] * double(map[pix[1]]) +
         w[2] * double(map[pix[2]]) + w[3] * double(map[pix[3]]);
}

}  // namespace hpx
}  // namespace clm
