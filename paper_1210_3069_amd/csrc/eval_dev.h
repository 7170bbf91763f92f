// Gradient and covariant Hessian of the patch potential u0 + du at a point
// (Sec. 3.2 last paragraphs, App. A): 4th-order finite differences of the
// raw partials psi_t', psi_p', psi_t't', psi_p'p', psi_t'p' at the four
// cells around the point, bilinear interpolation to the point, metric terms
// at the point's own theta', rotation to the global (theta-hat, phi-hat)
// basis.  Shared by the shear evaluation and the ray update.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "healpix_dev.h"

namespace clm {

struct PatchField {
  const double* rot;   // [nbundle][9]
  const double* u0;    // [nbundle][(n+2)^2] with ghosts
  const void* du;      // [nbundle][n^2] of T
  int n;
  double L, delta;
};

// u = u0 + du at cell (i, j), i, j in [-1, n]; du across the patch face is
// the negative of the interior cell it faces (zero face value).
template <typename T>
__device__ __forceinline__ double patch_u(const double* u0, const T* du, int n, int i, int j) {
  const double a = u0[(i + 1) * (n + 2) + (j + 1)];
  int ii = i, jj = j;
  double sg = 1.0;
  if (ii < 0) { ii = 0; sg = -1.0; }
  if (ii > n - 1) { ii = n - 1; sg = -1.0; }
  if (jj < 0) { jj = 0; sg = -1.0; }
  if (jj > n - 1) { jj = n - 1; sg = -1.0; }
  return a + sg * double(du[ii * n + jj]);
}

// 4th-order first- and second-derivative stencils at cell c of n along one
// axis: offsets o[k] = first + k and weights in units of 1/12.
struct Stencil {
  int first, len;
  double w[6];
};

__device__ __forceinline__ Stencil d1_stencil(int c, int n) {
  Stencil s;
  if (c >= 1 && c <= n - 2) {
    s.first = -2; s.len = 5;
    s.w[0] = 1; s.w[1] = -8; s.w[2] = 0; s.w[3] = 8; s.w[4] = -1;
  } else if (c == 0) {  // nodes -1 .. 3
    s.first = -1; s.len = 5;
    s.w[0] = -3; s.w[1] = -10; s.w[2] = 18; s.w[3] = -6; s.w[4] = 1;
  } else {              // nodes -3 .. 1
    s.first = -3; s.len = 5;
    s.w[0] = -1; s.w[1] = 6; s.w[2] = -18; s.w[3] = 10; s.w[4] = 3;
  }
  s.w[5] = 0;
  return s;
}

__device__ __forceinline__ Stencil d2_stencil(int c, int n) {
  Stencil s;
  if (c >= 1 && c <= n - 2) {
    s.first = -2; s.len = 5;
    s.w[0] = -1; s.w[1] = 16; s.w[2] = -30; s.w[3] = 16; s.w[4] = -1; s.w[5] = 0;
  } else if (c == 0) {  // nodes -1 .. 4
    s.first = -1; s.len = 6;
    s.w[0] = 10; s.w[1] = -15; s.w[2] = -4; s.w[3] = 14; s.w[4] = -6; s.w[5] = 1;
  } else {              // nodes -4 .. 1
    s.first = -4; s.len = 6;
    s.w[0] = 1; s.w[1] = -6; s.w[2] = 14; s.w[3] = -4; s.w[4] = -15; s.w[5] = 10;
  }
  return s;
}

// Raw stencil sums at one cell: 12 h psi_t', 12 h psi_p', 12 h^2 psi_t't',
// 12 h^2 psi_p'p', 144 h^2 psi_t'p'.
struct Partials {
  double pt, pp, ptt, ppp, ptp;
};

// Stencil sums at cell (i, j) with the general (edge-aware) stencils.  Only
// cells within two of the patch face take them; the loops stay rolled so
// this path does not raise the register count of the centred one.
template <typename T>
__device__ __forceinline__ Partials partials_general(const double* u0, const T* du, int n,
                                                     int i, int j) {
  const Stencil a1 = d1_stencil(i, n), b1 = d1_stencil(j, n);
  const Stencil a2 = d2_stencil(i, n), b2 = d2_stencil(j, n);
  Partials r{0, 0, 0, 0, 0};
#pragma unroll 1
  for (int k = 0; k < 6; ++k) {
    if (k < a1.len) {
      r.pt += a1.w[k] * patch_u(u0, du, n, i + a1.first + k, j);
      r.pp += b1.w[k] * patch_u(u0, du, n, i, j + b1.first + k);
    }
    if (k < a2.len) r.ptt += a2.w[k] * patch_u(u0, du, n, i + a2.first + k, j);
    if (k < b2.len) r.ppp += b2.w[k] * patch_u(u0, du, n, i, j + b2.first + k);
  }
#pragma unroll 1
  for (int k = 0; k < a1.len; ++k) {
    if (a1.w[k] == 0) continue;
    double row = 0;
#pragma unroll 1
    for (int q = 0; q < b1.len; ++q)
      row += b1.w[q] * patch_u(u0, du, n, i + a1.first + k, j + b1.first + q);
    r.ptp += a1.w[k] * row;
  }
  return r;
}

// g = (g_t, g_p), U = (U_tt, U_pp, U_tp) of psi at unit vector v in patch b,
// global basis.  Returns false when the bilinear footprint leaves the patch.
template <typename T>
__device__ bool eval_patch(const PatchField& P, int64_t b, double vx, double vy, double vz,
                           double g[2], double U[3]) {
  const double pi = 3.14159265358979323846;
  const double* R = P.rot + 9 * b;
  const double px = R[0] * vx + R[1] * vy + R[2] * vz;
  const double py = R[3] * vx + R[4] * vy + R[5] * vz;
  const double pz = R[6] * vx + R[7] * vy + R[8] * vz;
  const double sp_ = sqrt(px * px + py * py);  // sin theta'
  // theta' = pi/2 - asin(cos theta') and phi' = atan(py / px): series near
  // the patch centre, where every point of the bundle lies
  const double thp = pi / 2 - hpx::asin_small(pz);
  const double php = hpx::dphi_of(px, py, 1.0, 0.0);
  const int n = P.n;
  const double ih = 1.0 / P.delta;
  const double fi = (thp - (pi / 2 - P.L / 2)) * ih - 0.5;
  const double fj = (php + P.L / 2) * ih - 0.5;
  const double ffi = floor(fi), ffj = floor(fj);
  if (!(ffi >= 0 && ffi <= n - 2 && ffj >= 0 && ffj <= n - 2)) return false;
  const int i0 = int(ffi), j0 = int(ffj);
  const double t = fi - ffi, s = fj - ffj;
  const double* u0 = P.u0 + size_t(b) * (n + 2) * (n + 2);
  const T* du = static_cast<const T*>(P.du) + size_t(b) * n * n;
  // bilinear interpolation of the four cells' stencil sums, accumulated as
  // each cell's sums are formed (the interpolation is linear); the 1/(12 h),
  // 1/(12 h^2), 1/(144 h^2) factors are applied once afterwards
  double Pv0 = 0, Pv1 = 0, Pv2 = 0, Pv3 = 0, Pv4 = 0;
  if (i0 >= 2 && i0 + 3 <= n - 1 && j0 >= 2 && j0 + 3 <= n - 1) {
    // centred stencils only, over the 6 x 6 window of u around the four
    // cells (rows and columns i0-2 .. i0+3, j0-2 .. j0+3).  The bilinear
    // weights and the 1-D stencils combine into per-row and per-column
    // weight vectors (the 2-D stencils are products of 1-D ones), so each
    // sum is a row weight times a column weight times u, taken row by row.
    const double t0 = 1 - t, t1 = t, s0 = 1 - s, s1 = s;
    // first derivative (1, -8, 0, 8, -1) and second (-1, 16, -30, 16, -1)
    // about window rows 2 and 3, weighted t0 and t1
    const double r1[6] = {t0, -8 * t0 + t1, -8 * t1, 8 * t0, -t0 + 8 * t1, -t1};
    const double r2[6] = {-t0, 16 * t0 - t1, -30 * t0 + 16 * t1, 16 * t0 - 30 * t1,
                          -t0 + 16 * t1, -t1};
    const double c1[6] = {s0, -8 * s0 + s1, -8 * s1, 8 * s0, -s0 + 8 * s1, -s1};
    const double c2[6] = {-s0, 16 * s0 - s1, -30 * s0 + 16 * s1, 16 * s0 - 30 * s1,
                          -s0 + 16 * s1, -s1};
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const double* ur = u0 + (i0 - 2 + r + 1) * (n + 2) + (j0 - 2 + 1);
      const T* dr = du + (i0 - 2 + r) * n + (j0 - 2);
      double w[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) w[c] = ur[c] + double(dr[c]);
      const double wi = s0 * w[2] + s1 * w[3];  // interpolated along the row
      double w1 = 0;                            // first derivative along the row
#pragma unroll
      for (int c = 0; c < 6; ++c) w1 += c1[c] * w[c];
      Pv0 += r1[r] * wi;
      Pv2 += r2[r] * wi;
      Pv4 += r1[r] * w1;
      if (r == 2 || r == 3) {
        double w2 = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) w2 += c2[c] * w[c];
        const double tr = r == 2 ? t0 : t1;
        Pv1 += tr * w1;
        Pv3 += tr * w2;
      }
    }
  } else {
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
      const Partials c = partials_general<T>(u0, du, n, i0 + (k >> 1), j0 + (k & 1));
      const double bw = ((k >> 1) ? t : 1 - t) * ((k & 1) ? s : 1 - s);
      Pv0 += bw * c.pt;
      Pv1 += bw * c.pp;
      Pv2 += bw * c.ptt;
      Pv3 += bw * c.ppp;
      Pv4 += bw * c.ptp;
    }
  }
  const double i1 = ih / 12, i2 = ih * ih / 12;
  const double Pv[5] = {Pv0 * i1, Pv1 * i1, Pv2 * i2, Pv3 * i2, Pv4 * (i2 / 12)};
  // covariant components in the patch frame at the point (App. A)
  const double st = sp_, ct = pz, ist = 1.0 / st;
  const double gpt = Pv[0], gpp = Pv[1] * ist;
  const double Utt = Pv[2];
  const double Upp = Pv[3] * ist * ist + (ct * ist) * Pv[0];
  const double Utp = Pv[4] * ist - ct * Pv[1] * ist * ist;
  // patch basis at the point, in global coordinates: R^T (theta'-hat, phi'-hat)
  const double cpp = px * ist, spp = py * ist;
  const double et_p[3] = {ct * cpp, ct * spp, -st};
  const double ep_p[3] = {-spp, cpp, 0.0};
  double etp[3], epp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    etp[k] = R[k] * et_p[0] + R[3 + k] * et_p[1] + R[6 + k] * et_p[2];
    epp[k] = R[k] * ep_p[0] + R[3 + k] * ep_p[1] + R[6 + k] * ep_p[2];
  }
  // global basis at the point
  const double sg = sqrt(vx * vx + vy * vy), isg = 1.0 / sg;
  const double cph = vx * isg, sph = vy * isg;
  const double et[3] = {vz * cph, vz * sph, -sg};
  const double ep[3] = {-sph, cph, 0.0};
  const double q00 = et[0] * etp[0] + et[1] * etp[1] + et[2] * etp[2];
  const double q01 = et[0] * epp[0] + et[1] * epp[1] + et[2] * epp[2];
  const double q10 = ep[0] * etp[0] + ep[1] * etp[1] + ep[2] * etp[2];
  const double q11 = ep[0] * epp[0] + ep[1] * epp[1] + ep[2] * epp[2];
  g[0] = q00 * gpt + q01 * gpp;
  g[1] = q10 * gpt + q11 * gpp;
  // U = Q U' Q^T
  const double a00 = q00 * Utt + q01 * Utp, a01 = q00 * Utp + q01 * Upp;
  const double a10 = q10 * Utt + q11 * Utp, a11 = q10 * Utp + q11 * Upp;
  U[0] = a00 * q00 + a01 * q01;
  U[1] = a10 * q10 + a11 * q11;
  U[2] = a00 * q10 + a01 * q11;
  return true;
}

}  // namespace clm
