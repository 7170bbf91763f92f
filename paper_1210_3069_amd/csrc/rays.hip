// Multiple-plane ray propagation on the sphere (Sec. 2.2, App. B, App. D).
//
// Ray state is structure-of-arrays in NESTED pixel order of the fine grid,
// so the rays of one bundle are contiguous and their patch is bundle =
// ray >> shift (Sec. 3.1).  One thread per ray: gather g and U from the
// bundle's patch, rotate the direction (eq. betaprop), move to the next
// plane (eq. posprop), step the Jacobian (eq. Atraj) and parallel transport
// both Jacobians to the new position (App. B).  Geometry in float64,
// Jacobians stored as float32 and combined in float64.
#include <cmath>

#include "clm_internal.h"
#include "eval_dev.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlock = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;

__global__ void k_rays_init(int64_t Nf, int64_t n, double* th, double* ph, double* beta,
                            float* A, float* Ap) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double z, st, phi;
  hpx::pix2ang_ring(Nf, hpx::nest2ring(Nf, i), z, st, phi);
  th[i] = atan2(st, z);
  ph[i] = phi;
  beta[i] = st * cos(phi);
  beta[n + i] = st * sin(phi);
  beta[2 * n + i] = z;
  const float I4[4] = {1.f, 0.f, 0.f, 1.f};
  for (int k = 0; k < 4; ++k) {
    A[k * n + i] = I4[k];
    Ap[k * n + i] = I4[k];
  }
}

// v rotated counter-clockwise about unit axis k by the angle with cosine c
// and sine s (Rodrigues); omc = 1 - c.
__device__ __forceinline__ void rotate_cs(const double k[3], double c, double s, double omc,
                                          const double v[3], double out[3]) {
  const double kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2];
  const double cx = k[1] * v[2] - k[2] * v[1];
  const double cy = k[2] * v[0] - k[0] * v[2];
  const double cz = k[0] * v[1] - k[1] * v[0];
  out[0] = v[0] * c + cx * s + k[0] * kv * omc;
  out[1] = v[1] * c + cy * s + k[1] * kv * omc;
  out[2] = v[2] * c + cz * s + k[2] * kv * omc;
}

// v rotated by angle w counter-clockwise about unit axis k (Rodrigues).
__device__ __forceinline__ void rotate(const double k[3], double w, const double v[3],
                                       double out[3]) {
  double s, c;
  sincos(w, &s, &c);
  const double kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2];
  const double cx = k[1] * v[2] - k[2] * v[1];
  const double cy = k[2] * v[0] - k[0] * v[2];
  const double cz = k[0] * v[1] - k[1] * v[0];
  out[0] = v[0] * c + cx * s + k[0] * kv * (1.0 - c);
  out[1] = v[1] * c + cy * s + k[1] * kv * (1.0 - c);
  out[2] = v[2] * c + cz * s + k[2] * kv * (1.0 - c);
}

// theta-hat and phi-hat at unit vector v
__device__ __forceinline__ void basis(const double v[3], double et[3], double ep[3]) {
  const double s = sqrt(v[0] * v[0] + v[1] * v[1]);
  const double cp = v[0] / s, sp = v[1] / s;
  et[0] = v[2] * cp; et[1] = v[2] * sp; et[2] = -s;
  ep[0] = -sp; ep[1] = cp; ep[2] = 0.0;
}

// App. B: the rotation that carries unit vector n0 to n1 about n0 x n1,
// applied to the basis (et0, ep0) at n0 and projected on the basis at n1:
// M_kl = e_k(n1) . R e_l(n0).  A tensor transports as M X M^T.
__device__ __forceinline__ void transport_matrix(const double n0[3], const double et0[3],
                                                 const double ep0[3], const double n1[3],
                                                 double M[4]) {
  double et1[3], ep1[3];
  basis(n1, et1, ep1);
  double ax[3] = {n0[1] * n1[2] - n0[2] * n1[1], n0[2] * n1[0] - n0[0] * n1[2],
                  n0[0] * n1[1] - n0[1] * n1[0]};
  const double sn = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
  double rt[3], rp[3];
  if (sn > 0) {
    ax[0] /= sn; ax[1] /= sn; ax[2] /= sn;
    // the angle between the unit vectors: cosine n0.n1, sine |n0 x n1|;
    // 1 - cos = sin^2 / (1 + cos) without cancellation
    const double cw = n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2];
    const double omc = sn * sn / (1.0 + cw);
    rotate_cs(ax, cw, sn, omc, et0, rt);
    rotate_cs(ax, cw, sn, omc, ep0, rp);
  } else {
    for (int k = 0; k < 3; ++k) { rt[k] = et0[k]; rp[k] = ep0[k]; }
  }
  M[0] = et1[0] * rt[0] + et1[1] * rt[1] + et1[2] * rt[2];
  M[1] = et1[0] * rp[0] + et1[1] * rp[1] + et1[2] * rp[2];
  M[2] = ep1[0] * rt[0] + ep1[1] * rt[1] + ep1[2] * rt[2];
  M[3] = ep1[0] * rp[0] + ep1[1] * rp[1] + ep1[2] * rp[2];
}

// M X M^T of a row-major 2 x 2 tensor
__device__ __forceinline__ void transport_tensor(const double M[4], const double X[4],
                                                 double out[4]) {
  const double t00 = M[0] * X[0] + M[1] * X[2], t01 = M[0] * X[1] + M[1] * X[3];
  const double t10 = M[2] * X[0] + M[3] * X[2], t11 = M[2] * X[1] + M[3] * X[3];
  out[0] = t00 * M[0] + t01 * M[1];
  out[1] = t00 * M[2] + t01 * M[3];
  out[2] = t10 * M[0] + t11 * M[1];
  out[3] = t10 * M[2] + t11 * M[3];
}

struct RayArgs {
  PatchField P;
  const double* D;   // pure-SHT planes: [5][n] g_t, g_p, U_tt, U_pp, U_tp at the RING
                     // pixel centres of the ray grid
  hpx::Rings rf;     // ... and that grid's ring tables
  const int* pmap;   // partial sky: the domain's bundles (their rays only), or nullptr
  int64_t nlaunch;   // rays the grid covers (n, or the domain's)
  int shift;
  int64_t n;
  double chi_m, chi_m1;  // chi_m, chi_{m+1}
  double c, d;           // c_m, d_m of eq. Atraj
  double* th;
  double* ph;
  double* beta;
  float* A;
  float* Ap;
  int* status;
};

// Pure-SHT planes: g and U (U_tt, U_pp, U_tp) at the ray nv (cos theta ct,
// sin theta st, phi in [0, 2 pi)) from the fields at the pixel centres: the
// four-point HEALPix interpolation of the values transported from each
// pixel centre to the ray (App. B), as for the Jacobians at galaxy images.
__device__ __forceinline__ void pixel_field(const RayArgs& a, const double nv[3], double ct,
                                            double st, double ph, double g[2], double U[3]) {
  int pix[4];
  double wt[4];
  hpx::interp_weights(a.rf, ct, st, ph, pix, wt);
  const int64_t n = a.n;
  g[0] = g[1] = 0.0;
  U[0] = U[1] = U[2] = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int64_t r = pix[q];
    double zq, sq, pq;
    hpx::pix2ang_ring(a.rf.N, r, zq, sq, pq);
    const double nq[3] = {sq * cos(pq), sq * sin(pq), zq};
    double et[3], ep[3], M[4], T[4];
    basis(nq, et, ep);
    transport_matrix(nq, et, ep, nv, M);
    const double g0 = a.D[r], g1 = a.D[n + r];
    const double X[4] = {a.D[2 * n + r], a.D[4 * n + r], a.D[4 * n + r], a.D[3 * n + r]};
    transport_tensor(M, X, T);
    g[0] += wt[q] * (M[0] * g0 + M[1] * g1);
    g[1] += wt[q] * (M[2] * g0 + M[3] * g1);
    U[0] += wt[q] * T[0];
    U[1] += wt[q] * T[3];
    U[2] += wt[q] * T[1];
  }
}

// SHT: the plane is a pure-SHT plane (fields at the pixel centres, a.D);
// else an SHT+MG plane (patches of multigrid precision T).
template <typename T, bool SHT>
__global__ __launch_bounds__(kBlock) void k_ray_update(RayArgs a) {
  // the rays of one bundle (a NESTED range) stay on one XCD
  const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
  if (c >= a.nlaunch) return;
  const int64_t i =
      a.pmap ? (int64_t(a.pmap[c >> a.shift]) << a.shift) | (c & ((int64_t(1) << a.shift) - 1))
             : c;
  const int64_t n = a.n;
  double st, ct, sp, cp;
  sincos(a.th[i], &st, &ct);
  sincos(a.ph[i], &sp, &cp);
  const double nv[3] = {st * cp, st * sp, ct};
  double g[2], U[3];
  if constexpr (SHT) {
    pixel_field(a, nv, ct, st, a.ph[i], g, U);
  } else if (!eval_patch<T>(a.P, i >> a.shift, nv[0], nv[1], nv[2], g, U)) {
    atomicOr(a.status, ST_LEFT_PATCH);
    for (int k = 0; k < 4; ++k) a.A[k * n + i] = NAN;
    return;
  }
  double et[3], ep[3];
  basis(nv, et, ep);
  // eq. betaprop with the deflection d = -grad psi
  double b[3] = {a.beta[i], a.beta[n + i], a.beta[2 * n + i]};
  const double dv[3] = {-(g[0] * et[0] + g[1] * ep[0]), -(g[0] * et[1] + g[1] * ep[1]),
                        -(g[0] * et[2] + g[1] * ep[2])};
  const double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  if (dn > 0) {
    double k[3] = {nv[1] * dv[2] - nv[2] * dv[1], nv[2] * dv[0] - nv[0] * dv[2],
                   nv[0] * dv[1] - nv[1] * dv[0]};
    const double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    k[0] /= kn; k[1] /= kn; k[2] /= kn;
    double out[3];
    rotate(k, dn, b, out);
    b[0] = out[0]; b[1] = out[1]; b[2] = out[2];
  }
  // eq. posprop: |x + lambda beta| = chi_{m+1}, lambda > 0, cancellation-free root
  const double x[3] = {a.chi_m * nv[0], a.chi_m * nv[1], a.chi_m * nv[2]};
  const double bb = x[0] * b[0] + x[1] * b[1] + x[2] * b[2];
  const double q = a.chi_m1 * a.chi_m1 - a.chi_m * a.chi_m;
  const double lam = q / (bb + sqrt(bb * bb + q));
  double xn[3] = {x[0] + lam * b[0], x[1] + lam * b[1], x[2] + lam * b[2]};
  const double xl = sqrt(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2]);
  const double nn[3] = {xn[0] / xl, xn[1] / xl, xn[2] / xl};
  // eq. Atraj: A^(m+1) = (1 - c) A^(m-1) + c A^(m) - d U A^(m)
  double A0[4], Ap0[4];
  for (int k = 0; k < 4; ++k) {
    A0[k] = double(a.A[k * n + i]);
    Ap0[k] = double(a.Ap[k * n + i]);
  }
  const double Um[4] = {U[0], U[2], U[2], U[1]};
  double An[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      const double UA = Um[2 * r] * A0[c] + Um[2 * r + 1] * A0[2 + c];
      An[2 * r + c] = (1.0 - a.c) * Ap0[2 * r + c] + a.c * A0[2 * r + c] - a.d * UA;
    }
  // App. B: rotate the old basis along the great circle n -> n', project on
  // the new basis, A <- M A M^T for both Jacobians
  double M[4];
  transport_matrix(nv, et, ep, nn, M);
  auto transport = [&](const double X[4], float* dst) {
    double Y[4];
    transport_tensor(M, X, Y);
    for (int k = 0; k < 4; ++k) dst[k * n + i] = float(Y[k]);
  };
  transport(A0, a.Ap);
  transport(An, a.A);
  double phn = hpx::atan2_r(nn[1], nn[0]);
  if (phn < 0) phn += kTwoPi;
  a.th[i] = hpx::atan2_r(sqrt(nn[0] * nn[0] + nn[1] * nn[1]), nn[2]);
  a.ph[i] = phn;
  a.beta[i] = b[0];
  a.beta[n + i] = b[1];
  a.beta[2 * n + i] = b[2];
}

__device__ __forceinline__ double r_of(double x, double K) {
  if (K > 0) return sin(sqrt(K) * x) / sqrt(K);
  if (K < 0) return sinh(sqrt(-K) * x) / sqrt(-K);
  return x;
}

struct GalArgs {
  hpx::Rings rf;
  const int* r2n_f;
  int64_t nray;
  const float* A;
  const float* Ap;
  const double* th;
  const double* ph;
  const double* chi;
  float* Ag;
  int64_t ngal;
  double lo, hi;          // shell [lo, hi)
  int k;                  // shell index
  double chi_km1, chi_k;  // chi_{k-1}, chi_k
  double K;
};

// eq. gatraj: A_g = (1 - w) A^(k-1) + w A^(k), w = D_k D_{k-1,g} / (D_g D_{k-1,k}),
// the ray Jacobians taken by HEALPix linear interpolation on the image-plane
// grid at the galaxy position; shell 0 gets the identity.
__global__ void k_galaxies(GalArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.ngal) return;
  const double cg = a.chi[i];
  if (!(cg >= a.lo && cg < a.hi)) return;
  const int64_t ng = a.ngal;
  if (a.k == 0) {
    a.Ag[i] = 1.f; a.Ag[ng + i] = 0.f; a.Ag[2 * ng + i] = 0.f; a.Ag[3 * ng + i] = 1.f;
    return;
  }
  const double w = r_of(a.chi_k, a.K) * r_of(cg - a.chi_km1, a.K) /
                   (r_of(cg, a.K) * r_of(a.chi_k - a.chi_km1, a.K));
  int pix[4];
  double wt[4];
  double s_th, c_th;
  sincos(a.th[i], &s_th, &c_th);
  const double ph = a.ph[i] - kTwoPi * floor(a.ph[i] / kTwoPi);
  hpx::interp_weights(a.rf, c_th, s_th, ph, pix, wt);
  double Ai[4] = {0, 0, 0, 0}, Api[4] = {0, 0, 0, 0};
  for (int q = 0; q < 4; ++q) {
    const int64_t r = a.r2n_f[pix[q]];
    for (int k = 0; k < 4; ++k) {
      Ai[k] += wt[q] * double(a.A[k * a.nray + r]);
      Api[k] += wt[q] * double(a.Ap[k * a.nray + r]);
    }
  }
  for (int k = 0; k < 4; ++k) a.Ag[k * ng + i] = float((1.0 - w) * Api[k] + w * Ai[k]);
}

// ---------------------------------------------------------------- images
// The grid search for galaxy images (Sec. 2.3, Sec. 3.3, App. D).  The
// image-plane triangles join the pixel centres of consecutive rings: the
// two rings' centres merged in azimuth, each merge step adding the
// triangle of the current pair and the next vertex; the four pixels of
// each polar ring close the caps.  A triangle of the band between rings A
// and B that advances on A from vertex j to j + 1 has its apex at the last
// vertex of B before A's vertex j + 1 in azimuth, found in integers from
// the rings' pixel counts and half-pixel shifts.
struct ImgArgs {
  hpx::Rings rf;
  const int* r2n_f;
  int64_t nray;
  const double* rth;      // ray angular positions at chi_k
  const double* rph;
  const double* beta;     // [3][nray]
  const float* A;
  const float* Ap;
  const double* th;       // galaxies
  const double* ph;
  const double* chi;
  float* Ag;
  double* th_img;
  double* ph_img;
  int* found;
  int64_t ngal;
  double lo, hi;          // shell [lo, hi)
  int k;
  double chi_km1, chi_k, K;
  double radius;          // search radius around the predicted image (rad)
};

struct RingGeo {
  int n, first, s;        // pixels, first pixel, half-pixel shift of the azimuths
  double z, st, phi0;
};

__device__ __forceinline__ RingGeo ring_geo(const hpx::Rings& R, int q) {
  RingGeo g;
  g.n = R.ri[2 * q];
  g.first = R.ri[2 * q + 1];
  g.z = R.rt[4 * q];
  g.st = R.rt[4 * q + 1];
  g.phi0 = R.rt[4 * q + 3];
  g.s = g.phi0 != 0.0 ? 1 : 0;
  return g;
}

__device__ __forceinline__ void ring_vec(const RingGeo& g, int j, double v[3]) {
  double sp, cp;
  sincospi(2.0 * (double(j) + 0.5 * g.s) / double(g.n), &sp, &cp);
  v[0] = g.st * cp;
  v[1] = g.st * sp;
  v[2] = g.z;
}

// Last vertex of ring B before vertex jn of ring A in azimuth (cyclic).
__device__ __forceinline__ int pred_vertex(int jn, const RingGeo& a, const RingGeo& b) {
  const int64_t X = (2 * int64_t(jn) + a.s) * b.n - int64_t(b.s) * a.n;
  const int64_t d = 2 * int64_t(a.n);
  int64_t k = X >= 0 ? (X + d - 1) / d - 1 : -((-X) / d) - 1;
  k %= b.n;
  if (k < 0) k += b.n;
  return int(k);
}

// A ray moved along its direction from radius c0 to c1 (the root of
// eq. posprop of least |lambda|), as a unit vector.
__device__ __forceinline__ void ray_at(const ImgArgs& a, int64_t r, double c1, double out[3],
                                       double nr[3]) {
  double st, ct, sp, cp;
  sincos(a.rth[r], &st, &ct);
  sincos(a.rph[r], &sp, &cp);
  nr[0] = st * cp;
  nr[1] = st * sp;
  nr[2] = ct;
  const double b3[3] = {a.beta[r], a.beta[a.nray + r], a.beta[2 * a.nray + r]};
  const double x[3] = {a.chi_k * nr[0], a.chi_k * nr[1], a.chi_k * nr[2]};
  const double bb = x[0] * b3[0] + x[1] * b3[1] + x[2] * b3[2];
  const double q = c1 * c1 - a.chi_k * a.chi_k;
  const double lam = q / (bb + sqrt(bb * bb + q));
  double y[3] = {x[0] + lam * b3[0], x[1] + lam * b3[1], x[2] + lam * b3[2]};
  const double yl = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
  out[0] = y[0] / yl;
  out[1] = y[1] / yl;
  out[2] = y[2] / yl;
}

// Triangle (RING pixels pa, pb, pc with image-plane vectors va, vb, vc):
// true, with the image, when the galaxy g lies in its source triangle
// (barycentric coordinates >= 0 after gnomonic projection about g).
__device__ bool try_triangle(const ImgArgs& a, const double g[3], double cg, const int pix[3],
                             const double (&vimg)[3][3], double img[3]) {
  double P[3][3];
  for (int i = 0; i < 3; ++i) {
    double sv[3], nr[3];
    ray_at(a, a.r2n_f[pix[i]], cg, sv, nr);
    const double dg = sv[0] * g[0] + sv[1] * g[1] + sv[2] * g[2];
    if (!(dg > 0.0)) return false;
    for (int c = 0; c < 3; ++c) P[i][c] = sv[c] / dg - g[c];
  }
  double e1[3], e2[3], r[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = P[1][c] - P[0][c];
    e2[c] = P[2][c] - P[0][c];
    r[c] = -P[0][c];
  }
  const double m00 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
  const double m01 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
  const double m11 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
  const double r0 = r[0] * e1[0] + r[1] * e1[1] + r[2] * e1[2];
  const double r1 = r[0] * e2[0] + r[1] * e2[1] + r[2] * e2[2];
  const double det = m00 * m11 - m01 * m01;
  if (!(det > 0.0)) return false;
  const double b1 = (r0 * m11 - r1 * m01) / det;
  const double b2 = (m00 * r1 - m01 * r0) / det;
  const double b0 = 1.0 - b1 - b2;
  if (!(b0 >= 0.0 && b1 >= 0.0 && b2 >= 0.0)) return false;
  const double b[3] = {b0, b1, b2};
  double s3[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const double d = vimg[i][0] * g[0] + vimg[i][1] * g[1] + vimg[i][2] * g[2];
    for (int c = 0; c < 3; ++c) s3[c] += b[i] * vimg[i][c] / d;
  }
  const double l = sqrt(s3[0] * s3[0] + s3[1] * s3[1] + s3[2] * s3[2]);
  for (int c = 0; c < 3; ++c) img[c] = s3[c] / l;
  return true;
}

// The triangles of the bands whose rings lie within `radius` of the unit
// vector c, in azimuth windows around c, nearest first (the central band,
// then the neighbours on both sides; in a band the nearest vertices
// first); stops at the first triangle whose source triangle holds g.
__device__ bool search_images(const ImgArgs& a, const double g[3], double cg, const double c[3],
                              double radius, double img[3]) {
  const hpx::Rings& R = a.rf;
  const int N = R.N, nring = R.nring;
  const double pi = 3.14159265358979323846;
  const double zc = c[2], rc = sqrt(c[0] * c[0] + c[1] * c[1]);
  double phc = hpx::atan2_r(c[1], c[0]);
  if (phc < 0) phc += 2.0 * pi;
  const hpx::GlobalRingTab tab{R, 0.0};
  const int gc = hpx::ring_above(tab, zc);
  // ring spacing is at most about 1.2 / N in colatitude
  const int W = int(radius * N * 1.25) + 1;
  const double dphi = radius / fmax(rc, 1e-300) + pi / (2.0 * N);
  for (int dq = 0; dq <= 2 * W; ++dq) {
    const int q = gc + ((dq & 1) ? -(dq + 1) / 2 : dq / 2);
    if (q < -1 || q > nring - 1) continue;
    if (q == -1 || q == nring - 1) {
      const RingGeo cap = ring_geo(R, q == -1 ? 0 : nring - 1);
      double v[4][3];
      for (int j = 0; j < 4; ++j) ring_vec(cap, j, v[j]);
      const int order[2][3] = {{0, 1, 2}, {0, 2, 3}};
      for (int t = 0; t < 2; ++t) {
        int pix[3];
        double vi[3][3];
        for (int i = 0; i < 3; ++i) {
          // the vertex order does not change the test
          const int j = order[t][i];
          pix[i] = cap.first + j;
          for (int cc = 0; cc < 3; ++cc) vi[i][cc] = v[j][cc];
        }
        if (try_triangle(a, g, cg, pix, vi, img)) return true;
      }
      continue;
    }
    const RingGeo A = ring_geo(R, q), B = ring_geo(R, q + 1);
    // vertices j of each ring around the azimuth of c, nearest first
    // (the window is capped at a full ring: near the poles dphi is large)
    const int ha = int(fmin(dphi * A.n / (2.0 * pi), double(A.n))) + 1;
    const int hb = int(fmin(dphi * B.n / (2.0 * pi), double(B.n))) + 1;
    const int na = 2 * ha + 1 >= A.n ? A.n : 2 * ha + 1;
    const int nb = 2 * hb + 1 >= B.n ? B.n : 2 * hb + 1;
    const int ja = int(floor(phc * A.n / (2.0 * pi) - 0.5 * A.s));
    const int jb = int(floor(phc * B.n / (2.0 * pi) - 0.5 * B.s));
    for (int t = 0; t < na + nb; ++t) {
      const bool sa = t < na;
      const RingGeo& P = sa ? A : B;
      const RingGeo& Q = sa ? B : A;
      const int o = sa ? t : t - na;
      int j = (sa ? ja : jb) + ((o & 1) ? -(o + 1) / 2 : o / 2);
      j %= P.n;
      if (j < 0) j += P.n;
      const int jn = j + 1 == P.n ? 0 : j + 1;
      const int kq = pred_vertex(jn, P, Q);
      int pix[3] = {P.first + j, Q.first + kq, P.first + jn};
      double vi[3][3];
      ring_vec(P, j, vi[0]);
      ring_vec(Q, kq, vi[1]);
      ring_vec(P, jn, vi[2]);
      if (try_triangle(a, g, cg, pix, vi, img)) return true;
    }
  }
  return false;
}

// Four-point interpolation at the image of the ray Jacobians, each
// transported from its ray's position to the image (App. B), and eq. gatraj.
__device__ void image_jacobian(const ImgArgs& a, const double img[3], double w, double Ag[4]) {
  const double pi = 3.14159265358979323846;
  const double rho = sqrt(img[0] * img[0] + img[1] * img[1]);
  double ph = hpx::atan2_r(img[1], img[0]);
  if (ph < 0) ph += 2.0 * pi;
  int pix[4];
  double wt[4];
  hpx::interp_weights(a.rf, img[2], rho, ph, pix, wt);
  double S[4] = {0, 0, 0, 0}, Sp[4] = {0, 0, 0, 0};
  for (int q = 0; q < 4; ++q) {
    const int64_t r = a.r2n_f[pix[q]];
    double st, ct, sp, cp;
    sincos(a.rth[r], &st, &ct);
    sincos(a.rph[r], &sp, &cp);
    const double nv[3] = {st * cp, st * sp, ct};
    double et[3], ep[3], M[4];
    basis(nv, et, ep);
    transport_matrix(nv, et, ep, img, M);
    auto add = [&](const float* src, double acc[4]) {
      const double X[4] = {double(src[r]), double(src[a.nray + r]), double(src[2 * a.nray + r]),
                           double(src[3 * a.nray + r])};
      double T[4];
      transport_tensor(M, X, T);
      for (int c = 0; c < 4; ++c) acc[c] += wt[q] * T[c];
    };
    add(a.A, S);
    add(a.Ap, Sp);
  }
  for (int c = 0; c < 4; ++c) Ag[c] = (1.0 - w) * Sp[c] + w * S[c];
}

// One galaxy per thread: the image search around a predicted image (the
// galaxy moved by the offset between its pixel's image and source
// positions), then once more around the galaxy itself with twice the
// radius; galaxies not found get NaN and found = 0.
__global__ __launch_bounds__(kBlock) void k_galaxy_images(ImgArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.ngal) return;
  const double cg = a.chi[i];
  if (!(cg >= a.lo && cg < a.hi)) return;
  const int64_t ng = a.ngal;
  if (a.k == 0) {
    a.th_img[i] = a.th[i];
    a.ph_img[i] = a.ph[i];
    a.found[i] = 1;
    a.Ag[i] = 1.f; a.Ag[ng + i] = 0.f; a.Ag[2 * ng + i] = 0.f; a.Ag[3 * ng + i] = 1.f;
    return;
  }
  double st, ct, sp, cp;
  sincos(a.th[i], &st, &ct);
  sincos(a.ph[i], &sp, &cp);
  const double g[3] = {st * cp, st * sp, ct};
  // predicted image: g plus the image - source offset of the pixel at g
  const double pi = 3.14159265358979323846;
  double ph = a.ph[i] - 2.0 * pi * floor(a.ph[i] / (2.0 * pi));
  int pix4[4];
  double w4[4];
  hpx::interp_weights(a.rf, ct, st, ph, pix4, w4);
  int best = 0;
  for (int q = 1; q < 4; ++q)
    if (w4[q] > w4[best]) best = q;
  double z0, s0, p0;
  hpx::pix2ang_ring(a.rf.N, pix4[best], z0, s0, p0);
  const double v0[3] = {s0 * cos(p0), s0 * sin(p0), z0};
  double src0[3], nr0[3];
  ray_at(a, a.r2n_f[pix4[best]], cg, src0, nr0);
  double c[3] = {g[0] + v0[0] - src0[0], g[1] + v0[1] - src0[1], g[2] + v0[2] - src0[2]};
  const double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  c[0] /= cl; c[1] /= cl; c[2] /= cl;
  double img[3];
  bool ok = search_images(a, g, cg, c, a.radius, img);
  if (!ok) ok = search_images(a, g, cg, g, 2.0 * a.radius, img);
  if (!ok) {
    a.th_img[i] = NAN;
    a.ph_img[i] = NAN;
    a.found[i] = 0;
    for (int q = 0; q < 4; ++q) a.Ag[q * ng + i] = NAN;
    return;
  }
  const double w = r_of(a.chi_k, a.K) * r_of(cg - a.chi_km1, a.K) /
                   (r_of(cg, a.K) * r_of(a.chi_k - a.chi_km1, a.K));
  double Ag[4];
  image_jacobian(a, img, w, Ag);
  for (int q = 0; q < 4; ++q) a.Ag[q * ng + i] = float(Ag[q]);
  double phi = hpx::atan2_r(img[1], img[0]);
  if (phi < 0) phi += 2.0 * pi;
  a.th_img[i] = hpx::atan2_r(sqrt(img[0] * img[0] + img[1] * img[1]), img[2]);
  a.ph_img[i] = phi;
  a.found[i] = 1;
}

// ------------------------------------------------------ final-plane fields
// Sec. 5: kappa, gamma_1, gamma_2, omega of eq. invmagmat on the ray grid.
// Ray p (NESTED pixel p of the image plane) gives the value at its pixel
// centre; its Jacobian, held in the basis at the ray's position, is
// transported there first (App. B).  Output: RING-order maps [4][n].
__global__ __launch_bounds__(kBlock) void k_jacobian_fields(int64_t N, int64_t n,
                                                            const double* th, const double* ph,
                                                            const float* A, double* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t r = hpx::nest2ring(N, p);
  double z, st1, phi;
  hpx::pix2ang_ring(N, r, z, st1, phi);
  const double n1[3] = {st1 * cos(phi), st1 * sin(phi), z};
  double st, ct, sp, cp;
  sincos(th[p], &st, &ct);
  sincos(ph[p], &sp, &cp);
  const double n0[3] = {st * cp, st * sp, ct};
  double et[3], ep[3], M[4], T[4];
  basis(n0, et, ep);
  transport_matrix(n0, et, ep, n1, M);
  const double X[4] = {double(A[p]), double(A[n + p]), double(A[2 * n + p]),
                       double(A[3 * n + p])};
  transport_tensor(M, X, T);
  out[r] = 1.0 - 0.5 * (T[0] + T[3]);
  out[n + r] = 0.5 * (T[3] - T[0]);
  out[2 * n + r] = -0.5 * (T[1] + T[2]);
  out[3 * n + r] = 0.5 * (T[1] - T[2]);
}

}  // namespace

clm_status jacobian_fields(Plan* p, const clm_rays* r, double* out, hipStream_t s) {
  const int64_t n = r->n;
  CLM_TIMED(p, s, "jacobian_fields");
  hipLaunchKernelGGL(k_jacobian_fields, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, int64_t(p->d.nside_sht), n, r->theta, r->phi, r->A, out);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status galaxy_images(Plan* p, const double* chi, int nchi, int k, double K,
                         const clm_rays* r, const clm_galaxies* gl, double radius,
                         double* th_img, double* ph_img, int* found, hipStream_t s) {
  const int N = nchi - 1;
  auto edge = [&](int e) { return e == 0 ? 0.0 : 0.5 * (chi[e - 1] + chi[e]); };
  ImgArgs a;
  a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, p->d.nside_fine};
  a.r2n_f = p->r2n_f;
  a.nray = r->n;
  a.rth = r->theta;
  a.rph = r->phi;
  a.beta = r->beta;
  a.A = r->A;
  a.Ap = r->A_prev;
  a.th = gl->theta;
  a.ph = gl->phi;
  a.chi = gl->chi;
  a.Ag = gl->A;
  a.th_img = th_img;
  a.ph_img = ph_img;
  a.found = found;
  a.ngal = gl->n;
  a.k = k;
  a.lo = edge(k);
  a.hi = k < N ? edge(k + 1) : INFINITY;
  a.chi_km1 = k >= 1 ? chi[k - 1] : 0.0;
  a.chi_k = k <= N ? chi[k] : 0.0;
  a.K = K;
  a.radius = radius > 0 ? radius : 2.0 * std::sqrt(4.0 * 3.14159265358979323846 /
                                                   double(p->npix_f));
  CLM_TIMED(p, s, "galaxy_images");
  hipLaunchKernelGGL(k_galaxy_images, dim3((gl->n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status rays_init(Plan* p, const clm_rays* r, hipStream_t s) {
  hipLaunchKernelGGL(k_rays_init, dim3((r->n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     int64_t(p->d.nside_fine), r->n, r->theta, r->phi, r->beta, r->A, r->A_prev);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

static double r_host(double x, double K) {
  if (K > 0) return std::sin(std::sqrt(K) * x) / std::sqrt(K);
  if (K < 0) return std::sinh(std::sqrt(-K) * x) / std::sqrt(-K);
  return x;
}

clm_status ray_update(Plan* p, int slot, const double* chi, int nchi, int m, double K,
                      const clm_rays* r, hipStream_t s) {
  (void)nchi;
  RayArgs a{};
  if (p->mg) {
    a.P = PatchField{p->rot, p->slots[slot].u0, p->slots[slot].du, p->n, p->L, p->delta};
    a.shift = p->bundle_shift;
  } else {
    // the plane's fields at the pixel centres are in p->deriv
    a.D = p->deriv;
    a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, p->d.nside_fine};
  }
  a.n = r->n;
  a.nlaunch = r->n;
  if (p->mg && p->domain) {
    a.pmap = p->dom_map;
    a.nlaunch = p->nactive << p->bundle_shift;
  }
  a.chi_m = chi[m];
  a.chi_m1 = chi[m + 1];
  // eq. Atraj with chi_{-1} = 0: c_m = D_m/D_{m+1} * D_{m-1,m+1}/D_{m-1,m},
  // d_m = D_{m,m+1}/D_{m+1}
  const double cm1 = m == 0 ? 0.0 : chi[m - 1];
  a.c = (r_host(chi[m], K) / r_host(chi[m + 1], K)) *
        (r_host(chi[m + 1] - cm1, K) / r_host(chi[m] - cm1, K));
  a.d = r_host(chi[m + 1] - chi[m], K) / r_host(chi[m + 1], K);
  a.th = r->theta;
  a.ph = r->phi;
  a.beta = r->beta;
  a.A = r->A;
  a.Ap = r->A_prev;
  a.status = p->status_dev;
  const dim3 g(unsigned((a.nlaunch + kBlock - 1) / kBlock));
  CLM_TIMED(p, s, "ray_update");
  if (!p->mg)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ray_update<double, true>), g, dim3(kBlock), 0, s, a);
  else if (p->fp64mg)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ray_update<double, false>), g, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ray_update<float, false>), g, dim3(kBlock), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status galaxies_shell(Plan* p, const double* chi, int nchi, int k, double K,
                          const clm_rays* r, const clm_galaxies* gl, hipStream_t s) {
  // shell edges: 0, midpoints between consecutive planes, and above the
  // last plane everything (chi_0 .. chi_{N-1} planes, chi_N the target)
  const int N = nchi - 1;
  auto edge = [&](int e) { return e == 0 ? 0.0 : 0.5 * (chi[e - 1] + chi[e]); };
  GalArgs a;
  a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, p->d.nside_fine};
  a.r2n_f = p->r2n_f;
  a.nray = r->n;
  a.A = r->A;
  a.Ap = r->A_prev;
  a.th = gl->theta;
  a.ph = gl->phi;
  a.chi = gl->chi;
  a.Ag = gl->A;
  a.ngal = gl->n;
  a.k = k;
  a.lo = edge(k);
  a.hi = k < N ? edge(k + 1) : INFINITY;
  a.chi_km1 = k >= 1 ? chi[k - 1] : 0.0;
  a.chi_k = k <= N ? chi[k] : 0.0;
  a.K = K;
  CLM_TIMED(p, s, "galaxies");
  hipLaunchKernelGGL(k_galaxies, dim3((gl->n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace clm
