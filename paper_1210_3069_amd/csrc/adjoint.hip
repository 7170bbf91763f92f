// Transpose of the kappa -> (gradient, covariant Hessian at points) map of
// the SHT+MG solve, for gradients of losses such as the shear chi^2.
//
// With the geometry, the readings and the number of V-cycles fixed the map
// is linear in kappa (the SHT boundary data are linear in kappa too), so its
// transpose needs no state of the forward solve.  The steps of Sec. 3.2 are
// transposed in reverse order:
//   evaluation at points (bilinear weights, 4th-order stencils, App. A
//   metric terms, rotation)                    -> k_adj_eval (scatter)
//   u = u0 + du, du ghosts = -interior          -> k_adj_split
//   fixed V-cycles from du = 0                  -> mg_transpose (per level)
//   f' = 2 interp(kappa') - L u0, u0 from psi_SHT (cells, face ghosts)
//                                               -> k_adj_setup_cells / _ghosts
//   analysis, Poisson factor, synthesis         -> sht_adjoint (sht.hip)
//   degrade to the SHT grid, demean             -> k_adj_degrade, k_sub_mean
// Everything runs in FP64 on plain per-level arrays (no temporal blocking).
#include <cmath>

#include "clm_internal.h"
#include "eval_dev.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlk = 256;
constexpr double kPi = 3.14159265358979323846;

inline dim3 grid_for(int64_t n) { return dim3(unsigned((n + kBlk - 1) / kBlk)); }

// Row coefficients of a level: s_m, s_p, s_c, area per row.
struct Rows {
  const double* c;
  int n;
  __device__ double sm(int i) const { return c[4 * i]; }
  __device__ double sp(int i) const { return c[4 * i + 1]; }
  __device__ double isc(int i) const { return 1.0 / c[4 * i + 2]; }
  __device__ double A(int i) const { return c[4 * i + 3]; }
  // full diagonal: a neighbour across the patch face is the ghost -u
  __device__ double D(int i, int j) const {
    double d = sm(i) + sp(i) + 2.0 * isc(i);
    if (i == 0) d += sm(i);
    if (i == n - 1) d += sp(i);
    if (j == 0) d += isc(i);
    if (j == n - 1) d += isc(i);
    return d;
  }
};

// -------------------------------------------------------- evaluation^T
struct EvalTArgs {
  const double* rot;
  double* ubar;       // [nbundle][(n+2)^2]
  const double* th;
  const double* ph;
  const double* gbar; // [2][npts]
  const double* hbar; // [3][npts]: U_tt, U_pp, U_tp
  int64_t npts, Nb;
  int n;
  double L, delta;
  int* status;
};

// The raw-partial adjoints pbar at cell (i, j) scattered through the
// stencils of eval_patch into the (n+2)^2 field (ghost ring at -1 and n).
__device__ void partials_T(double* ub, int n, int i, int j, double h, const double pb[5]) {
  const Stencil a1 = d1_stencil(i, n), b1 = d1_stencil(j, n);
  const Stencil a2 = d2_stencil(i, n), b2 = d2_stencil(j, n);
  const int G = n + 2;
  auto at = [&](int r, int c) -> double* { return ub + (r + 1) * G + (c + 1); };
  for (int k = 0; k < a1.len; ++k)
    atomicAdd(at(i + a1.first + k, j), a1.w[k] * pb[0] / (12 * h));
  for (int k = 0; k < b1.len; ++k)
    atomicAdd(at(i, j + b1.first + k), b1.w[k] * pb[1] / (12 * h));
  for (int k = 0; k < a2.len; ++k)
    atomicAdd(at(i + a2.first + k, j), a2.w[k] * pb[2] / (12 * h * h));
  for (int k = 0; k < b2.len; ++k)
    atomicAdd(at(i, j + b2.first + k), b2.w[k] * pb[3] / (12 * h * h));
  for (int k = 0; k < a1.len; ++k) {
    if (a1.w[k] == 0) continue;
    for (int q = 0; q < b1.len; ++q)
      atomicAdd(at(i + a1.first + k, j + b1.first + q),
                a1.w[k] * b1.w[q] * pb[4] / (144 * h * h));
  }
}

__global__ __launch_bounds__(kBlk) void k_adj_eval(EvalTArgs a) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.npts) return;
  double st0, ct0, sp0, cp0;
  sincos(a.th[k], &st0, &ct0);
  sincos(a.ph[k], &sp0, &cp0);
  const double vx = st0 * cp0, vy = st0 * sp0, vz = ct0;
  const int64_t b = hpx::ang2nest(a.Nb, ct0, a.ph[k]);
  const double* R = a.rot + 9 * b;
  const double px = R[0] * vx + R[1] * vy + R[2] * vz;
  const double py = R[3] * vx + R[4] * vy + R[5] * vz;
  const double pz = R[6] * vx + R[7] * vy + R[8] * vz;
  const double st = sqrt(px * px + py * py), ct = pz;
  const double thp = atan2(st, pz), php = atan2(py, px);
  const int n = a.n;
  const double h = a.delta;
  const double fi = (thp - (kPi / 2 - a.L / 2)) / h - 0.5;
  const double fj = (php + a.L / 2) / h - 0.5;
  const double ffi = floor(fi), ffj = floor(fj);
  if (!(ffi >= 0 && ffi <= n - 2 && ffj >= 0 && ffj <= n - 2)) {
    atomicOr(a.status, ST_LEFT_PATCH);
    return;
  }
  const int i0 = int(ffi), j0 = int(ffj);
  const double t = fi - ffi, s = fj - ffj;
  // Q: global (theta-hat, phi-hat) against the patch basis at the point
  const double cpp = px / st, spp = py / st;
  const double et_p[3] = {ct * cpp, ct * spp, -st};
  const double ep_p[3] = {-spp, cpp, 0.0};
  double etp[3], epp[3];
  for (int q = 0; q < 3; ++q) {
    etp[q] = R[q] * et_p[0] + R[3 + q] * et_p[1] + R[6 + q] * et_p[2];
    epp[q] = R[q] * ep_p[0] + R[3 + q] * ep_p[1] + R[6 + q] * ep_p[2];
  }
  const double sg = sqrt(vx * vx + vy * vy);
  const double cph = vx / sg, sph = vy / sg;
  const double et[3] = {vz * cph, vz * sph, -sg};
  const double ep[3] = {-sph, cph, 0.0};
  const double q00 = et[0] * etp[0] + et[1] * etp[1] + et[2] * etp[2];
  const double q01 = et[0] * epp[0] + et[1] * epp[1] + et[2] * epp[2];
  const double q10 = ep[0] * etp[0] + ep[1] * etp[1] + ep[2] * etp[2];
  const double q11 = ep[0] * epp[0] + ep[1] * epp[1] + ep[2] * epp[2];
  // g = Q g', U = Q U' Q^T: g'bar = Q^T gbar, U'bar = Q^T Ubar Q with Ubar
  // symmetric (U_tp bar split over both off-diagonal entries)
  const double gb0 = a.gbar[k], gb1 = a.gbar[a.npts + k];
  const double u00 = a.hbar[k], u11 = a.hbar[a.npts + k], u01 = 0.5 * a.hbar[2 * a.npts + k];
  const double gpt = q00 * gb0 + q10 * gb1, gpp = q01 * gb0 + q11 * gb1;
  // M = Ubar Q, then Q^T M
  const double m00 = u00 * q00 + u01 * q10, m01 = u00 * q01 + u01 * q11;
  const double m10 = u01 * q00 + u11 * q10, m11 = u01 * q01 + u11 * q11;
  const double U00 = q00 * m00 + q10 * m10, U01 = q00 * m01 + q10 * m11;
  const double U10 = q01 * m00 + q11 * m10, U11 = q01 * m01 + q11 * m11;
  const double off = U01 + U10;
  double pb[5];
  pb[0] = gpt + (ct / st) * U11;
  pb[1] = gpp / st - ct / (st * st) * off;
  pb[2] = U00;
  pb[3] = U11 / (st * st);
  pb[4] = off / st;
  double* ub = a.ubar + size_t(b) * (n + 2) * (n + 2);
  const double w[4] = {(1 - t) * (1 - s), (1 - t) * s, t * (1 - s), t * s};
  for (int c = 0; c < 4; ++c) {
    double q[5];
    for (int e = 0; e < 5; ++e) q[e] = w[c] * pb[e];
    partials_T(ub, n, i0 + (c >> 1), j0 + (c & 1), h, q);
  }
}

// du-bar on the interior: the field bar plus minus each ghost it reflects.
__global__ void k_adj_split(const double* ubar, int n, int64_t np, double* dub) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * n * n) return;
  const int64_t b = t / (int64_t(n) * n);
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const int G = n + 2;
  const double* u = ubar + size_t(b) * G * G;
  auto at = [&](int r, int q) { return u[(r + 1) * G + (q + 1)]; };
  double v = at(i, j);
  if (i == 0) v -= at(-1, j);
  if (i == n - 1) v -= at(n, j);
  if (j == 0) v -= at(i, -1);
  if (j == n - 1) v -= at(i, n);
  if (i == 0 && j == 0) v -= at(-1, -1);
  if (i == 0 && j == n - 1) v -= at(-1, n);
  if (i == n - 1 && j == 0) v -= at(n, -1);
  if (i == n - 1 && j == n - 1) v -= at(n, n);
  dub[t] = v;
}

// -------------------------------------------------------- multigrid^T
// Transposed red-black half sweep of colour col on a level:
//   out = in with colour-col cells zeroed, plus for every other cell the
//   coefficients its colour-col neighbours give it times in/D there;
//   fbar -= A in / D on colour-col cells.
__global__ void k_hs_T(Rows r, int64_t np, int col, const double* in, double* out,
                       double* fbar) {
  const int n = r.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * n * n) return;
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const double* x = in + (t - c);
  if (((i + j) & 1) == col) {
    out[t] = 0.0;
    fbar[t] -= r.A(i) * x[c] / r.D(i, j);
    return;
  }
  double v = x[c];
  if (i > 0) v += r.sp(i - 1) * x[c - n] / r.D(i - 1, j);
  if (i < n - 1) v += r.sm(i + 1) * x[c + n] / r.D(i + 1, j);
  if (j > 0) v += r.isc(i) * x[c - 1] / r.D(i, j - 1);
  if (j < n - 1) v += r.isc(i) * x[c + 1] / r.D(i, j + 1);
  out[t] = v;
}

// y += s L0^T x (L0: the level operator on a correction with zero face
// values, rows scaled by 1 / area).
__global__ void k_L0_T(Rows r, int64_t np, const double* xin, double s, double* y) {
  const int n = r.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * n * n) return;
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const double* x = xin + (t - c);
  double v = -r.D(i, j) * x[c] / r.A(i);
  if (i > 0) v += r.sp(i - 1) * x[c - n] / r.A(i - 1);
  if (i < n - 1) v += r.sm(i + 1) * x[c + n] / r.A(i + 1);
  if (j > 0) v += r.isc(i) * x[c - 1] / r.A(i);
  if (j < n - 1) v += r.isc(i) * x[c + 1] / r.A(i);
  y[t] += s * v;
}

// x_fine += s R^T y_coarse (area-weighted restriction).
__global__ void k_restrict_T(Rows rf, int64_t np, const double* yc, double s, double* xf) {
  const int n = rf.n, nc = n / 2;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * n * n) return;
  const int64_t b = t / (int64_t(n) * n);
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const int I = i >> 1, J = j >> 1;
  const double a0 = rf.A(2 * I), a1 = rf.A(2 * I + 1);
  xf[t] += s * rf.A(i) / (2.0 * (a0 + a1)) * yc[size_t(b) * nc * nc + I * nc + J];
}

// e_coarse = P^T x_fine (bilinear 9/3/3/1, direct injection on the
// outermost fine ring); gather over the 4 x 4 fine window of a coarse cell.
__global__ void k_prolong_T(int n, int64_t np, const double* xf, double* ec) {
  const int nc = n / 2;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * nc * nc) return;
  const int64_t b = t / (int64_t(nc) * nc);
  const int c = int(t % (int64_t(nc) * nc)), I = c / nc, J = c % nc;
  const double* x = xf + size_t(b) * n * n;
  double v = 0.0;
  for (int r = 2 * I - 1; r <= 2 * I + 2; ++r) {
    if (r < 0 || r >= n) continue;
    const double wr = (r >> 1) == I ? 0.75 : 0.25;
    for (int q = 2 * J - 1; q <= 2 * J + 2; ++q) {
      if (q < 0 || q >= n) continue;
      const bool ring = r == 0 || r == n - 1 || q == 0 || q == n - 1;
      const bool own = (r >> 1) == I && (q >> 1) == J;
      if (ring) {
        if (own) v += x[r * n + q];
      } else {
        v += wr * ((q >> 1) == J ? 0.75 : 0.25) * x[r * n + q];
      }
    }
  }
  ec[t] = v;
}

// fbar = Cinv^T ubar on the coarsest 4 x 4 level.
__global__ void k_coarsest_T(const double* cinv, int64_t np, const double* ub, double* fb) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * 16) return;
  const int64_t b = t / 16;
  const int k = int(t % 16);
  double v = 0.0;
  for (int q = 0; q < 16; ++q) v += cinv[q * 16 + k] * ub[b * 16 + q];
  fb[t] = v;
}

__global__ void k_axpy(int64_t n, double s, const double* x, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] += s * x[t];
}

__global__ void k_fill(int64_t n, double v, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = v;
}

// -------------------------------------------------------- setup^T
struct SetupTArgs {
  const double* rot;
  const double* ubar;   // [np][(n+2)^2]: u0 bar as accumulated
  const double* fpb;    // [np][n^2]: f' bar
  Rows r;
  int64_t np;
  double L, delta;
  hpx::Rings rs, rf;
  double* psibar;       // SHT RING maps: ncopy private copies of npix_s each
  int64_t npix_s;
  int ncopy;
  double* kbar;         // fine RING map
};

__device__ void patch_point(const double* R, double thp, double php, double& z, double& rho,
                            double& ph) {
  double st, ct, sp, cp;
  sincos(thp, &st, &ct);
  sincos(php, &sp, &cp);
  const double x = st * cp, y = st * sp;
  const double vx = R[0] * x + R[3] * y + R[6] * ct;
  const double vy = R[1] * x + R[4] * y + R[7] * ct;
  z = R[2] * x + R[5] * y + R[8] * ct;
  rho = sqrt(vx * vx + vy * vy);
  ph = atan2(vy, vx);
  if (ph < 0) ph += 2.0 * kPi;
}

__device__ void scatter(const hpx::Rings& R, double* map, double z, double rho, double ph,
                        double v) {
  int pix[4];
  double w[4];
  hpx::interp_weights(R, z, rho, ph, pix, w);
  for (int c = 0; c < 4; ++c) atomicAdd(map + pix[c], w[c] * v);
}

// u0 bar at (i, j) in [-1, n]^2 after f' = f - L u0 (L reads the stored
// ghost ring of u0).
__device__ double u0bar_at(const SetupTArgs& a, const double* ub, const double* fb, int i,
                           int j) {
  const int n = a.r.n, G = n + 2;
  double v = ub[(i + 1) * G + (j + 1)];
  auto f = [&](int r, int q) { return fb[r * n + q] / a.r.A(r); };
  if (i >= 0 && i < n && j >= 0 && j < n) v += (a.r.sm(i) + a.r.sp(i) + 2.0 * a.r.isc(i)) * f(i, j);
  // cells whose stencil reads (i, j), with minus sign of -L
  if (i + 1 >= 0 && i + 1 < n && j >= 0 && j < n) v -= a.r.sm(i + 1) * f(i + 1, j);
  if (i - 1 >= 0 && i - 1 < n && j >= 0 && j < n) v -= a.r.sp(i - 1) * f(i - 1, j);
  if (i >= 0 && i < n && j + 1 >= 0 && j + 1 < n) v -= a.r.isc(i) * f(i, j + 1);
  if (i >= 0 && i < n && j - 1 >= 0 && j - 1 < n) v -= a.r.isc(i) * f(i, j - 1);
  return v;
}

// Interior cells: u0 = interp(psi) and the ghosts' -u0(adjacent) folded in;
// f = 2 interp(kappa') with f bar = f' bar.
__global__ void k_adj_setup_cells(SetupTArgs a) {
  const int n = a.r.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.np * n * n) return;
  const int64_t b = t / (int64_t(n) * n);
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const int G = n + 2;
  const double* ub = a.ubar + size_t(b) * G * G;
  const double* fb = a.fpb + size_t(b) * n * n;
  double v = u0bar_at(a, ub, fb, i, j);
  if (i == 0) v -= u0bar_at(a, ub, fb, -1, j);
  if (i == n - 1) v -= u0bar_at(a, ub, fb, n, j);
  if (j == 0) v -= u0bar_at(a, ub, fb, i, -1);
  if (j == n - 1) v -= u0bar_at(a, ub, fb, i, n);
  if (i == 0 && j == 0) v -= u0bar_at(a, ub, fb, -1, -1);
  if (i == 0 && j == n - 1) v -= u0bar_at(a, ub, fb, -1, n);
  if (i == n - 1 && j == 0) v -= u0bar_at(a, ub, fb, n, -1);
  if (i == n - 1 && j == n - 1) v -= u0bar_at(a, ub, fb, n, n);
  const double* R = a.rot + 9 * b;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  double z, rho, ph;
  patch_point(R, th0 + (i + 0.5) * a.delta, ph0 + (j + 0.5) * a.delta, z, rho, ph);
  // each block adds into its own copy of the small SHT-grid map: millions of
  // cells map to each SHT pixel, and one shared map serialises the atomics
  scatter(a.rs, a.psibar + (blockIdx.x % a.ncopy) * a.npix_s, z, rho, ph, v);
  scatter(a.rf, a.kbar, z, rho, ph, 2.0 * fb[c]);
}

// out[p] = sum of the ncopy private copies at p.
__global__ void k_sum_copies(int ncopy, int64_t n, const double* in, double* out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double v = 0.0;
  for (int k = 0; k < ncopy; ++k) v += in[k * n + t];
  out[t] = v;
}

// Ghost cells: u0_g = 2 b - u0(adjacent), b = interp(psi) on the face
// midpoint (corner ghosts: the patch corner).
__global__ void k_adj_setup_ghosts(SetupTArgs a) {
  const int n = a.r.n, G = n + 2;
  const int per = 4 * n + 4;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.np * per) return;
  const int64_t b = t / per;
  const int k = int(t % per);
  int gi, gj;
  if (k < n) { gi = -1; gj = k; }
  else if (k < 2 * n) { gi = n; gj = k - n; }
  else if (k < 3 * n) { gi = k - 2 * n; gj = -1; }
  else if (k < 4 * n) { gi = k - 3 * n; gj = n; }
  else { const int q = k - 4 * n; gi = (q & 2) ? n : -1; gj = (q & 1) ? n : -1; }
  const double* ub = a.ubar + size_t(b) * G * G;
  const double* fb = a.fpb + size_t(b) * n * n;
  const double v = u0bar_at(a, ub, fb, gi, gj);
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  const double thp = gi < 0 ? th0 : gi == n ? th0 + a.L : th0 + (gi + 0.5) * a.delta;
  const double php = gj < 0 ? ph0 : gj == n ? ph0 + a.L : ph0 + (gj + 0.5) * a.delta;
  double z, rho, ph;
  patch_point(a.rot + 9 * b, thp, php, z, rho, ph);
  scatter(a.rs, a.psibar + (blockIdx.x % a.ncopy) * a.npix_s, z, rho, ph, 2.0 * v);
}

// -------------------------------------------------------- degrade^T, demean^T
// fine kappa' bar += SHT-grid bar of the parent / (children per parent).
__global__ void k_adj_degrade(const double* ks, int64_t npix_f, const int* r2n_f, int shift,
                              int64_t Ns, double inv_k, double* kb) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npix_f) return;
  const int64_t parent = int64_t(r2n_f[p]) >> shift;
  kb[p] += ks[hpx::nest2ring(Ns, parent)] * inv_k;
}

__global__ void k_sub_mean(int64_t n, const double* red, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] -= red[1023];
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

Rows rows(Plan* p, int l) { return Rows{p->coef + p->lev[l].crow, p->n >> l}; }

// Transpose of one V-cycle on level l: ubar_out in adj_u[l] -> ubar_in in
// adj_u[l], fbar added to adj_f[l] (the caller zeroes it).
clm_status vcycle_T(Plan* p, int l, hipStream_t s) {
  const int n = p->n >> l;
  const int64_t np = p->nbundle, cells = np * n * n;
  double* u = p->adj_u[l];
  double* v = p->adj_v[l];
  double* f = p->adj_f[l];
  const Rows r = rows(p, l);
  if (n <= 4) {
    hipLaunchKernelGGL(k_coarsest_T, grid_for(np * 16), dim3(kBlk), 0, s, p->cinv, np, u, f);
    CLM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill, grid_for(cells), dim3(kBlk), 0, s, cells, 0.0, u);
    CLM_LAUNCH_CHECK();
    return CLM_OK;
  }
  auto smooth_T = [&](int sweeps) -> clm_status {
    for (int k = 0; k < sweeps; ++k)
      for (int col = 1; col >= 0; --col) {
        hipLaunchKernelGGL(k_hs_T, grid_for(cells), dim3(kBlk), 0, s, r, np, col, u, v, f);
        CLM_LAUNCH_CHECK();
        std::swap(u, v);
      }
    return CLM_OK;
  };
  clm_status st;
  if ((st = smooth_T(p->d.nu_post)) != CLM_OK) return st;
  // coarse level l + 1: e = P^T ubar; ubar_H out = e
  const int nc = n / 2;
  const int64_t ccells = np * nc * nc;
  double* uH = p->adj_u[l + 1];
  double* fH = p->adj_f[l + 1];
  double* e = p->adj_w[l + 1];
  hipLaunchKernelGGL(k_prolong_T, grid_for(ccells), dim3(kBlk), 0, s, n, np, u, e);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fill, grid_for(ccells), dim3(kBlk), 0, s, ccells, 0.0, uH);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_axpy, grid_for(ccells), dim3(kBlk), 0, s, ccells, 1.0, e, uH);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fill, grid_for(ccells), dim3(kBlk), 0, s, ccells, 0.0, fH);
  CLM_LAUNCH_CHECK();
  if ((st = vcycle_T(p, l + 1, s)) != CLM_OK) return st;
  // ubar_bar = -e + ubar_H in + L_H^T fbar_H  (into e)
  hipLaunchKernelGGL(k_axpy, grid_for(ccells), dim3(kBlk), 0, s, ccells, -2.0, e, e);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_axpy, grid_for(ccells), dim3(kBlk), 0, s, ccells, 1.0, p->adj_u[l + 1], e);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_L0_T, grid_for(ccells), dim3(kBlk), 0, s, rows(p, l + 1), np, fH, 1.0, e);
  CLM_LAUNCH_CHECK();
  // u += R^T ubar_bar; r = R^T fbar_H: f += r, u -= L^T r  (r in v)
  hipLaunchKernelGGL(k_restrict_T, grid_for(cells), dim3(kBlk), 0, s, r, np, e, 1.0, u);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fill, grid_for(cells), dim3(kBlk), 0, s, cells, 0.0, v);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_restrict_T, grid_for(cells), dim3(kBlk), 0, s, r, np, fH, 1.0, v);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_axpy, grid_for(cells), dim3(kBlk), 0, s, cells, 1.0, v, f);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_L0_T, grid_for(cells), dim3(kBlk), 0, s, r, np, v, -1.0, u);
  CLM_LAUNCH_CHECK();
  if ((st = smooth_T(p->d.nu_pre)) != CLM_OK) return st;
  // the smoothing ping-pong may have left the result in the partner array
  if (u != p->adj_u[l]) {
    hipLaunchKernelGGL(k_fill, grid_for(cells), dim3(kBlk), 0, s, cells, 0.0, p->adj_u[l]);
    CLM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_axpy, grid_for(cells), dim3(kBlk), 0, s, cells, 1.0, u, p->adj_u[l]);
    CLM_LAUNCH_CHECK();
  }
  return CLM_OK;
}

}  // namespace

clm_status shear_adjoint(Plan* p, const double* th, const double* ph, int64_t npts,
                         const double* gbar, const double* hbar, hipStream_t s) {
  if (npts == 0) return CLM_OK;
  EvalTArgs a;
  a.rot = p->rot;
  a.ubar = p->adj_ubar;
  a.th = th;
  a.ph = ph;
  a.gbar = gbar;
  a.hbar = hbar;
  a.npts = npts;
  a.Nb = p->d.nside_bundle;
  a.n = p->n;
  a.L = p->L;
  a.delta = p->delta;
  a.status = p->status_dev;
  {
    CLM_TIMED(p, s, "adj_eval");
    hipLaunchKernelGGL(k_adj_eval, grid_for(npts), dim3(kBlk), 0, s, a);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status poisson_adjoint(Plan* p, double* dkappa, hipStream_t s) {
  const int n = p->n;
  const int64_t np = p->nbundle, cells = np * n * n;
  const size_t G = size_t(n + 2) * (n + 2);
  clm_status st;
  // du bar on the interior; f' bar = sum over cycles of V^T
  hipLaunchKernelGGL(k_adj_split, grid_for(cells), dim3(kBlk), 0, s, p->adj_ubar, n, np,
                     p->adj_u[0]);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fill, grid_for(cells), dim3(kBlk), 0, s, cells, 0.0, p->adj_f[0]);
  CLM_LAUNCH_CHECK();
  {
    CLM_TIMED(p, s, "adj_mg");
    for (int cyc = 0; cyc < p->d.mg_vcycles; ++cyc)
      if ((st = vcycle_T(p, 0, s)) != CLM_OK) return st;
  }
  // setup^T into the SHT-grid (private copies) and fine maps
  const int64_t npriv = int64_t(p->adj_ncopy) * p->npix_s;
  hipLaunchKernelGGL(k_fill, grid_for(npriv), dim3(kBlk), 0, s, npriv, 0.0, p->adj_psi_priv);
  CLM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fill, grid_for(p->npix_f), dim3(kBlk), 0, s, p->npix_f, 0.0, dkappa);
  CLM_LAUNCH_CHECK();
  SetupTArgs a;
  a.rot = p->rot;
  a.ubar = p->adj_ubar;
  a.fpb = p->adj_f[0];
  a.r = rows(p, 0);
  a.np = np;
  a.L = p->L;
  a.delta = p->delta;
  a.rs = hpx::Rings{p->ring_s, p->ringi_s, p->ringx_s, p->nring_s, p->d.nside_sht};
  a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, p->d.nside_fine};
  a.psibar = p->adj_psi_priv;
  a.npix_s = p->npix_s;
  a.ncopy = p->adj_ncopy;
  a.kbar = dkappa;
  {
    CLM_TIMED(p, s, "adj_setup");
    hipLaunchKernelGGL(k_adj_setup_cells, grid_for(cells), dim3(kBlk), 0, s, a);
    hipLaunchKernelGGL(k_adj_setup_ghosts, grid_for(np * (4 * n + 4)), dim3(kBlk), 0, s, a);
    hipLaunchKernelGGL(k_sum_copies, grid_for(p->npix_s), dim3(kBlk), 0, s, p->adj_ncopy,
                       p->npix_s, static_cast<const double*>(p->adj_psi_priv), p->adj_psi);
  }
  CLM_LAUNCH_CHECK();
  // SHT^T: psi_SHT bar -> kappa_SHT bar
  if ((st = sht_adjoint(p, p->adj_psi, p->adj_alm, p->adj_ks, s)) != CLM_OK) return st;
  // degrade^T (or identity) into the fine map, then demean^T
  const int64_t ratio = p->d.nside_fine / p->d.nside_sht;
  int shift = 0;
  while ((int64_t(1) << shift) < ratio * ratio) ++shift;
  hipLaunchKernelGGL(k_adj_degrade, grid_for(p->npix_f), dim3(kBlk), 0, s, p->adj_ks, p->npix_f,
                     p->r2n_f, shift, int64_t(p->d.nside_sht), 1.0 / double(ratio * ratio),
                     dkappa);
  CLM_LAUNCH_CHECK();
  if ((st = plane_mean(p, dkappa, 1, s)) != CLM_OK) return st;
  hipLaunchKernelGGL(k_sub_mean, grid_for(p->npix_f), dim3(kBlk), 0, s, p->npix_f, p->red,
                     dkappa);
  CLM_LAUNCH_CHECK();
  // the accumulator starts again from zero
  hipLaunchKernelGGL(k_fill, grid_for(int64_t(np) * G), dim3(kBlk), 0, s, int64_t(np) * G, 0.0,
                     p->adj_ubar);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace clm
