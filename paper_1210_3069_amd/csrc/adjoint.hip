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
//   fixed V-cycles from du = 0                  -> vcycle_T per cycle: smoothing
//                                                  (k_smooth_T, LDS tiles, with
//                                                  the coarse correction as its
//                                                  prologue), k_prolong_T,
//                                                  k_corr_T, k_coarsest_T
//   f' = 2 interp(kappa') - L u0, u0 from psi_SHT (cells, face ghosts)
//                                               -> k_adj_setup_cells / _ghosts
//   analysis, Poisson factor, synthesis         -> sht_adjoint (sht.hip)
//   degrade to the SHT grid, demean             -> k_adj_degrade, k_sub_mean
// Everything runs in FP64 on plain per-level arrays; the smoothing blocks
// several half sweeps in LDS.
#include <cmath>

#include "clm_internal.h"
#include "eval_dev.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlk = 256;
constexpr double kPi = 3.14159265358979323846;

inline dim3 grid_for(int64_t n) { return dim3(unsigned((n + kBlk - 1) / kBlk)); }

// Row coefficients of a level: s_m, s_p, s_c, area per row (c), and the
// reciprocals 1 / s_c, 1 / area (q), so that no kernel divides per cell.
struct Rows {
  const double* c;
  const double* q;
  int n;
  __device__ double sm(int i) const { return c[4 * i]; }
  __device__ double sp(int i) const { return c[4 * i + 1]; }
  __device__ double isc(int i) const { return q[4 * i]; }
  __device__ double A(int i) const { return c[4 * i + 3]; }
  __device__ double rA(int i) const { return q[4 * i + 1]; }
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
  // the point's patch coordinates exactly as the forward evaluation takes them
  const double thp = kPi / 2 - hpx::asin_small(pz), php = hpx::dphi_of(px, py, 1.0, 0.0);
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
// Transposed red-black smoothing.  One half sweep of colour c maps (x, fbar)
// to (y, fbar'):
//   colour-c cells:     y = 0, fbar -= A x / D;
//   other cells:        y = x + sum over their colour-c neighbours q of
//                       (q's stencil coefficient towards the cell) x_q / D_q.
// A launch runs S successive half sweeps on a tile of TT^2 cells held in LDS
// with a halo of S cells.  Every half sweep updates the same set of cells
// (rows 1 .. W-2 of the W^2 LDS region); the cells near the region's edge
// that lose their inputs hold garbage, which moves inwards one cell per half
// sweep and never reaches the tile.  Cells are kept in LDS scaled by 1 / D
// while they are read as colour-c cells, so an update reads its neighbours
// as they are.  The cells of a row are taken in pairs (2q, 2q + 1): a pair
// holds one cell of each colour, and one thread owns it in every half
// sweep, accumulating the pair's f bar in registers.
//
// The launch that starts the transposed pre-smoothing first applies, on
// every loaded cell, the transpose of the coarse-grid correction of the
// forward cycle (area-weighted restriction R and level operator L0):
//   v = R^T fbar_H,  u += R^T e - L0^T v,  fbar += v.
template <int TT, int S, int NT>
struct SmGeom {
  static constexpr int W = TT + 2 * S;          // LDS side
  static constexpr int HP = W / 2;              // column pairs per row
  static constexpr int NPair = (W - 2) * HP;    // pairs of rows 1 .. W-2
  static constexpr int P = (NPair + NT - 1) / NT;   // pairs per thread
  static constexpr int Ld = (W * W + NT - 1) / NT;  // loads per thread
  static constexpr int R = W + 2;               // row-table rows (one more each side)
  static constexpr int C = TT / 2 + S + 2;      // coarse rows / columns under a tile
  // dynamic LDS: tile, row table (8 per row), coarse e and fbar_H
  static constexpr size_t Lds = 8 * (size_t(W) * W + 8 * R + 2 * C * C);
  static_assert(S % 2 == 0 && S >= 2, "half sweeps come in whole sweeps");
};

struct SmoothTArgs {
  Rows r;             // this level
  int tiles;          // tiles per patch side
  int c0;             // colour of the first half sweep
  int remap;          // XCD-contiguous block order
  const double* in;   // [np][n][n] u bar
  double* out;        // [np][n][n]
  double* fbar;       // [np][n][n], updated in place
  const double* e;    // coarse u-bar correction [np][n/2][n/2], or null
  const double* fH;   // coarse f bar [np][n/2][n/2] (with e)
};

template <int TT, int S, int NT>
__global__ __launch_bounds__(NT) void k_smooth_T(SmoothTArgs a) {
  using G = SmGeom<TT, S, NT>;
  constexpr int W = G::W, HP = G::HP, RR = G::R, CC = G::C;
  extern __shared__ double sm_[];
  double* X = sm_;                 // [W][W]
  // per row: s_m, s_p, 1/s_c, area, 1/area, R^T weight, and 1/D for the
  // interior columns and for the two face columns (levels have n >= 8);
  // zero on rows outside the patch
  double* RT = X + W * W;          // [8][RR]
  double* CE = RT + 8 * RR;        // [CC][CC] coarse e
  double* CF = CE + CC * CC;       // [CC][CC] coarse fbar_H
  const int n = a.r.n, tid = threadIdx.x;
  // Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // range of tiles so that neighbouring tiles share its L2 for their halos.
  int64_t bid = blockIdx.x;
  if (a.remap) {
    const int64_t per = gridDim.x / 8;
    bid = (bid & 7) * per + (bid >> 3);
  }
  const int t2 = a.tiles * a.tiles;
  const int64_t b = bid / t2;
  const int tt = int(bid - b * t2);
  const int i0 = (tt / a.tiles) * TT, j0 = (tt % a.tiles) * TT;
  const size_t base = size_t(b) * n * n;
  auto inside = [&](int i, int j) { return unsigned(i) < unsigned(n) && unsigned(j) < unsigned(n); };
  // pair m of this thread: LDS row r (1 .. W-2), first column 2q
  auto pair_rq = [&](int m, int& r, int& q) {
    const int k = tid + m * NT;
    r = 1 + k / HP;
    q = k - (r - 1) * HP;
    return k < G::NPair;
  };
  auto in_tile = [&](int r, int q) { return r >= S && r < S + TT && 2 * q >= S && 2 * q < S + TT; };
  // all global loads first: u bar on the tile and its halo (0 outside the
  // patch), f bar of the pairs of the tile this thread owns
  double xv[G::Ld];
#pragma unroll
  for (int m = 0; m < G::Ld; ++m) {
    const int idx = tid + m * NT;
    const int ri = idx / W, rj = idx - ri * W;
    const int i = i0 + ri - S, j = j0 + rj - S;
    xv[m] = idx < W * W && inside(i, j) ? a.in[base + size_t(i) * n + j] : 0.0;
  }
  double2 fb[G::P];
#pragma unroll
  for (int m = 0; m < G::P; ++m) {
    int r, q;
    const bool ok = pair_rq(m, r, q) && in_tile(r, q);
    fb[m] = ok ? *reinterpret_cast<const double2*>(a.fbar + base + size_t(i0 + r - S) * n +
                                                   j0 + 2 * q - S)
               : make_double2(0.0, 0.0);
  }
  for (int k = tid; k < RR; k += NT) {
    const int i = i0 - S - 1 + k;
    const bool ok = i >= 0 && i < n;
    const double d = ok ? a.r.D(i, 1) : 1.0;  // row faces included, no column face
    const int I2 = i & ~1;
    RT[0 * RR + k] = ok ? a.r.sm(i) : 0.0;
    RT[1 * RR + k] = ok ? a.r.sp(i) : 0.0;
    RT[2 * RR + k] = ok ? a.r.isc(i) : 0.0;
    RT[3 * RR + k] = ok ? a.r.A(i) : 0.0;
    RT[4 * RR + k] = ok ? a.r.rA(i) : 0.0;
    RT[5 * RR + k] = ok ? a.r.A(i) / (2.0 * (a.r.A(I2) + a.r.A(I2 + 1))) : 0.0;
    RT[6 * RR + k] = ok ? 1.0 / d : 0.0;
    RT[7 * RR + k] = ok ? 1.0 / (d + a.r.isc(i)) : 0.0;
  }
  // coarse tiles under rows / columns i0 - S - 1 .. i0 + TT + S
  const int nc = n >> 1;
  constexpr int CW = ((TT + S) >> 1) + ((S + 2) >> 1) + 1;
  static_assert(CW <= CC, "coarse tile");
  const int cI0 = (i0 >> 1) - ((S + 2) >> 1), cJ0 = (j0 >> 1) - ((S + 2) >> 1);
  if (a.e) {
    constexpr int NC = (CW * CW + NT - 1) / NT;
    const size_t cb = size_t(b) * nc * nc;
    double ce[NC], cf[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const int idx = tid + m * NT;
      const int ci = idx / CW, cj = idx - ci * CW;
      const int I = cI0 + ci, J = cJ0 + cj;
      const bool ok = idx < CW * CW && I >= 0 && I < nc && J >= 0 && J < nc;
      ce[m] = ok ? a.e[cb + size_t(I) * nc + J] : 0.0;
      cf[m] = ok ? a.fH[cb + size_t(I) * nc + J] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      const int idx = tid + m * NT;
      if (idx >= CW * CW) continue;
      const int ci = idx / CW, cj = idx - ci * CW;
      CE[ci * CC + cj] = ce[m];
      CF[ci * CC + cj] = cf[m];
    }
  }
  __syncthreads();
  // row-table entry t of global row i
  auto rt = [&](int t, int i) { return RT[t * RR + i - (i0 - S - 1)]; };
  // 1 / full diagonal at (i, j)
  auto diag = [&](int i, int j) { return rt(j == 0 || j == n - 1 ? 7 : 6, i); };
  // coarse value of the cell (i, j)
  auto cv = [&](const double* Cm, int i, int j) {
    return Cm[((i >> 1) - cI0) * CC + (j >> 1) - cJ0];
  };
  // R^T fbar_H at a cell of the patch
  auto vv = [&](int i, int j) { return rt(5, i) * cv(CF, i, j); };
#pragma unroll
  for (int m = 0; m < G::Ld; ++m) {
    const int idx = tid + m * NT;
    if (idx >= W * W) continue;
    const int ri = idx / W, rj = idx - ri * W;
    const int i = i0 + ri - S, j = j0 + rj - S;
    double x = xv[m];
    if (inside(i, j)) {
      if (a.e) {
        // u += R^T e - L0^T v at (i, j); full diagonal D (faces: ghost = -u)
        const double ra = rt(4, i), is = rt(2, i);
        double d = rt(0, i) + rt(1, i) + 2.0 * is;
        if (i == 0) d += rt(0, i);
        if (i == n - 1) d += rt(1, i);
        if (j == 0) d += is;
        if (j == n - 1) d += is;
        double l0 = -d * vv(i, j) * ra;
        if (i > 0) l0 += rt(1, i - 1) * vv(i - 1, j) * rt(4, i - 1);
        if (i < n - 1) l0 += rt(0, i + 1) * vv(i + 1, j) * rt(4, i + 1);
        if (j > 0) l0 += is * vv(i, j - 1) * ra;
        if (j < n - 1) l0 += is * vv(i, j + 1) * ra;
        x += rt(5, i) * cv(CE, i, j) - l0;
      }
      // the first half sweep reads its colour-c0 cells scaled by 1 / D
      if (((ri + rj) & 1) == a.c0) x *= diag(i, j);
    }
    X[idx] = x;
  }
  if (a.e) {
#pragma unroll
    for (int m = 0; m < G::P; ++m) {
      int r, q;
      if (!pair_rq(m, r, q) || !in_tile(r, q)) continue;
      const int i = i0 + r - S, j = j0 + 2 * q - S;
      fb[m].x += vv(i, j);
      fb[m].y += vv(i, j + 1);
    }
  }
  __syncthreads();
  double vlast[G::P];
#pragma unroll
  for (int h = 0; h < S; ++h) {
    const int c = a.c0 ^ (h & 1);
#pragma unroll
    for (int m = 0; m < G::P; ++m) {
      int r, q;
      if (!pair_rq(m, r, q)) continue;
      const int second = (1 + c + r) & 1;  // the pair's cell not of colour c
      const int col = 2 * q + second;
      const int i = i0 + r - S, j = j0 + col - S;
      if (!inside(i, j)) continue;
      const int x = r * W + col, k = r + 1;
      double v = h == 0 ? X[x] : 0.0;
      v += RT[1 * RR + k - 1] * X[x - W] + RT[0 * RR + k + 1] * X[x + W] +
           RT[2 * RR + k] * (X[x - 1] + X[x + 1]);
      const bool tile = in_tile(r, q);
      const double A = RT[3 * RR + k];
      double fd = 0.0;
      // this cell was of colour c0 in the first half sweep
      if (h == 1) fd -= A * X[x];
      if (h < S - 1) {
        const double z = v * diag(i, j);
        X[x] = z;
        fd -= A * z;
      } else {
        vlast[m] = v;
      }
      if (tile) {
        if (second) fb[m].y += fd;
        else fb[m].x += fd;
      }
    }
    if (h < S - 1) __syncthreads();
  }
  // the last half sweep's colour is zero; the other cells hold its results
  const int clast = a.c0 ^ ((S - 1) & 1);
#pragma unroll
  for (int m = 0; m < G::P; ++m) {
    int r, q;
    if (!pair_rq(m, r, q) || !in_tile(r, q)) continue;
    const size_t g = base + size_t(i0 + r - S) * n + j0 + 2 * q - S;
    const int second = (1 + clast + r) & 1;
    *reinterpret_cast<double2*>(a.out + g) =
        second ? make_double2(0.0, vlast[m]) : make_double2(vlast[m], 0.0);
    *reinterpret_cast<double2*>(a.fbar + g) = fb[m];
  }
}

// e = -e + u bar_H + L0^T f bar_H on a coarse level (L0: the level operator
// on a correction with zero face values, rows scaled by 1 / area).
__global__ void k_corr_T(Rows r, int64_t np, const double* uH, const double* xin, double* e) {
  const int n = r.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * n * n) return;
  const int c = int(t % (int64_t(n) * n)), i = c / n, j = c % n;
  const double* x = xin + (t - c);
  double v = -r.D(i, j) * x[c] * r.rA(i);
  if (i > 0) v += r.sp(i - 1) * x[c - n] * r.rA(i - 1);
  if (i < n - 1) v += r.sm(i + 1) * x[c + n] * r.rA(i + 1);
  if (j > 0) v += r.isc(i) * x[c - 1] * r.rA(i);
  if (j < n - 1) v += r.isc(i) * x[c + 1] * r.rA(i);
  e[t] = uH[t] - e[t] + v;
}

// e_coarse = P^T x_fine (bilinear 9/3/3/1, direct injection on the
// outermost fine ring); gather over the 4 x 4 fine window of a coarse cell.
// The coarse cycle then starts from u bar_H = e and f bar_H = 0.
__global__ void k_prolong_T(int n, int64_t np, const double* xf, double* ec, double* uH,
                            double* fH) {
  const int nc = n / 2;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * nc * nc) return;
  const int64_t b = t / (int64_t(nc) * nc);
  const int c = int(t % (int64_t(nc) * nc)), I = c / nc, J = c % nc;
  const double* x = xf + size_t(b) * n * n;
  // the 4 x 4 fine window, every load issued before any is used (indices
  // clamped into the patch; cells outside it add nothing)
  double xv[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int r = min(max(2 * I - 1 + a, 0), n - 1), q = min(max(2 * J - 1 + c4, 0), n - 1);
      xv[a][c4] = x[r * n + q];
    }
  double v = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = 2 * I - 1 + a;
    const double wr = (r >> 1) == I ? 0.75 : 0.25;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int q = 2 * J - 1 + c4;
      if (r < 0 || r >= n || q < 0 || q >= n) continue;
      const bool ring = r == 0 || r == n - 1 || q == 0 || q == n - 1;
      const bool own = (r >> 1) == I && (q >> 1) == J;
      if (ring) {
        if (own) v += xv[a][c4];
      } else {
        v += wr * ((q >> 1) == J ? 0.75 : 0.25) * xv[a][c4];
      }
    }
  }
  ec[t] = v;
  uH[t] = v;
  fH[t] = 0.0;
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
  auto f = [&](int r, int q) { return fb[r * n + q] * a.r.rA(r); };
  if (i >= 0 && i < n && j >= 0 && j < n) v += (a.r.sm(i) + a.r.sp(i) + 2.0 * a.r.isc(i)) * f(i, j);
  // cells whose stencil reads (i, j), with minus sign of -L
  if (i + 1 >= 0 && i + 1 < n && j >= 0 && j < n) v -= a.r.sm(i + 1) * f(i + 1, j);
  if (i - 1 >= 0 && i - 1 < n && j >= 0 && j < n) v -= a.r.sp(i - 1) * f(i - 1, j);
  if (i >= 0 && i < n && j + 1 >= 0 && j + 1 < n) v -= a.r.isc(i) * f(i, j + 1);
  if (i >= 0 && i < n && j - 1 >= 0 && j - 1 < n) v -= a.r.isc(i) * f(i, j - 1);
  return v;
}

// Block-local accumulation of scattered map contributions: an open-addressed
// hash table in LDS keyed by pixel.  A block adds its contributions there and
// then issues one global atomic per distinct pixel (neighbouring cells share
// most of their interpolation pixels).  A contribution that finds no slot
// within kProbe probes goes to the map directly.
constexpr int kProbe = 16;

template <int LG>
struct LdsMapAcc {
  static constexpr int HS = 1 << LG;
  int* key;      // [HS], -1: empty
  double* val;   // [HS]
  __device__ void clear() {
    for (int s = threadIdx.x; s < HS; s += blockDim.x) {
      key[s] = -1;
      val[s] = 0.0;
    }
  }
  __device__ void add(double* map, int pix, double v) {
    unsigned h = (unsigned(pix) * 2654435761u) >> (32 - LG);
    for (int k = 0; k < kProbe; ++k) {
      const int old = atomicCAS(&key[h], -1, pix);
      if (old == -1 || old == pix) {
        atomicAdd(&val[h], v);
        return;
      }
      h = (h + 1) & (HS - 1);
    }
    atomicAdd(map + pix, v);
  }
  __device__ void flush(double* map) const {
    for (int s = threadIdx.x; s < HS; s += blockDim.x)
      if (key[s] >= 0) atomicAdd(map + key[s], val[s]);
  }
};

// Interior cells: u0 = interp(psi) and the ghosts' -u0(adjacent) folded in;
// f = 2 interp(kappa') with f bar = f' bar.  A block takes a 16 x 16 tile
// of one patch (patches of 8^2 cells: 4 whole patches), so that its cells
// share interpolation pixels.
constexpr int kSetupTile = 16;

__global__ __launch_bounds__(kBlk) void k_adj_setup_cells(SetupTArgs a) {
  static_assert(kBlk == kSetupTile * kSetupTile, "one cell per thread");
  __shared__ int pk[256], fk[1024];
  __shared__ double pv[256], fv[1024];
  LdsMapAcc<8> accp{pk, pv};
  LdsMapAcc<10> accf{fk, fv};
  accp.clear();
  accf.clear();
  const int n = a.r.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool live = t < a.np * n * n;
  int64_t b;
  int i, j;
  if (n >= kSetupTile) {
    const int nt = n / kSetupTile;
    const int64_t tile = int64_t(blockIdx.x);
    b = tile / (int64_t(nt) * nt);
    const int tl = int(tile - b * nt * nt);
    i = (tl / nt) * kSetupTile + threadIdx.x / kSetupTile;
    j = (tl % nt) * kSetupTile + threadIdx.x % kSetupTile;
  } else {
    b = t / (int64_t(n) * n);
    const int c = int(t - b * n * n);
    i = c / n;
    j = c % n;
  }
  // each block adds into its own copy of the small SHT-grid map: millions of
  // cells map to each SHT pixel, and one shared map serialises the atomics
  double* psib = a.psibar + (blockIdx.x % a.ncopy) * a.npix_s;
  __syncthreads();
  if (live) {
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
    int pix[4];
    double w[4];
    hpx::interp_weights(a.rs, z, rho, ph, pix, w);
    for (int c = 0; c < 4; ++c) accp.add(psib, pix[c], w[c] * v);
    const double fv2 = 2.0 * fb[i * n + j];
    hpx::interp_weights(a.rf, z, rho, ph, pix, w);
    for (int c = 0; c < 4; ++c) accf.add(a.kbar, pix[c], w[c] * fv2);
  }
  __syncthreads();
  accp.flush(psib);
  accf.flush(a.kbar);
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

// Reciprocal row table (1 / s_c, 1 / area, two unused) of every level, laid
// out like the coefficient table.
__global__ void k_rrows(int64_t nrows, const double* c, double* q) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const double* r = c + 4 * t;
  q[4 * t] = 1.0 / r[2];
  q[4 * t + 1] = 1.0 / r[3];
  q[4 * t + 2] = 0.0;
  q[4 * t + 3] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

Rows rows(Plan* p, int l) {
  return Rows{p->coef + p->lev[l].crow, p->adj_rrows + p->lev[l].crow, p->n >> l};
}

template <int TT, int S, int NT>
clm_status launch_smooth_T(Plan* p, const SmoothTArgs& a, int64_t nblk, hipStream_t s) {
  using G = SmGeom<TT, S, NT>;
  const auto kern = k_smooth_T<TT, S, NT>;
  clm_status st = lds_opt_in(p, reinterpret_cast<const void*>(kern), G::Lds);
  if (st != CLM_OK) return st;
  hipLaunchKernelGGL(kern, dim3(unsigned(nblk)), dim3(NT), G::Lds, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

template <int TT, int NT>
clm_status launch_smooth_T(Plan* p, const SmoothTArgs& a, int S, int64_t nblk, hipStream_t s) {
  return S == 4 ? launch_smooth_T<TT, 4, NT>(p, a, nblk, s)
                : launch_smooth_T<TT, 2, NT>(p, a, nblk, s);
}

// Transposed smoothing of level l (n >= 8): 2 nu half sweeps, the first of
// colour 1, in launches of 4 half sweeps and a last one of 2 for odd nu; the
// first launch applies the coarse-correction transpose when e is given.
// Tiles are 64^2 cells, or the whole patch on smaller levels.  u and v swap
// per launch.
clm_status smooth_T(Plan* p, int l, int nu, const double* e, const double* fH, double*& u,
                    double*& v, double* f, hipStream_t s) {
  const int n = p->n >> l;
  const int T = std::min(64, n);
  SmoothTArgs a;
  a.r = rows(p, l);
  a.tiles = n / T;
  a.fbar = f;
  a.e = e;
  a.fH = fH;
  const int64_t nblk = int64_t(p->nbundle) * a.tiles * a.tiles;
  a.remap = nblk % 8 == 0;
  int left = 2 * nu;
  a.c0 = 1;
  while (left > 0) {
    const int S = left >= 4 ? 4 : 2;
    a.in = u;
    a.out = v;
    clm_status st;
    switch (T) {
      case 64: st = launch_smooth_T<64, 512>(p, a, S, nblk, s); break;
      case 32: st = launch_smooth_T<32, 256>(p, a, S, nblk, s); break;
      case 16: st = launch_smooth_T<16, 128>(p, a, S, nblk, s); break;
      case 8: st = launch_smooth_T<8, 64>(p, a, S, nblk, s); break;
      default: return fail(p, CLM_EINVAL, "smoothing level side must be a power of 2 >= 8");
    }
    if (st != CLM_OK) return st;
    std::swap(u, v);
    left -= S;
    a.e = nullptr;
    a.fH = nullptr;
  }
  return CLM_OK;
}

// Transpose of one V-cycle on level l: ubar_out in adj_u[l] -> ubar_in in
// adj_u[l], fbar added to adj_f[l] (the caller zeroes it).
clm_status vcycle_T(Plan* p, int l, hipStream_t s) {
  const int n = p->n >> l;
  const int64_t np = p->nbundle, cells = np * n * n;
  double* u = p->adj_u[l];
  double* v = p->adj_v[l];
  double* f = p->adj_f[l];
  if (n <= 4) {
    hipLaunchKernelGGL(k_coarsest_T, grid_for(np * 16), dim3(kBlk), 0, s, p->cinv, np, u, f);
    CLM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill, grid_for(cells), dim3(kBlk), 0, s, cells, 0.0, u);
    CLM_LAUNCH_CHECK();
    return CLM_OK;
  }
  clm_status st;
  if ((st = smooth_T(p, l, p->d.nu_post, nullptr, nullptr, u, v, f, s)) != CLM_OK) return st;
  // coarse level l + 1: e = P^T ubar; ubar_H out = e
  const int nc = n / 2;
  const int64_t ccells = np * nc * nc;
  double* uH = p->adj_u[l + 1];
  double* fH = p->adj_f[l + 1];
  double* e = p->adj_w[l + 1];
  hipLaunchKernelGGL(k_prolong_T, grid_for(ccells), dim3(kBlk), 0, s, n, np, u, e, uH, fH);
  CLM_LAUNCH_CHECK();
  if ((st = vcycle_T(p, l + 1, s)) != CLM_OK) return st;
  // ubar_bar = -e + ubar_H in + L_H^T fbar_H  (into e)
  hipLaunchKernelGGL(k_corr_T, grid_for(ccells), dim3(kBlk), 0, s, rows(p, l + 1), np,
                     static_cast<const double*>(uH), static_cast<const double*>(fH), e);
  CLM_LAUNCH_CHECK();
  // u += R^T ubar_bar, v = R^T fbar_H: f += v, u -= L0^T v; then smoothing
  if ((st = smooth_T(p, l, p->d.nu_pre, e, fH, u, v, f, s)) != CLM_OK) return st;
  // the smoothing ping-pong may have left the result in the partner array
  if (u != p->adj_u[l])
    CLM_HIP(hipMemcpyAsync(p->adj_u[l], u, size_t(cells) * 8, hipMemcpyDeviceToDevice, s));
  return CLM_OK;
}

}  // namespace

clm_status adjoint_tables(Plan* p) {
  int64_t nrows = 0;
  for (int l = 0; l < p->nlev; ++l) nrows += p->n >> l;
  hipLaunchKernelGGL(k_rrows, grid_for(nrows), dim3(kBlk), 0, 0, nrows,
                     static_cast<const double*>(p->coef), p->adj_rrows);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

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
