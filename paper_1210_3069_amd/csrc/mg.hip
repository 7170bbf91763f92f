// Multigrid refinement of the SHT potential on rotated patches (Sec. 3.2).
//
// One patch per ray bundle: rotated so the bundle centre is at
// (theta', phi') = (pi/2, 0), n x n cells with Delta theta' = Delta phi'.
// The unknown is the correction du = u - u0 to the interpolated SHT
// potential, zero on the patch faces; the finite-volume 5-point Laplacian
// uses exact cell areas, so a ghost across the patch face equals minus the
// interior cell (Dirichlet value on the face).  An FAS V-cycle: nu_pre
// red-black Gauss-Seidel sweeps (red = (i+j) even first), residual, area-
// weighted ("strictly conservative") restriction of du and of the residual,
// coarse source L_H ubar + rbar, recursion down to 4 x 4 solved exactly,
// bilinear prolongation of u_H - ubar with direct injection on the
// outermost fine ring, nu_post sweeps.
//
// Data layout in HBM: every level is [patch][i][j] row-major with j (phi')
// fastest, no ghost storage.  Levels wider than kLdsLevelMax are streamed
// through LDS in kTile x kTile tiles with a halo of 2 nu + 1 cells, so all
// sweeps of a smoothing pass, the residual and the restriction happen in one
// read and one write of the level (temporal blocking; the halo makes the
// tile interior identical to the global sweep).  Levels <= kLdsLevelMax of
// a patch are solved by one workgroup entirely in LDS.
#include <cmath>

#include "clm_internal.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

// Logical block index: consecutive logical blocks (tiles of one patch) are
// kept on one XCD (hardware dispatches blocks round-robin over 8 XCDs).
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// ------------------------------------------------------------ patch setup
// u0 = interp(psi_SHT) at the cell centres; ghost u0 = 2 b - u0(adjacent)
// with b = interp(psi_SHT) at the face midpoint (corner: patch corner);
// f' = 2 (interp(kappa) - mean) - L u0 at the cell centres, float64.
struct SetupArgs {
  int n, ntile, tile;
  double L, delta;
  const double* rot;
  const double* coef;  // level-0 rows
  hpx::Rings rs, rf;
  const double* psi_s;
  const void* kappa;
  int kappa_fp64;
  const double* red;   // red[1023] = mean of kappa
  double* u0;          // [patch][(n+2)^2]
  void* fprime;        // [patch][n^2] of T
};

// Global direction of the patch point with sin/cos of theta' and phi':
// v = R^T (sin th' cos ph', sin th' sin ph', cos th'); returns z = cos theta,
// rho = sin theta and the azimuth offset from a reference azimuth with
// cosine/sine (cr, sr).
__device__ __forceinline__ void patch_dir(const double* R, double st, double ct, double sp,
                                          double cp, double cr, double sr, double& z,
                                          double& rho, double& dph) {
  const double x = st * cp, y = st * sp;
  const double vx = R[0] * x + R[3] * y + R[6] * ct;
  const double vy = R[1] * x + R[4] * y + R[7] * ct;
  z = R[2] * x + R[5] * y + R[8] * ct;
  rho = sqrt(vx * vx + vy * vy);
  dph = hpx::dphi_of(vx, vy, cr, sr);
}

// Rings of the two grids a setup block may copy to LDS (the tile's z range
// plus one cell of slack; blocks whose range is wider read the global
// tables).
constexpr int kRingCapF = 256, kRingCapS = 64;
constexpr int kSetupBlock = 512;

template <int CAP>
struct RingStore {
  double z[CAP], s[CAP], t[CAP], k[CAP], g[CAP + 1];
  int n[CAP], f[CAP];
  __device__ hpx::LdsRingTab tab() {
    hpx::LdsRingTab r;
    r.zq = z; r.sq = s; r.tq = t; r.kq = k; r.gq = g; r.nq = n; r.fq = f;
    return r;
  }
};

// Reference azimuth of a setup block (the region centre's).
struct PhiRef {
  double phi, c, s;
};

// Pass 1 visits every cell of the tile plus one ring once: direction, u0 and
// (interior cells) the source f, written to the f' array; pass 2 fills the
// patch ghosts from the face values; pass 3 forms f' = f - L u0 (the thread
// that wrote f reads it back).
template <typename T, int TILE, typename TS, typename TF>
__device__ void setup_passes(const SetupArgs& a, const TS& rs, const TF& rf, double* shu,
                             const double* trig, const double* R, const PhiRef& pr,
                             int64_t patch, int i0, int j0) {
  constexpr int RR = TILE + 2;
  const int n = a.n;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  const double mean = a.red[1023];
  const size_t G = size_t(n + 2);
  double* u0 = a.u0 + size_t(patch) * G * G;
  T* fp = static_cast<T*>(a.fprime) + size_t(patch) * n * n;
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    double v = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      double z, rho, dph;
      patch_dir(R, trig[4 * li], trig[4 * li + 1], trig[4 * lj + 2], trig[4 * lj + 3], pr.c,
                pr.s, z, rho, dph);
      int ps[4];
      double ws[4];
      hpx::interp_weights_t(rs, z, rho, dph, ps, ws);
      if (li >= 1 && li <= TILE && lj >= 1 && lj <= TILE) {
        int pf[4];
        double wf[4];
        hpx::interp_weights_t(rf, z, rho, dph, pf, wf);
        double k4[4];
        if (a.kappa_fp64) {
          const double* km = static_cast<const double*>(a.kappa);
          for (int c = 0; c < 4; ++c) k4[c] = km[pf[c]];
        } else {
          const float* km = static_cast<const float*>(a.kappa);
          for (int c = 0; c < 4; ++c) k4[c] = km[pf[c]];
        }
        v = ws[0] * a.psi_s[ps[0]] + ws[1] * a.psi_s[ps[1]] + ws[2] * a.psi_s[ps[2]] +
            ws[3] * a.psi_s[ps[3]];
        const double kv = wf[0] * k4[0] + wf[1] * k4[1] + wf[2] * k4[2] + wf[3] * k4[3];
        fp[size_t(gi) * n + gj] = T(2.0 * (kv - mean));
      } else {
        v = ws[0] * a.psi_s[ps[0]] + ws[1] * a.psi_s[ps[1]] + ws[2] * a.psi_s[ps[2]] +
            ws[3] * a.psi_s[ps[3]];
      }
    }
    shu[idx] = v;
  }
  __syncthreads();
  // ghost cells of the region (on the patch boundary); only blocks at the
  // patch faces have any
  if (i0 == -1 || j0 == -1 || i0 + TILE + 1 == n || j0 + TILE + 1 == n) {
    for (int idx = threadIdx.x; idx < 4 * RR; idx += blockDim.x) {
      // the region's outer ring: rows 0 and RR-1, then columns 0 and RR-1
      const int side = idx / RR, r = idx % RR;
      const int li = side == 0 ? 0 : side == 1 ? RR - 1 : r;
      const int lj = side == 2 ? 0 : side == 3 ? RR - 1 : r;
      if (side >= 2 && (r == 0 || r == RR - 1)) continue;  // corners once
      const int gi = i0 + li, gj = j0 + lj;
      const bool gI = gi == -1 || gi == n, gJ = gj == -1 || gj == n;
      if (!(gI || gJ)) continue;
      double thp, php;
      int ai = li, aj = lj;  // adjacent interior cell
      if (gI) { thp = gi < 0 ? th0 : th0 + a.L; ai = gi < 0 ? li + 1 : li - 1; }
      else    { thp = th0 + (gi + 0.5) * a.delta; }
      if (gJ) { php = gj < 0 ? ph0 : ph0 + a.L; aj = gj < 0 ? lj + 1 : lj - 1; }
      else    { php = ph0 + (gj + 0.5) * a.delta; }
      double st, ct, sp, cp, z, rho, dph;
      sincos(thp, &st, &ct);
      sincos(php, &sp, &cp);
      patch_dir(R, st, ct, sp, cp, pr.c, pr.s, z, rho, dph);
      const double b = hpx::interp_t(rs, a.psi_s, z, rho, dph);
      shu[li * RR + lj] = 2.0 * b - shu[ai * RR + aj];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    // write u0: the tile's cells, plus the patch ghosts beside this tile
    const bool own_i = (li >= 1 && li <= TILE) || (gi == -1) || (gi == n);
    const bool own_j = (lj >= 1 && lj <= TILE) || (gj == -1) || (gj == n);
    if (own_i && own_j) u0[size_t(gi + 1) * G + (gj + 1)] = shu[idx];
    if (!(li >= 1 && li <= TILE && lj >= 1 && lj <= TILE)) continue;
    const double* c = a.coef + 4 * gi;
    const double u = shu[idx];
    const double Lu = (c[0] * (shu[idx - RR] - u) + c[1] * (shu[idx + RR] - u) +
                       (shu[idx - 1] - 2.0 * u + shu[idx + 1]) / c[2]) / c[3];
    T* fo = fp + size_t(gi) * n + gj;
    *fo = T(double(*fo) - Lu);
  }
}

// One block per TILE x TILE tile (TILE = 64, or the whole patch if smaller),
// sin/cos of theta' and phi' tabulated per row and column.  The block first
// bounds cos(theta) over its region, takes the region centre's azimuth as
// reference and copies the rings of both grids that can bracket the region
// into LDS.
template <typename T, int TILE>
__global__ __launch_bounds__(kSetupBlock) void k_patch_setup(SetupArgs a) {
  constexpr int RR = TILE + 2;
  __shared__ double shu[RR * RR];
  __shared__ double trig[4 * RR];  // sin/cos th'_row, ph'_col
  __shared__ RingStore<kRingCapF> ringf;
  __shared__ RingStore<kRingCapS> rings;
  __shared__ double zred[2 * (kSetupBlock / 64)];
  __shared__ PhiRef pref;
  __shared__ int rng[5];
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int ti = tt / a.ntile, tj = tt % a.ntile;
  const int i0 = ti * TILE - 1, j0 = tj * TILE - 1;
  const double* R = a.rot + 9 * patch;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  for (int r = threadIdx.x; r < RR; r += blockDim.x) {
    sincos(th0 + (i0 + r + 0.5) * a.delta, &trig[4 * r], &trig[4 * r + 1]);
    sincos(ph0 + (j0 + r + 0.5) * a.delta, &trig[4 * r + 2], &trig[4 * r + 3]);
  }
  __syncthreads();
  // z range of the region's cell centres; every point interpolated lies
  // within half a cell of one of them
  double zlo = 2.0, zhi = -2.0;
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const double st = trig[4 * li], ct = trig[4 * li + 1];
    const double z = R[2] * st * trig[4 * lj + 3] + R[5] * st * trig[4 * lj + 2] + R[8] * ct;
    zlo = fmin(zlo, z);
    zhi = fmax(zhi, z);
  }
  for (int o = 32; o >= 1; o >>= 1) {
    zlo = fmin(zlo, __shfl_xor(zlo, o));
    zhi = fmax(zhi, __shfl_xor(zhi, o));
  }
  if ((threadIdx.x & 63) == 0) {
    zred[2 * (threadIdx.x >> 6)] = zlo;
    zred[2 * (threadIdx.x >> 6) + 1] = zhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSetupBlock / 64; ++w) {
      zlo = fmin(zlo, zred[2 * w]);
      zhi = fmax(zhi, zred[2 * w + 1]);
    }
    const double lo = zlo - a.delta, hi = zhi + a.delta;
    const hpx::GlobalRingTab gs{a.rs, 0.0}, gf{a.rf, 0.0};
    const int bs = max(0, hpx::ring_above(gs, hi));
    const int ts = min(a.rs.nring - 1, hpx::ring_above(gs, lo) + 1);
    const int bf = max(0, hpx::ring_above(gf, hi));
    const int tf = min(a.rf.nring - 1, hpx::ring_above(gf, lo) + 1);
    rng[0] = bs; rng[1] = ts; rng[2] = bf; rng[3] = tf;
    rng[4] = (ts - bs + 1 <= kRingCapS) && (tf - bf + 1 <= kRingCapF);
    // reference azimuth: the region centre's, in [0, 2 pi)
    double sc, cc, sp, cp;
    sincos(th0 + (i0 + 0.5 * RR) * a.delta, &sc, &cc);
    sincos(ph0 + (j0 + 0.5 * RR) * a.delta, &sp, &cp);
    const double x = sc * cp, y = sc * sp;
    const double vx = R[0] * x + R[3] * y + R[6] * cc;
    const double vy = R[1] * x + R[4] * y + R[7] * cc;
    const double rc = sqrt(vx * vx + vy * vy);
    if (rc > 1e-12) {
      double ph = atan2(vy, vx);
      if (ph < 0) ph += 2.0 * kPi;
      pref.phi = ph;
      pref.c = vx / rc;
      pref.s = vy / rc;
    } else {
      pref.phi = 0.0;
      pref.c = 1.0;
      pref.s = 0.0;
    }
  }
  __syncthreads();
  const PhiRef pr = pref;
  if (rng[4]) {
    hpx::LdsRingTab ts = rings.tab(), tf = ringf.tab();
    ts.fill(a.rs, rng[0], rng[1], pr.phi);
    tf.fill(a.rf, rng[2], rng[3], pr.phi);
    __syncthreads();
    setup_passes<T, TILE>(a, ts, tf, shu, trig, R, pr, patch, i0, j0);
  } else {
    setup_passes<T, TILE>(a, hpx::GlobalRingTab{a.rs, pr.phi}, hpx::GlobalRingTab{a.rf, pr.phi},
                          shu, trig, R, pr, patch, i0, j0);
  }
}

// ------------------------------------------------------------ tile kernels
// A 64 x 64 tile plus an even halo of HH cells per side is processed by one
// workgroup.  The region is cut into 2 x 2 quads aligned with the cells of
// the next coarser level; each thread owns up to IT quads and keeps their
// four u values and four sources f in registers.  u is mirrored in LDS,
// columns split by parity (row stride Q) so that neighbouring quads of a
// row sit at consecutive LDS addresses.  A red-black half sweep updates the
// two cells of a quad that have the sweep's colour; their in-quad neighbours
// come from registers, the others from LDS.  Cells outside the patch are
// zero and never updated; a neighbour across the patch face is accounted
// for in the diagonal (zero face value).
constexpr int kTileBlock = 512;

template <typename T>
struct TileArgs {
  int n, ntile, nu;
  const double* coef;   // this level's rows
  const T* u_in;        // level iterate in (nullptr: zero), or ubar (level >= 1 pre)
  const T* f_in;        // source f (level 0 pre, all post), or rbar (level >= 1 pre)
  T* u_out;
  T* f_out;             // level >= 1 pre: the formed source
  T* ubar_out;          // pre: restricted iterate for the next level
  T* rbar_out;          // pre: restricted residual
  const T* uc;          // post: coarse result u_H
  const T* ubarc;       // post: coarse ubar
  int fas_source;       // pre on level >= 1: f = L u_in + f_in
};

template <typename T, int HH>
struct QT {
  static_assert(HH % 2 == 0, "quads must align with the coarse level");
  static constexpr int RR = kTile + 2 * HH;    // region side
  static constexpr int Q = RR / 2;             // quads per side
  static constexpr int NQ = Q * Q;
  static constexpr int IT = (NQ + kTileBlock - 1) / kTileBlock;
  static constexpr int QH = HH / 2;            // first interior quad
};

// Two adjacent cells of a row (even column, so the pair is aligned).
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ void load2(const T* p, T& a, T& b) {
  const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type*>(p);
  a = v.x;
  b = v.y;
}

template <typename T>
__device__ __forceinline__ void store2(T* p, T a, T b) {
  typename Vec2<T>::type v;
  v.x = a;
  v.y = b;
  *reinterpret_cast<typename Vec2<T>::type*>(p) = v;
}

template <typename T, int RR>
struct QLds {
  T uE[RR * (RR / 2)], uO[RR * (RR / 2)];
  T sm[RR], sp[RR], isc[RR], A[RR], rD[RR];
};

template <typename T, int RR>
__device__ __forceinline__ T& qcell(QLds<T, RR>& t, int li, int lj) {
  return ((lj & 1) ? t.uO : t.uE)[li * (RR / 2) + (lj >> 1)];
}

template <typename T, int RR>
__device__ __forceinline__ void qload_rows(QLds<T, RR>& t, const double* coef, int n, int i0) {
  for (int r = threadIdx.x; r < RR; r += kTileBlock) {
    const int gi = i0 + r;
    T sm = T(0), sp = T(0), isc = T(0), A = T(1), rD = T(0);
    if (gi >= 0 && gi < n) {
      const double* c = coef + 4 * gi;
      sm = T(c[0]);
      sp = T(c[1]);
      isc = T(1.0 / c[2]);
      A = T(c[3]);
      rD = T(1.0 / (c[0] + c[1] + 2.0 / c[2]));
    }
    t.sm[r] = sm; t.sp[r] = sp; t.isc[r] = isc; t.A[r] = A; t.rD[r] = rD;
  }
}

// Quad-owning thread state.
template <typename T, int IT>
struct QRegs {
  T u[IT][4];   // (a, b) -> 2a + b
  T f[IT][4];
};

// Load u (registers and LDS) and f (registers) of the owned quads.
template <typename T, int HH>
__device__ __forceinline__ void qload(QLds<T, QT<T, HH>::RR>& t, QRegs<T, QT<T, HH>::IT>& r,
                                      const T* u_in, const T* f_in, size_t pbase, int n,
                                      int i0, int j0) {
  using G = QT<T, HH>;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const int q = threadIdx.x + it * kTileBlock;
    const int qi = q / G::Q, qj = q - qi * G::Q;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int gi = i0 + 2 * qi + a, gj = j0 + 2 * qj;
      const bool in = q < G::NQ && gi >= 0 && gi < n && gj >= 0 && gj < n;
      T u0 = T(0), u1 = T(0), f0 = T(0), f1 = T(0);
      if (in) {
        const size_t g = pbase + size_t(gi) * n + gj;
        if (u_in) load2(u_in + g, u0, u1);
        load2(f_in + g, f0, f1);
      }
      r.u[it][2 * a] = u0; r.u[it][2 * a + 1] = u1;
      r.f[it][2 * a] = f0; r.f[it][2 * a + 1] = f1;
      if (q < G::NQ) {
        const int li = 2 * qi + a;
        t.uE[li * G::Q + qj] = u0;
        t.uO[li * G::Q + qj] = u1;
      }
    }
  }
}

// (L u) at cell (a, b) of quad (qi, qj): in-quad neighbours from registers,
// the others from LDS; zero face value across the patch boundary.
template <typename T, int HH>
__device__ __forceinline__ T qlap(QLds<T, QT<T, HH>::RR>& t, const T* u4, int qi, int qj, int a,
                                  int b, int i0, int j0, int n) {
  constexpr int RR = QT<T, HH>::RR;
  const int li = 2 * qi + a, lj = 2 * qj + b;
  const int gi = i0 + li, gj = j0 + lj;
  const T c = u4[2 * a + b];
  T up = a ? u4[b] : (li > 0 ? qcell(t, li - 1, lj) : T(0));
  T dn = a ? (li < RR - 1 ? qcell(t, li + 1, lj) : T(0)) : u4[2 + b];
  T lf = b ? u4[2 * a] : (lj > 0 ? qcell(t, li, lj - 1) : T(0));
  T rt = b ? (lj < RR - 1 ? qcell(t, li, lj + 1) : T(0)) : u4[2 * a + 1];
  if (gi == 0) up = -c;
  if (gi == n - 1) dn = -c;
  if (gj == 0) lf = -c;
  if (gj == n - 1) rt = -c;
  return (t.sm[li] * (up - c) + t.sp[li] * (dn - c) + (lf - T(2) * c + rt) * t.isc[li]) / t.A[li];
}

// Red-black half sweep: the two cells of colour `color` in every owned quad
// (i0, j0 even, so the colour of (a, b) is (a + b) % 2).
template <typename T, int HH>
__device__ __forceinline__ void qsweep(QLds<T, QT<T, HH>::RR>& t, QRegs<T, QT<T, HH>::IT>& r,
                                       int color, int i0, int j0, int n) {
  using G = QT<T, HH>;
  constexpr int RR = G::RR;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const int q = threadIdx.x + it * kTileBlock;
    if (q >= G::NQ) continue;
    const int qi = q / G::Q, qj = q - qi * G::Q;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int a = s, b = (color + s) & 1;   // (0, color) and (1, 1 - color)
      const int li = 2 * qi + a, lj = 2 * qj + b;
      if (li == 0 || li == RR - 1 || lj == 0 || lj == RR - 1) continue;
      const int gi = i0 + li, gj = j0 + lj;
      if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
      T* u4 = r.u[it];
      const T up = a ? u4[b] : qcell(t, li - 1, lj);
      const T dn = a ? qcell(t, li + 1, lj) : u4[2 + b];
      const T lf = b ? u4[2 * a] : qcell(t, li, lj - 1);
      const T rt = b ? qcell(t, li, lj + 1) : u4[2 * a + 1];
      const T sm = t.sm[li], sp = t.sp[li], isc = t.isc[li];
      const T num = sm * up + sp * dn + isc * (lf + rt) - t.A[li] * r.f[it][2 * a + b];
      T v;
      if (gi == 0 || gi == n - 1 || gj == 0 || gj == n - 1) {
        T diag = sm + sp + T(2) * isc;
        if (gi == 0) diag += sm;
        if (gi == n - 1) diag += sp;
        if (gj == 0) diag += isc;
        if (gj == n - 1) diag += isc;
        v = num / diag;
      } else {
        v = num * t.rD[li];
      }
      u4[2 * a + b] = v;
      qcell(t, li, lj) = v;
    }
  }
}

template <typename T, int HH>
__global__ __launch_bounds__(kTileBlock) void k_mg_pre(TileArgs<T> a) {
  using G = QT<T, HH>;
  __shared__ QLds<T, G::RR> t;
  QRegs<T, G::IT> r;
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int i0 = (tt / a.ntile) * kTile - HH, j0 = (tt % a.ntile) * kTile - HH;
  const int n = a.n;
  const size_t pbase = size_t(patch) * n * n;
  qload_rows(t, a.coef, n, i0);
  qload<T, HH>(t, r, a.u_in, a.f_in, pbase, n, i0, j0);
  __syncthreads();
  if (a.fas_source) {
    // f = L_H ubar + rbar on the in-patch cells away from the region edge
#pragma unroll
    for (int it = 0; it < G::IT; ++it) {
      const int q = threadIdx.x + it * kTileBlock;
      if (q >= G::NQ) continue;
      const int qi = q / G::Q, qj = q - qi * G::Q;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int li = 2 * qi + (c >> 1), lj = 2 * qj + (c & 1);
        const int gi = i0 + li, gj = j0 + lj;
        if (li >= 1 && li <= G::RR - 2 && lj >= 1 && lj <= G::RR - 2 && gi >= 0 && gi < n &&
            gj >= 0 && gj < n)
          r.f[it][c] += qlap<T, HH>(t, r.u[it], qi, qj, c >> 1, c & 1, i0, j0, n);
      }
    }
  }
  for (int s = 0; s < a.nu; ++s) {
    qsweep<T, HH>(t, r, 0, i0, j0, n);
    __syncthreads();
    qsweep<T, HH>(t, r, 1, i0, j0, n);
    __syncthreads();
  }
  // interior quads: store u (and f), residual, area-weighted restriction
  const int nc = n / 2;
  const size_t cbase = size_t(patch) * nc * nc;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const int q = threadIdx.x + it * kTileBlock;
    const int qi = q / G::Q, qj = q - qi * G::Q;
    if (q >= G::NQ || qi < G::QH || qi >= G::QH + kTile / 2 || qj < G::QH ||
        qj >= G::QH + kTile / 2)
      continue;
    const int gi = i0 + 2 * qi, gj = j0 + 2 * qj;
    const size_t g = pbase + size_t(gi) * n + gj;
    store2(a.u_out + g, r.u[it][0], r.u[it][1]);
    store2(a.u_out + g + n, r.u[it][2], r.u[it][3]);
    if (a.fas_source) {
      store2(a.f_out + g, r.f[it][0], r.f[it][1]);
      store2(a.f_out + g + n, r.f[it][2], r.f[it][3]);
    }
    T res[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      res[c] = r.f[it][c] - qlap<T, HH>(t, r.u[it], qi, qj, c >> 1, c & 1, i0, j0, n);
    const int li = 2 * qi;
    const T a0 = t.A[li], a1 = t.A[li + 1];
    const T den = T(2) * (a0 + a1);
    const size_t gc = cbase + size_t(gi / 2) * nc + gj / 2;
    a.ubar_out[gc] = (a0 * (r.u[it][0] + r.u[it][1]) + a1 * (r.u[it][2] + r.u[it][3])) / den;
    a.rbar_out[gc] = (a0 * (res[0] + res[1]) + a1 * (res[2] + res[3])) / den;
  }
}

// Coarse correction e = u_H - ubar prolonged to a fine cell: bilinear
// (9, 3, 3, 1)/16 of the parent and its neighbours toward the child, direct
// injection of the parent on the outermost fine ring.
template <typename T, typename EF>
__device__ __forceinline__ T prolong_cell(int gi, int gj, int n, EF e) {
  const int I = gi >> 1, J = gj >> 1;
  if (gi == 0 || gi == n - 1 || gj == 0 || gj == n - 1) return e(I, J);
  const int di = (gi & 1) ? 1 : -1, dj = (gj & 1) ? 1 : -1;
  return (T(9) * e(I, J) + T(3) * e(I + di, J) + T(3) * e(I, J + dj) + e(I + di, J + dj)) /
         T(16);
}

template <typename T, int HH>
__global__ __launch_bounds__(kTileBlock) void k_mg_post(TileArgs<T> a) {
  using G = QT<T, HH>;
  constexpr int CR = G::Q + 2;  // coarse cells covering the region quads +- 1
  __shared__ QLds<T, G::RR> t;
  __shared__ T e[CR * CR];
  QRegs<T, G::IT> r;
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int i0 = (tt / a.ntile) * kTile - HH, j0 = (tt % a.ntile) * kTile - HH;
  const int n = a.n, nc = n / 2;
  const size_t pbase = size_t(patch) * n * n, cbase = size_t(patch) * nc * nc;
  const int ci0 = i0 / 2 - 1, cj0 = j0 / 2 - 1;  // i0, j0 even
  qload_rows(t, a.coef, n, i0);
  qload<T, HH>(t, r, a.u_in, a.f_in, pbase, n, i0, j0);
  for (int item = threadIdx.x; item < CR * CR; item += kTileBlock) {
    const int I = ci0 + item / CR, J = cj0 + item % CR;
    T v = T(0);
    if (I >= 0 && I < nc && J >= 0 && J < nc) {
      const size_t g = cbase + size_t(I) * nc + J;
      v = a.uc[g] - a.ubarc[g];
    }
    e[item] = v;
  }
  __syncthreads();
  auto ef = [&](int I, int J) { return e[(I - ci0) * CR + (J - cj0)]; };
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const int q = threadIdx.x + it * kTileBlock;
    if (q >= G::NQ) continue;
    const int qi = q / G::Q, qj = q - qi * G::Q;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int li = 2 * qi + (c >> 1), lj = 2 * qj + (c & 1);
      const int gi = i0 + li, gj = j0 + lj;
      if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
      r.u[it][c] += prolong_cell<T>(gi, gj, n, ef);
      qcell(t, li, lj) = r.u[it][c];
    }
  }
  __syncthreads();
  for (int s = 0; s < a.nu; ++s) {
    qsweep<T, HH>(t, r, 0, i0, j0, n);
    __syncthreads();
    qsweep<T, HH>(t, r, 1, i0, j0, n);
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const int q = threadIdx.x + it * kTileBlock;
    const int qi = q / G::Q, qj = q - qi * G::Q;
    if (q >= G::NQ || qi < G::QH || qi >= G::QH + kTile / 2 || qj < G::QH ||
        qj >= G::QH + kTile / 2)
      continue;
    const size_t g = pbase + size_t(i0 + 2 * qi) * n + (j0 + 2 * qj);
    store2(a.u_out + g, r.u[it][0], r.u[it][1]);
    store2(a.u_out + g + n, r.u[it][2], r.u[it][3]);
  }
}

// ------------------------------------------------------------ LDS levels
// One workgroup per patch runs the V-cycle below level K entirely in LDS:
// per level l: u, f (and ubar for l > K) as row-major n_l x n_l arrays, and
// the level's row coefficients (s_m, s_p, 1/s_c, area, interior 1/diag).
struct LdsLevels {
  int K, nlev, n0;        // first level handled here, number of levels, its size
  size_t crow[16];        // coefficient row offsets per level (absolute level index)
};

template <typename T>
struct LdsArgs {
  LdsLevels lv;
  int nu1, nu2;
  const double* coef;
  const double* cinv;     // 16 x 16 inverse of the coarsest operator
  const T* u_in;          // K = 0: du (nullptr = zero); K > 0: ubar_K
  const T* f_in;          // K = 0: f'; K > 0: rbar_K
  T* u_out;
  int fas_source;
};

template <typename T>
struct LRows {
  const T* sm;
  const T* sp;
  const T* isc;
  const T* A;
  const T* rD;
};

// (L u)_ij, zero face value across the patch boundary.
template <typename T>
__device__ __forceinline__ T lap_g(const T* u, int n, int i, int j, const LRows<T>& r) {
  const T uc = u[i * n + j];
  const T up = i > 0 ? u[(i - 1) * n + j] : -uc;
  const T dn = i < n - 1 ? u[(i + 1) * n + j] : -uc;
  const T lf = j > 0 ? u[i * n + j - 1] : -uc;
  const T rt = j < n - 1 ? u[i * n + j + 1] : -uc;
  return (r.sm[i] * (up - uc) + r.sp[i] * (dn - uc) + (lf - T(2) * uc + rt) * r.isc[i]) / r.A[i];
}

template <typename T>
__device__ void lds_smooth(T* u, const T* f, int n, int lg, const LRows<T>& r, int sweeps) {
  const int half = n >> 1;
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      for (int idx = threadIdx.x; idx < n * half; idx += kBlock) {
        const int i = idx >> (lg - 1);
        const int j = 2 * (idx & (half - 1)) + ((color + i) & 1);
        const T sm = r.sm[i], sp = r.sp[i], isc = r.isc[i];
        T num = -r.A[i] * f[i * n + j];
        T lr = T(0);
        bool edge = false;
        if (i > 0) num += sm * u[(i - 1) * n + j]; else edge = true;
        if (i < n - 1) num += sp * u[(i + 1) * n + j]; else edge = true;
        if (j > 0) lr += u[i * n + j - 1]; else edge = true;
        if (j < n - 1) lr += u[i * n + j + 1]; else edge = true;
        num += lr * isc;
        if (edge) {
          T diag = sm + sp + T(2) * isc;
          if (i == 0) diag += sm;
          if (i == n - 1) diag += sp;
          if (j == 0) diag += isc;
          if (j == n - 1) diag += isc;
          u[i * n + j] = num / diag;
        } else {
          u[i * n + j] = num * r.rD[i];
        }
      }
      __syncthreads();
    }
  }
}

// Pointers of level l inside the LDS block (levels K .. l-1 precede it).
template <typename T>
struct LLevel {
  T* u;
  T* f;
  T* b;
  LRows<T> r;
};

template <typename T>
__device__ __forceinline__ LLevel<T> lds_level(unsigned char* smem, int K, int n0, int l) {
  T* q = reinterpret_cast<T*>(smem);
  for (int k = K; k < l; ++k) {
    const int nn = n0 >> (k - K);
    q += nn * nn * (k > K ? 3 : 2) + 5 * nn;
  }
  const int nn = n0 >> (l - K);
  LLevel<T> v;
  v.u = q;
  v.f = q + nn * nn;
  v.b = l > K ? q + 2 * nn * nn : nullptr;
  T* rows = q + nn * nn * (l > K ? 3 : 2);
  v.r = LRows<T>{rows, rows + nn, rows + 2 * nn, rows + 3 * nn, rows + 4 * nn};
  return v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_lds(LdsArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int64_t patch = xcd_block();
  const int K = a.lv.K, nl = a.lv.nlev, n0 = a.lv.n0;
  for (int l = K; l < nl; ++l) {
    const int nn = n0 >> (l - K);
    const LLevel<T> L = lds_level<T>(smem, K, n0, l);
    T* rows = const_cast<T*>(L.r.sm);
    for (int i = threadIdx.x; i < nn; i += kBlock) {
      const double* c = a.coef + a.lv.crow[l] + 4 * i;
      rows[i] = T(c[0]);
      rows[nn + i] = T(c[1]);
      rows[2 * nn + i] = T(1.0 / c[2]);
      rows[3 * nn + i] = T(c[3]);
      rows[4 * nn + i] = T(1.0 / (c[0] + c[1] + 2.0 / c[2]));
    }
  }
  int lg0 = 0;
  while ((1 << lg0) < n0) ++lg0;
  const size_t g0 = size_t(patch) * n0 * n0;
  {
    const LLevel<T> L = lds_level<T>(smem, K, n0, K);
    for (int idx = threadIdx.x; idx < n0 * n0; idx += kBlock) {
      L.u[idx] = a.u_in ? a.u_in[g0 + idx] : T(0);
      L.f[idx] = a.f_in[g0 + idx];
    }
    __syncthreads();
    if (a.fas_source) {
      // f = L ubar + rbar (reads u only, writes f only)
      for (int idx = threadIdx.x; idx < n0 * n0; idx += kBlock)
        L.f[idx] += lap_g(L.u, n0, idx >> lg0, idx & (n0 - 1), L.r);
      __syncthreads();
    }
  }
  // down
  for (int l = K; l < nl - 1; ++l) {
    const int lg = lg0 - (l - K);
    const int nn = 1 << lg, nc = nn >> 1;
    const LLevel<T> L = lds_level<T>(smem, K, n0, l);
    const LLevel<T> C = lds_level<T>(smem, K, n0, l + 1);
    lds_smooth(L.u, L.f, nn, lg, L.r, a.nu1);
    for (int idx = threadIdx.x; idx < nc * nc; idx += kBlock) {
      const int I = idx >> (lg - 1), J = idx & (nc - 1);
      T r[4], uu[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = 2 * I + (k >> 1), j = 2 * J + (k & 1);
        uu[k] = L.u[i * nn + j];
        r[k] = L.f[i * nn + j] - lap_g(L.u, nn, i, j, L.r);
      }
      const T a0 = L.r.A[2 * I], a1 = L.r.A[2 * I + 1];
      const T den = T(2) * (a0 + a1);
      const T ub = (a0 * (uu[0] + uu[1]) + a1 * (uu[2] + uu[3])) / den;
      C.b[idx] = ub;
      C.u[idx] = ub;
      C.f[idx] = (a0 * (r[0] + r[1]) + a1 * (r[2] + r[3])) / den;
    }
    __syncthreads();
    // f_H = L_H ubar + rbar
    for (int idx = threadIdx.x; idx < nc * nc; idx += kBlock)
      C.f[idx] += lap_g(C.u, nc, idx >> (lg - 1), idx & (nc - 1), C.r);
    __syncthreads();
  }
  // coarsest: exact solve (float64)
  {
    const LLevel<T> L = lds_level<T>(smem, K, n0, nl - 1);
    double v = 0.0;
    if (threadIdx.x < 16) {
      for (int k = 0; k < 16; ++k) v += a.cinv[threadIdx.x * 16 + k] * double(L.f[k]);
    }
    __syncthreads();
    if (threadIdx.x < 16) L.u[threadIdx.x] = T(v);
    __syncthreads();
  }
  // up
  for (int l = nl - 2; l >= K; --l) {
    const int lg = lg0 - (l - K);
    const int nn = 1 << lg, nc = nn >> 1;
    const LLevel<T> L = lds_level<T>(smem, K, n0, l);
    const LLevel<T> C = lds_level<T>(smem, K, n0, l + 1);
    auto ef = [&](int I, int J) { return C.u[I * nc + J] - C.b[I * nc + J]; };
    for (int idx = threadIdx.x; idx < nn * nn; idx += kBlock)
      L.u[idx] += prolong_cell<T>(idx >> lg, idx & (nn - 1), nn, ef);
    __syncthreads();
    lds_smooth(L.u, L.f, nn, lg, L.r, a.nu2);
  }
  {
    const LLevel<T> L = lds_level<T>(smem, K, n0, K);
    for (int idx = threadIdx.x; idx < n0 * n0; idx += kBlock) a.u_out[g0 + idx] = L.u[idx];
  }
}

// ------------------------------------------------------------ potential out
template <typename T>
__global__ void k_potential(const double* u0, const T* du, int n, int64_t first, int64_t np,
                            double* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(n) * n;
  if (i >= np * per) return;
  const int64_t pp = first + i / per;
  const int c = int(i % per), ci = c / n, cj = c % n;
  out[i] = u0[pp * (n + 2) * (n + 2) + (ci + 1) * (n + 2) + cj + 1] + double(du[pp * per + c]);
}

template <typename K>
clm_status allow_lds(Plan* p, K kernel, size_t bytes) {
  if (bytes > 65536)
    CLM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  return CLM_OK;
}

// Tile kernels are compiled per halo width: pre-smoothing needs 2 nu + 1
// cells (nu sweeps plus the residual), post-smoothing 2 nu.
template <typename T, int HH, bool PRE>
clm_status launch_tile_hh(Plan* p, const TileArgs<T>& a, int64_t np, hipStream_t s) {
  constexpr int RR = kTile + 2 * HH;
  const dim3 grid(unsigned(np * a.ntile * a.ntile));
  (void)RR;
  if (PRE)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_pre<T, HH>), grid, dim3(kTileBlock), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_post<T, HH>), grid, dim3(kTileBlock), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

template <typename T, bool PRE>
clm_status launch_tile(Plan* p, const TileArgs<T>& a, int64_t np, hipStream_t s) {
  // halo: 2 nu + 1 (pre: sweeps plus the residual) or 2 nu (post), rounded
  // up to even so that quads align with the coarse cells
  const int hh = PRE ? 2 * a.nu + 2 : 2 * a.nu;
  switch (hh) {
    case 2: return launch_tile_hh<T, 2, PRE>(p, a, np, s);
    case 4: return launch_tile_hh<T, 4, PRE>(p, a, np, s);
    case 6: return launch_tile_hh<T, 6, PRE>(p, a, np, s);
    case 8: return launch_tile_hh<T, 8, PRE>(p, a, np, s);
    case 10: return launch_tile_hh<T, 10, PRE>(p, a, np, s);
  }
  return fail(p, CLM_EUNSUPPORTED, "sweep count outside 1..4");
}

template <typename T>
clm_status run_mg(Plan* p, const void* kappa, int kappa_fp64, int slot, hipStream_t s) {
  const clm_plan_desc& d = p->d;
  Slot& sl = p->slots[slot];
  const int n = p->n;
  const int64_t np = p->nbundle;
  // patch setup
  {
    SetupArgs a;
    a.n = n;
    a.tile = n < kTile ? n : kTile;
    a.ntile = n / a.tile;
    a.L = p->L;
    a.delta = p->delta;
    a.rot = p->rot;
    a.coef = p->coef + p->lev[0].crow;
    a.rs = hpx::Rings{p->ring_s, p->ringi_s, p->ringx_s, p->nring_s, d.nside_sht};
    a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, d.nside_fine};
    a.psi_s = sl.psi_s;
    a.kappa = kappa;
    a.kappa_fp64 = kappa_fp64;
    a.red = p->red;
    a.u0 = sl.u0;
    a.fprime = p->fprime;
    const dim3 grid(unsigned(np * a.ntile * a.ntile));
    {
      CLM_TIMED(p, s, "patch_setup");
      switch (a.tile) {
        case 64: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_setup<T, 64>), grid, dim3(kSetupBlock), 0, s, a); break;
        case 32: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_setup<T, 32>), grid, dim3(kSetupBlock), 0, s, a); break;
        case 16: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_setup<T, 16>), grid, dim3(kSetupBlock), 0, s, a); break;
        default: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_setup<T, 8>), grid, dim3(kSetupBlock), 0, s, a); break;
      }
    }
    CLM_LAUNCH_CHECK();
  }
  T* du = static_cast<T*>(sl.du);
  T* dt = static_cast<T*>(p->dutmp);
  const T* fp = static_cast<const T*>(p->fprime);
  const int K = p->ktile;

  LdsArgs<T> la{};
  la.lv.K = K;
  la.lv.nlev = p->nlev;
  la.lv.n0 = n >> K;
  for (int l = 0; l < p->nlev && l < 16; ++l) la.lv.crow[l] = p->lev[l].crow;
  la.nu1 = d.nu_pre;
  la.nu2 = d.nu_post;
  la.coef = p->coef;
  la.cinv = p->cinv;
  size_t lds_elems = 0;
  for (int l = K; l < p->nlev; ++l) {
    const size_t nn = size_t(n >> l);
    lds_elems += nn * nn * (l > K ? 3 : 2) + 5 * nn;
  }
  const size_t lds_bytes = lds_elems * sizeof(T);
  if (allow_lds(p, k_mg_lds<T>, lds_bytes) != CLM_OK) return CLM_EHIP;

  auto tile_args = [&](int l, bool pre) {
    TileArgs<T> a{};
    a.n = n >> l;
    a.ntile = a.n / kTile;
    a.nu = pre ? d.nu_pre : d.nu_post;
    a.coef = p->coef + p->lev[l].crow;
    return a;
  };
  for (int cyc = 0; cyc < d.mg_vcycles; ++cyc) {
    const bool first = cyc == 0;
    if (K == 0) {
      la.u_in = first ? nullptr : du;
      la.f_in = fp;
      la.u_out = du;
      la.fas_source = 0;
      {
        CLM_TIMED(p, s, "mg_lds");
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_lds<T>), dim3(np), dim3(kBlock), lds_bytes, s,
                           la);
      }
      CLM_LAUNCH_CHECK();
      continue;
    }
    // pre-smoothing, residual and restriction on the tile levels
    for (int l = 0; l < K; ++l) {
      TileArgs<T> a = tile_args(l, true);
      if (l == 0) {
        a.u_in = first ? nullptr : du;
        a.f_in = fp;
        a.u_out = dt;
        a.fas_source = 0;
      } else {
        a.u_in = static_cast<T*>(p->ubar[l]);
        a.f_in = static_cast<T*>(p->rbar[l]);
        a.u_out = static_cast<T*>(p->ulev[l]);
        a.f_out = static_cast<T*>(p->flev[l]);
        a.fas_source = 1;
      }
      a.ubar_out = static_cast<T*>(p->ubar[l + 1]);
      a.rbar_out = static_cast<T*>(p->rbar[l + 1]);
      {
        CLM_TIMED(p, s, l == 0 ? "mg_pre_l0" : "mg_pre_l1+");
        const clm_status st = launch_tile<T, true>(p, a, np, s);
        if (st != CLM_OK) return st;
      }
    }
    // the LDS-resident levels
    la.u_in = static_cast<T*>(p->ubar[K]);
    la.f_in = static_cast<T*>(p->rbar[K]);
    la.u_out = static_cast<T*>(p->ulev[K]);
    la.fas_source = 1;
    {
      CLM_TIMED(p, s, "mg_lds");
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_lds<T>), dim3(np), dim3(kBlock), lds_bytes, s, la);
    }
    CLM_LAUNCH_CHECK();
    // prolongation, correction and post-smoothing back up
    for (int l = K - 1; l >= 0; --l) {
      TileArgs<T> a = tile_args(l, false);
      a.uc = static_cast<T*>(l + 1 == K ? p->ulev[K] : p->ulev2[l + 1]);
      a.ubarc = static_cast<T*>(p->ubar[l + 1]);
      if (l == 0) {
        a.u_in = dt;
        a.f_in = fp;
        a.u_out = du;
      } else {
        a.u_in = static_cast<T*>(p->ulev[l]);
        a.f_in = static_cast<T*>(p->flev[l]);
        a.u_out = static_cast<T*>(p->ulev2[l]);
      }
      {
        CLM_TIMED(p, s, l == 0 ? "mg_post_l0" : "mg_post_l1+");
        const clm_status st = launch_tile<T, false>(p, a, np, s);
        if (st != CLM_OK) return st;
      }
    }
  }
  return CLM_OK;
}

}  // namespace

clm_status mg_solve(Plan* p, const void* kappa, int kappa_fp64, int slot, hipStream_t s) {
  if (p->nlev > 16) return fail(p, CLM_EUNSUPPORTED, "too many multigrid levels");
  return p->fp64mg ? run_mg<double>(p, kappa, kappa_fp64, slot, s)
                   : run_mg<float>(p, kappa, kappa_fp64, slot, s);
}

clm_status mg_patch_potential(Plan* p, int slot, int64_t first, int64_t np, double* out,
                              hipStream_t s) {
  const int64_t total = np * p->n * p->n;
  const dim3 g((total + kBlock - 1) / kBlock);
  if (p->fp64mg)
    hipLaunchKernelGGL(k_potential<double>, g, dim3(kBlock), 0, s, p->slots[slot].u0,
                       static_cast<const double*>(p->slots[slot].du), p->n, first, np, out);
  else
    hipLaunchKernelGGL(k_potential<float>, g, dim3(kBlock), 0, s, p->slots[slot].u0,
                       static_cast<const float*>(p->slots[slot].du), p->n, first, np, out);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace clm
