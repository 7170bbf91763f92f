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
#include <algorithm>
#include <cmath>

#include "clm_internal.h"
#include "healpix_dev.h"

namespace clm {
namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

// Element i of an array whose base is the same for the whole workgroup, as
// an unsigned 32-bit byte offset (level arrays of a patch stay far below
// 2^30 elements): the access takes the base in scalar registers and one
// offset register, with no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T* at(T* base, unsigned i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * unsigned(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T* at(const T* base, unsigned i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * unsigned(sizeof(T)));
}

// ------------------------------------------------------------ patch setup
// u0 = interp(psi_SHT) at the cell centres; ghost u0 = 2 b - u0(adjacent)
// with b = interp(psi_SHT) at the face midpoint (corner: patch corner);
// f' = 2 (interp(kappa) - mean) - L u0 at the cell centres, float64.
// Geometry of one setup tile's region, fixed by the plan: the ring ranges of
// both grids that can bracket its points, whether both fit the LDS ring
// stores, and the reference azimuth (the region centre's).
struct SetupMeta {
  double phi, c, s;      // reference azimuth in [0, 2 pi), its cosine and sine
  int bs, ts, bf, tf;    // SHT-grid rings bs .. ts, fine-grid rings bf .. tf
  int lds, pad;
};
static_assert(sizeof(SetupMeta) == kSetupMetaBytes, "setup record size");

struct SetupArgs {
  int n, ntile, tile;
  int ring_shift;       // log2(nside_fine / nside_sht)
  double L, delta;
  const double* rot;
  const double* coef;  // level-0 rows
  hpx::Rings rs, rf;
  const double* psi_s;
  const void* kappa;   // fine map, or nullptr: f = -2 mean (particles add the rest)
  int kappa_fp64;
  const double* red;   // red[1023] = mean of kappa
  const double* spad;  // psi_s with padded rings (pad_s), read in the common case
  const void* kpad;    // kappa with padded rings (pad_f), its type
  int pad_s, pad_f;
  double* u0;          // [patch][(n+2)^2]
  void* fprime;        // [patch][n^2] of T
  SetupMeta* meta;     // [patch][tile]
  const int* pmap;     // partial sky: the domain's patches (nullptr: all)
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
constexpr int kRingCapF = 192, kRingCapS = 96;
constexpr int kSetupBlock = 512;
constexpr int kLdsBlock = 512;

// The setup's common case: azimuth offsets from the tile's reference
// azimuth below asin(kSetupSeries) (the series asin), so that a ring of n
// pixels is read at most asin(kSetupSeries) n / (2 pi) < 0.0319 nside pixels
// beyond either end (n <= 4 nside); setup_ring_pad covers that.
constexpr double kSetupSeries = 0.05;

// Reference azimuth of a setup block (the region centre's).
struct PhiRef {
  double phi, c, s;
};

// Pass 1 visits every cell of the tile plus one ring once: direction, u0 and
// (interior cells) the source f, kept in LDS (fsh, float32 form) or written
// to the f' array and read back by the same thread; pass 2 fills the patch
// ghosts from the face values; pass 3 forms f' = f - L u0.  The SHT grid's
// rings are the fine grid's rings ratio, 2 ratio, ... (nested HEALPix), so
// the SHT ring index follows from the fine one: floor((g_f + 1) / ratio) - 1.
// This pass 1 reads the global ring tables (regions wider than the LDS
// ring stores); setup_pass1_rec below is the LDS form.
template <typename T, int TILE, typename TS, typename TF>
__device__ void setup_pass1(const SetupArgs& a, const TS& rs, const TF& rf, double* shu,
                            T* fsh, const double* rowc, const double* colc, const double* R,
                            const PhiRef& pr, int64_t patch, int i0, int j0) {
  constexpr int RR = TILE + 2;
  const int n = a.n;
  const double mean = a.red[1023];
  T* fp = static_cast<T*>(a.fprime) + size_t(patch) * n * n;
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    double v = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      double z, rho, dph;
      patch_dir(R, rowc[12 * li + 9], rowc[12 * li + 10], colc[2 * lj + 1], colc[2 * lj], pr.c,
                pr.s, z, rho, dph);
      const int gf = hpx::ring_above(rf, z);
      const int gs = min(max(((gf + 1) >> a.ring_shift) - 1, rs.lo()), rs.hi());
      int ps[4];
      double ws[4];
      hpx::interp_weights_g(rs, gs, z, rho, dph, ps, ws);
      if (li >= 1 && li <= TILE && lj >= 1 && lj <= TILE) {
        int pf[4];
        double wf[4];
        hpx::interp_weights_g(rf, gf, z, rho, dph, pf, wf);
        double k4[4] = {0.0, 0.0, 0.0, 0.0};  // no map: the source comes from particles
        if (!a.kappa) {
        } else if (a.kappa_fp64) {
          const double* km = static_cast<const double*>(a.kappa);
          for (int c = 0; c < 4; ++c) k4[c] = km[pf[c]];
        } else {
          const float* km = static_cast<const float*>(a.kappa);
          for (int c = 0; c < 4; ++c) k4[c] = km[pf[c]];
        }
        v = ws[0] * a.psi_s[ps[0]] + ws[1] * a.psi_s[ps[1]] + ws[2] * a.psi_s[ps[2]] +
            ws[3] * a.psi_s[ps[3]];
        const double kv = wf[0] * k4[0] + wf[1] * k4[1] + wf[2] * k4[2] + wf[3] * k4[3];
        if (fsh)
          fsh[(li - 1) * TILE + (lj - 1)] = T(2.0 * (kv - mean));
        else
          fp[size_t(gi) * n + gj] = T(2.0 * (kv - mean));
      } else {
        v = ws[0] * a.psi_s[ps[0]] + ws[1] * a.psi_s[ps[1]] + ws[2] * a.psi_s[ps[2]] +
            ws[3] * a.psi_s[ps[3]];
      }
    }
    shu[idx] = v;
  }
}

// Passes 2 and 3 (after pass 1 filled shu and the sources): the patch
// ghosts from the face values, then f' = f - L u0 and the u0 writes.  prow
// holds per tile row c_minus, c_plus, 1 / s_c, 1 / area.
template <typename T, int TILE>
__device__ void setup_passes23(const SetupArgs& a, double* shu, const T* fsh,
                               const double* prow, const double* R, const PhiRef& pr,
                               int64_t patch, int i0, int j0) {
  constexpr int RR = TILE + 2;
  const int n = a.n;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  const size_t G = size_t(n + 2);
  double* u0 = a.u0 + size_t(patch) * G * G;
  T* fp = static_cast<T*>(a.fprime) + size_t(patch) * n * n;
  const hpx::GlobalRingTab rs{a.rs, pr.phi};
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
    if (own_i && own_j) *at(u0, unsigned((gi + 1) * (n + 2) + gj + 1)) = shu[idx];
    if (!(li >= 1 && li <= TILE && lj >= 1 && lj <= TILE)) continue;
    const double* q = prow + 4 * (li - 1);  // c_minus, c_plus, 1 / s_c, 1 / A of the row
    const double u = shu[idx];
    const double Lu = (q[0] * (shu[idx - RR] - u) + q[1] * (shu[idx + RR] - u) +
                       (shu[idx - 1] - 2.0 * u + shu[idx + 1]) * q[2]) * q[3];
    T* fo = at(fp, unsigned(gi * n + gj));
    const double f = fsh ? double(fsh[(li - 1) * TILE + (lj - 1)]) : double(*fo);
    *fo = T(f - Lu);
  }
}

// ---- setup with the ring stores as records (the LDS case)
// One ring of a block's LDS ring store: everything the interpolation reads
// for that ring in one 64-byte record, so each access is one base address.
struct alignas(16) SetupRing {
  double z, s;     // cos theta, sin theta
  double k, t0;    // n / (2 pi); (phi_ref - phi0) n / (2 pi)
  double gbelow;   // 1 / (theta_{q+1} - theta_q) (last ring: 1 / (pi - theta_q))
  double off;      // fine rings: theta_q - theta of the SHT ring above them
                   // (0 above the first SHT ring); 0 for SHT rings
  int n, first;    // pixels; the ring's pixel 0 in the padded map
};
static_assert(sizeof(SetupRing) == 64, "ring record size");

// Ring-table view of a record store for hpx::ring_above.
struct RecTab {
  const SetupRing* r;
  int base, top, nr, NN;
  __device__ __forceinline__ int N() const { return NN; }
  __device__ __forceinline__ double z(int q) const { return r[q - base].z; }
  __device__ __forceinline__ int qmin() const { return base; }
  __device__ __forceinline__ int qmax() const { return top; }
  __device__ __forceinline__ int lo() const { return base > 0 ? base : -1; }
  __device__ __forceinline__ int hi() const { return top == nr - 1 ? top : top - 1; }
};

// All threads of the block: rings b .. t of grid R (padded by pad pixels per
// side) into the record store; fine rings (shift >= 0) also get their offset
// to the SHT ring above, from the SHT grid's theta column rt_s.
__device__ void fill_records(SetupRing* st, const hpx::Rings& R, int b, int t, double phi_ref,
                             int shift, const double* rt_s, int pad) {
  for (int k = threadIdx.x; k <= t - b; k += blockDim.x) {
    const int q = b + k;
    SetupRing r;
    r.z = R.rt[4 * q];
    r.s = R.rt[4 * q + 1];
    r.k = R.rx[2 * q];
    r.t0 = (phi_ref - R.rt[4 * q + 3]) * R.rx[2 * q];
    r.gbelow = R.rx[2 * (q + 1) + 1];
    r.off = 0.0;
    if (shift >= 0) {
      const int gs = ((q + 1) >> shift) - 1;
      r.off = R.rt[4 * q + 2] - (gs >= 0 ? rt_s[4 * gs + 2] : 0.0);
    }
    r.n = R.ri[2 * q];
    r.first = R.ri[2 * q + 1] + (2 * q + 1) * pad;
    st[k] = r;
  }
}

// Element p of a map whose base is the same for the whole wave: the index
// enters as an unsigned 32-bit byte offset (pixel counts stay far below
// 2^28), so the load takes the uniform base in scalar registers and one
// offset register, with no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T map_at(const T* base, int p) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     unsigned(p) * unsigned(sizeof(T)));
}

// Pixels p and p + 1 of a map in one load (element alignment only).
template <typename T>
struct alignas(sizeof(T)) Pair {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Pair<T> pair_at(const T* base, int p) {
  return *reinterpret_cast<const Pair<T>*>(reinterpret_cast<const char*>(base) +
                                           unsigned(p) * unsigned(sizeof(T)));
}

// HEALPix bilinear interpolation of a ring-padded map between rings A
// (above) and B (below) at theta - theta_A = dth and azimuth offset dphi
// (|dphi| < asin kSetupSeries, which the padding covers): in each ring the
// pixels i = floor(t), i + 1 around t = (phi - phi_0) n / (2 pi), weight
// t - i on the second; along theta weight dth / (theta_B - theta_A) on ring
// B.  The same weights as the general path, in linear-interpolation form.
template <typename M>
__device__ __forceinline__ double pair_interp(const M* map, const SetupRing& A,
                                              const SetupRing& B, double dth, double dphi) {
  const double ta = fma(dphi, A.k, A.t0), tb = fma(dphi, B.k, B.t0);
  const double fa = floor(ta), fb = floor(tb);
  const Pair<M> pa = pair_at(map, A.first + int(fa));
  const Pair<M> pb = pair_at(map, B.first + int(fb));
  const double va = fma(ta - fa, double(pa.y) - double(pa.x), double(pa.x));
  const double vb = fma(tb - fb, double(pb.y) - double(pb.x), double(pb.x));
  return fma(dth * A.gbelow, vb - va, va);
}

// Pass 1 of the setup with record stores: the global direction of a cell
// from per-row coefficients (z, and the cos/sin-weighted components along
// the reference azimuth, each A + B cos phi' + C sin phi') and the column's
// cos/sin phi'; rho and 1 / rho from the hardware reciprocal square root
// refined by two Newton steps; the azimuth offset as asin(sn / rho).  The
// fine-grid theta offset comes from its upper ring, the SHT grid's from it
// plus the tabulated difference of the two rings' colatitudes.  Cells with
// an azimuth offset below asin kSetupSeries and rings in the stores (the
// common case) interpolate the ring-padded maps; the others (poles, wide
// regions) take the general path on the global tables and the plain maps.
template <typename T, int TILE>
__device__ void setup_pass1_rec(const SetupArgs& a, const SetupRing* rf, const SetupMeta& m,
                                const SetupRing* rs, double* shu, T* fsh, const double* rowc,
                                const double* colc, const PhiRef& pr, int64_t patch, int i0,
                                int j0) {
  constexpr int RR = TILE + 2;
  const int n = a.n;
  const double mean = a.red[1023];
  T* fp = static_cast<T*>(a.fprime) + size_t(patch) * n * n;
  const RecTab tf{rf, m.bf, m.tf, a.rf.nring, a.rf.N};
  const hpx::GlobalRingTab gfs{a.rf, pr.phi}, gss{a.rs, pr.phi};
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx - li * RR;
    const int gi = i0 + li, gj = j0 + lj;
    double v = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      const double* rc = rowc + 12 * li;
      const double cp = colc[2 * lj], sp = colc[2 * lj + 1];
      const double z = fma(rc[2], sp, fma(rc[1], cp, rc[0]));
      const double cs = fma(rc[5], sp, fma(rc[4], cp, rc[3]));
      const double sn = fma(rc[8], sp, fma(rc[7], cp, rc[6]));
      const double r2 = fma(cs, cs, sn * sn);
      double rho = 0.0, irho = 0.0, dphi;
      bool fast = r2 > 1e-20;
      if (fast) {
        // Goldschmidt iterations on the hardware estimate of 1 / sqrt(r2)
        const double y = __builtin_amdgcn_rsq(r2);
        double g = r2 * y, h = 0.5 * y;
        double e = fma(-g, h, 0.5);
        g = fma(g, e, g);
        h = fma(h, e, h);
        e = fma(-g, h, 0.5);
        g = fma(g, e, g);
        h = fma(h, e, h);
        rho = g;
        irho = 2.0 * h;
      } else {
        rho = sqrt(r2);
      }
      const double sd = sn * irho;
      const bool series = fast && cs > 0.0 && fabs(sd) < kSetupSeries;
      if (series) {
        dphi = hpx::asin_series(sd);
      } else {
        dphi = hpx::atan2_r(sn, cs);
        if (!fast) rho = sqrt(r2);
      }
      const int gf = hpx::ring_above(tf, z);
      const bool inner = li >= 1 && li <= TILE && lj >= 1 && lj <= TILE;
      const int gsr = ((gf + 1) >> a.ring_shift) - 1;
      double kv = 0.0;  // no map: the source comes from particles
      if (series && gf >= m.bf && gf < m.tf) {
        const SetupRing& A = rf[gf - m.bf];
        const double dthf = hpx::asin_small(fma(rho, A.z, -z * A.s));
        if (inner && a.kappa) {
          const SetupRing& B = rf[gf - m.bf + 1];
          kv = a.kappa_fp64 ? pair_interp(static_cast<const double*>(a.kpad), A, B, dthf, dphi)
                            : pair_interp(static_cast<const float*>(a.kpad), A, B, dthf, dphi);
        }
        if (gsr >= m.bs && gsr < m.ts) {
          v = pair_interp(a.spad, rs[gsr - m.bs], rs[gsr - m.bs + 1], dthf + A.off, dphi);
        } else {
          int ps[4];
          double ws[4];
          hpx::interp_weights_g(gss, min(max(gsr, -1), a.rs.nring - 1), z, rho, dphi, ps, ws);
          v = ws[0] * map_at(a.psi_s, ps[0]) + ws[1] * map_at(a.psi_s, ps[1]) +
              ws[2] * map_at(a.psi_s, ps[2]) + ws[3] * map_at(a.psi_s, ps[3]);
        }
      } else {
        int ps[4];
        double ws[4];
        if (inner && a.kappa) {
          int pf[4];
          double wf[4];
          hpx::interp_weights_g(gfs, gf, z, rho, dphi, pf, wf);
          if (a.kappa_fp64) {
            const double* km = static_cast<const double*>(a.kappa);
            kv = wf[0] * map_at(km, pf[0]) + wf[1] * map_at(km, pf[1]) +
                 wf[2] * map_at(km, pf[2]) + wf[3] * map_at(km, pf[3]);
          } else {
            const float* km = static_cast<const float*>(a.kappa);
            kv = wf[0] * double(map_at(km, pf[0])) + wf[1] * double(map_at(km, pf[1])) +
                 wf[2] * double(map_at(km, pf[2])) + wf[3] * double(map_at(km, pf[3]));
          }
        }
        hpx::interp_weights_g(gss, min(max(gsr, -1), a.rs.nring - 1), z, rho, dphi, ps, ws);
        v = ws[0] * map_at(a.psi_s, ps[0]) + ws[1] * map_at(a.psi_s, ps[1]) +
            ws[2] * map_at(a.psi_s, ps[2]) + ws[3] * map_at(a.psi_s, ps[3]);
      }
      if (inner) {
        if (fsh)
          fsh[(li - 1) * TILE + (lj - 1)] = T(2.0 * (kv - mean));
        else
          fp[size_t(gi) * n + gj] = T(2.0 * (kv - mean));
      }
    }
    shu[idx] = v;
  }
}

// The region of setup tile lb (TILE x TILE cells plus one ring) of its patch:
// patch index and the region's first cell (i0, j0).
struct SetupTile {
  int64_t patch;
  int i0, j0;
};

__device__ __forceinline__ SetupTile setup_tile(int64_t lb, int ntile, int tile) {
  const int tpp = ntile * ntile;
  const int tt = int(lb % tpp);
  return SetupTile{lb / tpp, (tt / ntile) * tile - 1, (tt % ntile) * tile - 1};
}

// Built once per plan, one block per setup tile: bound cos(theta) over the
// region, pick the rings of both grids that can bracket its points, and take
// the region centre's azimuth as reference.  z = cos(distance to the pole)
// has no extremum inside the region unless a pole lies in it (then the range
// opens up to it), so the region's boundary cells bound it to within half a
// cell (the largest gap from a boundary point to the nearest boundary
// centre); every point interpolated lies within half a cell of a cell centre.
constexpr int kMetaBlock = 256;

__global__ __launch_bounds__(kMetaBlock) void k_setup_meta(SetupArgs a) {
  __shared__ double zred[2 * (kMetaBlock / 64)];
  const int64_t lb = blockIdx.x;
  const SetupTile st = setup_tile(lb, a.ntile, a.tile);
  const int RR = a.tile + 2;
  const double* R = a.rot + 9 * st.patch;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  double zlo = 2.0, zhi = -2.0;
  for (int idx = threadIdx.x; idx < 4 * (RR - 1); idx += blockDim.x) {
    const int side = idx / (RR - 1), r = idx % (RR - 1);
    const int li = side == 0 ? 0 : side == 1 ? r : side == 2 ? RR - 1 : RR - 1 - r;
    const int lj = side == 0 ? r : side == 1 ? RR - 1 : side == 2 ? RR - 1 - r : 0;
    double s_t, c_t, s_p, c_p;
    sincos(th0 + (st.i0 + li + 0.5) * a.delta, &s_t, &c_t);
    sincos(ph0 + (st.j0 + lj + 0.5) * a.delta, &s_p, &c_p);
    const double z = R[2] * s_t * c_p + R[5] * s_t * s_p + R[8] * c_t;
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
  if (threadIdx.x != 0) return;
  for (int w = 1; w < kMetaBlock / 64; ++w) {
    zlo = fmin(zlo, zred[2 * w]);
    zhi = fmax(zhi, zred[2 * w + 1]);
  }
  // region centre; a pole closer to it than the region's side may lie in it
  double sc, cc, sp, cp;
  sincos(th0 + (st.i0 + 0.5 * RR) * a.delta, &sc, &cc);
  sincos(ph0 + (st.j0 + 0.5 * RR) * a.delta, &sp, &cp);
  const double x = sc * cp, y = sc * sp;
  const double zc = R[2] * x + R[5] * y + R[8] * cc;
  const double cr = cos(RR * a.delta);
  if (zc > cr) zhi = 1.0;
  if (zc < -cr) zlo = -1.0;
  const double lo = zlo - 2.0 * a.delta, hi = zhi + 2.0 * a.delta;
  const hpx::GlobalRingTab gs{a.rs, 0.0}, gf{a.rf, 0.0};
  SetupMeta m;
  m.bs = max(0, hpx::ring_above(gs, hi));
  m.ts = min(a.rs.nring - 1, hpx::ring_above(gs, lo) + 1);
  m.bf = max(0, hpx::ring_above(gf, hi));
  m.tf = min(a.rf.nring - 1, hpx::ring_above(gf, lo) + 1);
  m.lds = (m.ts - m.bs + 1 <= kRingCapS) && (m.tf - m.bf + 1 <= kRingCapF);
  m.pad = 0;
  // reference azimuth: the region centre's, in [0, 2 pi)
  const double vx = R[0] * x + R[3] * y + R[6] * cc;
  const double vy = R[1] * x + R[4] * y + R[7] * cc;
  const double rc = sqrt(vx * vx + vy * vy);
  if (rc > 1e-12) {
    double ph = atan2(vy, vx);
    if (ph < 0) ph += 2.0 * kPi;
    m.phi = ph;
    m.c = vx / rc;
    m.s = vy / rc;
  } else {
    m.phi = 0.0;
    m.c = 1.0;
    m.s = 0.0;
  }
  a.meta[lb] = m;
}

// One block per TILE x TILE tile (TILE = 64, or the whole patch if smaller).
// Per region row: sin/cos theta' and the coefficients of the cell direction
// in cos/sin phi'; per column cos/sin phi'.  The block copies the rings of
// both grids that its plan-time record names into LDS as ring records (or
// reads the global tables when they do not fit).
template <typename T, int TILE>
__global__ __launch_bounds__(kSetupBlock) void k_patch_setup(SetupArgs a) {
  constexpr int RR = TILE + 2;
  __shared__ double shu[RR * RR];
  __shared__ double rowc[12 * RR];   // z, cs, sn: A, B, C each; sin, cos theta'; pad
  __shared__ double colc[2 * RR];    // cos, sin phi'
  __shared__ double prow[4 * TILE];  // c_minus, c_plus, 1 / s_c, 1 / area per tile row
  __shared__ SetupRing recf[kRingCapF];
  __shared__ SetupRing recs[kRingCapS];
  __shared__ T fshm[sizeof(T) == 4 ? TILE * TILE : 1];
  T* fsh = sizeof(T) == 4 ? fshm : nullptr;
  const int64_t lc = xcd_block();
  const int64_t tpp = int64_t(a.ntile) * a.ntile;
  const int64_t lb = patch_of(a.pmap, lc / tpp) * tpp + lc % tpp;  // this tile's record
  const SetupTile st = setup_tile(lb, a.ntile, TILE);
  const int64_t patch = st.patch;
  const int i0 = st.i0, j0 = st.j0;
  const double* R = a.rot + 9 * patch;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  // a copy in registers: a reference to global memory would be reloaded
  // after every global store of the cell loop (it may alias them)
  const SetupMeta m = a.meta[lb];
  const PhiRef pr{m.phi, m.c, m.s};
  for (int r = threadIdx.x; r < RR; r += blockDim.x) {
    double s_t, c_t, s_p, c_p;
    sincos(th0 + (i0 + r + 0.5) * a.delta, &s_t, &c_t);
    sincos(ph0 + (j0 + r + 0.5) * a.delta, &s_p, &c_p);
    colc[2 * r] = c_p;
    colc[2 * r + 1] = s_p;
    // v = R^T (s_t c_p, s_t s_p, c_t); cs, sn: v_x, v_y turned by the
    // reference azimuth (cs = v_x c + v_y s, sn = v_y c - v_x s)
    double* rc = rowc + 12 * r;
    rc[0] = R[8] * c_t;
    rc[1] = R[2] * s_t;
    rc[2] = R[5] * s_t;
    rc[3] = (R[6] * pr.c + R[7] * pr.s) * c_t;
    rc[4] = (R[0] * pr.c + R[1] * pr.s) * s_t;
    rc[5] = (R[3] * pr.c + R[4] * pr.s) * s_t;
    rc[6] = (R[7] * pr.c - R[6] * pr.s) * c_t;
    rc[7] = (R[1] * pr.c - R[0] * pr.s) * s_t;
    rc[8] = (R[4] * pr.c - R[3] * pr.s) * s_t;
    rc[9] = s_t;
    rc[10] = c_t;
    rc[11] = 0.0;
  }
  for (int r = threadIdx.x; r < TILE; r += blockDim.x) {
    const double* c = a.coef + 4 * (i0 + 1 + r);
    prow[4 * r] = c[0];
    prow[4 * r + 1] = c[1];
    prow[4 * r + 2] = 1.0 / c[2];
    prow[4 * r + 3] = 1.0 / c[3];
  }
  if (m.lds) {
    fill_records(recs, a.rs, m.bs, m.ts, pr.phi, -1, nullptr, a.pad_s);
    fill_records(recf, a.rf, m.bf, m.tf, pr.phi, a.ring_shift, a.rs.rt, a.pad_f);
    __syncthreads();
    setup_pass1_rec<T, TILE>(a, recf, m, recs, shu, fsh, rowc, colc, pr, patch, i0, j0);
  } else {
    __syncthreads();
    setup_pass1<T, TILE>(a, hpx::GlobalRingTab{a.rs, pr.phi}, hpx::GlobalRingTab{a.rf, pr.phi},
                         shu, fsh, rowc, colc, R, pr, patch, i0, j0);
  }
  setup_passes23<T, TILE>(a, shu, fsh, prow, R, pr, patch, i0, j0);
}

// Ring padding of a RING-ordered map for the setup's common case: ring q
// (n pixels from first) becomes pixels -pad .. n + pad - 1 at first + 2 q pad
// onward, pixel i holding pixel i mod n.  One block row per ring.
template <typename M>
__global__ __launch_bounds__(kBlock) void k_pad_rings(const M* src, M* dst, const int* ri,
                                                      int pad) {
  const int q = blockIdx.y;
  const int n = ri[2 * q], first = ri[2 * q + 1];
  const int w = n + 2 * pad;
  const int64_t base = int64_t(first) + 2 * int64_t(q) * pad;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < w; i += gridDim.x * kBlock) {
    int k = (i - pad) % n;
    k += k < 0 ? n : 0;
    dst[base + i] = src[first + k];
  }
}

template <typename M>
void pad_rings(const M* src, M* dst, const int* ri, int nring, int nside, int pad,
               hipStream_t s) {
  const int wmax = 4 * nside + 2 * pad;
  const dim3 grid(unsigned(std::min((wmax + kBlock - 1) / kBlock, 64)), unsigned(nring));
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pad_rings<M>), grid, dim3(kBlock), 0, s, src, dst, ri, pad);
}

// ------------------------------------------------------------ tile kernels
// A 64 x 64 tile plus an even halo of HH cells per side is processed by one
// workgroup.  The region is cut into 2 x 2 quads aligned with the cells of
// the next coarser level.  A thread owns IT quads of one quad row (columns
// tr, tr + TPR, ...), so it keeps that row pair's coefficients once, and per
// quad the four u values, the four sources times the cell area (A f) and
// the four reciprocal diagonals, all in registers.  u is mirrored in LDS,
// columns split by parity, with a guard ring of zeros, so that every
// neighbour a quad reads sits at a fixed offset from one base index.  Cells
// outside the patch carry a zero reciprocal diagonal and zero source, so
// they stay zero; a neighbour across the patch face enters only through the
// diagonal (zero face value).  Cells near the region edge read the guard
// zeros; the halo is wide enough that this never reaches the tile.
constexpr int kTileBlock = 512;

template <typename T>
struct TileArgs {
  int n, ntile, nu;
  int lgt;              // log2(ntile): tile levels have a power-of-two size
  int nu2;              // fused post + pre: the pre-smoothing sweeps
  const double* coef;   // this level's rows
  const T* rowt;        // this level's row table (8 values per row)
  const T* u_in;        // level iterate in (nullptr: zero), or ubar (level >= 1 pre)
  const T* f_in;        // source (level 0: f'; level >= 1 post: A f), or rbar (level >= 1 pre)
  T* u_out;
  T* f_out;             // level >= 1 pre: the formed source, times the cell area
  T* ubar_out;          // pre: restricted iterate for the next level
  T* rbar_out;          // pre: restricted residual
  const T* uc;          // post: coarse result u_H
  const T* ubarc;       // post: coarse ubar
  int fas_source;       // pre on level >= 1: A f = A L u_in + A f_in
  int f_scaled;         // f_in already holds A f
  const int* done;      // epsilon rule: patches that stopped (nullptr: none)
  const int* pmap;      // partial sky: the domain's patches (nullptr: all)
};

// Quads per region side, threads per workgroup and threads per quad row.
// The widest halos (fused smoothing) take 1024 threads with TPR = 2 S mod 64,
// S = Q + 2 the LDS row stride: a wave's quad rows, 2 S floats apart, then
// land on successive banks of the 64-bank LDS (no bank conflicts in the
// sweeps).  The others take 512 threads and the fewest quads per thread,
// which measured faster than the conflict-free mapping on 1024 threads.
constexpr int tile_q(int hh) { return (kTile + 2 * hh) / 2; }
constexpr int tile_threads(int hh) { return hh >= 10 ? 2 * kTileBlock : kTileBlock; }
constexpr int quads_per_thread(int q, int nt) {
  int it = 1;
  while (q * ((q + it - 1) / it) > nt) ++it;
  return it;
}
constexpr int tile_tpr(int hh) {
  return hh >= 10 ? (2 * (tile_q(hh) + 2)) % 64
                  : (tile_q(hh) + quads_per_thread(tile_q(hh), kTileBlock) - 1) /
                        quads_per_thread(tile_q(hh), kTileBlock);
}

template <typename T, int HH>
struct QT {
  static_assert(HH % 2 == 0, "quads must align with the coarse level");
  static constexpr int RR = kTile + 2 * HH;    // region side
  static constexpr int Q = RR / 2;             // quads per side
  static constexpr int NT = tile_threads(HH);
  static constexpr int TPR = tile_tpr(HH);       // threads per quad row
  static constexpr int IT = (Q + TPR - 1) / TPR; // quads per thread
  static_assert(TPR >= 8 && Q * TPR <= NT, "quad rows must fit the workgroup");
  static constexpr int QH = HH / 2;            // first interior quad
  static constexpr int S = Q + 2;              // parity-array row stride (guard columns)
  static constexpr int PAR = (RR + 2) * S;     // cells per parity array (guard rows)
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

// LDS of a tile: u of cell (li, lj) at (lj & 1) * PAR + (li + 1) * S + (lj >> 1) + 1;
// per region row the coefficients, the term er that a patch face above or
// below the row adds to the diagonal (ghost = -u: the missing neighbour's
// coefficient), and the reciprocal diagonals of the row's cells away from
// the side faces (rD) and on a side face (rD1, one more isc); per region
// column cf = 1 on a side face of the patch, else 0.  Tile levels have at
// least 128 cells per side, so no column lies on both side faces.
template <typename T, int HH>
struct QLds {
  using G = QT<T, HH>;
  T u[2 * G::PAR];
  T sm[G::RR], sp[G::RR], isc[G::RR], A[G::RR], er[G::RR], rD[G::RR], rD1[G::RR];
  T cf[G::RR];
  T rden[G::Q];   // 1 / (2 (A_2k + A_2k+1)): area weight of a quad row pair
};

// A thread's quad row pair (qi): rows 2 qi and 2 qi + 1 of the region.
template <typename T>
struct QRow {
  T sm0, sp0, is0, sm1, sp1, is1;
  int qi;
  bool live;
};

// Per owned quad (qi, qj): cells c = 2a + b at (2 qi + a, 2 qj + b).  b is
// the LDS index of cell (2 qi - 1, 2 qj); every neighbour outside the quad
// is at a fixed offset from it.  Regions start at even cells and levels have
// an even size, so a quad lies wholly inside or wholly outside the patch:
// the quads outside (in false) hold u = 0 in LDS and are never updated, and
// their registers are never read.
template <typename T>
struct Quad {
  T u[4], ft[4], rD[4];
  int b, qj;
  bool live, in, edge;  // edge: a cell of the quad lies on the patch boundary
};


// Row table of the region (rows i0 .. i0 + RR - 1 of the level's table,
// defaults outside the patch), the side-face flags of its columns and the
// zero guard ring of both parity arrays.
template <typename T>
struct alignas(8 * sizeof(T)) Row8 {
  T v[8];
};

template <typename T, int HH>
__device__ __forceinline__ void qload_rows(QLds<T, HH>& t, const T* rowt, int n, int i0, int j0) {
  using G = QT<T, HH>;
  static_assert(G::RR <= G::NT, "one region row per thread");
  const Row8<T>* rows = reinterpret_cast<const Row8<T>*>(rowt);
  const int r = threadIdx.x;
  if (r < G::RR) {
    // both loads first (the quad-pair weight of quad row r: row 2 r)
    const int gi = i0 + r, gp = i0 + 2 * r;  // i0 is even
    const bool rin = gi >= 0 && gi < n, pin = r < G::Q && gp >= 0 && gp + 1 < n;
    const Row8<T> w = rows[min(max(gi, 0), n - 1)];
    const T rd = rowt[8 * min(max(gp, 0), n - 2) + 7];
    const int gj = j0 + r;
    t.sm[r] = rin ? w.v[0] : T(0);
    t.sp[r] = rin ? w.v[1] : T(0);
    t.isc[r] = rin ? w.v[2] : T(0);
    t.A[r] = rin ? w.v[3] : T(1);
    t.er[r] = rin ? w.v[4] : T(0);
    t.rD[r] = rin ? w.v[5] : T(1);
    t.rD1[r] = rin ? w.v[6] : T(1);
    t.cf[r] = (gj == 0 || gj == n - 1) ? T(1) : T(0);
    if (r < G::Q) t.rden[r] = pin ? rd : T(0.25);
  }
  // the guard ring of both parity arrays is zero (every region cell is
  // written by its quad)
  constexpr int NG = 2 * G::S + 2 * G::RR;
  for (int k = threadIdx.x; k < 2 * NG; k += G::NT) {
    const int par = k / NG, g = k - par * NG;
    int idx;
    if (g < 2 * G::S)
      idx = (g < G::S ? 0 : (G::RR + 1) * G::S) + (g % G::S);
    else {
      const int h = g - 2 * G::S, r = 1 + (h >> 1);
      idx = r * G::S + ((h & 1) ? G::S - 1 : 0);
    }
    t.u[par * G::PAR + idx] = T(0);
  }
}

// The thread's row pair and quads, and the global loads of the u and
// (unscaled) source of its quads inside the patch, issued before anything
// waits.  u_in and f_in point at this patch's level array (u_in nullptr:
// zero).
template <typename T, int HH>
__device__ __forceinline__ void qissue(QRow<T>& rw, Quad<T> (&qd)[QT<T, HH>::IT],
                                       const T* u_in, const T* f_in, int n, int i0, int j0) {
  using G = QT<T, HH>;
  const int qi = threadIdx.x / G::TPR, tr = threadIdx.x - qi * G::TPR;
  rw.live = qi < G::Q;
  rw.qi = rw.live ? qi : 0;
  const int gi0 = i0 + 2 * rw.qi;
  const bool rin = rw.live && gi0 >= 0 && gi0 < n;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    Quad<T>& Qd = qd[it];
    const int qj = tr + it * G::TPR;
    Qd.live = rw.live && qj < G::Q;
    Qd.qj = Qd.live ? qj : 0;
    Qd.b = 2 * rw.qi * G::S + Qd.qj + 1;
    const int gj = j0 + 2 * Qd.qj;
    Qd.in = rin && Qd.live && gj >= 0 && gj < n;
    Qd.edge = gi0 == 0 || gi0 + 1 == n - 1 || gj == 0 || gj + 1 == n - 1;
    if (Qd.in) {
      // the second row through its own (uniform) base: one offset register
      const unsigned g = unsigned(gi0 * n + gj);
      load2(at(f_in, g), Qd.ft[0], Qd.ft[1]);
      load2(at(f_in + n, g), Qd.ft[2], Qd.ft[3]);
      if (u_in) {
        load2(at(u_in, g), Qd.u[0], Qd.u[1]);
        load2(at(u_in + n, g), Qd.u[2], Qd.u[3]);
      } else {
        Qd.u[0] = Qd.u[1] = Qd.u[2] = Qd.u[3] = T(0);
      }
    }
  }
}

// After the row table is visible: the row pair's coefficients, and per
// quad inside the patch A f (unless f_in held it) and the reciprocal
// diagonals (one more isc on a side face: column 0 is the even cell of its
// quad, column n - 1 the odd one).
template <typename T, int HH>
__device__ __forceinline__ void qfinish(const QLds<T, HH>& t, QRow<T>& rw,
                                        Quad<T> (&qd)[QT<T, HH>::IT], bool f_scaled, int n,
                                        int i0, int j0) {
  using G = QT<T, HH>;
  const int li = 2 * rw.qi;
  rw.sm0 = t.sm[li]; rw.sp0 = t.sp[li]; rw.is0 = t.isc[li];
  rw.sm1 = t.sm[li + 1]; rw.sp1 = t.sp[li + 1]; rw.is1 = t.isc[li + 1];
  const T A0 = f_scaled ? T(1) : t.A[li], A1 = f_scaled ? T(1) : t.A[li + 1];
  const T rd0 = t.rD[li], rd1 = t.rD[li + 1], re0 = t.rD1[li], re1 = t.rD1[li + 1];
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    Quad<T>& Qd = qd[it];
    if (!Qd.in) continue;
    const int gj = j0 + 2 * Qd.qj;
    const bool side0 = gj == 0, side1 = gj + 1 == n - 1;
    if (!f_scaled) {
      Qd.ft[0] *= A0;
      Qd.ft[1] *= A0;
      Qd.ft[2] *= A1;
      Qd.ft[3] *= A1;
    }
    Qd.rD[0] = side0 ? re0 : rd0;
    Qd.rD[1] = side1 ? re0 : rd0;
    Qd.rD[2] = side0 ? re1 : rd1;
    Qd.rD[3] = side1 ? re1 : rd1;
  }
}

// Write the owned quads' u to LDS.
template <typename T, int HH>
__device__ __forceinline__ void qput(QLds<T, HH>& t, const Quad<T> (&qd)[QT<T, HH>::IT]) {
  using G = QT<T, HH>;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const Quad<T>& Qd = qd[it];
    if (!Qd.live) continue;
    T* ub = t.u + Qd.b;
    if (Qd.in) {
      ub[G::S] = Qd.u[0];
      ub[G::PAR + G::S] = Qd.u[1];
      ub[2 * G::S] = Qd.u[2];
      ub[G::PAR + 2 * G::S] = Qd.u[3];
    } else {
      ub[G::S] = T(0);
      ub[G::PAR + G::S] = T(0);
      ub[2 * G::S] = T(0);
      ub[G::PAR + 2 * G::S] = T(0);
    }
  }
}

// Gauss-Seidel value of one cell: (s_m u_up + s_p u_down + isc (u_left +
// u_right) - A f) / D, accumulated from -A f so that each product fuses.
template <typename T>
__device__ __forceinline__ T gs_update(T sm, T up, T sp, T dn, T isc, T lr, T af, T rd) {
  return fma(isc, lr, fma(sp, dn, fma(sm, up, -af))) * rd;
}

// Red-black half sweep over the owned quads.
template <typename T, int HH>
__device__ __forceinline__ void qsweep(QLds<T, HH>& t, const QRow<T>& rw,
                                       Quad<T> (&qd)[QT<T, HH>::IT], int color) {
  using G = QT<T, HH>;
  constexpr int S = G::S, P = G::PAR;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    Quad<T>& Qd = qd[it];
    if (!Qd.in) continue;
    T* ub = t.u + Qd.b;
    if (color == 0) {
      const T up = ub[0], lf = ub[P + S - 1], dn = ub[P + 3 * S], rt = ub[2 * S + 1];
      const T v0 = gs_update(rw.sm0, up, rw.sp0, Qd.u[2], rw.is0, lf + Qd.u[1], Qd.ft[0], Qd.rD[0]);
      const T v3 = gs_update(rw.sm1, Qd.u[1], rw.sp1, dn, rw.is1, Qd.u[2] + rt, Qd.ft[3], Qd.rD[3]);
      Qd.u[0] = v0;
      Qd.u[3] = v3;
      ub[S] = v0;
      ub[P + 2 * S] = v3;
    } else {
      const T up = ub[P], rt = ub[S + 1], dn = ub[3 * S], lf = ub[P + 2 * S - 1];
      const T v1 = gs_update(rw.sm0, up, rw.sp0, Qd.u[3], rw.is0, Qd.u[0] + rt, Qd.ft[1], Qd.rD[1]);
      const T v2 = gs_update(rw.sm1, Qd.u[0], rw.sp1, dn, rw.is1, lf + Qd.u[3], Qd.ft[2], Qd.rD[2]);
      Qd.u[1] = v1;
      Qd.u[2] = v2;
      ub[P + S] = v1;
      ub[2 * S] = v2;
    }
  }
}

// A (L u) of the four cells of a quad in difference form (neighbour minus
// centre, which keeps the float32 residual free of cancellation); a
// neighbour across the patch face is the ghost -u, so its coefficient
// enters twice.
template <typename T, int HH>
__device__ __forceinline__ void qalap(const QLds<T, HH>& t, const QRow<T>& rw, const Quad<T>& Qd,
                                      T AL[4]) {
  using G = QT<T, HH>;
  constexpr int S = G::S, P = G::PAR;
  const T* ub = t.u + Qd.b;
  const T* u = Qd.u;
  const T er0 = t.er[2 * rw.qi], er1 = t.er[2 * rw.qi + 1];
  const T cf0 = t.cf[2 * Qd.qj], cf1 = t.cf[2 * Qd.qj + 1];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const T nb0 = c == 0 ? ub[0] : c == 1 ? ub[P] : c == 2 ? u[0] : u[1];
    const T nb1 = c == 0 ? u[2] : c == 1 ? u[3] : c == 2 ? ub[3 * S] : ub[P + 3 * S];
    const T nb2 = c == 0 ? ub[P + S - 1] : c == 1 ? u[0] : c == 2 ? ub[P + 2 * S - 1] : u[2];
    const T nb3 = c == 0 ? u[1] : c == 1 ? ub[S + 1] : c == 2 ? u[3] : ub[2 * S + 1];
    const int aa = c >> 1, bb = c & 1;
    const T sm = aa ? rw.sm1 : rw.sm0, sp = aa ? rw.sp1 : rw.sp0, isc = aa ? rw.is1 : rw.is0;
    const T x = u[c];
    AL[c] = sm * (nb0 - x) + sp * (nb1 - x) + isc * ((nb2 - x) + (nb3 - x));
    // the face terms (quads on the patch boundary only): er of the row,
    // isc on a side-face column
    if (Qd.edge) AL[c] -= ((aa ? er1 : er0) + isc * (bb ? cf1 : cf0)) * x;
  }
}

template <typename T, int HH>
__device__ __forceinline__ bool interior_quad(const QRow<T>& rw, const Quad<T>& Qd) {
  using G = QT<T, HH>;
  return Qd.in && rw.qi >= G::QH && rw.qi < G::QH + kTile / 2 && Qd.qj >= G::QH &&
         Qd.qj < G::QH + kTile / 2;
}

// End of pre-smoothing: the interior quads store u (and A f), form the
// residual and the area-weighted restrictions of u and of the residual.
template <typename T, int HH>
__device__ __forceinline__ void pre_epilogue(const TileArgs<T>& a, const QLds<T, HH>& t,
                                             const QRow<T>& rw,
                                             const Quad<T> (&qd)[QT<T, HH>::IT], int i0, int j0,
                                             size_t pbase, size_t cbase) {
  using G = QT<T, HH>;
  const int n = a.n, nc = n / 2;
  T* uo = a.u_out + pbase;
  T* ubo = a.ubar_out + cbase;
  T* rbo = a.rbar_out + cbase;
  const int li = 2 * rw.qi;
  const T a0 = t.A[li], a1 = t.A[li + 1], rden = t.rden[rw.qi];
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const Quad<T>& Qd = qd[it];
    if (!interior_quad<T, HH>(rw, Qd)) continue;
    const int gi = i0 + li, gj = j0 + 2 * Qd.qj;
    const unsigned g = unsigned(gi * n + gj);
    store2(at(uo, g), Qd.u[0], Qd.u[1]);
    store2(at(uo + n, g), Qd.u[2], Qd.u[3]);
    if (a.fas_source) {
      T* fo = a.f_out + pbase;
      store2(at(fo, g), Qd.ft[0], Qd.ft[1]);
      store2(at(fo + n, g), Qd.ft[2], Qd.ft[3]);
    }
    // A r = A f - A L u, summed over the quad (formed at all four cells:
    // in float32 the cells the last half sweep updated carry the rounding
    // of that update, which the coarse correction must see)
    T AL[4];
    qalap<T, HH>(t, rw, Qd, AL);
    const T ar = ((Qd.ft[0] - AL[0]) + (Qd.ft[1] - AL[1])) + ((Qd.ft[2] - AL[2]) + (Qd.ft[3] - AL[3]));
    const unsigned gc = unsigned((gi / 2) * nc + gj / 2);
    *at(ubo, gc) = (a0 * (Qd.u[0] + Qd.u[1]) + a1 * (Qd.u[2] + Qd.u[3])) * rden;
    *at(rbo, gc) = ar * rden;
  }
}

// Coarse correction e = u_H - ubar on the coarse cells covering the region
// (+- 1 cell), then added to the owned quads: bilinear (9, 3, 3, 1)/16 of
// the parent and its neighbours toward the child, direct injection of the
// parent on the outermost fine ring.  corr_issue loads the thread's items
// (clamped into the patch) without waiting; corr_store writes them to LDS,
// zero outside the patch.
template <typename T, int HH>
struct CorrIn {
  static constexpr int CR = QT<T, HH>::Q + 2;
  // LDS row stride of the staged correction: on the conflict-free quad
  // mapping (TPR threads per quad row) a stride congruent to TPR modulo 64
  // puts a wave's rows on successive banks, as in the sweeps
  static constexpr int ES = HH >= 10 ? CR + ((QT<T, HH>::TPR - CR) % 64 + 64) % 64 : CR;
  // the region's first coarse column, (tile) 32 - HH / 2 - 1, is even when
  // HH / 2 is odd: then coarse columns pair up (an even one and the next,
  // both inside or both outside the patch) and each item is a pair
  static constexpr bool PAIR = (HH / 2) % 2 == 1;
  static constexpr int CW = PAIR ? CR / 2 : CR;  // items per row
  static constexpr int NE = (CR * CW + QT<T, HH>::NT - 1) / QT<T, HH>::NT;
  static constexpr int EV = PAIR ? 2 : 1;        // values per item
  T uc[NE * EV], ub[NE * EV];
};

template <typename T, int HH>
__device__ __forceinline__ void corr_issue(const TileArgs<T>& a, CorrIn<T, HH>& c, size_t cbase,
                                           int i0, int j0) {
  using C = CorrIn<T, HH>;
  const int nc = a.n / 2, ci0 = i0 / 2 - 1, cj0 = j0 / 2 - 1;  // i0, j0 even
#pragma unroll
  for (int k = 0; k < C::NE; ++k) {
    const int item = min(int(threadIdx.x) + k * QT<T, HH>::NT, C::CR * C::CW - 1);
    const int r = item / C::CW, q = item - r * C::CW;
    const int I = min(max(ci0 + r, 0), nc - 1);
    if constexpr (C::PAIR) {
      const int J = min(max(cj0 + 2 * q, 0), nc - 2);
      const unsigned g = unsigned(I * nc + J);
      load2(at(a.uc + cbase, g), c.uc[2 * k], c.uc[2 * k + 1]);
      load2(at(a.ubarc + cbase, g), c.ub[2 * k], c.ub[2 * k + 1]);
    } else {
      const int J = min(max(cj0 + q, 0), nc - 1);
      const unsigned g = unsigned(I * nc + J);
      c.uc[k] = *at(a.uc + cbase, g);
      c.ub[k] = *at(a.ubarc + cbase, g);
    }
  }
}

template <typename T, int HH>
__device__ __forceinline__ void corr_store(T* e, const CorrIn<T, HH>& c, int n, int i0, int j0) {
  using C = CorrIn<T, HH>;
  const int nc = n / 2, ci0 = i0 / 2 - 1, cj0 = j0 / 2 - 1;
#pragma unroll
  for (int k = 0; k < C::NE; ++k) {
    const int item = int(threadIdx.x) + k * QT<T, HH>::NT;
    if (item >= C::CR * C::CW) break;
    const int r = item / C::CW, q = item - r * C::CW;
    const int I = ci0 + r;
    if constexpr (C::PAIR) {
      const int J = cj0 + 2 * q;
      const bool in = I >= 0 && I < nc && J >= 0 && J < nc;
      e[r * C::ES + 2 * q] = in ? c.uc[2 * k] - c.ub[2 * k] : T(0);
      e[r * C::ES + 2 * q + 1] = in ? c.uc[2 * k + 1] - c.ub[2 * k + 1] : T(0);
    } else {
      const int J = cj0 + q;
      e[r * C::ES + q] = (I >= 0 && I < nc && J >= 0 && J < nc) ? c.uc[k] - c.ub[k] : T(0);
    }
  }
}

template <typename T, int HH>
__device__ __forceinline__ void apply_correction(const T* e, const QRow<T>& rw,
                                                 Quad<T> (&qd)[QT<T, HH>::IT], int i0, int j0,
                                                 int n) {
  using G = QT<T, HH>;
  constexpr int CR = CorrIn<T, HH>::ES;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    Quad<T>& Qd = qd[it];
    if (!Qd.in) continue;
    const T* ec = e + (rw.qi + 1) * CR + (Qd.qj + 1);
    const T c = ec[0];
    const T nu = ec[-CR], nd = ec[CR], nl = ec[-1], nr = ec[1];
    const T ul = ec[-CR - 1], ur = ec[-CR + 1], dl = ec[CR - 1], dr = ec[CR + 1];
    const T p[4] = {(T(9) * c + T(3) * (nu + nl) + ul) * T(0.0625),
                    (T(9) * c + T(3) * (nu + nr) + ur) * T(0.0625),
                    (T(9) * c + T(3) * (nd + nl) + dl) * T(0.0625),
                    (T(9) * c + T(3) * (nd + nr) + dr) * T(0.0625)};
    const int gi = i0 + 2 * rw.qi, gj = j0 + 2 * Qd.qj;
    if (Qd.edge) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ci = gi + (k >> 1), cj = gj + (k & 1);
        const bool ring = ci == 0 || ci == n - 1 || cj == 0 || cj == n - 1;
        Qd.u[k] += ring ? c : p[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) Qd.u[k] += p[k];
    }
  }
}

template <typename T, int HH>
__global__ __launch_bounds__(tile_threads(HH)) void k_mg_pre(TileArgs<T> a) {
  using G = QT<T, HH>;
  __shared__ QLds<T, HH> t;
  QRow<T> rw;
  Quad<T> qd[G::IT];
  const int64_t lb = xcd_block();
  const int64_t patch = patch_of(a.pmap, lb >> (2 * a.lgt));
  const int tt = int(lb & ((int64_t(1) << (2 * a.lgt)) - 1));
  if (a.done && a.done[patch]) return;
  const int i0 = (tt >> a.lgt) * kTile - HH, j0 = (tt & (a.ntile - 1)) * kTile - HH;
  const int n = a.n, nc = n / 2;
  const size_t pbase = size_t(patch) * n * n, cbase = size_t(patch) * nc * nc;
  qissue<T, HH>(rw, qd, a.u_in ? a.u_in + pbase : nullptr, a.f_in + pbase, n, i0, j0);
  qload_rows(t, a.rowt, n, i0, j0);
  __syncthreads();
  qfinish<T, HH>(t, rw, qd, false, n, i0, j0);
  qput<T, HH>(t, qd);
  __syncthreads();
  if (a.fas_source) {
    // A f = A L_H ubar + A rbar on the in-patch cells
#pragma unroll
    for (int it = 0; it < G::IT; ++it) {
      Quad<T>& Qd = qd[it];
      if (!Qd.in) continue;
      T AL[4];
      qalap<T, HH>(t, rw, Qd, AL);
#pragma unroll
      for (int c = 0; c < 4; ++c) Qd.ft[c] += AL[c];
    }
    __syncthreads();
  }
  for (int s = 0; s < a.nu; ++s) {
    qsweep<T, HH>(t, rw, qd, 0);
    __syncthreads();
    qsweep<T, HH>(t, rw, qd, 1);
    __syncthreads();
  }
  pre_epilogue<T, HH>(a, t, rw, qd, i0, j0, pbase, cbase);
}

template <typename T, int HH>
__global__ __launch_bounds__(tile_threads(HH)) void k_mg_post(TileArgs<T> a) {
  using G = QT<T, HH>;
  constexpr int CR = G::Q + 2;  // coarse cells covering the region quads +- 1
  __shared__ QLds<T, HH> t;
  __shared__ T e[CR * CorrIn<T, HH>::ES];
  QRow<T> rw;
  Quad<T> qd[G::IT];
  const int64_t lb = xcd_block();
  const int64_t patch = patch_of(a.pmap, lb >> (2 * a.lgt));
  const int tt = int(lb & ((int64_t(1) << (2 * a.lgt)) - 1));
  const int i0 = (tt >> a.lgt) * kTile - HH, j0 = (tt & (a.ntile - 1)) * kTile - HH;
  const int n = a.n, nc = n / 2;
  const size_t pbase = size_t(patch) * n * n, cbase = size_t(patch) * nc * nc;
  if (a.done && a.done[patch]) return;
  CorrIn<T, HH> ci;
  qissue<T, HH>(rw, qd, a.u_in + pbase, a.f_in + pbase, n, i0, j0);
  corr_issue<T, HH>(a, ci, cbase, i0, j0);
  qload_rows(t, a.rowt, n, i0, j0);
  corr_store<T, HH>(e, ci, n, i0, j0);
  __syncthreads();
  qfinish<T, HH>(t, rw, qd, a.f_scaled != 0, n, i0, j0);
  apply_correction<T, HH>(e, rw, qd, i0, j0, n);
  qput<T, HH>(t, qd);
  __syncthreads();
  for (int s = 0; s < a.nu; ++s) {
    qsweep<T, HH>(t, rw, qd, 0);
    __syncthreads();
    qsweep<T, HH>(t, rw, qd, 1);
    __syncthreads();
  }
  T* uo = a.u_out + pbase;
#pragma unroll
  for (int it = 0; it < G::IT; ++it) {
    const Quad<T>& Qd = qd[it];
    if (!interior_quad<T, HH>(rw, Qd)) continue;
    const unsigned g = unsigned((i0 + 2 * rw.qi) * n + (j0 + 2 * Qd.qj));
    store2(at(uo, g), Qd.u[0], Qd.u[1]);
    store2(at(uo + n, g), Qd.u[2], Qd.u[3]);
  }
}

// Finest level: the post-smoothing of one V-cycle and the pre-smoothing of
// the next in one pass.  The region carries the halos of both (2 (nu_post +
// nu_pre) + 2 cells: every sweep plus the residual), so the corrected and
// smoothed iterate of the finished cycle never leaves LDS; the kernel writes
// what the next cycle's pre-smoothing writes: u and the restrictions of u
// and of the residual.
template <typename T, int HH>
__global__ __launch_bounds__(tile_threads(HH)) void k_mg_postpre(TileArgs<T> a) {
  using G = QT<T, HH>;
  constexpr int CR = G::Q + 2;
  __shared__ QLds<T, HH> t;
  __shared__ T e[CR * CorrIn<T, HH>::ES];
  QRow<T> rw;
  Quad<T> qd[G::IT];
  const int64_t lb = xcd_block();
  const int64_t patch = patch_of(a.pmap, lb >> (2 * a.lgt));
  const int tt = int(lb & ((int64_t(1) << (2 * a.lgt)) - 1));
  const int i0 = (tt >> a.lgt) * kTile - HH, j0 = (tt & (a.ntile - 1)) * kTile - HH;
  const int n = a.n, nc = n / 2;
  const size_t pbase = size_t(patch) * n * n, cbase = size_t(patch) * nc * nc;
  CorrIn<T, HH> ci;
  qissue<T, HH>(rw, qd, a.u_in + pbase, a.f_in + pbase, n, i0, j0);
  corr_issue<T, HH>(a, ci, cbase, i0, j0);
  qload_rows(t, a.rowt, n, i0, j0);
  corr_store<T, HH>(e, ci, n, i0, j0);
  __syncthreads();
  qfinish<T, HH>(t, rw, qd, false, n, i0, j0);
  apply_correction<T, HH>(e, rw, qd, i0, j0, n);
  qput<T, HH>(t, qd);
  __syncthreads();
  for (int s = 0; s < a.nu + a.nu2; ++s) {
    qsweep<T, HH>(t, rw, qd, 0);
    __syncthreads();
    qsweep<T, HH>(t, rw, qd, 1);
    __syncthreads();
  }
  pre_epilogue<T, HH>(a, t, rw, qd, i0, j0, pbase, cbase);
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

// ------------------------------------------------------------ LDS levels
// One workgroup per patch runs the V-cycle below level K entirely in LDS:
// 512 threads, so the 64^2 level's half-sweeps take four cells per thread
// (fewer threads sit idle on the coarser levels, and in float32 three such
// workgroups share a CU's LDS, against two of 1024 threads).  Per level l:
// u, f (and ubar for l > K) as row-major n_l x n_l arrays, and the level's
// row coefficients (s_m, s_p, 1/s_c, area, the reciprocal diagonals of the
// row's cells off and on a side face, with the face terms of rows 0 and
// n - 1 included, and 1/area).
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
  const int* done;        // epsilon rule: patches that stopped (nullptr: none)
  const int* pmap;        // partial sky: the domain's patches (nullptr: all)
};

template <typename T>
struct LRows {
  const T* sm;
  const T* sp;
  const T* isc;
  const T* A;
  const T* rD;
  const T* rDs;
  const T* iA;
};

// (L u)_ij, zero face value across the patch boundary (the ghost -u); a
// missing neighbour is read at the cell itself, so no load is predicated.
template <typename T>
__device__ __forceinline__ T lap_g(const T* u, int n, int i, int j, const LRows<T>& r) {
  const int c = i * n + j;
  const T uc = u[c];
  const bool ui = i > 0, di = i < n - 1, lj = j > 0, rj = j < n - 1;
  const T upv = u[ui ? c - n : c], dnv = u[di ? c + n : c];
  const T lfv = u[lj ? c - 1 : c], rtv = u[rj ? c + 1 : c];
  const T up = ui ? upv : -uc, dn = di ? dnv : -uc, lf = lj ? lfv : -uc, rt = rj ? rtv : -uc;
  return (r.sm[i] * (up - uc) + r.sp[i] * (dn - uc) + (lf - T(2) * uc + rt) * r.isc[i]) * r.iA[i];
}

// Red-black sweeps: a neighbour across the patch face is zero (the ghost
// -u enters through the diagonal, which the row's reciprocals include).
// Each thread keeps one row (its coefficients and face flags in registers)
// and cpt cells of the colour in it, columns q, q + tpr, ... of the colour;
// a missing neighbour is read at the cell itself and weighted by zero, so no
// load is predicated.
template <typename T>
__device__ void lds_smooth(T* u, const T* f, int n, int lg, const LRows<T>& r, int sweeps) {
  const int half = n >> 1;
  const int cpt = max(1, (n * half) / kLdsBlock);  // powers of two
  const int tpr = half / cpt;
  const int i = threadIdx.x / tpr, q = threadIdx.x - i * tpr;
  const bool live = i < n;
  const int ii = live ? i : 0;
  const T sm = i > 0 ? r.sm[ii] : T(0), sp = i < n - 1 ? r.sp[ii] : T(0);
  const T isc = r.isc[ii], A = r.A[ii], rd = r.rD[ii], rds = r.rDs[ii];
  const int om = i > 0 ? -n : 0, op = i < n - 1 ? n : 0;
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      if (live) {
        const int par = (color + i) & 1;
        for (int k = 0; k < cpt; ++k) {
          const int j = 2 * (q + tpr * k) + par;
          const int c = ii * n + j;
          const bool lfin = j > 0, rtin = j < n - 1;
          const T lf = u[lfin ? c - 1 : c], rt = u[rtin ? c + 1 : c];
          const T lr = (lfin ? lf : T(0)) + (rtin ? rt : T(0));
          const T num = fma(isc, lr, fma(sp, u[c + op], fma(sm, u[c + om], -A * f[c])));
          u[c] = num * (lfin && rtin ? rd : rds);
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
    q += nn * nn * (k > K ? 3 : 2) + 7 * nn;
  }
  const int nn = n0 >> (l - K);
  LLevel<T> v;
  v.u = q;
  v.f = q + nn * nn;
  v.b = l > K ? q + 2 * nn * nn : nullptr;
  T* rows = q + nn * nn * (l > K ? 3 : 2);
  v.r = LRows<T>{rows,          rows + nn,     rows + 2 * nn, rows + 3 * nn,
                 rows + 4 * nn, rows + 5 * nn, rows + 6 * nn};
  return v;
}

template <typename T>
__global__ __launch_bounds__(kLdsBlock) void k_mg_lds(LdsArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int64_t patch = patch_of(a.pmap, xcd_block());
  if (a.done && a.done[patch]) return;
  const int K = a.lv.K, nl = a.lv.nlev, n0 = a.lv.n0;
  for (int l = K; l < nl; ++l) {
    const int nn = n0 >> (l - K);
    const LLevel<T> L = lds_level<T>(smem, K, n0, l);
    T* rows = const_cast<T*>(L.r.sm);
    for (int i = threadIdx.x; i < nn; i += kLdsBlock) {
      const double* c = a.coef + a.lv.crow[l] + 4 * i;
      const double is = 1.0 / c[2];
      const double d = c[0] + c[1] + 2.0 * is + (i == 0 ? c[0] : 0.0) + (i == nn - 1 ? c[1] : 0.0);
      rows[i] = T(c[0]);
      rows[nn + i] = T(c[1]);
      rows[2 * nn + i] = T(is);
      rows[3 * nn + i] = T(c[3]);
      rows[4 * nn + i] = T(1.0 / d);
      rows[5 * nn + i] = T(1.0 / (d + is));
      rows[6 * nn + i] = T(1.0 / c[3]);
    }
  }
  int lg0 = 0;
  while ((1 << lg0) < n0) ++lg0;
  const size_t g0 = size_t(patch) * n0 * n0;
  {
    const LLevel<T> L = lds_level<T>(smem, K, n0, K);
    const T* ui = a.u_in ? a.u_in + g0 : nullptr;
    const T* fi = a.f_in + g0;
    for (int idx = threadIdx.x; idx < n0 * n0; idx += kLdsBlock) {
      L.u[idx] = ui ? *at(ui, unsigned(idx)) : T(0);
      L.f[idx] = *at(fi, unsigned(idx));
    }
    __syncthreads();
    if (a.fas_source) {
      // f = L ubar + rbar (reads u only, writes f only)
      for (int idx = threadIdx.x; idx < n0 * n0; idx += kLdsBlock)
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
    for (int idx = threadIdx.x; idx < nc * nc; idx += kLdsBlock) {
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
    for (int idx = threadIdx.x; idx < nc * nc; idx += kLdsBlock)
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
    // the coarse correction e = u_H - ubar once per coarse cell (ubar is not
    // needed again in this cycle)
    for (int idx = threadIdx.x; idx < nc * nc; idx += kLdsBlock) C.b[idx] = C.u[idx] - C.b[idx];
    __syncthreads();
    auto ef = [&](int I, int J) { return C.b[I * nc + J]; };
    for (int idx = threadIdx.x; idx < nn * nn; idx += kLdsBlock)
      L.u[idx] += prolong_cell<T>(idx >> lg, idx & (nn - 1), nn, ef);
    __syncthreads();
    lds_smooth(L.u, L.f, nn, lg, L.r, a.nu2);
  }
  {
    const LLevel<T> L = lds_level<T>(smem, K, n0, K);
    T* uo = a.u_out + g0;
    for (int idx = threadIdx.x; idx < n0 * n0; idx += kLdsBlock) *at(uo, unsigned(idx)) = L.u[idx];
  }
}

// ------------------------------------------------------------ epsilon rule
// epsilon = ||r_h|| / ||tau|| per patch (Sec. 3.2 stopping rule):
// r_h = f' - L_h du on the finest level, tau = L_H(R du) - R(L_h du) on the
// first coarse level, area-weighted RMS, accumulated in FP64.  One block per
// tile of kEpsTC^2 coarse cells stages the fine correction (with its ghost
// ring) and the restricted field in LDS and writes four partial sums; a
// second kernel adds a patch's partials in a fixed order and applies the
// threshold.
constexpr int kEpsTC = kEpsTile;

template <typename T>
struct EpsArgs {
  int n;                // finest cells per side
  int tc;               // coarse cells per tile side, min(kEpsTC, n / 2): 4, 8, 16
  int ntile;            // tiles per side
  const double* c0;     // finest-level rows (s_m, s_p, s_c, area)
  const double* c1;     // first coarse level rows
  const T* du;
  const T* fp;
  const int* done;      // patches that already stopped
  double* part;         // [patch][tile][4]: sum A r^2, sum A, sum A_H tau^2, sum A_H
  const int* pmap;      // partial sky: the domain's patches (nullptr: all)
};

template <typename T, int TC>
__global__ __launch_bounds__(kBlock) void k_mg_eps(EpsArgs<T> a) {
  constexpr int FS = 2 * TC + 4, CS = TC + 2, NW = kBlock / 64;
  static_assert(TC * TC <= kBlock && FS <= 64, "one coarse cell per thread");
  __shared__ double F[FS * FS];
  __shared__ double U[CS * CS];
  // rows: fine (s_m, s_p, 1/s_c, 1/A, A) for rows 2 I0 .. 2 (I0 + TC) - 1;
  // coarse (s_m, s_p, 1/s_c, 1/A, A) for rows I0 .. I0 + TC - 1; restriction
  // weights (w0, w1) for coarse rows I0 - 1 .. I0 + TC
  __shared__ double RF[5][2 * TC], RC[5][TC], RW[2][CS];
  __shared__ double red[4][NW];
  const int tiles = a.ntile * a.ntile;
  const int64_t patch = patch_of(a.pmap, blockIdx.x / tiles);
  const int tile = blockIdx.x % tiles;
  if (a.done[patch]) return;
  const int n = a.n, nc = n / 2;
  const int I0 = (tile / a.ntile) * TC, J0 = (tile % a.ntile) * TC;
  const T* x = a.du + size_t(patch) * n * n;
  const T* f = a.fp + size_t(patch) * n * n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool cell = int(threadIdx.x) < TC * TC;
  const int li = threadIdx.x / TC, lj = threadIdx.x % TC, I = I0 + li, J = J0 + lj;
  // this thread's four f' values, requested before anything waits
  double fq[4] = {0.0, 0.0, 0.0, 0.0};
  if (cell)
    for (int q = 0; q < 4; ++q)
      fq[q] = double(f[size_t(2 * I + (q >> 1)) * n + 2 * J + (q & 1)]);
  // fine rows / columns 2 I0 - 2 .. 2 (I0 + TC) + 1, one row per wave; the
  // face ghost is -du of the cell it faces; cells two beyond the face are
  // never used
  constexpr int ROWS = (FS + NW - 1) / NW;
  double fv[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int r = wv + k * NW;
    const int i = 2 * I0 - 2 + r, j = 2 * J0 - 2 + lane;
    double v = 0.0;
    if (r < FS && lane < FS && i >= -1 && i <= n && j >= -1 && j <= n) {
      const int ii = min(max(i, 0), n - 1), jj = min(max(j, 0), n - 1);
      const bool gi = ii != i, gj = jj != j;
      if (!(gi && gj)) {
        v = double(x[size_t(ii) * n + jj]);
        if (gi || gj) v = -v;
      }
    }
    fv[k] = v;
  }
  if (threadIdx.x < 2 * TC) {
    const double* c = a.c0 + 4 * (2 * I0 + threadIdx.x);
    RF[0][threadIdx.x] = c[0];
    RF[1][threadIdx.x] = c[1];
    RF[2][threadIdx.x] = 1.0 / c[2];
    RF[3][threadIdx.x] = 1.0 / c[3];
    RF[4][threadIdx.x] = c[3];
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + TC) {
    const int t = threadIdx.x - 64;
    const double* c = a.c1 + 4 * (I0 + t);
    RC[0][t] = c[0];
    RC[1][t] = c[1];
    RC[2][t] = 1.0 / c[2];
    RC[3][t] = 1.0 / c[3];
    RC[4][t] = c[3];
  } else if (threadIdx.x >= 128 && threadIdx.x < 128 + CS) {
    const int t = threadIdx.x - 128, Ic = min(max(I0 - 1 + t, 0), nc - 1);
    const double a0 = a.c0[4 * (2 * Ic) + 3], a1 = a.c0[4 * (2 * Ic + 1) + 3];
    const double h = 1.0 / (2.0 * (a0 + a1));
    RW[0][t] = a0 * h;
    RW[1][t] = a1 * h;
  }
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int r = wv + k * NW;
    if (r < FS && lane < FS) F[r * FS + lane] = fv[k];
  }
  __syncthreads();
  // area-weighted restriction R du on coarse rows I0 - 1 .. I0 + TC
  for (int k = threadIdx.x; k < CS * CS; k += kBlock) {
    const int r = k / CS, c = k % CS, Ic = I0 - 1 + r, Jc = J0 - 1 + c;
    double v = 0.0;
    if (Ic >= 0 && Ic < nc && Jc >= 0 && Jc < nc) {
      const double* q = F + (2 * r) * FS + 2 * c;
      v = RW[0][r] * (q[0] + q[1]) + RW[1][r] * (q[FS] + q[FS + 1]);
    }
    U[k] = v;
  }
  __syncthreads();
  double sr = 0.0, sa = 0.0, st = 0.0, sb = 0.0;
  if (cell) {
    const double* uc = U + (li + 1) * CS + lj + 1;
    const double u = uc[0];
    // coarse ghosts: the negative of the interior cell (zero face value)
    const double up = I > 0 ? uc[-CS] : -u, dn = I < nc - 1 ? uc[CS] : -u;
    const double lf = J > 0 ? uc[-1] : -u, rt = J < nc - 1 ? uc[1] : -u;
    const double LH =
        (RC[0][li] * (up - u) + RC[1][li] * (dn - u) + (lf - 2.0 * u + rt) * RC[2][li]) *
        RC[3][li];
    double lh[4];
    for (int q = 0; q < 4; ++q) {
      const int fr = 2 * li + (q >> 1);
      const double* v = F + (fr + 2) * FS + 2 * lj + 2 + (q & 1);
      const double w = v[0];
      lh[q] = (RF[0][fr] * (v[-FS] - w) + RF[1][fr] * (v[FS] - w) +
               (v[-1] - 2.0 * w + v[1]) * RF[2][fr]) * RF[3][fr];
      const double rr = fq[q] - lh[q];
      sr += RF[4][fr] * rr * rr;
      sa += RF[4][fr];
    }
    const double tau = LH - (RW[0][li + 1] * (lh[0] + lh[1]) + RW[1][li + 1] * (lh[2] + lh[3]));
    st += RC[4][li] * tau * tau;
    sb += RC[4][li];
  }
  double v4[4] = {sr, sa, st, sb};
  for (int m = 0; m < 4; ++m) {
    double v = v4[m];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[m][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += red[threadIdx.x][w];
    a.part[(size_t(patch) * tiles + tile) * 4 + threadIdx.x] = v;
  }
}

struct EpsFinal {
  int tiles;
  double eps;
  int cycle;            // V-cycles run so far
  const double* part;
  int* done;
  int* cycles;
  double* eps_out;
  int* active;          // patches still above the threshold (added to)
  int* status;          // latched conditions (ST_NONFINITE)
  const int* pmap;      // partial sky: the domain's patches (nullptr: all)
};

// one wave per patch: partial sums added in a fixed order
__global__ __launch_bounds__(64) void k_mg_eps_final(EpsFinal a) {
  const int64_t patch = patch_of(a.pmap, blockIdx.x);
  if (a.done[patch]) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < a.tiles; t += 64)
    for (int m = 0; m < 4; ++m) v[m] += a.part[(size_t(patch) * a.tiles + t) * 4 + m];
  for (int m = 0; m < 4; ++m)
    for (int o = 32; o >= 1; o >>= 1) v[m] += __shfl_xor(v[m], o);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(v[0] / v[1]), nt = sqrt(v[2] / v[3]);
  const double e = nt > 0.0 ? nr / nt : (nr > 0.0 ? INFINITY : 0.0);
  a.eps_out[patch] = e;
  a.cycles[patch] = a.cycle;
  if (!isfinite(v[0]) || !isfinite(v[2])) {
    // a non-finite residual or truncation norm: latch it and stop the patch
    atomicOr(a.status, ST_NONFINITE);
    a.done[patch] = 1;
  } else if (e < a.eps)
    a.done[patch] = 1;
  else
    atomicAdd(a.active, 1);
}

__global__ void k_fill_int(int64_t n, int v, int* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = v;
}

__global__ void k_fill_f64(int64_t n, double v, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = v;
}

__global__ void k_notconv(int64_t n, const int* pmap, const int* done, int* status) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n && !done[patch_of(pmap, t)]) atomicOr(status, ST_NOTCONV);
}

// y[patch] = v for the n patches of a domain (pmap) or the first n
__global__ void k_fill_patches(int64_t n, const int* pmap, int v, int* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[patch_of(pmap, t)] = v;
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
  return lds_opt_in(p, reinterpret_cast<const void*>(kernel), bytes);
}

// Tile kernels are compiled per halo width: pre-smoothing needs 2 nu + 1
// cells (nu sweeps plus the residual), post-smoothing 2 nu.
template <typename T, int HH, bool PRE>
clm_status launch_tile_hh(Plan* p, const TileArgs<T>& a, int64_t np, hipStream_t s) {
  constexpr int RR = kTile + 2 * HH;
  const dim3 grid(unsigned(np * a.ntile * a.ntile));
  (void)RR;
  if (PRE)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_pre<T, HH>), grid, dim3(QT<T, HH>::NT), 0, s, a);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_post<T, HH>), grid, dim3(QT<T, HH>::NT), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

template <typename T>
clm_status launch_postpre(Plan* p, const TileArgs<T>& a, int64_t np, hipStream_t s) {
  const dim3 grid(unsigned(np * a.ntile * a.ntile));
  switch (2 * (a.nu + a.nu2) + 2) {
    case 6:
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_postpre<T, 6>), grid, dim3(QT<T, 6>::NT), 0, s,
                         a);
      break;
    case 8:
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_postpre<T, 8>), grid, dim3(QT<T, 8>::NT), 0, s,
                         a);
      break;
    case 10:
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_postpre<T, 10>), grid, dim3(QT<T, 10>::NT), 0, s,
                         a);
      break;
    default:
      return fail(p, CLM_EUNSUPPORTED, "fused smoothing needs nu_pre + nu_post <= 4");
  }
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

// The plan's patch geometry as the setup kernels take it.
SetupArgs setup_geometry(const Plan* p) {
  const clm_plan_desc& d = p->d;
  SetupArgs a{};
  a.n = p->n;
  a.tile = p->n < kTile ? p->n : kTile;
  a.ntile = p->n / a.tile;
  a.L = p->L;
  a.delta = p->delta;
  a.rot = p->rot;
  a.coef = p->coef + p->lev[0].crow;
  a.rs = hpx::Rings{p->ring_s, p->ringi_s, p->ringx_s, p->nring_s, d.nside_sht};
  a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->ringx_f, p->nring_f, d.nside_fine};
  a.ring_shift = 0;
  while ((d.nside_sht << a.ring_shift) < d.nside_fine) ++a.ring_shift;
  a.meta = reinterpret_cast<SetupMeta*>(p->setup_meta);
  return a;
}

template <typename T>
clm_status run_mg(Plan* p, const void* kappa, int kappa_fp64, int slot, hipStream_t s,
                  const clm_particles* parts) {
  const clm_plan_desc& d = p->d;
  Slot& sl = p->slots[slot];
  const int n = p->n;
  const int64_t np = p->nbundle;
  // the patches the grids cover: the domain's (pm maps compact indices to
  // patches) or all of them
  const int64_t na = p->domain ? p->nactive : np;
  const int* pm = p->domain ? p->dom_map : nullptr;
  // patch setup
  {
    SetupArgs a = setup_geometry(p);
    a.pmap = pm;
    a.psi_s = sl.psi_s;
    a.kappa = kappa;
    a.kappa_fp64 = kappa_fp64;
    a.spad = p->spad;
    a.kpad = p->kpad;
    a.pad_s = p->pad_s;
    a.pad_f = p->pad_f;
    pad_rings(sl.psi_s, p->spad, p->ringi_s, p->nring_s, p->d.nside_sht, p->pad_s, s);
    if (kappa && kappa_fp64)
      pad_rings(static_cast<const double*>(kappa), static_cast<double*>(p->kpad), p->ringi_f,
                p->nring_f, p->d.nside_fine, p->pad_f, s);
    else if (kappa)
      pad_rings(static_cast<const float*>(kappa), static_cast<float*>(p->kpad), p->ringi_f,
                p->nring_f, p->d.nside_fine, p->pad_f, s);
    CLM_LAUNCH_CHECK();
    a.red = p->red;
    a.u0 = sl.u0;
    a.fprime = p->fprime;
    const dim3 grid(unsigned(na * a.ntile * a.ntile));
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
  // particles: their deposition on the patch cells completes the source
  if (parts) {
    const clm_status st = patch_deposit(p, parts, s);
    if (st != CLM_OK) return st;
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
  la.pmap = pm;
  size_t lds_elems = 0;
  for (int l = K; l < p->nlev; ++l) {
    const size_t nn = size_t(n >> l);
    lds_elems += nn * nn * (l > K ? 3 : 2) + 7 * nn;
  }
  const size_t lds_bytes = lds_elems * sizeof(T);
  if (allow_lds(p, k_mg_lds<T>, lds_bytes) != CLM_OK) return CLM_EHIP;

  // epsilon rule (mg_vcycles == 0): every patch runs V-cycles until its
  // epsilon drops below mg_eps, at most mg_max_vcycles; patches that stopped
  // skip the remaining cycles, so the host never waits on the device
  const bool eps_mode = d.mg_vcycles == 0;
  const int ncyc = eps_mode ? d.mg_max_vcycles : d.mg_vcycles;
  const int* done = eps_mode ? p->mg_done_dev : nullptr;
  auto tile_args = [&](int l, bool pre) {
    TileArgs<T> a{};
    a.n = n >> l;
    a.ntile = a.n / kTile;
    a.lgt = 0;
    while ((1 << a.lgt) < a.ntile) ++a.lgt;
    a.nu = pre ? d.nu_pre : d.nu_post;
    a.coef = p->coef + p->lev[l].crow;
    a.rowt = static_cast<const T*>(p->rowt) + 2 * p->lev[l].crow;
    a.done = done;
    a.pmap = pm;
    return a;
  };
  // per-patch convergence record: patches outside a domain report 0 cycles
  // and NaN
  const dim3 gfill(unsigned((np + kBlock - 1) / kBlock));
  const dim3 gfa(unsigned((na + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_fill_f64, gfill, dim3(kBlock), 0, s, np, double(NAN), p->mg_eps_dev);
  if (eps_mode) {
    hipLaunchKernelGGL(k_fill_int, gfill, dim3(kBlock), 0, s, np, 0, p->mg_done_dev);
    hipLaunchKernelGGL(k_fill_int, gfill, dim3(kBlock), 0, s, np, 0, p->mg_cycles_dev);
  } else {
    if (pm) hipLaunchKernelGGL(k_fill_int, gfill, dim3(kBlock), 0, s, np, 0, p->mg_cycles_dev);
    hipLaunchKernelGGL(k_fill_patches, gfa, dim3(kBlock), 0, s, na, pm, d.mg_vcycles,
                       p->mg_cycles_dev);
  }
  CLM_LAUNCH_CHECK();
  la.done = done;
  const int eps_tc = std::min(kEpsTC, n / 2), eps_nt = (n / 2) / eps_tc;
  auto eps_eval = [&](int cycle) -> clm_status {
    EpsArgs<T> e{};
    e.n = n;
    e.tc = eps_tc;
    e.ntile = eps_nt;
    e.c0 = p->coef + p->lev[0].crow;
    e.c1 = p->coef + p->lev[1].crow;
    e.du = du;
    e.fp = fp;
    e.done = p->mg_done_dev;
    e.part = p->mg_eps_part;
    e.pmap = pm;
    EpsFinal g{};
    g.tiles = eps_nt * eps_nt;
    g.eps = d.mg_eps;
    g.cycle = cycle;
    g.part = p->mg_eps_part;
    g.done = p->mg_done_dev;
    g.cycles = p->mg_cycles_dev;
    g.eps_out = p->mg_eps_dev;
    g.active = p->mg_active_dev;
    g.status = p->status_dev;
    g.pmap = pm;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, int64_t(1), 0, p->mg_active_dev);
    {
      CLM_TIMED(p, s, "mg_eps");
      const dim3 ge(unsigned(na * g.tiles));
      if (eps_tc == 16)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_eps<T, 16>), ge, dim3(kBlock), 0, s, e);
      else if (eps_tc == 8)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_eps<T, 8>), ge, dim3(kBlock), 0, s, e);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_eps<T, 4>), ge, dim3(kBlock), 0, s, e);
      hipLaunchKernelGGL(k_mg_eps_final, dim3(unsigned(na)), dim3(64), 0, s, g);
    }
    CLM_LAUNCH_CHECK();
    return CLM_OK;
  };
  bool all_done = false;
  // With a fixed cycle count the finest level's post-smoothing of a cycle
  // and the pre-smoothing of the next run as one kernel; the pre-smoothed
  // iterate then alternates between du and dt, starting so that the last
  // cycle's post-smoothing reads dt and writes du.
  const bool fuse = !eps_mode && K >= 1 && d.nu_pre + d.nu_post <= 4;
  T* cur = fuse && ((ncyc - 1) & 1) ? du : dt;  // pre-smoothed finest iterate
  bool have_pre = false;                        // formed by the fused kernel
  if (fuse && !p->ubar1b) return fail(p, CLM_EHIP, "fused smoothing without its buffers");
  // the restricted iterate of level l (level 1 alternates with ubar1b under
  // fused smoothing)
  void* ub1 = K >= 1 ? p->ubar[1] : nullptr;
  auto ubar_at = [&](int l) { return static_cast<T*>(l == 1 ? ub1 : p->ubar[l]); };
  for (int cyc = 0; cyc < ncyc; ++cyc) {
    const bool first = cyc == 0;
    if (eps_mode && !first) {
      // epsilon after cyc cycles; stop once every patch is below mg_eps
      const clm_status st = eps_eval(cyc);
      if (st != CLM_OK) return st;
      CLM_HIP(hipMemcpyAsync(p->mg_active_host, p->mg_active_dev, sizeof(int),
                             hipMemcpyDeviceToHost, s));
      CLM_HIP(hipStreamSynchronize(s));
      if (*p->mg_active_host == 0) {
        all_done = true;
        break;
      }
    }
    if (K == 0) {
      la.u_in = first ? nullptr : du;
      la.f_in = fp;
      la.u_out = du;
      la.fas_source = 0;
      {
        CLM_TIMED(p, s, "mg_lds");
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_lds<T>), dim3(na), dim3(kLdsBlock), lds_bytes, s,
                           la);
      }
      CLM_LAUNCH_CHECK();
      continue;
    }
    // pre-smoothing, residual and restriction on the tile levels
    for (int l = 0; l < K; ++l) {
      if (l == 0 && have_pre) continue;
      TileArgs<T> a = tile_args(l, true);
      if (l == 0) {
        a.u_in = first ? nullptr : du;
        a.f_in = fp;
        a.u_out = cur;
        a.fas_source = 0;
      } else {
        a.u_in = ubar_at(l);
        a.f_in = static_cast<T*>(p->rbar[l]);
        a.u_out = static_cast<T*>(p->ulev[l]);
        a.f_out = static_cast<T*>(p->flev[l]);
        a.fas_source = 1;
      }
      a.ubar_out = ubar_at(l + 1);
      a.rbar_out = static_cast<T*>(p->rbar[l + 1]);
      {
        CLM_TIMED(p, s, l == 0 ? "mg_pre_l0" : "mg_pre_l1+");
        const clm_status st = launch_tile<T, true>(p, a, na, s);
        if (st != CLM_OK) return st;
      }
    }
    // the LDS-resident levels
    la.u_in = ubar_at(K);
    la.f_in = static_cast<T*>(p->rbar[K]);
    la.u_out = static_cast<T*>(p->ulev[K]);
    la.fas_source = 1;
    {
      CLM_TIMED(p, s, "mg_lds");
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_lds<T>), dim3(na), dim3(kLdsBlock), lds_bytes, s, la);
    }
    CLM_LAUNCH_CHECK();
    // prolongation, correction and post-smoothing back up
    for (int l = K - 1; l >= 0; --l) {
      TileArgs<T> a = tile_args(l, false);
      a.uc = static_cast<T*>(l + 1 == K ? p->ulev[K] : p->ulev2[l + 1]);
      a.ubarc = ubar_at(l + 1);
      if (l == 0 && fuse && cyc + 1 < ncyc) {
        // post-smoothing of this cycle + pre-smoothing of the next
        T* nxt = cur == dt ? du : dt;
        a.nu = d.nu_post;
        a.nu2 = d.nu_pre;
        a.u_in = cur;
        a.f_in = fp;
        a.u_out = nxt;
        // the correction reads this cycle's restricted iterate (a.ubarc);
        // the next cycle's goes to the other level-1 array
        void* ub1n = ub1 == p->ubar[1] ? p->ubar1b : p->ubar[1];
        a.ubar_out = static_cast<T*>(ub1n);
        a.rbar_out = static_cast<T*>(p->rbar[1]);
        {
          CLM_TIMED(p, s, "mg_postpre_l0");
          const clm_status st = launch_postpre<T>(p, a, na, s);
          if (st != CLM_OK) return st;
        }
        ub1 = ub1n;
        cur = nxt;
        have_pre = true;
        continue;
      }
      if (l == 0) {
        if (cur != dt) return fail(p, CLM_EHIP, "multigrid buffer order");
        a.u_in = dt;
        a.f_in = fp;
        a.u_out = du;
        have_pre = false;
      } else {
        a.u_in = static_cast<T*>(p->ulev[l]);
        a.f_in = static_cast<T*>(p->flev[l]);
        a.f_scaled = 1;
        a.u_out = static_cast<T*>(p->ulev2[l]);
      }
      {
        CLM_TIMED(p, s, l == 0 ? "mg_post_l0" : "mg_post_l1+");
        const clm_status st = launch_tile<T, false>(p, a, na, s);
        if (st != CLM_OK) return st;
      }
    }
  }
  if (eps_mode && !all_done) {
    const clm_status st = eps_eval(ncyc);
    if (st != CLM_OK) return st;
    hipLaunchKernelGGL(k_notconv, gfa, dim3(kBlock), 0, s, na, pm,
                       static_cast<const int*>(p->mg_done_dev), p->status_dev);
    CLM_LAUNCH_CHECK();
  }
  return CLM_OK;
}

}  // namespace

int setup_ring_pad(int nside) {
  // asin(kSetupSeries) 4 nside / (2 pi) = 0.03185 nside pixels beyond the
  // ring ends, one more for the pair, one for t0 in (-1, n)
  return int(std::ceil(0.032 * nside)) + 3;
}

int64_t setup_tiles(const Plan* p) {
  const int tile = p->n < kTile ? p->n : kTile;
  return p->nbundle * (p->n / tile) * (p->n / tile);
}

clm_status setup_tables(Plan* p, hipStream_t s) {
  const SetupArgs a = setup_geometry(p);
  const int64_t nt = setup_tiles(p);
  if (nt == 0) return CLM_OK;
  hipLaunchKernelGGL(k_setup_meta, dim3(unsigned(nt)), dim3(kMetaBlock), 0, s, a);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status mg_solve(Plan* p, const void* kappa, int kappa_fp64, int slot, hipStream_t s,
                    const clm_particles* parts) {
  if (p->nlev > 16) return fail(p, CLM_EUNSUPPORTED, "too many multigrid levels");
  return p->fp64mg ? run_mg<double>(p, kappa, kappa_fp64, slot, s, parts)
                   : run_mg<float>(p, kappa, kappa_fp64, slot, s, parts);
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
