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

// Row coefficients of a level in LDS, as T: s_m, s_p, 1/s_c, area.
template <typename T>
struct RowC {
  T sm, sp, isc, A;
};

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

__device__ __forceinline__ void patch_point(const double* R, double thp, double php,
                                            double& th, double& ph) {
  double st, ct, sp, cp;
  sincos(thp, &st, &ct);
  sincos(php, &sp, &cp);
  const double x = st * cp, y = st * sp, z = ct;
  const double vx = R[0] * x + R[3] * y + R[6] * z;
  const double vy = R[1] * x + R[4] * y + R[7] * z;
  const double vz = R[2] * x + R[5] * y + R[8] * z;
  th = atan2(sqrt(vx * vx + vy * vy), vz);
  ph = atan2(vy, vx);
  if (ph < 0) ph += 2.0 * kPi;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_patch_setup(SetupArgs a) {
  extern __shared__ double shu[];  // [(tile+2)^2] u0 over the tile and one halo ring
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int ti = tt / a.ntile, tj = tt % a.ntile;
  const int RR = a.tile + 2;
  const int i0 = ti * a.tile - 1, j0 = tj * a.tile - 1;
  const int n = a.n;
  const double* R = a.rot + 9 * patch;
  const double th0 = kPi / 2 - a.L / 2, ph0 = -a.L / 2;
  // interior cells of the region
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    double v = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      double th, ph;
      patch_point(R, th0 + (gi + 0.5) * a.delta, ph0 + (gj + 0.5) * a.delta, th, ph);
      v = hpx::interp(a.rs, a.psi_s, th, ph);
    }
    shu[idx] = v;
  }
  __syncthreads();
  // ghost cells of the region (on the patch boundary)
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    const bool gI = gi == -1 || gi == n, gJ = gj == -1 || gj == n;
    if (!(gI || gJ)) continue;
    if ((gI && (gj < -1 || gj > n)) || (gJ && (gi < -1 || gi > n))) continue;
    double thp, php;
    int ai = li, aj = lj;  // adjacent interior cell
    if (gI) { thp = gi < 0 ? th0 : th0 + a.L; ai = gi < 0 ? li + 1 : li - 1; }
    else    { thp = th0 + (gi + 0.5) * a.delta; }
    if (gJ) { php = gj < 0 ? ph0 : ph0 + a.L; aj = gj < 0 ? lj + 1 : lj - 1; }
    else    { php = ph0 + (gj + 0.5) * a.delta; }
    double th, ph;
    patch_point(R, thp, php, th, ph);
    const double b = hpx::interp(a.rs, a.psi_s, th, ph);
    shu[idx] = 2.0 * b - shu[ai * RR + aj];
  }
  __syncthreads();
  const double mean = a.red[1023];
  const size_t G = size_t(n + 2);
  double* u0 = a.u0 + size_t(patch) * G * G;
  T* fp = static_cast<T*>(a.fprime) + size_t(patch) * n * n;
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int li = idx / RR, lj = idx % RR;
    const int gi = i0 + li, gj = j0 + lj;
    const bool interior = li >= 1 && li <= a.tile && lj >= 1 && lj <= a.tile;
    // write u0: the tile's cells, plus the patch ghosts beside this tile
    const bool own_i = (li >= 1 && li <= a.tile) || (gi == -1) || (gi == n);
    const bool own_j = (lj >= 1 && lj <= a.tile) || (gj == -1) || (gj == n);
    if (own_i && own_j && gi >= -1 && gi <= n && gj >= -1 && gj <= n)
      u0[size_t(gi + 1) * G + (gj + 1)] = shu[idx];
    if (!interior) continue;
    double th, ph;
    patch_point(R, th0 + (gi + 0.5) * a.delta, ph0 + (gj + 0.5) * a.delta, th, ph);
    const double kv = a.kappa_fp64 ? hpx::interp(a.rf, static_cast<const double*>(a.kappa), th, ph)
                                   : hpx::interp(a.rf, static_cast<const float*>(a.kappa), th, ph);
    const double f = 2.0 * (kv - mean);
    const double* c = a.coef + 4 * gi;
    const double u = shu[idx];
    const double Lu = (c[0] * (shu[idx - RR] - u) + c[1] * (shu[idx + RR] - u) +
                       (shu[idx - 1] - 2.0 * u + shu[idx + 1]) / c[2]) / c[3];
    fp[size_t(gi) * n + gj] = T(f - Lu);
  }
}

// ------------------------------------------------------------ tile kernels
template <typename T>
struct TileArgs {
  int n, ntile, tile, hh, nu;
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

// Load rows of coefficients for region rows [i0, i0 + RR) into LDS.
template <typename T>
__device__ __forceinline__ void load_rows(const double* coef, int n, int i0, int RR, RowC<T>* rc) {
  for (int r = threadIdx.x; r < RR; r += blockDim.x) {
    const int gi = i0 + r;
    RowC<T> v{T(0), T(0), T(0), T(1)};
    if (gi >= 0 && gi < n) {
      const double* c = coef + 4 * gi;
      v.sm = T(c[0]); v.sp = T(c[1]); v.isc = T(1.0 / c[2]); v.A = T(c[3]);
    }
    rc[r] = v;
  }
}

// (L u)_ij for a cell of the region, faces of the patch as zero Dirichlet
// (a neighbour across the patch face is -u_ij).
template <typename T>
__device__ __forceinline__ T lap(const T* u, int RR, int li, int lj, int gi, int gj, int n,
                                 const RowC<T>& c) {
  const T uc = u[li * RR + lj];
  const T up = gi > 0 ? u[(li - 1) * RR + lj] : -uc;
  const T dn = gi < n - 1 ? u[(li + 1) * RR + lj] : -uc;
  const T lf = gj > 0 ? u[li * RR + lj - 1] : -uc;
  const T rt = gj < n - 1 ? u[li * RR + lj + 1] : -uc;
  return (c.sm * (up - uc) + c.sp * (dn - uc) + (lf - T(2) * uc + rt) * c.isc) / c.A;
}

// Gauss-Seidel solve of one cell (neighbours across the patch face fold
// into the diagonal).
template <typename T>
__device__ __forceinline__ T gs_cell(const T* u, const T* f, int RR, int li, int lj, int gi,
                                     int gj, int n, const RowC<T>& c) {
  T num = -c.A * f[li * RR + lj];
  T diag = c.sm + c.sp + T(2) * c.isc;
  if (gi > 0) num += c.sm * u[(li - 1) * RR + lj]; else diag += c.sm;
  if (gi < n - 1) num += c.sp * u[(li + 1) * RR + lj]; else diag += c.sp;
  T lr = T(0);
  if (gj > 0) lr += u[li * RR + lj - 1]; else diag += c.isc;
  if (gj < n - 1) lr += u[li * RR + lj + 1]; else diag += c.isc;
  num += lr * c.isc;
  return num / diag;
}

// One red-black half sweep over the region cells at distance >= 1 from the
// region edge that lie in the patch.
template <typename T>
__device__ __forceinline__ void half_sweep(T* u, const T* f, const RowC<T>* rc, int RR, int i0,
                                           int j0, int n, int color) {
  const int half = (RR - 1) / 2;  // cells of one colour per row, upper bound
  const int total = (RR - 2) * half;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int li = 1 + idx / half;
    const int gi = i0 + li;
    const int off = (color + gi + j0 + 1) & 1;
    const int lj = 1 + 2 * (idx % half) + off;
    const int gj = j0 + lj;
    if (lj > RR - 2 || gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
    u[li * RR + lj] = gs_cell(u, f, RR, li, lj, gi, gj, n, rc[li]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_pre(TileArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int RR = a.tile + 2 * a.hh;
  T* u = reinterpret_cast<T*>(smem);
  T* f = u + RR * RR;
  RowC<T>* rc = reinterpret_cast<RowC<T>*>(f + RR * RR);
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int i0 = (tt / a.ntile) * a.tile - a.hh, j0 = (tt % a.ntile) * a.tile - a.hh;
  const int n = a.n;
  const size_t pbase = size_t(patch) * n * n;
  load_rows(a.coef, n, i0, RR, rc);
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int gi = i0 + idx / RR, gj = j0 + idx % RR;
    const bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
    const size_t g = pbase + size_t(gi) * n + gj;
    u[idx] = (in && a.u_in) ? a.u_in[g] : T(0);
    f[idx] = in ? a.f_in[g] : T(0);
  }
  __syncthreads();
  if (a.fas_source) {
    // f = L_H ubar + rbar on the region cells away from its edge
    for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
      const int li = idx / RR, lj = idx % RR;
      const int gi = i0 + li, gj = j0 + lj;
      if (li < 1 || li > RR - 2 || lj < 1 || lj > RR - 2) continue;
      if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
      f[idx] += lap(u, RR, li, lj, gi, gj, n, rc[li]);
    }
    __syncthreads();
  }
  for (int s = 0; s < a.nu; ++s) {
    half_sweep(u, f, rc, RR, i0, j0, n, 0);
    __syncthreads();
    half_sweep(u, f, rc, RR, i0, j0, n, 1);
    __syncthreads();
  }
  // write the tile interior (and its source on coarse levels)
  for (int idx = threadIdx.x; idx < a.tile * a.tile; idx += blockDim.x) {
    const int li = a.hh + idx / a.tile, lj = a.hh + idx % a.tile;
    const size_t g = pbase + size_t(i0 + li) * n + (j0 + lj);
    a.u_out[g] = u[li * RR + lj];
    if (a.fas_source) a.f_out[g] = f[li * RR + lj];
  }
  // residual and area-weighted restriction of the tile interior
  const int th = a.tile / 2, nc = n / 2;
  const size_t cbase = size_t(patch) * nc * nc;
  for (int idx = threadIdx.x; idx < th * th; idx += blockDim.x) {
    const int ci = idx / th, cj = idx % th;
    const int li = a.hh + 2 * ci, lj = a.hh + 2 * cj;
    const int gi = i0 + li, gj = j0 + lj;
    T r[4], uu[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k >> 1, dj = k & 1;
      const int id = (li + di) * RR + lj + dj;
      uu[k] = u[id];
      r[k] = f[id] - lap(u, RR, li + di, lj + dj, gi + di, gj + dj, n, rc[li + di]);
    }
    const T a0 = rc[li].A, a1 = rc[li + 1].A;
    const T den = T(2) * (a0 + a1);
    const size_t gc = cbase + size_t(gi / 2) * nc + gj / 2;
    a.ubar_out[gc] = (a0 * (uu[0] + uu[1]) + a1 * (uu[2] + uu[3])) / den;
    a.rbar_out[gc] = (a0 * (r[0] + r[1]) + a1 * (r[2] + r[3])) / den;
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_post(TileArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int RR = a.tile + 2 * a.hh;
  const int CR = RR / 2 + 3;  // coarse rows/cols covering the region +- 1
  T* u = reinterpret_cast<T*>(smem);
  T* f = u + RR * RR;
  T* e = f + RR * RR;
  RowC<T>* rc = reinterpret_cast<RowC<T>*>(e + CR * CR);
  const int64_t lb = xcd_block();
  const int tpp = a.ntile * a.ntile;
  const int64_t patch = lb / tpp;
  const int tt = int(lb % tpp);
  const int i0 = (tt / a.ntile) * a.tile - a.hh, j0 = (tt % a.ntile) * a.tile - a.hh;
  const int n = a.n, nc = n / 2;
  const size_t pbase = size_t(patch) * n * n, cbase = size_t(patch) * nc * nc;
  const int ci0 = (i0 >> 1) - 1, cj0 = (j0 >> 1) - 1;  // floor division (i0 may be < 0)
  load_rows(a.coef, n, i0, RR, rc);
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int gi = i0 + idx / RR, gj = j0 + idx % RR;
    const bool in = gi >= 0 && gi < n && gj >= 0 && gj < n;
    const size_t g = pbase + size_t(gi) * n + gj;
    u[idx] = in ? a.u_in[g] : T(0);
    f[idx] = in ? a.f_in[g] : T(0);
  }
  for (int idx = threadIdx.x; idx < CR * CR; idx += blockDim.x) {
    const int I = ci0 + idx / CR, J = cj0 + idx % CR;
    T v = T(0);
    if (I >= 0 && I < nc && J >= 0 && J < nc) {
      const size_t g = cbase + size_t(I) * nc + J;
      v = a.uc[g] - a.ubarc[g];
    }
    e[idx] = v;
  }
  __syncthreads();
  auto ef = [&](int I, int J) { return e[(I - ci0) * CR + (J - cj0)]; };
  for (int idx = threadIdx.x; idx < RR * RR; idx += blockDim.x) {
    const int gi = i0 + idx / RR, gj = j0 + idx % RR;
    if (gi < 0 || gi >= n || gj < 0 || gj >= n) continue;
    u[idx] += prolong_cell<T>(gi, gj, n, ef);
  }
  __syncthreads();
  for (int s = 0; s < a.nu; ++s) {
    half_sweep(u, f, rc, RR, i0, j0, n, 0);
    __syncthreads();
    half_sweep(u, f, rc, RR, i0, j0, n, 1);
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < a.tile * a.tile; idx += blockDim.x) {
    const int li = a.hh + idx / a.tile, lj = a.hh + idx % a.tile;
    a.u_out[pbase + size_t(i0 + li) * n + (j0 + lj)] = u[li * RR + lj];
  }
}

// ------------------------------------------------------------ LDS levels
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
__device__ __forceinline__ T lap_g(const T* u, int n, int i, int j, const double* c) {
  const T uc = u[i * n + j];
  const T up = i > 0 ? u[(i - 1) * n + j] : -uc;
  const T dn = i < n - 1 ? u[(i + 1) * n + j] : -uc;
  const T lf = j > 0 ? u[i * n + j - 1] : -uc;
  const T rt = j < n - 1 ? u[i * n + j + 1] : -uc;
  return (T(c[0]) * (up - uc) + T(c[1]) * (dn - uc) + (lf - T(2) * uc + rt) * T(1.0 / c[2])) /
         T(c[3]);
}

template <typename T>
__device__ void lds_smooth(T* u, const T* f, int n, const double* coef, int sweeps) {
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      const int half = n / 2;
      for (int idx = threadIdx.x; idx < n * half; idx += blockDim.x) {
        const int i = idx / half;
        const int j = 2 * (idx % half) + ((color + i) & 1);
        const double* c = coef + 4 * i;
        const T sm = T(c[0]), sp = T(c[1]), isc = T(1.0 / c[2]), A = T(c[3]);
        T num = -A * f[i * n + j];
        T diag = sm + sp + T(2) * isc;
        if (i > 0) num += sm * u[(i - 1) * n + j]; else diag += sm;
        if (i < n - 1) num += sp * u[(i + 1) * n + j]; else diag += sp;
        T lr = T(0);
        if (j > 0) lr += u[i * n + j - 1]; else diag += isc;
        if (j < n - 1) lr += u[i * n + j + 1]; else diag += isc;
        num += lr * isc;
        u[i * n + j] = num / diag;
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_lds(LdsArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int64_t patch = xcd_block();
  const int K = a.lv.K, nl = a.lv.nlev;
  // LDS: per level l >= K: u[n_l^2], f[n_l^2], ubar[n_l^2] (l > K)
  T* base = reinterpret_cast<T*>(smem);
  T* U[16];
  T* Fv[16];
  T* B[16];
  {
    T* q = base;
    for (int l = K; l < nl; ++l) {
      const int nn = a.lv.n0 >> (l - K);
      U[l] = q; q += nn * nn;
      Fv[l] = q; q += nn * nn;
      if (l > K) { B[l] = q; q += nn * nn; }
    }
  }
  const int n0 = a.lv.n0;
  const size_t g0 = size_t(patch) * n0 * n0;
  for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x) {
    U[K][idx] = a.u_in ? a.u_in[g0 + idx] : T(0);
    Fv[K][idx] = a.f_in[g0 + idx];
  }
  __syncthreads();
  if (a.fas_source) {
    const double* c = a.coef + a.lv.crow[K];
    T tmp[16];
    int cnt = 0;
    for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x)
      tmp[cnt++] = lap_g(U[K], n0, idx / n0, idx % n0, c + 4 * (idx / n0));
    __syncthreads();
    cnt = 0;
    for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x) Fv[K][idx] += tmp[cnt++];
    __syncthreads();
  }
  // down
  for (int l = K; l < nl - 1; ++l) {
    const int nn = n0 >> (l - K), nc = nn / 2;
    const double* c = a.coef + a.lv.crow[l];
    const double* cc = a.coef + a.lv.crow[l + 1];
    lds_smooth(U[l], Fv[l], nn, c, a.nu1);
    for (int idx = threadIdx.x; idx < nc * nc; idx += blockDim.x) {
      const int I = idx / nc, J = idx % nc;
      T r[4], uu[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = 2 * I + (k >> 1), j = 2 * J + (k & 1);
        uu[k] = U[l][i * nn + j];
        r[k] = Fv[l][i * nn + j] - lap_g(U[l], nn, i, j, c + 4 * i);
      }
      const T a0 = T(c[4 * (2 * I) + 3]), a1 = T(c[4 * (2 * I + 1) + 3]);
      const T den = T(2) * (a0 + a1);
      const T ub = (a0 * (uu[0] + uu[1]) + a1 * (uu[2] + uu[3])) / den;
      B[l + 1][idx] = ub;
      U[l + 1][idx] = ub;
      Fv[l + 1][idx] = (a0 * (r[0] + r[1]) + a1 * (r[2] + r[3])) / den;
    }
    __syncthreads();
    // f_H = L_H ubar + rbar
    T tmp[4];
    int cnt = 0;
    for (int idx = threadIdx.x; idx < nc * nc; idx += blockDim.x)
      tmp[cnt++] = lap_g(U[l + 1], nc, idx / nc, idx % nc, cc + 4 * (idx / nc));
    __syncthreads();
    cnt = 0;
    for (int idx = threadIdx.x; idx < nc * nc; idx += blockDim.x) Fv[l + 1][idx] += tmp[cnt++];
    __syncthreads();
  }
  // coarsest: exact solve (float64)
  {
    const int l = nl - 1;
    double v = 0.0;
    if (threadIdx.x < 16) {
      for (int k = 0; k < 16; ++k) v += a.cinv[threadIdx.x * 16 + k] * double(Fv[l][k]);
    }
    __syncthreads();
    if (threadIdx.x < 16) U[l][threadIdx.x] = T(v);
    __syncthreads();
  }
  // up
  for (int l = nl - 2; l >= K; --l) {
    const int nn = n0 >> (l - K), nc = nn / 2;
    const T* uc = U[l + 1];
    const T* bc = B[l + 1];
    auto ef = [&](int I, int J) { return uc[I * nc + J] - bc[I * nc + J]; };
    for (int idx = threadIdx.x; idx < nn * nn; idx += blockDim.x)
      U[l][idx] += prolong_cell<T>(idx / nn, idx % nn, nn, ef);
    __syncthreads();
    lds_smooth(U[l], Fv[l], nn, a.coef + a.lv.crow[l], a.nu2);
  }
  for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x) a.u_out[g0 + idx] = U[K][idx];
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
    a.rs = hpx::Rings{p->ring_s, p->ringi_s, p->nring_s, d.nside_sht};
    a.rf = hpx::Rings{p->ring_f, p->ringi_f, p->nring_f, d.nside_fine};
    a.psi_s = sl.psi_s;
    a.kappa = kappa;
    a.kappa_fp64 = kappa_fp64;
    a.red = p->red;
    a.u0 = sl.u0;
    a.fprime = p->fprime;
    const size_t shm = size_t(a.tile + 2) * (a.tile + 2) * sizeof(double);
    if (allow_lds(p, k_patch_setup<T>, shm) != CLM_OK) return CLM_EHIP;
    {
      CLM_TIMED(p, s, "patch_setup");
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_patch_setup<T>), dim3(np * a.ntile * a.ntile),
                         dim3(kBlock), shm, s, a);
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
    lds_elems += nn * nn * (l > K ? 3 : 2);
  }
  const size_t lds_bytes = lds_elems * sizeof(T);
  if (allow_lds(p, k_mg_lds<T>, lds_bytes) != CLM_OK) return CLM_EHIP;

  auto tile_args = [&](int l, bool pre) {
    TileArgs<T> a{};
    a.n = n >> l;
    a.tile = kTile;
    a.ntile = a.n / kTile;
    a.nu = pre ? d.nu_pre : d.nu_post;
    a.hh = pre ? 2 * a.nu + 1 : 2 * a.nu;
    a.coef = p->coef + p->lev[l].crow;
    return a;
  };
  auto pre_bytes = [&](const TileArgs<T>& a) {
    const size_t RR = a.tile + 2 * a.hh;
    return 2 * RR * RR * sizeof(T) + RR * sizeof(RowC<T>);
  };
  auto post_bytes = [&](const TileArgs<T>& a) {
    const size_t RR = a.tile + 2 * a.hh, CR = RR / 2 + 3;
    return (2 * RR * RR + CR * CR) * sizeof(T) + RR * sizeof(RowC<T>);
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
      const size_t b = pre_bytes(a);
      if (allow_lds(p, k_mg_pre<T>, b) != CLM_OK) return CLM_EHIP;
      {
        CLM_TIMED(p, s, l == 0 ? "mg_pre_l0" : "mg_pre_l1+");
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_pre<T>), dim3(np * a.ntile * a.ntile),
                           dim3(kBlock), b, s, a);
      }
      CLM_LAUNCH_CHECK();
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
      const size_t b = post_bytes(a);
      if (allow_lds(p, k_mg_post<T>, b) != CLM_OK) return CLM_EHIP;
      {
        CLM_TIMED(p, s, l == 0 ? "mg_post_l0" : "mg_post_l1+");
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mg_post<T>), dim3(np * a.ntile * a.ntile),
                           dim3(kBlock), b, s, a);
      }
      CLM_LAUNCH_CHECK();
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
