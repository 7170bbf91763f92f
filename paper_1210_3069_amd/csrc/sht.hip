// Spherical-harmonic stage of the plane solve (Sec. 3.2): demean and
// degrade, ring DFTs, Legendre analysis and synthesis, the harmonic Poisson
// step and the pure-SHT derivative synthesis.  All float64.
//
// Layout: F and G are ring-major [ring][m] complex (m = 0..lmax); the
// Legendre kernels work one order m per workgroup with the north rings
// spread over the threads, so the three-term recurrence in l runs in
// registers and mirror rings are folded in with the (-1)^(l+m) parity.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "clm_internal.h"
#include "healpix_dev.h"

namespace clm {

// lambda_mm(theta_q) for the north rings, by the product recursion
// lambda_00 = 1/sqrt(4 pi), lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},
// with a scale exponent in units of 2^800 keeping the mantissa above 2^-400.
__global__ void k_lambda_mm(const double* rt, int H, int lmax, double* mant, int* scale) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= H) return;
  const double st = rt[4 * q + 1];
  double v = 0.28209479177387814347403972578039;  // 1/sqrt(4 pi)
  int s = 0;
  mant[q] = v;
  scale[q] = 0;
  const double tiny = 0x1p-400, big = 0x1p800;
  for (int m = 1; m <= lmax; ++m) {
    v *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
    if (fabs(v) < tiny) {
      v *= big;
      s -= 1;
    }
    mant[size_t(m) * H + q] = v;
    scale[size_t(m) * H + q] = s;
  }
}

namespace {

constexpr int kBlock = 256;

// FP64 Legendre workgroups: as many threads as the rings need, up to 1024
// (512 for 8 rings per thread, 256 for 16, whose registers allow no more).
// The per-m tables of a workgroup fill most of the LDS, so one workgroup
// runs per CU and its size sets the waves that hide the recurrence's
// latency.
constexpr int leg_threads_max(int rpt) { return rpt <= 4 ? 1024 : rpt == 8 ? 512 : 256; }
inline int round64(int v) { return (v + 63) / 64 * 64; }
constexpr double kPi = 3.14159265358979323846;
constexpr double kHuge = 0x1p400;    // rescale threshold of the scaled recurrence
constexpr double kSmall = 0x1p-800;  // rescale factor

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// v moved across lanes by a DPP pattern (both 32-bit halves); lanes of rows
// outside ROW_MASK read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROW_MASK, 0xF, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(
      static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sums over the 64 lanes of a wave of 16 values per lane at once, by
// recursive halving: at the exchanges with lane masks 32, 16 (shuffles), 15
// and 7 (row mirror, half-row mirror) a lane keeps half of its values, the
// half picked by one of its own lane bits (5, 4, 3, 2), adds the partner's
// copy of that half and hands over the other; masks 2 and 1 (quad permutes)
// then finish the sum.  The six masks span all six lane bits, so lane L ends
// with the wave total of value L >> 2.  17 exchanges instead of the 96 of
// sixteen separate reductions.
__device__ __forceinline__ double wave_sum16(const double (&v)[16]) {
  const int lane = threadIdx.x & 63;
  double v8[8], v4[4], v2[2];
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double send = b5 ? v[j] : v[j + 8], keep = b5 ? v[j + 8] : v[j];
    v8[j] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double send = b4 ? v8[j] : v8[j + 4], keep = b4 ? v8[j + 4] : v8[j];
    v4[j] = keep + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double send = b3 ? v4[j] : v4[j + 2], keep = b3 ? v4[j + 2] : v4[j];
    v2[j] = keep + dpp_move<0x140>(send);  // row_mirror: lane ^ 15 in its row
  }
  const double send = b2 ? v2[0] : v2[1], keep = b2 ? v2[1] : v2[0];
  double t = keep + dpp_move<0x141>(send);  // row_half_mirror: lane ^ 7
  t += dpp_move<0x4E>(t);                   // quad_perm [2, 3, 0, 1]: lane ^ 2
  t += dpp_move<0xB1>(t);                   // quad_perm [1, 0, 3, 2]: lane ^ 1
  return t;
}

// ---------------------------------------------------------------- mean
template <typename T>
__global__ void k_partial_sum(const T* x, int64_t n, double* out) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    acc += double(x[i]);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
    out[blockIdx.x] = s;
  }
}

// Also latches ST_NONFINITE when the sum is not finite: a NaN or infinite
// convergence value (or an overflowing sum) anywhere in the map.
__global__ void k_final_mean(double* red, int nb, double inv_n, int* status) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += red[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
    red[1023] = s * inv_n;
    if (!isfinite(s)) atomicOr(status, ST_NONFINITE);
  }
}

// kappa_s(p) = mean of the NESTED children of p at nside_fine, minus the
// mean of the fine map (mass-conserving degrade of the demeaned map).
template <typename T>
__global__ void k_degrade(const T* kap, int64_t Nf, int64_t npix_s, const int* r2n_s, int64_t k2,
                          const double* red, double* out) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= npix_s) return;
  const int64_t pn = r2n_s[r];
  double acc = 0.0;
  for (int64_t c = 0; c < k2; ++c) acc += double(kap[hpx::nest2ring(Nf, pn * k2 + c)]);
  out[r] = acc / double(k2) - red[1023];
}

// ---------------------------------------------------------------- ring DFTs
// Every HEALPix ring has n = 4k samples, so the twiddles e^{2 pi i t / n}
// come from a quarter-wave sine table s[r] = sin(2 pi r / n), r = 0..n/4,
// held in LDS: (n/4 + 1) doubles per ring.
// Quadrant q = t / Q and remainder r of 0 <= t < 4 Q, by comparisons.
__device__ __forceinline__ void quadrant(int t, int Q, int& q, int& r) {
  q = 0;
  r = t;
  if (r >= Q) { r -= Q; ++q; }
  if (r >= Q) { r -= Q; ++q; }
  if (r >= Q) { r -= Q; ++q; }
}

// a / d for 0 <= a < 2^22 and d >= 1: the float quotient is within one of
// the true one, and one comparison each way settles it.
__device__ __forceinline__ int div_small(int a, int d, float inv_d) {
  int q = int(float(a) * inv_d);
  const int r = a - q * d;
  if (r < 0)
    --q;
  else if (r >= d)
    ++q;
  return q;
}

// e^{2 pi i t / n}, 0 <= t < n = 4 Q, from the quarter-wave table.
__device__ __forceinline__ void twiddle(const double* sq, int Q, int t, double& c, double& s) {
  int q, r;
  quadrant(t, Q, q, r);
  const double sr = sq[r], cr = sq[Q - r];
  switch (q) {
    case 0: c = cr; s = sr; break;
    case 1: c = -sr; s = cr; break;
    case 2: c = -cr; s = -sr; break;
    default: c = sr; s = -cr; break;
  }
}

__device__ __forceinline__ void quarter_table(double* sq, int n) {
  const int Q = n / 4;
  for (int r = threadIdx.x; r <= Q; r += blockDim.x) sq[r] = sinpi(2.0 * double(r) / double(n));
}

// e^{sign 2 pi i t / n} for 0 <= t < n from the quarter-wave table.
__device__ __forceinline__ void unit(const double* sq, int Q, int t, int sign, double& c,
                                     double& s) {
  twiddle(sq, Q, t, c, s);
  s *= sign;
}

// Complex DFT of length h = 2^lg r (r odd) with kernel e^{sign 2 pi i jk/h},
// for a ring of n = 2h samples whose quarter-wave table is sq.  Stockham
// order, natural order in and out with no permutation pass: lg radix-2
// stages (stage s joins the pairs h/2 apart into sub-transforms of length
// 2^(s+1)), then one stage of direct p-point sums per odd prime factor p of
// r.  The stages ping-pong between the LDS arrays a (holding the input,
// overwritten) and b; the return value is the one holding the result.
// Complex values move as 16-byte pairs, and every stage reads consecutive
// elements per lane.  Twiddles of the odd stages advance by quadrant and
// remainder so their inner loops have no division.
__device__ double* dft_mixed(double* a, double* b, int h, int lg, int r, const double* sq, int n,
                             int sign) {
  const int Q = n / 4, hh = h / 2;
  double2* src = reinterpret_cast<double2*>(a);
  double2* dst = reinterpret_cast<double2*>(b);
  for (int st = 0; st < lg; ++st) {
    const int ns = 1 << st;
    for (int j = threadIdx.x; j < hh; j += blockDim.x) {
      const int k = j & (ns - 1);
      double c, s;
      unit(sq, Q, k * (h >> st), sign, c, s);  // e^{sign 2 pi i k / (2 ns)}
      const double2 x0 = src[j], x1 = src[j + hh];
      const double tr = x1.x * c - x1.y * s, ti = x1.x * s + x1.y * c;
      const int d = ((j >> st) << (st + 1)) + k;
      dst[d] = make_double2(x0.x + tr, x0.y + ti);
      dst[d + ns] = make_double2(x0.x - tr, x0.y - ti);
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
  }
  // odd prime factors, smallest first: stage of radix R on sub-transforms of
  // length ns; output item = jh ns R + u ns + k takes
  // sum_t Y_{jh ns + k + t h/R} e^{sign 2 pi i t (u ns + k) / (ns R)}
  int ns = 1 << lg, rr = r;
  for (int R = 3; rr > 1; R += 2) {
    while (rr % R == 0) {
      rr /= R;
      const int nsR = ns * R, hR = h / R, step = n / nsR;
      const float inv_nsR = 1.0f / float(nsR), inv_ns = 1.0f / float(ns);
      for (int item = threadIdx.x; item < h; item += blockDim.x) {
        const int jh = div_small(item, nsR, inv_nsR), rem = item - jh * nsR;
        const int u = div_small(rem, ns, inv_ns), k = rem - u * ns;
        const int j = jh * ns + k;
        int iq, ir;
        quadrant(rem * step, Q, iq, ir);  // angle step rem / (ns R) in units of 2 pi
        int q = 0, re = 0;
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < R; ++t) {
          const double2 z = src[j + t * hR];
          const double sr = sq[re], cr = sq[Q - re];
          const double uu = (q & 1) ? sr : cr, vv = (q & 1) ? cr : sr;
          const double c = (q == 1 || q == 2) ? -uu : uu;
          const double ss = sign * ((q >= 2) ? -vv : vv);
          ar += z.x * c - z.y * ss;
          ai += z.x * ss + z.y * c;
          re += ir;
          q += iq;
          if (re >= Q) {
            re -= Q;
            ++q;
          }
          q &= 3;
        }
        dst[item] = make_double2(ar, ai);
      }
      __syncthreads();
      double2* t = src;
      src = dst;
      dst = t;
      ns = nsR;
    }
  }
  return reinterpret_cast<double*>(src);
}

// h = n / 2 = 2^lg r with r odd.
__device__ __forceinline__ void half_split(int n, int& h, int& lg, int& r) {
  h = n / 2;
  lg = __ffs(h) - 1;
  r = h >> lg;
}

// Rings whose half length h = 2^lg r has odd prime factors summing above
// kDirectFactorSum use Bluestein's chirp transform instead of the direct odd
// stages (cost h times that sum):
// with w_k = e^{-i pi k^2 / h} and jk = (j^2 + k^2 - (k - j)^2) / 2,
// X_k = w_k sum_j (z_j w_j) conj(w_{k-j}), a cyclic convolution of length
// M = 2^lgM >= 2h - 1 done by two power-of-two FFTs and a product with the
// transform of the chirp filter, tabulated per ring length at plan time.
constexpr int kRingBlock = 1024;
// Rings whose odd prime factors sum to at most this take the direct stages
// (cost about h times that sum); the others Bluestein (about 56 h).
constexpr int kDirectFactorSum = 64;

__host__ __device__ inline int odd_factor_sum(int r) {
  int sum = 0;
  for (int p = 3; r > 1; p += 2)
    while (r % p == 0) {
      r /= p;
      sum += p;
    }
  return sum;
}

__host__ __device__ inline int lg_ceil(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// e^{sign 2 pi i t / M}, M = 4 * 2^lgQ, from the quarter-wave table of M.
__device__ __forceinline__ void unit_p2(const double* sq, int lgQ, int t, int sign, double& c,
                                        double& s) {
  const int Q = 1 << lgQ, q = (t >> lgQ) & 3, r = t & (Q - 1);
  const double sr = sq[r], cr = sq[Q - r];
  switch (q) {
    case 0: c = cr; s = sr; break;
    case 1: c = -sr; s = cr; break;
    case 2: c = -cr; s = -sr; break;
    default: c = sr; s = -cr; break;
  }
  s *= sign;
}

// Radix-2 decimation in frequency, kernel e^{-2 pi i jk / M}: natural
// order in, bit-reversed order out (in place, interleaved complex).
__device__ void fft_dif(double* A, int lgM, const double* sq) {
  const int M = 1 << lgM;
  for (int ls = lgM - 1; ls >= 0; --ls) {
    const int span = 1 << ls;
    for (int item = threadIdx.x; item < M / 2; item += blockDim.x) {
      const int kk = item & (span - 1), i0 = ((item >> ls) << (ls + 1)) + kk, i1 = i0 + span;
      double c, s;
      unit_p2(sq, lgM - 2, kk << (lgM - 1 - ls), -1, c, s);
      double2* A2 = reinterpret_cast<double2*>(A);
      const double2 x0 = A2[i0], x1 = A2[i1];
      const double dr = x0.x - x1.x, di = x0.y - x1.y;
      A2[i0] = make_double2(x0.x + x1.x, x0.y + x1.y);
      A2[i1] = make_double2(dr * c - di * s, dr * s + di * c);
    }
    __syncthreads();
  }
}

// Radix-2 decimation in time, kernel e^{+2 pi i jk / M}: bit-reversed order
// in, natural order out, unnormalised.
__device__ void fft_dit_inv(double* A, int lgM, const double* sq) {
  const int M = 1 << lgM;
  for (int ls = 0; ls < lgM; ++ls) {
    const int span = 1 << ls;
    for (int item = threadIdx.x; item < M / 2; item += blockDim.x) {
      const int kk = item & (span - 1), i0 = ((item >> ls) << (ls + 1)) + kk, i1 = i0 + span;
      double c, s;
      unit_p2(sq, lgM - 2, kk << (lgM - 1 - ls), +1, c, s);
      double2* A2 = reinterpret_cast<double2*>(A);
      const double2 x0 = A2[i0], x1 = A2[i1];
      const double tr = c * x1.x - s * x1.y, ti = c * x1.y + s * x1.x;
      A2[i0] = make_double2(x0.x + tr, x0.y + ti);
      A2[i1] = make_double2(x0.x - tr, x0.y - ti);
    }
    __syncthreads();
  }
}

// Chirp w_k = e^{-i pi k^2 / h} = c - i s, k^2 reduced modulo 2h exactly
// (k^2 < 2^53: the floating-point quotient is off by at most one, fixed by
// one comparison each way).
__device__ __forceinline__ void chirp(int k, int h, double& c, double& s) {
  const double k2 = double(k) * double(k), d = 2.0 * double(h);
  double q = k2 - d * floor(k2 * (1.0 / d));
  if (q < 0.0) q += d;
  if (q >= d) q -= d;
  sincospi(q * (1.0 / double(h)), &s, &c);
}

// A holds a_k = z_k w_k (k < h) and zeros up to M: on return A_k holds M times
// the cyclic convolution (a * b)_k, natural order; Bh = DFT_M(b) of the filter
// b_k = conj w_k (b_{M-k} = b_k), bit-reversed order.
__device__ void bluestein_core(double* A, int lgM, const double* sq, const double* Bh) {
  fft_dif(A, lgM, sq);
  double2* A2 = reinterpret_cast<double2*>(A);
  const double2* B2 = reinterpret_cast<const double2*>(Bh);
  for (int p = threadIdx.x; p < (1 << lgM); p += blockDim.x) {
    const double2 x = A2[p], y = B2[p];
    A2[p] = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
  }
  __syncthreads();
  fft_dit_inv(A, lgM, sq);
}

// Transform of the chirp filter for ring length lens[b] (one block each),
// written bit-reversed at blu + offs[b].
__global__ __launch_bounds__(kRingBlock) void k_blu_table(const int* lens, const int64_t* offs,
                                                          double* blu) {
  extern __shared__ double sm[];
  const int h = lens[blockIdx.x] / 2, lgM = lg_ceil(2 * h - 1), M = 1 << lgM;
  double* A = sm;
  double* sq = sm + 2 * M;
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    const int j = k < h ? k : (k > M - h ? M - k : -1);
    double c = 0.0, s = 0.0;
    if (j >= 0) chirp(j, h, c, s);
    A[2 * k] = c;  // conj w_j = c + i s
    A[2 * k + 1] = s;
  }
  quarter_table(sq, M);
  __syncthreads();
  fft_dif(A, lgM, sq);
  double* out = blu + offs[blockIdx.x];
  for (int k = threadIdx.x; k < 2 * M; k += blockDim.x) out[k] = A[k];
}

// e^{sign 2 pi i t / n} of a ring: from its quarter-wave table when it is
// in LDS (direct path), else by sincospi.
__device__ __forceinline__ void ring_unit(const double* sq, int n, int t, int sign, double& c,
                                          double& s) {
  if (sq) {
    unit(sq, n / 4, t, sign, c, s);
  } else {
    sincospi(2.0 * double(t) / double(n), &s, &c);
    s *= sign;
  }
}

// e^{i pi k / n} for 0 <= k < 2n on a ring whose azimuth offset is pi / n
// (shifted) or 0: e^{2 pi i (k/2) / n} from the quarter-wave table, times
// (c1, s1) = e^{i pi / n} for odd k.
__device__ __forceinline__ void half_unit(const double* sq, int n, int k, bool shifted, double c1,
                                          double s1, double& c, double& s) {
  if (!shifted) {
    c = 1.0;
    s = 0.0;
    return;
  }
  unit(sq, n / 4, k >> 1, +1, c, s);
  if (k & 1) {
    const double cc = c * c1 - s * s1;
    s = c * s1 + s * c1;
    c = cc;
  }
}

// F_m(q) = e^{-i m phi0_q} sum_j f_{q,j} e^{-2 pi i (m mod n) j / n}, m = 0..lmax
// (HEALPix aliasing for rings shorter than lmax + 1).  The real ring is read
// as h = n/2 complex samples z_j = f_2j + i f_2j+1, transformed with
// dft_mixed, and split: X_k = E_k + e^{-2 pi i k/n} O_k with
// E_k = (Z_k + conj Z_{h-k}) / 2, O_k = (Z_k - conj Z_{h-k}) / 2i, and
// X_{n-k} = conj X_k.
__global__ __launch_bounds__(kRingBlock) void k_ring_forward(const double* map, const double* rt,
                                                             const int* ri, const int64_t* boff,
                                                             const double* blu, int lmax,
                                                             double* F) {
  extern __shared__ double sm[];
  const int q = blockIdx.x;
  const int n = ri[2 * q], h = n / 2;
  const int64_t first = ri[2 * q + 1];
  const double phi0 = rt[4 * q + 3];
  double* out = F + size_t(q) * (lmax + 1) * 2;
  const int64_t bo = boff[q];
  const double* Z;           // [h] complex half-length transform, natural order
  const double* sq = nullptr;
  if (bo < 0) {
    double* x = sm;            // [n] real samples = [h] complex z
    double* Zs = sm + n;       // [h] complex
    double* sqn = sm + 2 * n;  // [n/4 + 1]
    for (int j = threadIdx.x; j < n; j += blockDim.x) x[j] = map[first + j];
    quarter_table(sqn, n);
    __syncthreads();
    int hh, lg, r;
    half_split(n, hh, lg, r);
    Z = dft_mixed(x, Zs, hh, lg, r, sqn, n, -1);
    sq = sqn;
  } else {
    const int lgM = lg_ceil(2 * h - 1), M = 1 << lgM;
    double* A = sm;            // [M] complex
    double* sqM = sm + 2 * M;  // [M/4 + 1]
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
      double ar = 0.0, ai = 0.0;
      if (k < h) {
        const double zr = map[first + 2 * k], zi = map[first + 2 * k + 1];
        double c, s;
        chirp(k, h, c, s);
        ar = zr * c + zi * s;
        ai = zi * c - zr * s;
      }
      A[2 * k] = ar;
      A[2 * k + 1] = ai;
    }
    quarter_table(sqM, M);
    __syncthreads();
    bluestein_core(A, lgM, sqM, blu + bo);
    const double inv = 1.0 / double(M);
    for (int k = threadIdx.x; k < h; k += blockDim.x) {
      double c, s;
      chirp(k, h, c, s);
      const double cr = A[2 * k] * inv, ci = A[2 * k + 1] * inv;
      A[2 * k] = cr * c + ci * s;
      A[2 * k + 1] = ci * c - cr * s;
    }
    __syncthreads();
    Z = A;
  }
  const float inv_n = 1.0f / float(n), inv_2n = 0.5f / float(n);
  // phi0 is pi / n (shifted ring) or 0
  const bool shifted = phi0 > 0.0;
  double c1 = 1.0, s1 = 0.0;
  if (sq) sincospi(1.0 / double(n), &s1, &c1);
  for (int m = threadIdx.x; m <= lmax; m += blockDim.x) {
    const int k = m - n * div_small(m, n, inv_n);  // m mod n
    const bool up = k > n / 2;
    const int kk = up ? n - k : k;       // X_k = conj X_{n-k}, kk <= h
    const int k1 = kk == h ? 0 : kk, k2 = kk == 0 ? 0 : h - kk;
    const double zr = Z[2 * k1], zi = Z[2 * k1 + 1];
    const double wr = Z[2 * k2], wi = -Z[2 * k2 + 1];  // conj Z_{h-k}
    const double er = 0.5 * (zr + wr), ei = 0.5 * (zi + wi);
    const double dr = zr - wr, di = zi - wi;
    const double orr = 0.5 * di, oi = -0.5 * dr;       // (Z - conj) / 2i
    double c, s;
    ring_unit(sq, n, kk, -1, c, s);
    double xr = er + c * orr - s * oi, xi = ei + c * oi + s * orr;
    if (up) xi = -xi;
    double sp, cp;
    if (sq)
      half_unit(sq, n, m - 2 * n * div_small(m, 2 * n, inv_2n), shifted, c1, s1, cp, sp);
    else
      sincos(double(m) * phi0, &sp, &cp);
    out[2 * m] = cp * xr + sp * xi;       // (cp - i sp)(xr + i xi)
    out[2 * m + 1] = cp * xi - sp * xr;
  }
}

// f_{q,j} = Re sum_{m=0}^{lmax} c_m G_m(q) e^{i m (phi0 + 2 pi j / n)}, c_0 = 1,
// c_m = 2; nf fields [nf][ring][m] -> [nf][npix].  Orders fold onto
// B_k = sum_{m = k mod n} c_m G_m e^{i m phi0}; the real part equals the
// transform of the Hermitian C_k = (B_k + conj B_{n-k}) / 2, done at half
// length: Y_k = (C_k + C_{k+h}) + i e^{2 pi i k/n} (C_k - C_{k+h}), z the
// inverse DFT of Y, f_2j = Re z_j, f_2j+1 = Im z_j.
__global__ __launch_bounds__(kRingBlock) void k_ring_inverse(const double* G, int nring,
                                                             const double* rt, const int* ri,
                                                             const int64_t* boff,
                                                             const double* blu, int lmax,
                                                             int64_t npix, int nf, double* out) {
  extern __shared__ double sm[];
  const int q = blockIdx.x;
  const int n = ri[2 * q];
  const int64_t first = ri[2 * q + 1];
  const double phi0 = rt[4 * q + 3];
  const int64_t bo = boff[q];
  // e^{i n phi0} = +-1: n phi0 is a multiple of pi on every HEALPix ring
  const double sig = cos(double(n) * phi0) > 0.0 ? 1.0 : -1.0;
  int h, lg, r;
  half_split(n, h, lg, r);
  const int lgM = bo < 0 ? 0 : lg_ceil(2 * h - 1), M = 1 << lgM;
  // direct path: Y [h] complex, Z [h] complex, quarter table of n;
  // Bluestein: A [M] complex, quarter table of M
  double* sq = bo < 0 ? sm + 2 * n : nullptr;
  double* sqM = sm + 2 * M;
  if (bo < 0)
    quarter_table(sq, n);
  else
    quarter_table(sqM, M);
  for (int fld = 0; fld < nf; ++fld) {
    const double* g = G + (size_t(fld) * nring + q) * (lmax + 1) * 2;
    __syncthreads();
    // B_k with (c, s) = e^{i k phi0}; e^{i (k + t n) phi0} = sig^t e^{i k phi0}
    auto bk = [&](int k, double c, double s, double& br, double& bi) {
      br = 0.0;
      bi = 0.0;
      double sg = 1.0;
      for (int m = k; m <= lmax; m += n) {
        const double cm = m == 0 ? sg : 2.0 * sg;
        const double gr = g[2 * m], gi = g[2 * m + 1];
        br += cm * (c * gr - s * gi);
        bi += cm * (c * gi + s * gr);
        sg *= sig;
      }
    };
    auto ck = [&](int k, double& cr, double& ci) {
      double ar, ai, br, bi, s, c;
      sincos(double(k) * phi0, &s, &c);
      bk(k, c, s, ar, ai);
      if (k == 0)
        bk(0, 1.0, 0.0, br, bi);
      else
        bk(n - k, sig * c, -sig * s, br, bi);  // e^{i (n - k) phi0} = sig conj e^{i k phi0}
      cr = 0.5 * (ar + br);
      ci = 0.5 * (ai - bi);
    };
    // Y_k = (C_k + C_{k+h}) + i e^{2 pi i k/n} (C_k - C_{k+h})
    auto yk = [&](int k, double& yr, double& yi) {
      double c1r, c1i, c2r, c2i;
      ck(k, c1r, c1i);
      ck(k + h, c2r, c2i);
      double c, s;
      ring_unit(sq, n, k, +1, c, s);
      const double dr = c1r - c2r, di = c1i - c2i;
      const double tr = c * dr - s * di, ti = c * di + s * dr;
      yr = (c1r + c2r) - ti;
      yi = (c1i + c2i) + tr;
    };
    if (bo < 0) {
      double* Y = sm;
      double* Z = sm + n;
      // B_k for 0 <= k < n into both work arrays: the m = k terms of four
      // indices are loaded together, the aliased m = k + t n (short rings)
      // after them
      double2* B = reinterpret_cast<double2*>(sm);
      const double2* g2 = reinterpret_cast<const double2*>(g);
      const bool shifted = sig < 0.0;  // phi0 = pi / n
      double c1, s1;
      sincospi(1.0 / double(n), &s1, &c1);
      constexpr int U = 4;
      for (int k0 = threadIdx.x; k0 < n; k0 += U * blockDim.x) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * blockDim.x;
          v[u] = k < n && k <= lmax ? g2[k] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * blockDim.x;
          if (k >= n) continue;
          const double c0 = k == 0 ? 1.0 : 2.0;
          double gr = c0 * v[u].x, gi = c0 * v[u].y, sg = sig;
          for (int m = k + n; m <= lmax; m += n) {
            const double2 w = g2[m];
            gr += 2.0 * sg * w.x;
            gi += 2.0 * sg * w.y;
            sg *= sig;
          }
          double c, s;
          half_unit(sq, n, k, shifted, c1, s1, c, s);
          B[k] = make_double2(c * gr - s * gi, c * gi + s * gr);
        }
      }
      __syncthreads();
      // Y_k and Y_{h-k} from B_k, B_{n-k}, B_{k+h}, B_{h-k}: the thread of k
      // alone reads and writes positions k and h - k (the others lie above h)
      for (int k = threadIdx.x; k <= h / 2; k += blockDim.x) {
        const double2 bk = B[k], bnk = B[k == 0 ? 0 : n - k];
        const double2 bkh = B[k + h], bhk = B[h - k];
        // C_j = (B_j + conj B_{n-j}) / 2
        const double2 ck = make_double2(0.5 * (bk.x + bnk.x), 0.5 * (bk.y - bnk.y));
        const double2 ckh = make_double2(0.5 * (bkh.x + bhk.x), 0.5 * (bkh.y - bhk.y));
        const double2 chk = make_double2(0.5 * (bhk.x + bkh.x), 0.5 * (bhk.y - bkh.y));
        const double2 cnk = make_double2(0.5 * (bnk.x + bk.x), 0.5 * (bnk.y - bk.y));
        auto yval = [&](int kk, double2 a, double2 b) {
          double c, s;
          ring_unit(sq, n, kk, +1, c, s);
          const double dr = a.x - b.x, di = a.y - b.y;
          const double tr = c * dr - s * di, ti = c * di + s * dr;
          return make_double2((a.x + b.x) - ti, (a.y + b.y) + tr);
        };
        const double2 yk0 = yval(k, ck, ckh);
        // Y_{h-k} from C_{h-k} and C_{n-k} (C_{h-k+h} = C_{n-k})
        const double2 yk1 = yval(h - k, chk, cnk);
        B[k] = yk0;
        if (k > 0 && h - k != k) B[h - k] = yk1;
      }
      __syncthreads();
      const double* Zr = dft_mixed(Y, Z, h, lg, r, sq, n, +1);
      for (int j = threadIdx.x; j < h; j += blockDim.x) {
        out[size_t(fld) * npix + first + 2 * j] = Zr[2 * j];
        out[size_t(fld) * npix + first + 2 * j + 1] = Zr[2 * j + 1];
      }
    } else {
      // the e^{+...} transform as conj(DFT^-(conj Y))
      double* A = sm;
      for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double ar = 0.0, ai = 0.0;
        if (k < h) {
          double yr, yi, c, s;
          yk(k, yr, yi);
          chirp(k, h, c, s);
          ar = yr * c - yi * s;    // (yr - i yi)(c - i s)
          ai = -yi * c - yr * s;
        }
        A[2 * k] = ar;
        A[2 * k + 1] = ai;
      }
      __syncthreads();
      bluestein_core(A, lgM, sqM, blu + bo);
      const double inv = 1.0 / double(M);
      for (int j = threadIdx.x; j < h; j += blockDim.x) {
        double c, s;
        chirp(j, h, c, s);
        const double cr = A[2 * j] * inv, ci = A[2 * j + 1] * inv;
        out[size_t(fld) * npix + first + 2 * j] = cr * c + ci * s;
        out[size_t(fld) * npix + first + 2 * j + 1] = -(ci * c - cr * s);
      }
    }
  }
}

// ---------------------------------------------------------------- Legendre
// Coefficients of lambda_l = a_l (z lambda_{l-1} - b_l lambda_{l-2}):
// a_l = sqrt((4l^2-1)/(l^2-m^2)), b_l = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
__device__ __forceinline__ void recur_coeffs(int m, int lmax, double* a, double* b) {
  for (int l = m + 2 + threadIdx.x; l <= lmax; l += blockDim.x) {
    const double L = l, M = m;
    a[l - m] = sqrt((4.0 * L * L - 1.0) / (L * L - M * M));
    b[l - m] = sqrt(((L - 1.0) * (L - 1.0) - M * M) / (4.0 * (L - 1.0) * (L - 1.0) - 1.0));
  }
}

// Per-ring recurrence state: p1 = lambda_{l-1}, p2 = lambda_{l-2}, scale s.
struct Recur {
  double p1, p2;
  int s;
};

__device__ __forceinline__ double recur_value(const Recur& r) { return r.s == 0 ? r.p1 : 0.0; }

// Advance from lambda_{l-1} to lambda_l (l >= m+2) for cos theta = z.
__device__ __forceinline__ void recur_step(Recur& r, double z, double a, double b) {
  const double p0 = a * (z * r.p1 - b * r.p2);
  r.p2 = r.p1;
  r.p1 = p0;
}

// The rescale of the scaled recurrence, applied after every kRecGroup
// values of l instead of after each: across a group the values grow by less
// than 2^(4 log2(2m)) (the largest factors, l near m near a pole), so from
// below 2^400 they stay far inside the FP64 range.  A value that the
// rescale at the threshold would already have counted (true size below
// 2^-350) then enters as 0 until the group ends.
constexpr int kRecGroup = 8;
__device__ __forceinline__ void recur_rescale(Recur& r) {
  if (r.s < 0 && fabs(r.p1) > kHuge) {
    r.p1 *= kSmall;
    r.p2 *= kSmall;
    r.s += 1;
  }
}

// a_lm = w sum_{north q} lambda_lm(theta_q) [F_m(q) + (-1)^(l+m) F_m(q')],
// the equator counted once; one workgroup per m.
template <int RPT>
__global__ __launch_bounds__(leg_threads_max(RPT)) void k_analysis(const double* F, const double* rt,
                                                     const double* lam_mant,
                                                     const int* lam_scale, int H, int nring,
                                                     int lmax, double w, double* alm) {
  extern __shared__ double sm[];
  const int m = blockIdx.x;
  const int nl = lmax - m + 1;
  double* a = sm;                 // [nl]
  double* b = sm + nl;            // [nl]
  double* part = sm + 2 * nl;     // [64][waves][2]
  const int nw = blockDim.x >> 6;
  recur_coeffs(m, lmax, a, b);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  double z[RPT], fpr[RPT], fpi[RPT], fmr[RPT], fmi[RPT];
  Recur st[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q < H) {
      z[k] = rt[4 * q];
      const int qm = nring - 1 - q;
      const double* fn = F + (size_t(q) * (lmax + 1) + m) * 2;
      const double* fs = F + (size_t(qm) * (lmax + 1) + m) * 2;
      if (qm != q) {
        fpr[k] = fn[0] + fs[0]; fpi[k] = fn[1] + fs[1];
        fmr[k] = fn[0] - fs[0]; fmi[k] = fn[1] - fs[1];
      } else {
        fpr[k] = fmr[k] = fn[0];
        fpi[k] = fmi[k] = fn[1];
      }
      st[k].p1 = lam_mant[size_t(m) * H + q];
      st[k].p2 = 0.0;
      st[k].s = lam_scale[size_t(m) * H + q];
    } else {
      z[k] = 0.0; fpr[k] = fpi[k] = fmr[k] = fmi[k] = 0.0;
      st[k].p1 = st[k].p2 = 0.0; st[k].s = -1;
    }
  }
  __syncthreads();
  for (int l0 = 0; l0 < nl; l0 += 64) {
    const int cnt = nl - l0 < 64 ? nl - l0 : 64;
    // eight l at a time: their real and imaginary ring sums reduced over
    // the wave together
    for (int c0 = 0; c0 < cnt; c0 += 8) {
      double acc[16];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int dl = l0 + c0 + cc;  // l - m
        double sr = 0.0, si = 0.0;
        if (c0 + cc < cnt) {
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            if (dl == 1) {
              // lambda_{m+1,m} = sqrt(2m+3) z lambda_mm
              st[k].p2 = st[k].p1;
              st[k].p1 = sqrt(2.0 * m + 3.0) * z[k] * st[k].p2;
            } else if (dl >= 2) {
              recur_step(st[k], z[k], a[dl], b[dl]);
            }
            const double v = recur_value(st[k]);
            if (dl & 1) { sr += v * fmr[k]; si += v * fmi[k]; }
            else        { sr += v * fpr[k]; si += v * fpi[k]; }
          }
        }
        acc[2 * cc] = sr;
        acc[2 * cc + 1] = si;
      }
      static_assert(kRecGroup == 8, "one rescale per group of eight l");
#pragma unroll
      for (int k = 0; k < RPT; ++k) recur_rescale(st[k]);
      const double tot = wave_sum16(acc);
      const int idx = lane >> 2;  // 2 cc + (0: real, 1: imaginary)
      const int c = c0 + (idx >> 1);
      if ((lane & 3) == 0 && c < cnt) part[(c * nw + wv) * 2 + (idx & 1)] = tot;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
      const int c = threadIdx.x;
      double sr = 0.0, si = 0.0;
      for (int v = 0; v < nw; ++v) {
        sr += part[(c * nw + v) * 2];
        si += part[(c * nw + v) * 2 + 1];
      }
      const size_t idx = size_t(m) * (2 * lmax + 1 - m) / 2 + (m + l0 + c);
      alm[2 * idx] = w * sr;
      alm[2 * idx + 1] = w * si;
    }
    __syncthreads();
  }
}

// E/B analysis of a shear field (Sec. 5: full-sky E/B decomposition of the
// final plane's shear).  With the spin-2 functions of the covariant Hessian
// (z = cos, s = sin theta, dlambda = d lambda / d theta)
//   X = (m^2/s^2 - l(l+1)/2) lambda - (z/s) dlambda,  Y = (m/s)(dlambda - (z/s) lambda),
// the shear of psi = Y_lm is gamma_1 = X e^{i m phi}, gamma_2 = i Y e^{i m phi};
// both basis fields have squared norm N_l^2/4, N_l^2 = (l-1) l (l+1) (l+2):
//   E_lm = (2/N_l) w sum_rings [X F1 - i Y F2],  B_lm = (2/N_l) w sum_rings [X F2 + i Y F1]
// for l >= 2 (0 below), F1, F2 the ring transforms of gamma_1, gamma_2.  On
// the mirror ring X keeps the sign (-1)^(l+m) of lambda and Y takes the
// opposite one.  One workgroup per m; four l per wave reduction.
template <int RPT>
__global__ __launch_bounds__(leg_threads_max(RPT)) void k_analysis_spin2(
    const double* F1, const double* F2, const double* rt, const double* lam_mant,
    const int* lam_scale, int H, int nring, int lmax, double w, double* E, double* B) {
  extern __shared__ double sm[];
  const int m = blockIdx.x;
  const int nl = lmax - m + 1;
  double* a = sm;                 // [nl]
  double* b = sm + nl;            // [nl]
  double* kc = sm + 2 * nl;       // [nl] k_l = sqrt((2l+1)(l^2-m^2)/(2l-1))
  double* part = sm + 3 * nl;     // [64][waves][4]
  const int nw = blockDim.x >> 6;
  recur_coeffs(m, lmax, a, b);
  for (int dl = threadIdx.x; dl < nl; dl += blockDim.x) {
    const double L = m + dl, M = m;
    kc[dl] = sqrt((2.0 * L + 1.0) * (L * L - M * M) / fmax(2.0 * L - 1.0, 1.0));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double M = m;
  // per ring: z, 1/s, and F1, F2 folded with the mirror ring (+: sum, -: difference)
  double z[RPT], is[RPT], f1p[RPT][2], f1m[RPT][2], f2p[RPT][2], f2m[RPT][2];
  Recur st[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q < H) {
      z[k] = rt[4 * q];
      is[k] = 1.0 / rt[4 * q + 1];
      const int qm = nring - 1 - q;
      const double* a1 = F1 + (size_t(q) * (lmax + 1) + m) * 2;
      const double* b1 = F1 + (size_t(qm) * (lmax + 1) + m) * 2;
      const double* a2 = F2 + (size_t(q) * (lmax + 1) + m) * 2;
      const double* b2 = F2 + (size_t(qm) * (lmax + 1) + m) * 2;
      for (int c = 0; c < 2; ++c) {
        if (qm != q) {
          f1p[k][c] = a1[c] + b1[c]; f1m[k][c] = a1[c] - b1[c];
          f2p[k][c] = a2[c] + b2[c]; f2m[k][c] = a2[c] - b2[c];
        } else {
          f1p[k][c] = f1m[k][c] = a1[c];
          f2p[k][c] = f2m[k][c] = a2[c];
        }
      }
      st[k].p1 = lam_mant[size_t(m) * H + q];
      st[k].p2 = 0.0;
      st[k].s = lam_scale[size_t(m) * H + q];
    } else {
      z[k] = 0.0; is[k] = 0.0;
      for (int c = 0; c < 2; ++c) f1p[k][c] = f1m[k][c] = f2p[k][c] = f2m[k][c] = 0.0;
      st[k].p1 = st[k].p2 = 0.0; st[k].s = -1;
    }
  }
  __syncthreads();
  for (int l0 = 0; l0 < nl; l0 += 64) {
    const int cnt = nl - l0 < 64 ? nl - l0 : 64;
    for (int c0 = 0; c0 < cnt; c0 += 4) {
      double acc[16];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int dl = l0 + c0 + cc;  // l - m
        double er = 0.0, ei = 0.0, br = 0.0, bi = 0.0;
        if (c0 + cc < cnt) {
          const double L = M + dl, kl = kc[dl], hl = 0.5 * L * (L + 1.0);
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            const double prev = dl == 0 ? 0.0 : recur_value(st[k]);  // lambda_{l-1}
            if (dl == 1) {
              st[k].p2 = st[k].p1;
              st[k].p1 = sqrt(2.0 * m + 3.0) * z[k] * st[k].p2;
            } else if (dl >= 2) {
              recur_step(st[k], z[k], a[dl], b[dl]);
            }
            const double v = recur_value(st[k]);
            const double zs = z[k] * is[k], ms = M * is[k];
            const double t = (L * z[k] * v - kl * prev) * is[k];
            const double X = (ms * ms - hl) * v - zs * t;
            const double Y = ms * (t - zs * v);
            const double* fx1 = (dl & 1) ? f1m[k] : f1p[k];   // X: parity of lambda
            const double* fx2 = (dl & 1) ? f2m[k] : f2p[k];
            const double* fy1 = (dl & 1) ? f1p[k] : f1m[k];   // Y: the opposite
            const double* fy2 = (dl & 1) ? f2p[k] : f2m[k];
            er += X * fx1[0] + Y * fy2[1];
            ei += X * fx1[1] - Y * fy2[0];
            br += X * fx2[0] - Y * fy1[1];
            bi += X * fx2[1] + Y * fy1[0];
          }
        }
        acc[4 * cc] = er;
        acc[4 * cc + 1] = ei;
        acc[4 * cc + 2] = br;
        acc[4 * cc + 3] = bi;
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) recur_rescale(st[k]);
      const double tot = wave_sum16(acc);
      const int idx = lane >> 2;  // 4 cc + (E re, E im, B re, B im)
      const int c = c0 + (idx >> 2);
      if ((lane & 3) == 0 && c < cnt) part[(c * nw + wv) * 4 + (idx & 3)] = tot;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
      const int c = threadIdx.x;
      double v4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int v = 0; v < nw; ++v)
        for (int j = 0; j < 4; ++j) v4[j] += part[(c * nw + v) * 4 + j];
      const double L = m + l0 + c;
      const double n2 = (L - 1.0) * L * (L + 1.0) * (L + 2.0);
      const double f = L >= 2.0 ? 2.0 * w / sqrt(n2) : 0.0;
      const size_t idx = size_t(m) * (2 * lmax + 1 - m) / 2 + (m + l0 + c);
      E[2 * idx] = f * v4[0];
      E[2 * idx + 1] = f * v4[1];
      B[2 * idx] = f * v4[2];
      B[2 * idx + 1] = f * v4[3];
    }
    __syncthreads();
  }
}

// C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1) of nf coefficient sets
// [nf][n_lm] complex into cl [nf][lmax+1]; one workgroup per (l, set), a
// fixed-order tree sum.
__global__ void k_spectrum(const double* alm, int64_t nalm, int lmax, double* cl) {
  __shared__ double red[256];
  const int l = blockIdx.x, f = blockIdx.y;
  const double* a = alm + size_t(f) * nalm * 2;
  double acc = 0.0;
  for (int m = threadIdx.x; m <= l; m += blockDim.x) {
    const size_t idx = size_t(m) * (2 * lmax + 1 - m) / 2 + l;
    const double p = a[2 * idx] * a[2 * idx] + a[2 * idx + 1] * a[2 * idx + 1];
    acc += m == 0 ? p : 2.0 * p;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cl[size_t(f) * (lmax + 1) + l] = red[0] / (2.0 * l + 1.0);
}

// psi_lm = -2 kappa_lm / (l (l+1)), psi_00 = 0
__global__ void k_poisson(double* alm, int lmax) {
  const int m = blockIdx.x;
  for (int l = m + threadIdx.x; l <= lmax; l += blockDim.x) {
    const size_t idx = size_t(m) * (2 * lmax + 1 - m) / 2 + l;
    const double f = l == 0 ? 0.0 : -2.0 / (double(l) * (double(l) + 1.0));
    alm[2 * idx] *= f;
    alm[2 * idx + 1] *= f;
  }
}

// G_m(q) = sum_l alm_lm lambda_lm(theta_q) on north ring q and its mirror.
// DERIV: also the theta-derivative sums needed for the pure-SHT gradient
// and Hessian:  G_t = sum dlambda, G_tt = sum d2lambda, with
// sin dlambda_l = l z lambda_l - sqrt((2l+1)(l^2-m^2)/(2l-1)) lambda_{l-1} and
// d2lambda = -cot dlambda - (l(l+1) - m^2/sin^2) lambda.
// Output fields (DERIV): 0 = G, 1 = G_t, 2 = G_tt  ([field][ring][m]).
template <bool DERIV>
__global__ __launch_bounds__(1024) void k_synthesis(const double* alm, const double* rt,
                                                      const double* lam_mant,
                                                      const int* lam_scale, int H, int nring,
                                                      int lmax, double* G) {
  extern __shared__ double sm[];
  const int m = blockIdx.x;
  const int nl = lmax - m + 1;
  double* a = sm;
  double* b = sm + nl;
  double* c = sm + 2 * nl;  // [nl][2] alm for this m
  recur_coeffs(m, lmax, a, b);
  const size_t base = size_t(m) * (2 * lmax + 1 - m) / 2 + m;
  for (int dl = threadIdx.x; dl < nl; dl += blockDim.x) {
    c[2 * dl] = alm[2 * (base + dl)];
    c[2 * dl + 1] = alm[2 * (base + dl) + 1];
  }
  __syncthreads();
  const int q = blockIdx.y * blockDim.x + threadIdx.x;
  if (q >= H) return;
  const double z = rt[4 * q], st = rt[4 * q + 1];
  Recur r;
  r.p1 = lam_mant[size_t(m) * H + q];
  r.p2 = 0.0;
  r.s = lam_scale[size_t(m) * H + q];
  double er = 0, ei = 0, orr = 0, oi = 0;     // even / odd (l+m) sums
  double ter = 0, tei = 0, tor = 0, toi = 0;  // dlambda sums
  double wer = 0, wei = 0, wor = 0, woi = 0;  // d2lambda sums
  const double M = m;
  for (int dl = 0; dl < nl; ++dl) {
    if (dl % kRecGroup == 0) recur_rescale(r);
    const double lm1 = r.s == 0 ? r.p1 : 0.0;  // lambda_{l-1} (valid for dl >= 1)
    if (dl == 1) {
      r.p2 = r.p1;
      r.p1 = sqrt(2.0 * m + 3.0) * z * r.p2;
    } else if (dl >= 2) {
      recur_step(r, z, a[dl], b[dl]);
    }
    const double v = recur_value(r);
    const double cr = c[2 * dl], ci = c[2 * dl + 1];
    if (dl & 1) { orr += v * cr; oi += v * ci; }
    else        { er += v * cr; ei += v * ci; }
    if (DERIV) {
      const double L = m + dl;
      const double prev = dl == 0 ? 0.0 : lm1;
      const double k = sqrt((2.0 * L + 1.0) * (L * L - M * M) / fmax(2.0 * L - 1.0, 1.0));
      const double d1 = (L * z * v - k * prev) / st;
      const double d2 = -(z / st) * d1 - L * (L + 1.0) * v + M * M * v / (st * st);
      if (dl & 1) { tor += d1 * cr; toi += d1 * ci; wor += d2 * cr; woi += d2 * ci; }
      else        { ter += d1 * cr; tei += d1 * ci; wer += d2 * cr; wei += d2 * ci; }
    }
  }
  const int qm = nring - 1 - q;
  const size_t fs = size_t(nring) * (lmax + 1) * 2;  // field stride
  double* gn = G + (size_t(q) * (lmax + 1) + m) * 2;
  double* gs = G + (size_t(qm) * (lmax + 1) + m) * 2;
  gn[0] = er + orr;
  gn[1] = ei + oi;
  if (qm != q) { gs[0] = er - orr; gs[1] = ei - oi; }
  if (DERIV) {
    // lambda'(pi - theta) = -(-1)^(l+m) lambda'(theta); lambda'' keeps the parity
    gn[fs] = ter + tor;
    gn[fs + 1] = tei + toi;
    gn[2 * fs] = wer + wor;
    gn[2 * fs + 1] = wei + woi;
    if (qm != q) {
      gs[fs] = tor - ter;
      gs[fs + 1] = toi - tei;
      gs[2 * fs] = wer - wor;
      gs[2 * fs + 1] = wei - woi;
    }
  }
}

// From the three synthesis fields build the five pixel-space sums
// psi_t (G_t), psi_p (i m G), psi_tt (G_tt), psi_pp (-m^2 G), psi_tp (i m G_t).
__global__ void k_phi_fields(const double* G3, int nring, int lmax, double* G5) {
  const size_t per = size_t(nring) * (lmax + 1);
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= per) return;
  const double m = double(i % (lmax + 1));
  const double gr = G3[2 * i], gi = G3[2 * i + 1];
  const double tr = G3[2 * (per + i)], ti = G3[2 * (per + i) + 1];
  const double wr = G3[2 * (2 * per + i)], wi = G3[2 * (2 * per + i) + 1];
  G5[2 * i] = tr;                  G5[2 * i + 1] = ti;                  // psi_t
  G5[2 * (per + i)] = -m * gi;     G5[2 * (per + i) + 1] = m * gr;      // psi_p
  G5[2 * (2 * per + i)] = wr;      G5[2 * (2 * per + i) + 1] = wi;      // psi_tt
  G5[2 * (3 * per + i)] = -m * m * gr; G5[2 * (3 * per + i) + 1] = -m * m * gi;  // psi_pp
  G5[2 * (4 * per + i)] = -m * ti; G5[2 * (4 * per + i) + 1] = m * tr;  // psi_tp
}

// Covariant gradient and Hessian (App. A) from raw derivative maps, written
// in RING or NESTED order.
template <typename TO>
__global__ void k_covariant(const double* D, int64_t npix, const double* rt, const int* ri,
                            int nring, const int* r2n, int nested, TO* grad, TO* hess) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  int lo = 0, hi = nring - 1;  // ring of pixel p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ri[2 * mid + 1] <= p) lo = mid; else hi = mid - 1;
  }
  const double z = rt[4 * lo], s = rt[4 * lo + 1];
  const double pt = D[p], pp = D[npix + p], ptt = D[2 * npix + p], ppp = D[3 * npix + p],
               ptp = D[4 * npix + p];
  const int64_t o = nested ? int64_t(r2n[p]) : p;
  grad[o] = TO(pt);
  grad[npix + o] = TO(pp / s);
  hess[o] = TO(ptt);
  hess[npix + o] = TO(ppp / (s * s) + (z / s) * pt);
  hess[2 * npix + o] = TO(ptp / s - z * pp / (s * s));
}

template <typename K>
clm_status allow_lds(Plan* p, K kernel, size_t bytes);

// Rings per thread of the analysis: 4 (each wave reduces its partial sums
// once per l, so fewer rings per thread pay that more often), fewer while
// the grid would hold under 16 waves per CU, more when one workgroup would
// not cover the H north rings.
int rpt_for(int H, int lmax) {
  int k = 4;
  while (k > 1 && int64_t(lmax + 1) * (H / (64 * k)) < 16 * 256) k >>= 1;
  while (k <= 16 && k * leg_threads_max(k) < H) k <<= 1;
  return k;
}

template <int RPT>
void launch_analysis(Plan* p, hipStream_t s, double* alm) {
  const int lmax = p->d.lmax;
  const int nt = std::min(leg_threads_max(RPT), round64((p->H + RPT - 1) / RPT));
  const size_t shm = (2 * size_t(lmax + 1) + 64 * size_t(nt / 64) * 2) * sizeof(double);
  (void)allow_lds(p, k_analysis<RPT>, shm);
  {
    CLM_TIMED(p, s, "sht_analysis");
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_analysis<RPT>), dim3(lmax + 1), dim3(nt), shm, s,
                       p->F, p->ring_s, p->lam_mant, p->lam_scale, p->H, p->nring_s, lmax,
                       4.0 * kPi / double(p->npix_s), alm);
  }
}

clm_status ring_forward(Plan* p, const double* map, double* F, hipStream_t s) {
  if (allow_lds(p, k_ring_forward, p->ring_lds) != CLM_OK) return CLM_EHIP;
  {
    CLM_TIMED(p, s, "sht_ring_forward");
    hipLaunchKernelGGL(k_ring_forward, dim3(p->nring_s), dim3(kRingBlock), p->ring_lds, s, map,
                       p->ring_s, p->ringi_s, p->blu_off, p->blu, p->d.lmax, F);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// LDS above 64 KiB needs an explicit opt-in per kernel.
template <typename K>
clm_status allow_lds(Plan* p, K kernel, size_t bytes) {
  return lds_opt_in(p, reinterpret_cast<const void*>(kernel), bytes);
}

clm_status synthesis(Plan* p, const double* alm, hipStream_t s) {
  const int lmax = p->d.lmax;
  const size_t shm = 4 * size_t(lmax + 1) * sizeof(double);
  const int nt = std::min(1024, round64(p->H));
  dim3 grid(lmax + 1, (p->H + nt - 1) / nt);
  if (allow_lds(p, k_synthesis<false>, shm) != CLM_OK) return CLM_EHIP;
  {
    CLM_TIMED(p, s, "sht_synthesis");
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_synthesis<false>), grid, dim3(nt), shm, s, alm,
                       p->ring_s, p->lam_mant, p->lam_scale, p->H, p->nring_s, lmax, p->G);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

clm_status ring_inverse(Plan* p, const double* G, int nf, double* out, hipStream_t s) {
  if (allow_lds(p, k_ring_inverse, p->ring_lds) != CLM_OK) return CLM_EHIP;
  {
    CLM_TIMED(p, s, "sht_ring_inverse");
    hipLaunchKernelGGL(k_ring_inverse, dim3(p->nring_s), dim3(kRingBlock), p->ring_lds, s, G,
                       p->nring_s, p->ring_s, p->ringi_s, p->blu_off, p->blu, p->d.lmax,
                       p->npix_s, nf, out);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace

// Ring-transform plan of the SHT grid: which rings take Bluestein's
// transform (offset of their chirp-filter table, else -1), the tables, and
// the dynamic LDS of the ring kernels (the largest ring's need).
clm_status ring_plan(Plan* p) {
  const int N = p->d.nside_sht, nr = p->nring_s;
  std::vector<int64_t> off(nr, -1);
  std::vector<int> lens;
  std::vector<int64_t> loff;
  int64_t total = 0;
  size_t lds = 0;
  for (int q = 0; q < nr; ++q) {
    const int ring = q + 1, i = std::min(ring, 4 * N - ring);
    const int n = i < N ? 4 * i : 4 * N, h = n / 2;
    int r = h;
    while (!(r & 1)) r >>= 1;
    if (odd_factor_sum(r) <= kDirectFactorSum) {
      lds = std::max(lds, size_t(2 * n + n / 4 + 1) * sizeof(double));
      continue;
    }
    size_t k = 0;
    while (k < lens.size() && lens[k] != n) ++k;
    if (k == lens.size()) {
      const int64_t M = int64_t(1) << lg_ceil(2 * h - 1);
      lens.push_back(n);
      loff.push_back(total);
      total += 2 * M;
      lds = std::max(lds, size_t(2 * M + M / 4 + 1) * sizeof(double));
    }
    off[q] = loff[k];
  }
  p->ring_lds = lds;
  if (hipMalloc(&p->blu_off, size_t(nr) * sizeof(int64_t)) != hipSuccess)
    return fail(p, CLM_ENOMEM, "hipMalloc failed (ring plan)");
  CLM_HIP(hipMemcpy(p->blu_off, off.data(), off.size() * 8, hipMemcpyHostToDevice));
  if (lens.empty() || lds > 160 * 1024) return CLM_OK;  // oversize: rejected at solve time
  if (hipMalloc(&p->blu, size_t(total) * sizeof(double)) != hipSuccess)
    return fail(p, CLM_ENOMEM, "hipMalloc failed (ring plan)");
  int* dl = nullptr;
  int64_t* dof = nullptr;
  CLM_HIP(hipMalloc(&dl, lens.size() * sizeof(int)));
  if (hipMalloc(&dof, loff.size() * sizeof(int64_t)) != hipSuccess) {
    (void)hipFree(dl);
    return fail(p, CLM_ENOMEM, "hipMalloc failed");
  }
  clm_status st = CLM_OK;
  if (hipMemcpy(dl, lens.data(), lens.size() * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(dof, loff.data(), loff.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      allow_lds(p, k_blu_table, lds) != CLM_OK) {
    st = fail(p, CLM_EHIP, "ring plan set-up failed");
  } else {
    hipLaunchKernelGGL(k_blu_table, dim3(unsigned(lens.size())), dim3(kRingBlock), lds, 0, dl,
                       dof, p->blu);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
      st = fail(p, CLM_EHIP, "ring plan kernel failed");
  }
  (void)hipFree(dl);
  (void)hipFree(dof);
  return st;
}

clm_status plane_mean(Plan* p, const void* kappa, int kappa_fp64, hipStream_t s) {
  const int nb = 1023;
  {
    CLM_TIMED(p, s, "mean");
    if (kappa_fp64)
      hipLaunchKernelGGL(k_partial_sum<double>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const double*>(kappa), p->npix_f, p->red);
    else
      hipLaunchKernelGGL(k_partial_sum<float>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const float*>(kappa), p->npix_f, p->red);
  }
  CLM_LAUNCH_CHECK();
  {
    CLM_TIMED(p, s, "mean");
    hipLaunchKernelGGL(k_final_mean, dim3(1), dim3(kBlock), 0, s, p->red, nb,
                       1.0 / double(p->npix_f), p->status_dev);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

namespace {

// Mean, demean + degrade to the SHT grid and the ring transforms into F.
clm_status sht_front(Plan* p, const void* kappa, int kappa_fp64, double* F, hipStream_t s) {
  const clm_plan_desc& d = p->d;
  if (p->ring_lds > 160 * 1024)
    return fail(p, CLM_EUNSUPPORTED, "ring transforms exceed the LDS for this nside");
  clm_status st = plane_mean(p, kappa, kappa_fp64, s);
  if (st != CLM_OK) return st;
  const int64_t ratio = d.nside_fine / d.nside_sht;
  const int64_t k2 = ratio * ratio;
  {
    CLM_TIMED(p, s, "degrade");
    if (kappa_fp64)
      hipLaunchKernelGGL(k_degrade<double>, dim3((p->npix_s + kBlock - 1) / kBlock),
                         dim3(kBlock), 0, s, static_cast<const double*>(kappa),
                         int64_t(d.nside_fine), p->npix_s, p->r2n_s, k2, p->red, p->kap_s);
    else
      hipLaunchKernelGGL(k_degrade<float>, dim3((p->npix_s + kBlock - 1) / kBlock),
                         dim3(kBlock), 0, s, static_cast<const float*>(kappa),
                         int64_t(d.nside_fine), p->npix_s, p->r2n_s, k2, p->red, p->kap_s);
  }
  CLM_LAUNCH_CHECK();
  return ring_forward(p, p->kap_s, F, s);
}

clm_status poisson(Plan* p, double* alm, hipStream_t s) {
  {
    CLM_TIMED(p, s, "sht_poisson");
    hipLaunchKernelGGL(k_poisson, dim3(p->d.lmax + 1), dim3(kBlock), 0, s, alm, p->d.lmax);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// a_lm of the ring transforms in p->F (FP64 Legendre analysis).
clm_status analysis(Plan* p, double* alm, hipStream_t s) {
  switch (rpt_for(p->H, p->d.lmax)) {
    case 1: launch_analysis<1>(p, s, alm); break;
    case 2: launch_analysis<2>(p, s, alm); break;
    case 4: launch_analysis<4>(p, s, alm); break;
    case 8: launch_analysis<8>(p, s, alm); break;
    case 16: launch_analysis<16>(p, s, alm); break;
    default: return fail(p, CLM_EUNSUPPORTED, "too many rings per thread");
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// y = x - y and y = y + x, elementwise.
__global__ void k_sub_from(int64_t n, const double* x, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t] - y[t];
}

__global__ void k_add_to(int64_t n, const double* x, double* y) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] += x[t];
}

}  // namespace

clm_status sht_solve(Plan* p, const void* kappa, int kappa_fp64, int slot, hipStream_t s,
                     bool psi_map) {
  clm_status st = sht_front(p, kappa, kappa_fp64, p->F, s);
  if (st != CLM_OK) return st;
  double* alm = p->slots[slot].alm;
  if ((st = analysis(p, alm, s)) != CLM_OK) return st;
  // Jacobi refinement: a <- a + A(f - S a), f the degraded, demeaned map
  for (int it = 0; it < p->d.analysis_iters; ++it) {
    if ((st = synthesis(p, alm, s)) != CLM_OK) return st;
    if ((st = ring_inverse(p, p->G, 1, p->iter_map, s)) != CLM_OK) return st;
    {
      CLM_TIMED(p, s, "sht_refine");
      hipLaunchKernelGGL(k_sub_from, dim3(unsigned((p->npix_s + kBlock - 1) / kBlock)),
                         dim3(kBlock), 0, s, p->npix_s, static_cast<const double*>(p->kap_s),
                         p->iter_map);
    }
    CLM_LAUNCH_CHECK();
    if ((st = ring_forward(p, p->iter_map, p->F, s)) != CLM_OK) return st;
    if ((st = analysis(p, p->iter_alm, s)) != CLM_OK) return st;
    {
      CLM_TIMED(p, s, "sht_refine");
      hipLaunchKernelGGL(k_add_to, dim3(unsigned((2 * p->nalm + kBlock - 1) / kBlock)),
                         dim3(kBlock), 0, s, 2 * p->nalm,
                         static_cast<const double*>(p->iter_alm), alm);
    }
    CLM_LAUNCH_CHECK();
  }
  if ((st = poisson(p, alm, s)) != CLM_OK) return st;
  if (!psi_map) return CLM_OK;
  if ((st = synthesis(p, alm, s)) != CLM_OK) return st;
  return ring_inverse(p, p->G, 1, p->slots[slot].psi_s, s);
}

// Transpose of (SHT-grid kappa -> analysis -> Poisson -> synthesis): with the
// uniform weight w = 4 pi / N_pix, synthesis^T is the unweighted analysis
// with the m >= 1 terms doubled and analysis^T is w times the synthesis with
// the m >= 1 terms halved; the factors cancel around the real diagonal
// Poisson step, so the transpose is the same chain applied to psi bar.
clm_status sht_adjoint(Plan* p, const double* psibar, double* alm, double* ksbar,
                       hipStream_t s) {
  clm_status st = ring_forward(p, psibar, p->F, s);
  if (st != CLM_OK) return st;
  const int rpt = rpt_for(p->H, p->d.lmax);
  switch (rpt) {
    case 1: launch_analysis<1>(p, s, alm); break;
    case 2: launch_analysis<2>(p, s, alm); break;
    case 4: launch_analysis<4>(p, s, alm); break;
    case 8: launch_analysis<8>(p, s, alm); break;
    case 16: launch_analysis<16>(p, s, alm); break;
    default: return fail(p, CLM_EUNSUPPORTED, "too many rings per thread");
  }
  CLM_LAUNCH_CHECK();
  if ((st = poisson(p, alm, s)) != CLM_OK) return st;
  if ((st = synthesis(p, alm, s)) != CLM_OK) return st;
  return ring_inverse(p, p->G, 1, ksbar, s);
}

clm_status sht_solve_batch(Plan* p, const void* kappa, int kappa_fp64, int first_slot,
                           int nplanes, hipStream_t s, bool psi_map) {
  if (nplanes < 1 || nplanes > p->batch) return fail(p, CLM_EINVAL, "batch size");
  const size_t nF = size_t(p->nring_s) * (p->d.lmax + 1) * 2;
  const size_t esz = kappa_fp64 ? 8 : 4;
  clm_status st;
  for (int k = 0; k < nplanes; ++k) {
    const char* kp = static_cast<const char*>(kappa) + size_t(k) * p->npix_f * esz;
    if ((st = sht_front(p, kp, kappa_fp64, p->Fb + k * nF, s)) != CLM_OK) return st;
  }
  if ((st = mfma_analysis(p, first_slot, nplanes, s)) != CLM_OK) return st;
  for (int k = 0; k < nplanes; ++k)
    if ((st = poisson(p, p->slots[first_slot + k].alm, s)) != CLM_OK) return st;
  if (!psi_map) return CLM_OK;
  if ((st = mfma_synthesis(p, first_slot, nplanes, s)) != CLM_OK) return st;
  for (int k = 0; k < nplanes; ++k)
    if ((st = ring_inverse(p, p->Gb + k * nF, 1, p->slots[first_slot + k].psi_s, s)) != CLM_OK)
      return st;
  return CLM_OK;
}

clm_status sht_solve_multi(Plan* const* ps, int n, const void* const* kappa,
                           const int32_t* kappa_fp64, const int32_t* nplanes, hipStream_t s) {
  int rounds = 0;
  for (int i = 0; i < n; ++i)
    rounds = std::max(rounds, (nplanes[i] + ps[i]->batch - 1) / ps[i]->batch);
  clm_status st;
  for (int r = 0; r < rounds; ++r) {
    MfmaGroup gs[4];
    int ng = 0;
    for (int i = 0; i < n; ++i) {
      Plan* p = ps[i];
      const int k0 = r * p->batch;
      if (k0 >= nplanes[i]) continue;
      const int nb = std::min(p->batch, nplanes[i] - k0);
      const size_t nF = size_t(p->nring_s) * (p->d.lmax + 1) * 2;
      const size_t esz = kappa_fp64[i] ? 8 : 4;
      for (int k = 0; k < nb; ++k) {
        const char* kp = static_cast<const char*>(kappa[i]) + size_t(k0 + k) * p->npix_f * esz;
        if ((st = sht_front(p, kp, kappa_fp64[i], p->Fb + k * nF, s)) != CLM_OK) return st;
      }
      gs[ng++] = MfmaGroup{p, k0, nb};
    }
    if ((st = mfma_analysis_multi(gs, ng, s)) != CLM_OK) return st;
    for (int g = 0; g < ng; ++g)
      for (int k = 0; k < gs[g].P; ++k)
        if ((st = poisson(gs[g].p, gs[g].p->slots[gs[g].first_slot + k].alm, s)) != CLM_OK)
          return st;
    if ((st = mfma_synthesis_multi(gs, ng, s)) != CLM_OK) return st;
    for (int g = 0; g < ng; ++g) {
      Plan* p = gs[g].p;
      const size_t nF = size_t(p->nring_s) * (p->d.lmax + 1) * 2;
      for (int k = 0; k < gs[g].P; ++k)
        if ((st = ring_inverse(p, p->Gb + k * nF, 1, p->slots[gs[g].first_slot + k].psi_s, s)) !=
            CLM_OK)
          return st;
    }
    // SHT+MG plans: the multigrid of each plane, after its mean is taken again
    for (int g = 0; g < ng; ++g) {
      Plan* p = gs[g].p;
      if (!p->mg) continue;
      const int i = int(std::find(ps, ps + n, p) - ps);
      const size_t esz = kappa_fp64[i] ? 8 : 4;
      for (int k = 0; k < gs[g].P; ++k) {
        const int slot = gs[g].first_slot + k;
        const char* kp = static_cast<const char*>(kappa[i]) + size_t(slot) * p->npix_f * esz;
        if ((st = plane_mean(p, kp, kappa_fp64[i], s)) != CLM_OK) return st;
        if ((st = mg_solve(p, kp, kappa_fp64[i], slot, s)) != CLM_OK) return st;
      }
    }
  }
  return CLM_OK;
}

// The raw partials psi_t, psi_p, psi_tt, psi_pp, psi_tp of slot `slot` at
// the RING pixel centres into p->deriv (FP64 synthesis).
clm_status fp64_raw_derivs(Plan* p, int slot, hipStream_t s) {
  // theta sums G, G_t, G_tt into fields 0..2 of G ([field][ring][m]); G is
  // sized for five fields in SHT-only plans
  const int lmax = p->d.lmax;
  const size_t per = size_t(p->nring_s) * (lmax + 1);
  {
    const size_t shm = 4 * size_t(lmax + 1) * sizeof(double);
    const int nt = std::min(1024, round64(p->H));
    dim3 grid(lmax + 1, (p->H + nt - 1) / nt);
    if (allow_lds(p, k_synthesis<true>, shm) != CLM_OK) return CLM_EHIP;
    {
      CLM_TIMED(p, s, "sht_deriv_synthesis");
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_synthesis<true>), grid, dim3(nt), shm, s,
                         p->slots[slot].alm, p->ring_s, p->lam_mant, p->lam_scale, p->H,
                         p->nring_s, lmax, p->G);
    }
    CLM_LAUNCH_CHECK();
  }
  // the five pixel-space sums, element-wise in place (each thread reads all
  // three inputs of its (ring, m) slot before writing the five outputs)
  {
    CLM_TIMED(p, s, "sht_deriv_fields");
    hipLaunchKernelGGL(k_phi_fields, dim3((per + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p->G,
                       p->nring_s, lmax, p->G);
  }
  CLM_LAUNCH_CHECK();
  return ring_inverse(p, p->G, 5, p->deriv, s);
}

clm_status sht_pixel_derivs(Plan* p, int slot, int order, int out_fp64, void* grad, void* hess,
                            hipStream_t s) {
  clm_status st = fp64_raw_derivs(p, slot, s);
  if (st != CLM_OK) return st;
  const dim3 g((p->npix_s + kBlock - 1) / kBlock);
  CLM_TIMED(p, s, "sht_covariant");
  if (out_fp64)
    hipLaunchKernelGGL(k_covariant<double>, g, dim3(kBlock), 0, s, p->deriv, p->npix_s,
                       p->ring_s, p->ringi_s, p->nring_s, p->r2n_s, order == CLM_ORDER_NESTED,
                       static_cast<double*>(grad), static_cast<double*>(hess));
  else
    hipLaunchKernelGGL(k_covariant<float>, g, dim3(kBlock), 0, s, p->deriv, p->npix_s,
                       p->ring_s, p->ringi_s, p->nring_s, p->r2n_s, order == CLM_ORDER_NESTED,
                       static_cast<float*>(grad), static_cast<float*>(hess));
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// The gradient and covariant Hessian of slot `slot` at the RING pixel
// centres, FP64, into p->deriv [5][npix] (g_t, g_p, U_tt, U_pp, U_tp): the
// fields a ray update through a pure-SHT plane interpolates.  In matrix-core
// plans the derivative synthesis of the slot (one plane); FP64 plans take the
// raw partials and make them covariant in place (each thread reads its five
// values before writing them).
clm_status sht_plane_fields(Plan* p, int slot, hipStream_t s) {
  clm_status st;
  if (p->batch > 0) {
    if ((st = mfma_deriv_synthesis(p, slot, 1, s)) != CLM_OK) return st;
    return ring_inverse(p, p->Gb, 5, p->deriv, s);
  }
  if ((st = fp64_raw_derivs(p, slot, s)) != CLM_OK) return st;
  const dim3 g((p->npix_s + kBlock - 1) / kBlock);
  CLM_TIMED(p, s, "sht_covariant");
  hipLaunchKernelGGL(k_covariant<double>, g, dim3(kBlock), 0, s, p->deriv, p->npix_s, p->ring_s,
                     p->ringi_s, p->nring_s, p->r2n_s, 0, p->deriv, p->deriv + 2 * p->npix_s);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// Fields of plane k of the latest derivative synthesis batch (Gb) into
// p->deriv.
clm_status sht_batch_fields(Plan* p, int k, hipStream_t s) {
  const size_t nF = size_t(p->nring_s) * (p->d.lmax + 1) * 2;
  return ring_inverse(p, p->Gb + 5 * k * nF, 5, p->deriv, s);
}

// The five derivative maps [5][npix] (g_t, g_p, U_tt, U_pp, U_tp, RING) to
// the caller's gradient [2][npix] and Hessian [3][npix] in RING or NESTED
// order.
template <typename TO>
__global__ void k_deriv_out(const double* D, int64_t npix, const int* r2n, int nested, TO* grad,
                            TO* hess) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const int64_t o = nested ? int64_t(r2n[p]) : p;
  grad[o] = TO(D[p]);
  grad[npix + o] = TO(D[npix + p]);
  hess[o] = TO(D[2 * npix + p]);
  hess[npix + o] = TO(D[3 * npix + p]);
  hess[2 * npix + o] = TO(D[4 * npix + p]);
}

// Gradient and covariant Hessian at every pixel for planes first_slot ..
// first_slot + nplanes - 1 of a pure-SHT plan: the matrix-core derivative
// synthesis of up to 8 planes per launch, then per plane five ring inverses
// and the reordering; FP64 plans run the FP64 synthesis plane by plane.
clm_status sht_pixel_derivs_batch(Plan* p, int first_slot, int nplanes, int order, int out_fp64,
                                  void* grad, void* hess, hipStream_t s) {
  const size_t esz = out_fp64 ? 8 : 4;
  const size_t npix = size_t(p->npix_s);
  char* g = static_cast<char*>(grad);
  char* h = static_cast<char*>(hess);
  clm_status st;
  if (p->batch == 0) {
    for (int k = 0; k < nplanes; ++k)
      if ((st = sht_pixel_derivs(p, first_slot + k, order, out_fp64, g + k * 2 * npix * esz,
                                 h + k * 3 * npix * esz, s)) != CLM_OK)
        return st;
    return CLM_OK;
  }
  const int dp = std::min(p->batch, mfma_deriv_planes());
  const size_t nF = size_t(p->nring_s) * (p->d.lmax + 1) * 2;
  const dim3 grid(unsigned((npix + kBlock - 1) / kBlock));
  for (int k0 = 0; k0 < nplanes; k0 += dp) {
    const int nb = std::min(dp, nplanes - k0);
    if ((st = mfma_deriv_synthesis(p, first_slot + k0, nb, s)) != CLM_OK) return st;
    for (int k = 0; k < nb; ++k) {
      if ((st = ring_inverse(p, p->Gb + 5 * k * nF, 5, p->deriv, s)) != CLM_OK) return st;
      const size_t pk = size_t(k0 + k);
      CLM_TIMED(p, s, "sht_deriv_out");
      if (out_fp64)
        hipLaunchKernelGGL(k_deriv_out<double>, grid, dim3(kBlock), 0, s, p->deriv,
                           int64_t(npix), p->r2n_s, order == CLM_ORDER_NESTED,
                           reinterpret_cast<double*>(g + pk * 2 * npix * esz),
                           reinterpret_cast<double*>(h + pk * 3 * npix * esz));
      else
        hipLaunchKernelGGL(k_deriv_out<float>, grid, dim3(kBlock), 0, s, p->deriv,
                           int64_t(npix), p->r2n_s, order == CLM_ORDER_NESTED,
                           reinterpret_cast<float*>(g + pk * 2 * npix * esz),
                           reinterpret_cast<float*>(h + pk * 3 * npix * esz));
    }
    CLM_LAUNCH_CHECK();
  }
  return CLM_OK;
}

// kappa, E, B, omega coefficients [4][n_lm] and spectra [4][lmax+1] of a
// ray state's final Jacobians on the plan's grid (Sec. 5).
clm_status sht_jacobian_spectra(Plan* p, const clm_rays* rays, double* alm, double* cl,
                                hipStream_t s) {
  if (p->H > 4 * leg_threads_max(4))
    return fail(p, CLM_EUNSUPPORTED, "spectra: at most 4096 north rings (Nside 2048)");
  const size_t npix = size_t(p->npix_s);
  clm_status st = jacobian_fields(p, rays, p->deriv, s);
  if (st != CLM_OK) return st;
  const int lmax = p->d.lmax;
  const size_t na = size_t(p->nalm) * 2;
  const int rpt = rpt_for(p->H, lmax);
  auto spin0 = [&](const double* map, double* out) -> clm_status {
    clm_status e = ring_forward(p, map, p->F, s);
    return e != CLM_OK ? e : analysis(p, out, s);
  };
  if ((st = spin0(p->deriv, alm)) != CLM_OK) return st;                       // kappa
  if ((st = spin0(p->deriv + 3 * npix, alm + 3 * na)) != CLM_OK) return st;  // omega
  if ((st = ring_forward(p, p->deriv + npix, p->F, s)) != CLM_OK) return st;
  if ((st = ring_forward(p, p->deriv + 2 * npix, p->G, s)) != CLM_OK) return st;
  {
    const int r2 = rpt < 4 ? rpt : 4;
    const int nt = std::min(leg_threads_max(r2), round64((p->H + r2 - 1) / r2));
    const size_t shm = (3 * size_t(lmax + 1) + 64 * size_t(nt / 64) * 4) * sizeof(double);
    const double w = 4.0 * kPi / double(p->npix_s);
    CLM_TIMED(p, s, "spin2_analysis");
    switch (r2) {
      case 1:
        if (allow_lds(p, k_analysis_spin2<1>, shm) != CLM_OK) return CLM_EHIP;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_analysis_spin2<1>), dim3(lmax + 1), dim3(nt), shm,
                           s, p->F, p->G, p->ring_s, p->lam_mant, p->lam_scale, p->H,
                           p->nring_s, lmax, w, alm + na, alm + 2 * na);
        break;
      case 2:
        if (allow_lds(p, k_analysis_spin2<2>, shm) != CLM_OK) return CLM_EHIP;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_analysis_spin2<2>), dim3(lmax + 1), dim3(nt), shm,
                           s, p->F, p->G, p->ring_s, p->lam_mant, p->lam_scale, p->H,
                           p->nring_s, lmax, w, alm + na, alm + 2 * na);
        break;
      default:
        if (allow_lds(p, k_analysis_spin2<4>, shm) != CLM_OK) return CLM_EHIP;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_analysis_spin2<4>), dim3(lmax + 1), dim3(nt), shm,
                           s, p->F, p->G, p->ring_s, p->lam_mant, p->lam_scale, p->H,
                           p->nring_s, lmax, w, alm + na, alm + 2 * na);
        break;
    }
  }
  CLM_LAUNCH_CHECK();
  {
    CLM_TIMED(p, s, "spectra");
    hipLaunchKernelGGL(k_spectrum, dim3(lmax + 1, 4), dim3(256), 0, s, alm, int64_t(p->nalm),
                       lmax, cl);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace clm

extern "C" clm_status clm_alm2map(const double* alm, int32_t lmax, int32_t nside, double* map,
                                  hipStream_t stream) {
  if (!alm || !map || lmax < 0 || nside < 1 || (nside & (nside - 1)) || nside > 8192)
    return CLM_EINVAL;
  clm_plan_desc d;
  clm_plan_desc_default(&d, nside);
  d.nside_sht = nside;
  d.lmax = lmax < 1 ? 1 : lmax;
  d.solver = CLM_SOLVER_SHT;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CLM_EHIP;
  clm_plan pl = nullptr;
  clm_status st = clm_plan_create(&d, dev, &pl);
  if (st != CLM_OK) return st;
  clm::Plan* p = pl;
  const size_t bytes = size_t(p->nalm) * 16;
  if (lmax < 1) {
    // lmax = 0: only a_00; pad a_10, a_11 with zeros
    (void)hipMemsetAsync(p->slots[0].alm, 0, bytes, stream);
    (void)hipMemcpyAsync(p->slots[0].alm, alm, 16, hipMemcpyDeviceToDevice, stream);
  } else {
    (void)hipMemcpyAsync(p->slots[0].alm, alm, bytes, hipMemcpyDeviceToDevice, stream);
  }
  st = clm::synthesis(p, p->slots[0].alm, stream);
  if (st == CLM_OK) st = clm::ring_inverse(p, p->G, 1, map, stream);
  if (hipStreamSynchronize(stream) != hipSuccess && st == CLM_OK) st = CLM_EHIP;
  clm_plan_destroy(pl);
  return st;
}

// ------------------------------------------------ allocation-free synthesis
// clm_alm2map_noalloc: the synthesis of clm_alm2map with every table and
// intermediate (ring geometry, chirp-filter transforms, lambda_mm starting
// values, the ring sums G) in one file-scope device array instead of plan
// workspace.  Sizes up to nside 256 / lmax 512 fit in it.
namespace clm {
namespace {

constexpr int kNaMaxNside = 256;
constexpr int kNaMaxLmax = 512;
constexpr size_t kNaScratchBytes = size_t(16) << 20;
constexpr int kNaMaxDevices = 64;

}  // namespace
}  // namespace clm

// One copy per GPU, held until the process ends.  In host code this name
// is only a stand-in for the symbol: the device address of each GPU's copy
// comes from hipGetSymbolAddress (na_scratch_ptr) and is the only address
// host code passes on.
static __device__ __align__(256) char scratch[clm::kNaScratchBytes];

namespace clm {
namespace {

std::mutex g_na_mutex;
char* g_na_ptr[kNaMaxDevices] = {};

// Device address of this GPU's scratch, looked up once per device with that
// device current.
hipError_t na_scratch_ptr(int dev, char** out) {
  std::lock_guard<std::mutex> lk(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_na_ptr[dev] = static_cast<char*>(q);
  }
  *out = g_na_ptr[dev];
  return hipSuccess;
}

// Ring geometry of the HEALPix grid N on the device, the definitions of the
// plan's host tables (Gorski et al. 2005): rt[4q..] = z, sin theta, theta,
// phi0 of ring q + 1; ri[2q..] = pixels, first pixel.
__global__ void k_ring_geom(int N, double* rt, int* ri) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 4 * N - 1) return;
  const int64_t i = q + 1;
  double z, st;
  int64_t n, first;
  bool shifted = true;
  if (i < N) {
    const double omz = double(i) * double(i) / (3.0 * N * N);
    z = 1.0 - omz;
    st = sqrt(omz * (1.0 + z));
    n = 4 * i;
    first = 2 * i * (i - 1);
  } else if (i <= 3 * N) {
    z = (4.0 * N - 2.0 * i) / (3.0 * N);
    st = sqrt((1.0 - z) * (1.0 + z));
    n = 4 * N;
    first = 2 * int64_t(N) * (N - 1) + 4 * int64_t(N) * (i - N);
    shifted = ((i - N) % 2) == 0;
  } else {
    const int64_t ip = 4 * N - i;
    const double opz = double(ip) * double(ip) / (3.0 * N * N);
    z = opz - 1.0;
    st = sqrt(opz * (2.0 - opz));
    n = 4 * ip;
    first = 12 * int64_t(N) * N - 2 * ip * (ip + 1);
  }
  rt[4 * q + 0] = z;
  rt[4 * q + 1] = st;
  rt[4 * q + 2] = atan2(st, z);
  rt[4 * q + 3] = shifted ? 3.14159265358979323846 / double(n) : 0.0;
  ri[2 * q + 0] = int(n);
  ri[2 * q + 1] = int(first);
}

// Size of the ring-transform plan of grid N: distinct Bluestein ring
// lengths, doubles of their filter tables, and the ring kernels' LDS.  The
// same rule as ring_plan; cap rings of one length come in north/south
// pairs, so lengths are first met in the north in increasing order.
struct NaRingPlan {
  int nlen = 0;
  int64_t total = 0;
  size_t lds = 0;
};

__host__ __device__ inline bool na_bluestein(int N, int q, int& n, int64_t& twoM) {
  const int ring = q + 1, i = ring < 4 * N - ring ? ring : 4 * N - ring;
  n = i < N ? 4 * i : 4 * N;
  const int h = n / 2;
  int r = h;
  while (!(r & 1)) r >>= 1;
  twoM = int64_t(2) << lg_ceil(2 * h - 1);
  return odd_factor_sum(r) > kDirectFactorSum;
}

NaRingPlan na_ring_plan(int N) {
  NaRingPlan rp;
  for (int q = 0; q < 2 * N; ++q) {  // north rings and the equator
    int n;
    int64_t twoM;
    if (na_bluestein(N, q, n, twoM)) {
      ++rp.nlen;
      rp.total += twoM;
      rp.lds = std::max(rp.lds, size_t(twoM + twoM / 8 + 1) * sizeof(double));
    } else {
      rp.lds = std::max(rp.lds, size_t(2 * n + n / 4 + 1) * sizeof(double));
    }
  }
  return rp;
}

// One thread: every ring's chirp-table offset (-1: direct stages), and the
// distinct lengths with their offsets, in the order na_ring_plan counts them.
__global__ void k_na_ring_scan(int N, int64_t* boff, int* lens, int64_t* offs) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int cnt = 0;
  int64_t total = 0;
  for (int q = 0; q < 4 * N - 1; ++q) {
    int n;
    int64_t twoM;
    if (!na_bluestein(N, q, n, twoM)) {
      boff[q] = -1;
      continue;
    }
    int k = 0;
    while (k < cnt && lens[k] != n) ++k;
    if (k == cnt) {
      lens[cnt] = n;
      offs[cnt] = total;
      total += twoM;
      ++cnt;
    }
    boff[q] = offs[k];
  }
}

}  // namespace
}  // namespace clm

extern "C" clm_status clm_alm2map_noalloc(const double* alm, int32_t lmax, int32_t nside,
                                          double* map, hipStream_t stream) {
  using namespace clm;
  if (!alm || !map || lmax < 1 || nside < 1 || (nside & (nside - 1))) return CLM_EINVAL;
  if (nside > kNaMaxNside || lmax > kNaMaxLmax) return CLM_EUNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CLM_EHIP;
  if (dev < 0 || dev >= kNaMaxDevices) return CLM_EUNSUPPORTED;
  char* base = nullptr;
  if (na_scratch_ptr(dev, &base) != hipSuccess) return CLM_EHIP;

  const int N = nside, nr = 4 * N - 1, H = 2 * N;
  const int64_t npix = 12 * int64_t(N) * N;
  const NaRingPlan rp = na_ring_plan(N);
  // carve the scratch: 256-byte aligned pieces
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base + off;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  double* rt = reinterpret_cast<double*>(take(size_t(nr) * 4 * 8));
  int* ri = reinterpret_cast<int*>(take(size_t(nr) * 2 * 4));
  int64_t* boff = reinterpret_cast<int64_t*>(take(size_t(nr) * 8));
  int* lens = reinterpret_cast<int*>(take(size_t(N) * 4));
  int64_t* loffs = reinterpret_cast<int64_t*>(take(size_t(N) * 8));
  double* blu = reinterpret_cast<double*>(take(size_t(rp.total) * 8));
  double* mant = reinterpret_cast<double*>(take(size_t(lmax + 1) * H * 8));
  int* scale = reinterpret_cast<int*>(take(size_t(lmax + 1) * H * 4));
  double* G = reinterpret_cast<double*>(take(size_t(nr) * (lmax + 1) * 16));
  const size_t shm_syn = 4 * size_t(lmax + 1) * sizeof(double);
  // at the largest sizes every kernel stays within the default 64 KiB of
  // dynamic LDS, so no attribute call is made here
  if (off > kNaScratchBytes || rp.lds > 65536 || shm_syn > 65536) return CLM_EUNSUPPORTED;

  hipLaunchKernelGGL(k_ring_geom, dim3((nr + 255) / 256), dim3(256), 0, stream, N, rt, ri);
  hipLaunchKernelGGL(k_na_ring_scan, dim3(1), dim3(64), 0, stream, N, boff, lens, loffs);
  if (rp.nlen > 0)
    hipLaunchKernelGGL(k_blu_table, dim3(unsigned(rp.nlen)), dim3(kRingBlock), rp.lds, stream,
                       lens, loffs, blu);
  hipLaunchKernelGGL(k_lambda_mm, dim3((H + 127) / 128), dim3(128), 0, stream, rt, H,
                     int(lmax), mant, scale);
  const int nt = std::min(1024, round64(H));
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_synthesis<false>), dim3(lmax + 1, (H + nt - 1) / nt),
                     dim3(nt), shm_syn, stream, alm, rt, mant, scale, H, nr, int(lmax), G);
  hipLaunchKernelGGL(k_ring_inverse, dim3(nr), dim3(kRingBlock), rp.lds, stream, G, nr, rt,
                     ri, boff, blu, int(lmax), npix, 1, map);
  return hipGetLastError() == hipSuccess ? CLM_OK : CLM_EHIP;
}
