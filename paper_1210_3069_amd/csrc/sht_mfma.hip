// Batched Legendre transforms on the matrix cores (Sec. 3.1: the a_lm sum
// over rings and its synthesis, in the SHT step of the SHT+MG solve).
//
// For a fixed m the analysis over P planes is a real matrix product
//   a[l][c] = sum_q lambda_lm(theta_q) X[q][c],   c = 2 p + (re, im),
// with X = F_m(q) + F_m(q') (l - m even) or F_m(q) - F_m(q') (l - m odd) on
// the north rings q and their mirrors q' (the equator counted once), and the
// synthesis is its transpose, G^{even/odd}[q][c] = sum_l lambda_lm(theta_q)
// psi[l][c], north = even + odd, south = even - odd.  The planes are the
// GEMM columns.  lambda_lm is never stored: each lane runs the scaled FP64
// recurrence of one ring, 32 values of l at a time, and the wave stages the
// values in LDS for the MFMA operands.
//
// Forms: FP32 (lambda and X rounded to float32, v_mfma_f32_16x16x4f32),
// BF16x3 (each float32 operand split into bf16 hi + lo, products hi*hi +
// hi*lo + lo*hi) and BF16x6 (split into hi + mid + lo, products hi*hi +
// hi*mid + mid*hi + hi*lo + lo*hi + mid*mid), both accumulated in float32
// on the double-K bf16 matrix instructions (v_mfma_f32_16x16x32_bf16 in the
// analysis, v_mfma_f32_32x32x16_bf16 in the synthesis).  The recurrence, its
// scaling and the final weights stay in FP64; the waves' partial sums are
// added in FP64.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "clm_internal.h"

namespace clm {
namespace {

constexpr double kHugeB = 0x1p400;    // rescale threshold of the scaled recurrence
constexpr double kSmallB = 0x1p-800;  // rescale factor
constexpr int kStep = 32;             // values of l generated per step (16 per parity)
constexpr int kCols = 32;             // GEMM columns: 2 x up to 16 planes
constexpr int kBlk = 256;
constexpr int kMaxGroups = 4;         // plans (grids) of one persistent launch

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum Form : int { kFP32 = 0, kBF16X3 = 1, kBF16X6 = 2 };

// bf16 terms of a split operand, and the products summed: (i, j) = term i
// of the lambda operand times term j of the other, smallest first.
template <int FORM> struct Split;
template <> struct Split<kBF16X3> {
  static constexpr int NS = 2, NP = 3;
  static constexpr int A[NP] = {1, 0, 0}, B[NP] = {0, 1, 0};
};
template <> struct Split<kBF16X6> {
  static constexpr int NS = 3, NP = 6;
  static constexpr int A[NP] = {1, 2, 0, 1, 0, 0}, B[NP] = {1, 0, 2, 0, 1, 0};
};
template <> struct Split<kFP32> { static constexpr int NS = 1, NP = 1; };

// Row stride (floats) of a wave's lambda tile [32 l][64 rings].  Analysis
// reads, per lane, row 2 i + parity at a column group; synthesis reads
// column 16 mb + i (float32) or 32 mt + i (bf16) at rows of one parity.
template <int FORM> struct AnaStride { static constexpr int S = 68; };
template <> struct AnaStride<kFP32> { static constexpr int S = 65; };
constexpr int kSynStride = 72;

// x = sum of NS bf16 terms (each the rounding of the remainder), into
// element e of the operand vectors t[0..NS-1].
template <int NS>
__device__ __forceinline__ void split_into(float x, bf8 (&t)[NS], int e) {
  float r = x;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const __bf16 h = __bf16(r);
    t[k][e] = h;
    r -= float(h);
  }
}

// One ring's recurrence for fixed m: p1 = the latest lambda, p2 the one
// before, scale exponent s (< 0: below 2^-800 relative to the true value).
struct Rec {
  double z, p1, p2;
  int s;
};

// One step of the recurrence (lambda_{m+1,m} = sqrt(2m+3) z lambda_mm, then
// lambda_l = a_l (z lambda_{l-1} - b_l lambda_{l-2})): the kStep values of l
// from dl0 of this lane's ring, as float (0 while the scale exponent is
// negative or beyond l_max),
// into rows 0 .. kStep - 1 of the wave's tile (row stride STRIDE floats).
// The step's coefficients arrive as one vector (lane t holding element
// 2 dl0 + t: a_l, b_l interleaved); the wave stages them in its LDS slot cs
// and every lane then reads each (a_l, b_l) pair from one address.  The
// scaled recurrence is rescaled once per step instead of at each value:
// over 32 consecutive values it grows by less than 2^(16 log2(2m) - 58)
// (the largest factors are the first ones, l near m, near a pole), so from
// below 2^400 it stays far below the FP64 range for any m below 2^37, and
// the rescale is by a power of two, so every value, and every float
// written, equals that of a rescale at the threshold value.
template <int STRIDE>
__device__ __forceinline__ void rec_step(Rec& r, int m, int dl0, int nl, double rcv, double* cs,
                                         float* tw, int lane) {
  cs[lane] = rcv;
  __builtin_amdgcn_wave_barrier();
  const double2* ab = reinterpret_cast<const double2*>(cs);
  if (dl0 == 0) {
#pragma unroll
    for (int d = 0; d < kStep; ++d) {
      if (d == 1) {
        r.p2 = r.p1;
        r.p1 = sqrt(2.0 * m + 3.0) * r.z * r.p2;
      } else if (d >= 2) {
        const double2 c = ab[d];
        const double p0 = c.x * (r.z * r.p1 - c.y * r.p2);
        r.p2 = r.p1;
        r.p1 = p0;
      }
      tw[d * STRIDE + lane] = (d < nl && r.s == 0) ? float(r.p1) : 0.0f;
    }
  } else {
#pragma unroll
    for (int d = 0; d < kStep; ++d) {
      const double2 c = ab[d];
      const double p0 = c.x * (r.z * r.p1 - c.y * r.p2);
      r.p2 = r.p1;
      r.p1 = p0;
      tw[d * STRIDE + lane] = (dl0 + d < nl && r.s == 0) ? float(r.p1) : 0.0f;
    }
  }
  if (r.s < 0 && fabs(r.p1) > kHugeB) {
    r.p1 *= kSmallB;
    r.p2 *= kSmallB;
    r.s += 1;
  }
}

// The recurrence coefficients of a step of kStep values of l are read with
// one vector load a step ahead, lane t holding rc[2 dl0 + t] (a_l, b_l
// interleaved), so the recurrence never waits on memory.
__device__ __forceinline__ double rc_fetch(const double* rc, int dl0, int nl, int lane) {
  const int t = 2 * dl0 + lane;
  return t < 2 * nl ? rc[t] : 0.0;
}


struct MfmaArgs {
  const double* F;         // analysis in: [P][nring][lmax+1] complex
  double* G;               // synthesis out: [P][nring][lmax+1] complex
  const double* rt;        // ring table [nring][4]
  const double* lam_mant;  // [lmax+1][H]
  const int* lam_scale;
  const double* rc;        // recurrence coefficients (a, b) per (l, m), alm order
  const double* rk;        // derivative coefficients k_l per (l, m), alm order
  const float* psi;        // synthesis in: [nalm][32] (column c = 2 p + re/im)
  float* part;             // analysis out with several ring blocks: [R][nalm][32]
  double* alm[16];         // analysis out with one ring block: per plane
  double w;                // analysis weight 4 pi / N_pix
  int64_t nalm;
  int H, nring, lmax, P;
  int nwv;                 // waves of a workgroup (64 rings each)
  int R;                   // ring blocks: ceil(H / (64 nwv))
};

// The work of one persistent launch: up to kMaxGroups grids (plans), whose
// items (m, ring block) are numbered group by group, m ascending (the
// largest sums first), ring block fastest; workgroups take the next item
// from a counter in device memory until none is left.
struct MfmaMulti {
  MfmaArgs g[kMaxGroups];
  int start[kMaxGroups + 1];  // first item of each group; start[ng] = all items
  int R[kMaxGroups];          // ring blocks of each group
  int ng;
  int* ctr;                   // zero before the launch
};

// The next item of a persistent workgroup (block-uniform), or -1.
__device__ __forceinline__ int next_item(const MfmaMulti& mm, int* slot, int& g, int& m,
                                         int& rb) {
  __syncthreads();  // every thread has read the previous item
  if (threadIdx.x == 0) *slot = atomicAdd(mm.ctr, 1);
  __syncthreads();
  const int t = *slot;
  if (t >= mm.start[mm.ng]) return -1;
  g = 0;
  while (g + 1 < mm.ng && t >= mm.start[g + 1]) ++g;
  const int lt = t - mm.start[g];
  const int R = mm.R[g];
  m = lt / R;
  rb = lt - m * R;
  return t;
}

__device__ __forceinline__ size_t alm_base(int m, int lmax) {
  return size_t(m) * (2 * lmax + 1 - m) / 2 + m;  // index of (l = m, m)
}

__device__ __forceinline__ Rec rec_start(const MfmaArgs& a, int m, int q) {
  Rec r{0.0, 0.0, 0.0, -1};
  if (q < a.H) {
    r.z = a.rt[4 * q];
    r.p1 = a.lam_mant[size_t(m) * a.H + q];
    r.s = a.lam_scale[size_t(m) * a.H + q];
  }
  return r;
}

// ---------------------------------------------------------------- analysis
// One item: order m, block of 64 NW rings; each wave owns 64 rings for all
// l and keeps their X in registers.  The waves' partial sums are added in a
// fixed order (results do not depend on scheduling).  With 8 waves two
// workgroups fit per CU, so one's recurrence runs beside the other's matrix
// products.
template <int FORM, int NW>
__device__ __forceinline__ void analysis_item(const MfmaArgs& a, int m, int rb, float* tiles,
                                              double* coefs) {
  constexpr int SA = AnaStride<FORM>::S;
  constexpr int NS = Split<FORM>::NS;
  constexpr int KB = FORM == kFP32 ? 16 : 2;   // k-blocks over the 64 rings
  constexpr int KW = FORM == kFP32 ? 4 : 32;   // rings per k-block
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nl = a.lmax - m + 1;
  const int qb = (rb * a.nwv + w) * 64;  // first ring of this wave
  float* tw = tiles + w * kStep * SA;
  double* cs = coefs + w * 2 * kStep;
  const double* rc = a.rc + 2 * alm_base(m, a.lmax);
  Rec r = rec_start(a, m, qb + l);

  // B operands: X^{even/odd} of the wave's rings for the 32 columns
  const size_t pstride = size_t(a.nring) * (a.lmax + 1) * 2;
  auto xval = [&](int ring, int c, int par) -> float {
    const int p = c >> 1, ri = c & 1;
    if (ring >= a.H || p >= a.P) return 0.0f;
    const double* Fp = a.F + p * pstride;
    const int qm = a.nring - 1 - ring;
    const double fn = Fp[(size_t(ring) * (a.lmax + 1) + m) * 2 + ri];
    if (qm == ring) return float(fn);
    const double fs = Fp[(size_t(qm) * (a.lmax + 1) + m) * 2 + ri];
    return float(par == 0 ? fn + fs : fn - fs);
  };
  float xs[2][KB][2];
  bf8 xb[2][KB][2][NS];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int c = (l & 15) + 16 * nb;
        if constexpr (FORM == kFP32) {
          xs[par][j][nb] = xval(qb + KW * j + (l >> 4), c, par);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            split_into<NS>(xval(qb + KW * j + 8 * (l >> 4) + e, c, par), xb[par][j][nb], e);
        }
      }

  double rcv = rc_fetch(rc, 0, nl, l);
  for (int dl0 = 0; dl0 < nl; dl0 += kStep) {
    const double rcn = rc_fetch(rc, dl0 + kStep, nl, l);  // next step's, in flight
    // lambda for dl0 .. dl0 + 31 of this lane's ring into the wave's tile
    rec_step<SA>(r, m, dl0, nl, rcv, cs, tw, l);
    rcv = rcn;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the tile is written
    f4 acc[2][2];
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[par][nb] = f4{0.f, 0.f, 0.f, 0.f};
    const int i = l & 15;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const float* row = tw + (2 * i + par) * SA;
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        if constexpr (FORM == kFP32) {
          const float av = row[KW * j + (l >> 4)];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[par][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, xs[par][j][nb],
                                                               acc[par][nb], 0, 0, 0);
        } else {
          // A: row i of the M tile, rings 8 (lane / 16) + e of the k-block
          bf8 ab[NS];
#pragma unroll
          for (int e = 0; e < 8; ++e) split_into<NS>(row[KW * j + 8 * (l >> 4) + e], ab, e);
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int q = 0; q < Split<FORM>::NP; ++q)
              acc[par][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  ab[Split<FORM>::A[q]], xb[par][j][nb][Split<FORM>::B[q]], acc[par][nb], 0, 0,
                  0);
        }
      }
    }
    // this wave's partial sums into its own tile as [par][nb][i4][lane]
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) tw[((par * 2 + nb) * 4 + i4) * 64 + l] = acc[par][nb][i4];
    __syncthreads();
    // sum over the waves (in FP64, fixed order); output row rr = local dl,
    // column c.  The C fragment of row 4 (lane / 16) + i4 of an M tile,
    // column lane % 16.
    for (int t = threadIdx.x; t < kStep * kCols; t += blockDim.x) {
      const int rr = t >> 5, c = t & 31;
      const int par = rr & 1, ii = rr >> 1;
      const int src = ((par * 2 + (c >> 4)) * 4 + (ii & 3)) * 64 + 16 * (ii >> 2) + (c & 15);
      double sum = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) sum += double(tiles[v * kStep * SA + src]);
      const int dl = dl0 + rr, p = c >> 1;
      if (dl < nl && p < a.P) {
        const size_t idx = alm_base(m, a.lmax) + dl;
        if (a.R == 1)
          a.alm[p][2 * idx + (c & 1)] = a.w * sum;
        else
          a.part[(size_t(rb) * a.nalm + idx) * kCols + c] = float(sum);
      }
    }
    __syncthreads();
  }
}

// The groups' arguments are copied to LDS once (indexing the kernel
// argument by the item's group would copy it to scratch memory).
__device__ __forceinline__ void load_groups(const MfmaMulti& mm, MfmaArgs* ga) {
  if (threadIdx.x == 0) {
    ga[0] = mm.g[0];
    ga[1] = mm.g[1];
    ga[2] = mm.g[2];
    ga[3] = mm.g[3];
  }
}

template <int FORM, int NW>
__global__ __launch_bounds__(64 * NW, 32 / NW) void k_analysis_mfma(MfmaMulti mm) {
  __shared__ float tiles[NW * kStep * AnaStride<FORM>::S];
  __shared__ __align__(16) double coefs[NW * 2 * kStep];
  __shared__ MfmaArgs ga[kMaxGroups];
  __shared__ int slot;
  load_groups(mm, ga);
  int g, m, rb;
  while (next_item(mm, &slot, g, m, rb) >= 0)
    analysis_item<FORM, NW>(ga[g], m, rb, tiles, coefs);
}

// Sum of the ring-block partials, weighted, into the planes' alm.
__global__ void k_analysis_reduce(MfmaArgs a, int R) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.nalm * kCols) return;
  const int64_t idx = t / kCols;
  const int c = int(t % kCols), p = c >> 1;
  if (p >= a.P) return;
  double s = 0.0;
  for (int k = 0; k < R; ++k) s += double(a.part[(size_t(k) * a.nalm + idx) * kCols + c]);
  a.alm[p][2 * idx + (c & 1)] = a.w * s;
}

// psi_lm of the P planes as float GEMM columns [nalm][32].
__global__ void k_pack_psi(MfmaArgs a, float* psi) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.nalm * kCols) return;
  const int64_t idx = t / kCols;
  const int c = int(t % kCols), p = c >> 1;
  psi[t] = p < a.P ? float(a.alm[p][2 * idx + (c & 1)]) : 0.0f;
}

// --------------------------------------------------------------- synthesis
// One item: order m, block of 64 NW rings; each wave owns 64 rings and sums
// over all l, even and odd l - m apart.
template <int FORM, int NW>
__device__ __forceinline__ void synthesis_item(const MfmaArgs& a, int m, int rb, float* tiles,
                                               double* coefs) {
  constexpr int SS = kSynStride;
  constexpr int NS = Split<FORM>::NS;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nl = a.lmax - m + 1;
  const int qb = (rb * a.nwv + w) * 64;
  float* tw = tiles + w * kStep * SS;
  double* cs = coefs + w * 2 * kStep;
  const double* rc = a.rc + 2 * alm_base(m, a.lmax);
  const float* pm = a.psi + alm_base(m, a.lmax) * kCols;
  Rec r = rec_start(a, m, qb + l);
  // float32 form: 16 x 16 tiles, acc[par][mb][nb] (rings 16 mb + ..,
  // columns 16 nb + ..); bf16 forms: 32 x 32 tiles, accb[par][mt] (rings
  // 32 mt + .., all 32 columns)
  f4 acc[2][4][2];
  f16v accb[2][2];
  if constexpr (FORM == kFP32) {
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[par][mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
  } else {
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 16; ++v) accb[par][mt][v] = 0.f;
  }
  const int i = l & 15, k = l >> 4;
  // psi operands of a step (bf16 forms: loaded before the step's recurrence
  // so that it hides their latency).  float32: per parity, 4 values of l (k-blocks) x 2
  // column blocks; bf16: per parity the 8 values of l 2 (8 (lane / 32) + e)
  // + parity at column lane % 32.
  auto psi_fetch = [&](int dl0, float (&v)[2][8]) {
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int dl, col;
        if constexpr (FORM == kFP32) {
          dl = dl0 + 2 * (4 * (e >> 1) + k) + par;
          col = i + 16 * (e & 1);
        } else {
          dl = dl0 + 2 * (8 * (l >> 5) + e) + par;
          col = l & 31;
        }
        v[par][e] = dl < nl ? pm[size_t(dl) * kCols + col] : 0.0f;
      }
  };
  float pv[2][8];
  double rcv = rc_fetch(rc, 0, nl, l);
  for (int dl0 = 0; dl0 < nl; dl0 += kStep) {
    const double rcn = rc_fetch(rc, dl0 + kStep, nl, l);  // next step's, in flight
    // float32: the operands are fetched after the recurrence, which keeps
    // them out of its register peak (fewer spills at 16 waves per
    // workgroup; the other waves of the CU hide their latency)
    if constexpr (FORM != kFP32) psi_fetch(dl0, pv);
    rec_step<SS>(r, m, dl0, nl, rcv, cs, tw, l);
    if constexpr (FORM == kFP32) psi_fetch(dl0, pv);
    rcv = rcn;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      if constexpr (FORM == kFP32) {
        // K blocks of 4 values of l of this parity: rows 2 (4 j + k) + par
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 2 * (4 * j + k) + par;
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            const float av = tw[row * SS + 16 * mb + i];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[par][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  av, pv[par][2 * j + nb], acc[par][mb][nb], 0, 0, 0);
          }
        }
      } else {
        // the 16 values of l of this parity as one K block: B row
        // 8 (lane / 32) + e, column lane % 32; A ring 32 mt + lane % 32
        bf8 bb[NS];
#pragma unroll
        for (int e = 0; e < 8; ++e) split_into<NS>(pv[par][e], bb, e);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          bf8 ab[NS];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            split_into<NS>(tw[(2 * (8 * (l >> 5) + e) + par) * SS + 32 * mt + (l & 31)], ab, e);
#pragma unroll
          for (int q = 0; q < Split<FORM>::NP; ++q)
            accb[par][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                ab[Split<FORM>::A[q]], bb[Split<FORM>::B[q]], accb[par][mt], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // tile reads done before the next step
  }
  const size_t pstride = size_t(a.nring) * (a.lmax + 1) * 2;
  auto put = [&](int q, int c, double e, double o) {
    const int p = c >> 1, ri = c & 1;
    if (q >= a.H || p >= a.P) return;
    const int qm = a.nring - 1 - q;
    double* Gp = a.G + p * pstride;
    Gp[(size_t(q) * (a.lmax + 1) + m) * 2 + ri] = e + o;
    if (qm != q) Gp[(size_t(qm) * (a.lmax + 1) + m) * 2 + ri] = e - o;
  };
  if constexpr (FORM == kFP32) {
    // C fragment: ring 16 mb + 4 (lane / 16) + i4, column lane % 16 + 16 nb
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          put(qb + 16 * mb + 4 * k + i4, i + 16 * nb, acc[0][mb][nb][i4], acc[1][mb][nb][i4]);
  } else {
    // C fragment of a 32 x 32 tile: column lane % 32, row
    // 8 (v / 4) + 4 (lane / 32) + v % 4 for element v
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        put(qb + 32 * mt + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3), l & 31, accb[0][mt][v],
            accb[1][mt][v]);
  }
}

template <int FORM, int NW>
__global__ __launch_bounds__(64 * NW) void k_synthesis_mfma(MfmaMulti mm) {
  __shared__ float tiles[NW * kStep * kSynStride];
  __shared__ __align__(16) double coefs[NW * 2 * kStep];
  __shared__ MfmaArgs ga[kMaxGroups];
  __shared__ int slot;
  load_groups(mm, ga);
  int g, m, rb;
  while (next_item(mm, &slot, g, m, rb) >= 0)
    synthesis_item<FORM, NW>(ga[g], m, rb, tiles, coefs);
}

// ----------------------------------------------------- derivative synthesis
// The pure-SHT solver's fields (Sec. 3.2, last paragraph; covariant
// components as in App. A): on every ring the m-coefficients of
//   g_t = psi_theta, g_p = psi_phi / sin, U_tt, U_pp, U_tp
// from psi_lm.  Per (ring, l) the recurrence generates, in FP64, four
// functions of theta (z = cos, s = sin):
//   lambda;
//   T = d lambda / d theta = (l z lambda_l - k_l lambda_{l-1}) / s,
//       k_l = sqrt((2l+1)(l^2-m^2)/(2l-1))  (from the Legendre equation);
//   X = (m^2/s^2 - l(l+1)/2) lambda - (z/s) T, so that
//       gamma_1 = (U_tt - U_pp)/2 = sum X psi e^{i m phi};
//   Y = (m/s) (T - (z/s) lambda), so that gamma_2 = U_tp = sum i Y psi e^{i m phi}.
// X and Y are the spin-2 functions (and T with (m/s) lambda the spin-1
// pair): their 1/s and 1/s^2 terms cancel inside the FP64 evaluation, so
// the rounded values keep float32 relative precision on the polar rings.
// They enter float32 matrix products with the GEMM columns psi_lm (8
// planes x re/im) and, for lambda only, l(l+1) psi_lm (the Laplacian:
// U_tt + U_pp = -sum l(l+1) psi_lm Y_lm):
//   G = sum lambda psi, L = sum lambda l(l+1) psi, T, X, Y = sum (T|X|Y) psi.
// Per ring then g_t = T, g_p = i (m/s) G, U_tt = X - L/2, U_pp = -X - L/2,
// U_tp = i Y.  On the mirror ring lambda, L and X take the sign (-1)^(l+m)
// of lambda, T and Y the opposite one.
constexpr int kStepD = 16;   // values of l per step (8 per parity: 2 K blocks)
constexpr int kPlanesD = 8;  // planes of one launch (32 columns: psi and l(l+1) psi)
constexpr int kTileD = kStepD * kSynStride;  // floats of one function's tile

// One step of kStepD values of l of this lane's ring: lambda, T, X, Y into
// the four tiles of the wave (rows d, column = lane).  The step's
// coefficients arrive as one vector: lanes 0..31 hold (a_l, b_l)
// interleaved, lanes 32..47 hold k_l; the wave stages them in LDS.  The
// rescale rule is that of rec_step over fewer values.
__device__ __forceinline__ void deriv_value(const Rec& r, double L, double kl, double zs,
                                            double is, double ms, double mms, bool ok,
                                            float* tw, int off) {
  const double t = L * zs * r.p1 - (kl * is) * r.p2;
  const double x = (mms - 0.5 * L * (L + 1.0)) * r.p1 - zs * t;
  const double y = ms * (t - zs * r.p1);
  tw[off] = ok ? float(r.p1) : 0.0f;
  tw[kTileD + off] = ok ? float(t) : 0.0f;
  tw[2 * kTileD + off] = ok ? float(x) : 0.0f;
  tw[3 * kTileD + off] = ok ? float(y) : 0.0f;
}

__device__ __forceinline__ void rec_step_deriv(Rec& r, int m, int dl0, int nl, double cv,
                                               double* cs, float* tw, int lane, double zs,
                                               double is, double ms, double mms) {
  cs[lane] = cv;
  __builtin_amdgcn_wave_barrier();
  const double2* ab = reinterpret_cast<const double2*>(cs);
  const double* kk = cs + 2 * kStepD;
  const double L0 = double(m + dl0);
  if (dl0 == 0) {
#pragma unroll
    for (int d = 0; d < kStepD; ++d) {
      if (d == 1) {
        r.p2 = r.p1;
        r.p1 = sqrt(2.0 * m + 3.0) * r.z * r.p2;
      } else if (d >= 2) {
        const double2 c = ab[d];
        const double p0 = c.x * (r.z * r.p1 - c.y * r.p2);
        r.p2 = r.p1;
        r.p1 = p0;
      }
      deriv_value(r, L0 + d, kk[d], zs, is, ms, mms, d < nl && r.s == 0, tw,
                  d * kSynStride + lane);
    }
  } else {
#pragma unroll
    for (int d = 0; d < kStepD; ++d) {
      const double2 c = ab[d];
      const double p0 = c.x * (r.z * r.p1 - c.y * r.p2);
      r.p2 = r.p1;
      r.p1 = p0;
      deriv_value(r, L0 + d, kk[d], zs, is, ms, mms, dl0 + d < nl && r.s == 0, tw,
                  d * kSynStride + lane);
    }
  }
  if (r.s < 0 && fabs(r.p1) > kHugeB) {
    r.p1 *= kSmallB;
    r.p2 *= kSmallB;
    r.s += 1;
  }
}

// The coefficients of the step at dl0 (layout of rec_step_deriv), loaded a
// step ahead.
__device__ __forceinline__ double dcoef_fetch(const double* rc, const double* rk, int dl0,
                                              int nl, int lane) {
  if (lane < 2 * kStepD) {
    const int t = 2 * dl0 + lane;
    return t < 2 * nl ? rc[t] : 0.0;
  }
  const int t = dl0 + lane - 2 * kStepD;
  return (lane < 3 * kStepD && t < nl) ? rk[t] : 0.0;
}

// psi_lm of up to kPlanesD planes as float GEMM columns [nalm][32]: column
// 2 p + re/im holds psi_lm of plane p, column 16 + 2 p + re/im holds
// l (l + 1) psi_lm.  One workgroup per m.
__global__ void k_pack_psi_deriv(MfmaArgs a, float* psi) {
  const int m = blockIdx.x;
  const int nl = a.lmax - m + 1;
  const size_t base = alm_base(m, a.lmax);
  for (int t = threadIdx.x; t < nl * kCols; t += blockDim.x) {
    const int dl = t >> 5, c = t & 31;
    const int cc = c & 15, p = cc >> 1;
    double v = 0.0;
    if (p < a.P) {
      v = a.alm[p][2 * (base + dl) + (cc & 1)];
      if (c >= 16) {
        const double L = double(m + dl);
        v *= L * (L + 1.0);
      }
    }
    psi[(base + dl) * kCols + c] = float(v);
  }
}

// One item: order m, block of 64 NW rings; each wave owns 64 rings.  Output
// G = [P][5 fields][nring][lmax+1] complex, fields g_t, g_p, U_tt, U_pp, U_tp.
template <int NW>
__device__ __forceinline__ void deriv_item(const MfmaArgs& a, int m, int rb, float* tiles,
                                           double* coefs) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nl = a.lmax - m + 1;
  const int qb = (rb * a.nwv + w) * 64;
  float* tw = tiles + w * 4 * kTileD;
  double* cs = coefs + w * 4 * kStepD;
  const double* rc = a.rc + 2 * alm_base(m, a.lmax);
  const double* rk = a.rk + alm_base(m, a.lmax);
  const float* pm = a.psi + alm_base(m, a.lmax) * kCols;
  Rec r = rec_start(a, m, qb + l);
  double is = 0.0;
  if (qb + l < a.H) is = 1.0 / a.rt[4 * (qb + l) + 1];
  const double zs = r.z * is, ms = double(m) * is, mms = ms * ms;
  // acc[par][mb][f]: rings 16 mb + .., f = lambda x psi, lambda x l(l+1) psi,
  // T x psi, X x psi, Y x psi (columns lane % 16 of the psi block)
  f4 acc[2][4][5];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int f = 0; f < 5; ++f) acc[par][mb][f] = f4{0.f, 0.f, 0.f, 0.f};
  const int i = l & 15, k = l >> 4;
  // psi operands of a step, per parity: K block j (values 2 (4 j + k) + par)
  // x column block nb (psi, l(l+1) psi), as element 2 j + nb
  auto psi_fetch = [&](int dl0, float (&v)[2][4]) {
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int dl = dl0 + 2 * (4 * (e >> 1) + k) + par;
        v[par][e] = dl < nl ? pm[size_t(dl) * kCols + i + 16 * (e & 1)] : 0.0f;
      }
  };
  float pv[2][4];
  double cv = dcoef_fetch(rc, rk, 0, nl, l);
  for (int dl0 = 0; dl0 < nl; dl0 += kStepD) {
    const double cn = dcoef_fetch(rc, rk, dl0 + kStepD, nl, l);  // next step's, in flight
    psi_fetch(dl0, pv);
    rec_step_deriv(r, m, dl0, nl, cv, cs, tw, l, zs, is, ms, mms);
    cv = cn;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the tiles are written
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = 2 * (4 * j + k) + par;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const float* ap = tw + row * kSynStride + 16 * mb + i;
          const float a0 = ap[0], a1 = ap[kTileD], a2 = ap[2 * kTileD], a3 = ap[3 * kTileD];
          const float b0 = pv[par][2 * j], b1 = pv[par][2 * j + 1];
          acc[par][mb][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[par][mb][0], 0, 0, 0);
          acc[par][mb][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[par][mb][1], 0, 0, 0);
          acc[par][mb][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[par][mb][2], 0, 0, 0);
          acc[par][mb][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b0, acc[par][mb][3], 0, 0, 0);
          acc[par][mb][4] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b0, acc[par][mb][4], 0, 0, 0);
        }
      }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // tile reads done before the next step
  }
  // C fragment: ring 16 mb + 4 (lane / 16) + i4, column lane % 16 = 2 p + ri.
  // Multiplying by i moves component ri to 1 - ri with sign (+ for ri = 0).
  const size_t fs = size_t(a.nring) * (a.lmax + 1) * 2;  // one field, doubles
  const int p = i >> 1, ri = i & 1;
  const double sg = ri == 0 ? 1.0 : -1.0;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int i4 = 0; i4 < 4; ++i4) {
      const int q = qb + 16 * mb + 4 * k + i4;
      if (q >= a.H || p >= a.P) continue;
      const double mos = double(m) / a.rt[4 * q + 1];
      const int qm = a.nring - 1 - q;
      double* Gp = a.G + size_t(p) * 5 * fs;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && qm == q) break;
        const double sn = h == 0 ? 1.0 : -1.0;  // even + sn odd
        const double G = double(acc[0][mb][0][i4]) + sn * double(acc[1][mb][0][i4]);
        const double L = double(acc[0][mb][1][i4]) + sn * double(acc[1][mb][1][i4]);
        const double T = sn * (double(acc[0][mb][2][i4]) + sn * double(acc[1][mb][2][i4]));
        const double X = double(acc[0][mb][3][i4]) + sn * double(acc[1][mb][3][i4]);
        const double Y = sn * (double(acc[0][mb][4][i4]) + sn * double(acc[1][mb][4][i4]));
        double* g = Gp + (size_t(h == 0 ? q : qm) * (a.lmax + 1) + m) * 2;
        g[ri] = T;
        g[fs + 1 - ri] = sg * mos * G;
        g[2 * fs + ri] = X - 0.5 * L;
        g[3 * fs + ri] = -X - 0.5 * L;
        g[4 * fs + 1 - ri] = sg * Y;
      }
    }
}

template <int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_deriv_mfma(MfmaMulti mm) {
  __shared__ float tiles[NW * 4 * kTileD];
  __shared__ __align__(16) double coefs[NW * 4 * kStepD];
  __shared__ MfmaArgs ga[kMaxGroups];
  __shared__ int slot;
  load_groups(mm, ga);
  int g, m, rb;
  while (next_item(mm, &slot, g, m, rb) >= 0) deriv_item<NW>(ga[g], m, rb, tiles, coefs);
}

// k_l = sqrt((2l+1)(l^2-m^2)/(2l-1)) per (l, m) in alm order (0 at l = m).
__global__ void k_deriv_table(int lmax, double* rk) {
  const int m = blockIdx.x;
  const size_t base = alm_base(m, lmax);
  for (int l = m + threadIdx.x; l <= lmax; l += blockDim.x) {
    const double L = l, M = m;
    rk[base + l - m] = sqrt((2.0 * L + 1.0) * (L * L - M * M) / fmax(2.0 * L - 1.0, 1.0));
  }
}

// Recurrence coefficients per (l, m) in alm order:
// a_l = sqrt((4l^2-1)/(l^2-m^2)), b_l = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
__global__ void k_recur_table(int lmax, double* rc) {
  const int m = blockIdx.x;
  const size_t base = alm_base(m, lmax);
  for (int l = m + 2 + threadIdx.x; l <= lmax; l += blockDim.x) {
    const double L = l, M = m;
    rc[2 * (base + l - m)] = sqrt((4.0 * L * L - 1.0) / (L * L - M * M));
    rc[2 * (base + l - m) + 1] =
        sqrt(((L - 1.0) * (L - 1.0) - M * M) / (4.0 * (L - 1.0) * (L - 1.0) - 1.0));
  }
}

MfmaArgs base_args(Plan* p, int first_slot, int P) {
  MfmaArgs a{};
  a.rt = p->ring_s;
  a.lam_mant = p->lam_mant;
  a.lam_scale = p->lam_scale;
  a.rc = p->rcoef;
  a.nalm = p->nalm;
  a.H = p->H;
  a.nring = p->nring_s;
  a.lmax = p->d.lmax;
  a.P = P;
  for (int k = 0; k < P; ++k) a.alm[k] = p->slots[first_slot + k].alm;
  return a;
}

int ring_blocks_nw(int H, int nw) { return (H + 64 * nw - 1) / (64 * nw); }

__global__ void k_zero_int(int* x) { *x = 0; }

// Workgroups of a persistent launch: as many as fit on the device at once
// (LDS and wave slots per CU), at most one per item.
int persistent_blocks(const Plan* p, size_t lds, int nw, int items) {
  int per_cu = int((160 * 1024) / (lds + 256));
  per_cu = std::min(per_cu, 32 / nw);
  per_cu = std::max(per_cu, 1);
  return std::max(1, std::min(items, per_cu * p->ncu));
}

// Shapes the autotuner chooses from: waves per workgroup.
constexpr int kAnaNW[] = {8, 16};
constexpr int kSynNW[] = {8, 12, 16};

template <int FORM, int NW>
void launch_ana(const MfmaMulti& mm, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_analysis_mfma<FORM, NW>), dim3(blocks), dim3(64 * NW), 0,
                     s, mm);
}

template <int FORM, int NW>
void launch_syn(const MfmaMulti& mm, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_synthesis_mfma<FORM, NW>), dim3(blocks), dim3(64 * NW), 0,
                     s, mm);
}

template <int FORM>
bool dispatch_ana(int nw, const MfmaMulti& mm, int blocks, hipStream_t s) {
  switch (nw) {
    case 8: launch_ana<FORM, 8>(mm, blocks, s); return true;
    case 16: launch_ana<FORM, 16>(mm, blocks, s); return true;
    default: return false;
  }
}

template <int FORM>
bool dispatch_syn(int nw, const MfmaMulti& mm, int blocks, hipStream_t s) {
  switch (nw) {
    case 8: launch_syn<FORM, 8>(mm, blocks, s); return true;
    case 12: launch_syn<FORM, 12>(mm, blocks, s); return true;
    case 16: launch_syn<FORM, 16>(mm, blocks, s); return true;
    default: return false;
  }
}

int form_of(const Plan* p) {
  return p->d.legendre_prec == CLM_BF16X3 ? kBF16X3
         : p->d.legendre_prec == CLM_BF16X6 ? kBF16X6 : kFP32;
}

// One persistent analysis launch over the groups (plan, first slot,
// planes), then the ring-block partial sums of each group that has several.
clm_status analysis_groups(const MfmaGroup* gs, int ng, int nw, hipStream_t s) {
  Plan* p = gs[0].p;
  MfmaMulti mm{};
  mm.ng = ng;
  mm.ctr = p->mfma_ctr;
  int items = 0;
  for (int k = 0; k < ng; ++k) {
    MfmaArgs& a = mm.g[k];
    a = base_args(gs[k].p, gs[k].first_slot, gs[k].P);
    a.F = gs[k].p->Fb;
    a.part = gs[k].p->apart;
    a.w = 4.0 * 3.14159265358979323846 / double(gs[k].p->npix_s);
    a.nwv = nw;
    a.R = ring_blocks_nw(a.H, nw);
    mm.R[k] = a.R;
    mm.start[k] = items;
    items += (a.lmax + 1) * a.R;
  }
  mm.start[ng] = items;
  const int form = form_of(p);
  const size_t lds = size_t(nw) * kStep * (form == kFP32 ? 65 : 68) * 4 + sizeof(mm.g);
  const int blocks = persistent_blocks(p, lds, nw, items);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, p->mfma_ctr);
  {
    CLM_TIMED(p, s, "sht_analysis_mfma");
    const bool ok = form == kBF16X3   ? dispatch_ana<kBF16X3>(nw, mm, blocks, s)
                    : form == kBF16X6 ? dispatch_ana<kBF16X6>(nw, mm, blocks, s)
                                      : dispatch_ana<kFP32>(nw, mm, blocks, s);
    if (!ok) return fail(p, CLM_EINVAL, "no analysis shape with that many waves");
  }
  CLM_LAUNCH_CHECK();
  for (int k = 0; k < ng; ++k) {
    const MfmaArgs& a = mm.g[k];
    if (a.R == 1) continue;
    const int64_t n = a.nalm * kCols;
    CLM_TIMED(p, s, "sht_analysis_reduce");
    hipLaunchKernelGGL(k_analysis_reduce, dim3(unsigned((n + kBlk - 1) / kBlk)), dim3(kBlk), 0,
                       s, a, a.R);
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

// psi_lm of each group packed as GEMM columns, then one persistent
// synthesis launch over the groups.
clm_status synthesis_groups(const MfmaGroup* gs, int ng, int nw, hipStream_t s) {
  Plan* p = gs[0].p;
  MfmaMulti mm{};
  mm.ng = ng;
  mm.ctr = p->mfma_ctr;
  int items = 0;
  for (int k = 0; k < ng; ++k) {
    MfmaArgs& a = mm.g[k];
    a = base_args(gs[k].p, gs[k].first_slot, gs[k].P);
    a.G = gs[k].p->Gb;
    a.psi = gs[k].p->psib;
    a.nwv = nw;
    a.R = ring_blocks_nw(a.H, nw);
    mm.R[k] = a.R;
    mm.start[k] = items;
    items += (a.lmax + 1) * a.R;
    const int64_t n = a.nalm * kCols;
    {
      CLM_TIMED(p, s, "sht_pack_psi");
      hipLaunchKernelGGL(k_pack_psi, dim3(unsigned((n + kBlk - 1) / kBlk)), dim3(kBlk), 0, s, a,
                         gs[k].p->psib);
    }
    CLM_LAUNCH_CHECK();
  }
  mm.start[ng] = items;
  const int form = form_of(p);
  const size_t lds = size_t(nw) * kStep * kSynStride * 4 + sizeof(mm.g);
  const int blocks = persistent_blocks(p, lds, nw, items);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, p->mfma_ctr);
  {
    CLM_TIMED(p, s, "sht_synthesis_mfma");
    const bool ok = form == kBF16X3   ? dispatch_syn<kBF16X3>(nw, mm, blocks, s)
                    : form == kBF16X6 ? dispatch_syn<kBF16X6>(nw, mm, blocks, s)
                                      : dispatch_syn<kFP32>(nw, mm, blocks, s);
    if (!ok) return fail(p, CLM_EINVAL, "no synthesis shape with that many waves");
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

template <int NW>
void launch_der(const MfmaMulti& mm, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_deriv_mfma<NW>), dim3(blocks), dim3(64 * NW), 0, s, mm);
}

constexpr int kDerNW[] = {4, 8};

// psi_lm of planes first_slot .. first_slot + P - 1 packed as GEMM columns,
// then one persistent derivative-synthesis launch; the five fields of plane
// k land in Gb + 5 k nF.
clm_status deriv_launch(Plan* p, int first_slot, int P, int nw, hipStream_t s) {
  if (P < 1 || P > kPlanesD) return fail(p, CLM_EINVAL, "1 to 8 planes per derivative synthesis");
  if (!p->dcoef) return fail(p, CLM_EINVAL, "derivative synthesis needs a pure-SHT plan");
  MfmaMulti mm{};
  mm.ng = 1;
  mm.ctr = p->mfma_ctr;
  MfmaArgs& a = mm.g[0];
  a = base_args(p, first_slot, P);
  a.G = p->Gb;
  a.psi = p->psib;
  a.rk = p->dcoef;
  a.nwv = nw;
  a.R = ring_blocks_nw(a.H, nw);
  mm.R[0] = a.R;
  mm.start[0] = 0;
  mm.start[1] = (a.lmax + 1) * a.R;
  {
    CLM_TIMED(p, s, "sht_pack_psi");
    hipLaunchKernelGGL(k_pack_psi_deriv, dim3(a.lmax + 1), dim3(kBlk), 0, s, a, p->psib);
  }
  CLM_LAUNCH_CHECK();
  const size_t lds = size_t(nw) * 4 * (kTileD * 4 + kStepD * 8) + sizeof(mm.g);
  const int blocks = persistent_blocks(p, lds, nw, mm.start[1]);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, p->mfma_ctr);
  {
    CLM_TIMED(p, s, "sht_deriv_mfma");
    switch (nw) {
      case 4: launch_der<4>(mm, blocks, s); break;
      case 8: launch_der<8>(mm, blocks, s); break;
      default: return fail(p, CLM_EINVAL, "no derivative-synthesis shape with that many waves");
    }
  }
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

}  // namespace

// Ring blocks of the analysis at the fewest waves the autotuner may pick
// (its partial sums are [R][nalm][32]).
int mfma_ring_blocks(int H) { return ring_blocks_nw(H, kAnaNW[0]); }

clm_status mfma_tables(Plan* p, hipStream_t s) {
  hipLaunchKernelGGL(k_recur_table, dim3(p->d.lmax + 1), dim3(kBlk), 0, s, p->d.lmax, p->rcoef);
  if (p->dcoef)
    hipLaunchKernelGGL(k_deriv_table, dim3(p->d.lmax + 1), dim3(kBlk), 0, s, p->d.lmax,
                       p->dcoef);
  CLM_LAUNCH_CHECK();
  return CLM_OK;
}

int mfma_deriv_planes() { return kPlanesD; }

clm_status mfma_deriv_synthesis(Plan* p, int first_slot, int P, hipStream_t s) {
  return deriv_launch(p, first_slot, P, p->der_nw, s);
}

clm_status mfma_analysis(Plan* p, int first_slot, int P, hipStream_t s) {
  const MfmaGroup g{p, first_slot, P};
  return analysis_groups(&g, 1, p->ana_nw, s);
}

clm_status mfma_synthesis(Plan* p, int first_slot, int P, hipStream_t s) {
  const MfmaGroup g{p, first_slot, P};
  return synthesis_groups(&g, 1, p->syn_nw, s);
}

clm_status mfma_analysis_multi(const MfmaGroup* gs, int ng, hipStream_t s) {
  if (ng < 1 || ng > kMaxGroups) return fail(gs[0].p, CLM_EINVAL, "1 to 4 plans per launch");
  return analysis_groups(gs, ng, gs[0].p->ana_nw, s);
}

clm_status mfma_synthesis_multi(const MfmaGroup* gs, int ng, hipStream_t s) {
  if (ng < 1 || ng > kMaxGroups) return fail(gs[0].p, CLM_EINVAL, "1 to 4 plans per launch");
  return synthesis_groups(gs, ng, gs[0].p->syn_nw, s);
}

// The autotuner: waves per workgroup of the analysis and of the synthesis,
// chosen by timing each shape on the plan's own buffers with a full batch
// (kept, for plans of the same device, grid, lmax, form and batch, for the
// life of the process).  Shapes given in the description are kept.
namespace {
struct TuneKey {
  int dev, nside, lmax, form, batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, nside, lmax, form, batch) <
           std::tie(o.dev, o.nside, o.lmax, o.form, o.batch);
  }
};
std::mutex g_tune_mutex;
std::map<TuneKey, std::tuple<int, int, int>> g_tuned;

template <typename F>
float time_launch(F f, clm_status& st) {
  hipEvent_t a = nullptr, b = nullptr;
  float best = 1e30f;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    st = CLM_EHIP;
    return best;
  }
  for (int rep = 0; rep < 3 && st == CLM_OK; ++rep) {
    (void)hipEventRecord(a, nullptr);
    st = f();
    (void)hipEventRecord(b, nullptr);
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      st = CLM_EHIP;
    if (rep > 0) best = std::min(best, ms);  // the first launch is a warm-up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}
}  // namespace

clm_status mfma_autotune(Plan* p) {
  const clm_plan_desc& d = p->d;
  const TuneKey key{p->device, d.nside_sht, d.lmax, form_of(p) + (p->mg ? 0 : 8), p->batch};
  int ana = d.mfma_ana_waves, syn = d.mfma_syn_waves;
  int der = p->mg ? p->der_nw : d.mfma_der_waves;
  {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      if (ana == 0) ana = std::get<0>(it->second);
      if (syn == 0) syn = std::get<1>(it->second);
      if (der == 0) der = std::get<2>(it->second);
    }
  }
  const size_t nF = size_t(p->nring_s) * (d.lmax + 1) * 2;
  if (ana == 0 || syn == 0 || der == 0) {
    if (hipMemset(p->Fb, 0, nF * p->batch * 8) != hipSuccess ||
        hipMemset(p->psib, 0, size_t(p->nalm) * kCols * 4) != hipSuccess)
      return fail(p, CLM_EHIP, "autotune set-up failed");
  }
  clm_status st = CLM_OK;
  const MfmaGroup g{p, 0, p->batch};
  if (ana == 0) {
    float best = 1e30f;
    for (int nw : kAnaNW) {
      const float t = time_launch([&] { return analysis_groups(&g, 1, nw, nullptr); }, st);
      if (st != CLM_OK) return st;
      p->tune_ms.push_back({std::string("analysis_waves_") + std::to_string(nw), t});
      if (t < best) { best = t; ana = nw; }
    }
  }
  if (syn == 0) {
    float best = 1e30f;
    for (int nw : kSynNW) {
      const float t = time_launch([&] { return synthesis_groups(&g, 1, nw, nullptr); }, st);
      if (st != CLM_OK) return st;
      p->tune_ms.push_back({std::string("synthesis_waves_") + std::to_string(nw), t});
      if (t < best) { best = t; syn = nw; }
    }
  }
  if (der == 0) {
    // on psi_lm = 0 (the slots' coefficients are not yet written)
    float best = 1e30f;
    const int P = std::min(p->batch, kPlanesD);
    for (int k = 0; k < P; ++k)
      if (hipMemset(p->slots[k].alm, 0, size_t(p->nalm) * 16) != hipSuccess)
        return fail(p, CLM_EHIP, "autotune set-up failed");
    for (int nw : kDerNW) {
      const float t = time_launch([&] { return deriv_launch(p, 0, P, nw, nullptr); }, st);
      if (st != CLM_OK) return st;
      p->tune_ms.push_back({std::string("derivative_waves_") + std::to_string(nw), t});
      if (t < best) { best = t; der = nw; }
    }
  }
  p->ana_nw = ana;
  p->syn_nw = syn;
  p->der_nw = der;
  p->d.mfma_ana_waves = ana;
  p->d.mfma_syn_waves = syn;
  if (!p->mg) p->d.mfma_der_waves = der;
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  g_tuned[key] = {ana, syn, der};
  return CLM_OK;
}

}  // namespace clm
