// Internal definitions shared by the library's translation units: the plan
// object, error plumbing and the launchers each stage exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "calclens_mi.h"

namespace clm {

// Device-side latched conditions (bit flags in plan->status_dev).
enum : int { ST_LEFT_PATCH = 1, ST_NONFINITE = 2, ST_NOTCONV = 4 };

// Epsilon rule: coarse cells per side of one partial-sum tile.
constexpr int kEpsTile = 16;

// Bytes of one patch-setup tile's geometry record.
constexpr int kSetupMetaBytes = 48;

// Largest multigrid level handled entirely inside one workgroup's LDS.
constexpr int kLdsLevelMax = 64;
// Interior side of the multigrid tiles streamed through LDS on larger levels.
constexpr int kTile = 64;

// Logical block index for grids whose neighbouring blocks share data: the
// hardware deals blocks round-robin over the 8 XCDs (each with its own L2),
// so block b is given logical index (b mod 8) (nb / 8) + b / 8 and each XCD
// runs one contiguous range of logical blocks.  Identity when the grid is
// not a multiple of 8.
// The patch (bundle) of compact index c under a partial-sky domain: the
// c-th entry of the sorted list of the domain's bundles, or c itself when
// the plan covers the whole sky (pmap = nullptr).
__device__ __forceinline__ int64_t patch_of(const int* pmap, int64_t c) {
  return pmap ? int64_t(pmap[c]) : c;
}

__device__ __forceinline__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

struct LevelGeom {
  int n;         // cells per side
  size_t crow;   // offset of this level's row coefficients (4 doubles per row)
};

struct Slot {
  double* alm = nullptr;     // [nalm] complex (2 doubles each)
  double* psi_s = nullptr;   // [npix_s]
  double* u0 = nullptr;      // [npatch][(n+2)^2], SHT+MG only
  void* du = nullptr;        // [npatch][n^2] of T, SHT+MG only
};

struct Plan {
  clm_plan_desc d{};
  int device = 0;
  bool mg = false;
  bool fp64mg = false;
  int64_t npix_f = 0, npix_s = 0, nalm = 0, nbundle = 0;
  int nring_s = 0, nring_f = 0, H = 0;  // rings; north rings incl. equator
  int n = 0, nlev = 0, ktile = 0;       // patch cells, levels, first LDS level
  int bundle_shift = 0;                 // ray NESTED index >> shift = bundle
  double side_b = 0, L = 0, delta = 0;
  std::vector<LevelGeom> lev;
  size_t bytes = 0;
  std::string err;

  // tables
  double* ring_s = nullptr;     // [nring_s][4]: z, sin theta, theta, phi0
  int* ringi_s = nullptr;       // [nring_s][2]: n, first
  double* ringx_s = nullptr;    // [nring_s + 1][2]: n/(2 pi), 1/(theta gap above)
  double* ring_f = nullptr;     // same for the fine grid
  int* ringi_f = nullptr;
  double* ringx_f = nullptr;
  int64_t* blu_off = nullptr;   // [nring_s] chirp-filter table offset (doubles), -1: direct
  double* blu = nullptr;        // chirp-filter transforms of the Bluestein rings
  size_t ring_lds = 0;          // dynamic LDS of the ring kernels
  std::vector<std::pair<const void*, size_t>> lds_set;  // LDS opt-ins made
  double* lam_mant = nullptr;   // [lmax+1][H] lambda_mm mantissa
  int* lam_scale = nullptr;     // [lmax+1][H] scale exponent (units of 2^800)
  int* r2n_s = nullptr;         // RING -> NESTED at nside_sht
  int* r2n_f = nullptr;         // RING -> NESTED at nside_fine
  double* rot = nullptr;        // [nbundle][9] patch rotations R_b
  double* coef = nullptr;       // level row coefficients
  // per level row, in the multigrid precision (8 values of T, rows as in
  // coef): s_m, s_p, 1 / s_c, area, the face term of the diagonal, the
  // reciprocal diagonals off and on a side face, and (even rows) the
  // quad-pair restriction weight 1 / (2 (A_i + A_i+1))
  void* rowt = nullptr;
  double* cinv = nullptr;       // [16*16] inverse of the coarsest operator
  double* rcoef = nullptr;      // [nalm][2] Legendre recurrence a_l, b_l (matrix-core SHT)
  double* dcoef = nullptr;      // [nalm] derivative coefficients k_l (pure-SHT matrix-core plans)

  // scratch
  double* kap_s = nullptr;      // [npix_s] degraded, demeaned kappa
  double* F = nullptr;          // [nring_s][lmax+1] complex
  double* G = nullptr;          // [5][nring_s][lmax+1] complex (synthesis)
  double* red = nullptr;        // [1024] reduction partials; red[1023] = mean
  // matrix-core SHT of a batch of planes (legendre_prec FP32 / BF16X3 / BF16X6)
  int batch = 0;                // planes per GEMM batch (<= 16)
  int ncu = 0;                  // compute units of the device
  int ana_nw = 8, syn_nw = 16;  // waves per workgroup of the matrix-core kernels
  int der_nw = 4;               // ... and of the derivative synthesis
  int* mfma_ctr = nullptr;      // work counter of their persistent launches
  std::vector<std::pair<std::string, float>> tune_ms;  // autotuner timings
  double* Fb = nullptr;         // [batch][nring_s][lmax+1] complex ring transforms
  double* Gb = nullptr;         // [batch][nring_s][lmax+1] complex synthesis sums; pure-SHT
                                // plans: at least [8][5] such fields (derivative synthesis)
  float* apart = nullptr;       // [ring blocks][nalm][32] analysis partial sums
  float* psib = nullptr;        // [nalm][32] psi_lm as GEMM columns
  double* deriv = nullptr;      // [5][npix_s] pure-SHT raw derivative maps
  double* iter_map = nullptr;   // [npix_s] analysis refinement: f - S a
  double* iter_alm = nullptr;   // [nalm] complex: its analysis
  void* fprime = nullptr;       // [npatch][n^2] T
  void* dutmp = nullptr;        // [npatch][n^2] T (ping-pong partner of du)
  // per coarser tile level k (1 .. ktile), and the LDS level ktile:
  std::vector<void*> ubar, rbar, flev, ulev, ulev2;
  // second level-1 ubar: the fused finest-level smoothing reads the
  // restricted iterate of its cycle from one and writes the next cycle's to
  // the other (one array would let a block read a neighbour's new values)
  void* ubar1b = nullptr;
  // per patch-setup tile (nbundle x tiles per patch): the ring ranges of both
  // grids that bracket the tile's region and its reference azimuth, which
  // depend on the plan's geometry only (kSetupMetaBytes each)
  char* setup_meta = nullptr;
  // the SHT potential and the fine map as the patch setup reads them in its
  // common case: every ring followed and preceded by pad_s (pad_f) copies of
  // its pixels from the other end, ring q starting at first_q + 2 q pad, so
  // that the two pixels around an azimuth sit side by side without a wrap
  double* spad = nullptr;       // [npix_s + 2 pad_s nring_s]
  void* kpad = nullptr;         // [npix_f + 2 pad_f nring_f], the fine map's type
  int pad_s = 0, pad_f = 0;
  int* status_dev = nullptr;
  double* mg_eps_dev = nullptr;   // [nbundle] epsilon ratio of the latest solve
  int* mg_cycles_dev = nullptr;   // [nbundle] V-cycles run
  int* mg_done_dev = nullptr;     // [nbundle] epsilon rule met
  // partial sky (clm_plan_set_domain): the multigrid, the evaluation and the
  // rays run over the domain's bundles only
  bool domain = false;            // false: the whole sky
  int64_t nactive = 0;            // bundles of the domain (nbundle without one)
  int* dom_map = nullptr;         // [nbundle] the domain's bundles, ascending
  int* dom_flag = nullptr;        // [nbundle] 1 inside the domain
  double* mg_eps_part = nullptr;  // epsilon rule: [nbundle][tiles][4] partial sums
  int* mg_active_dev = nullptr;   // epsilon rule: patches still above mg_eps
  int* mg_active_host = nullptr;  // pinned copy of mg_active_dev
  // adjoint workspace (desc.adjoint): u0 + du bar per patch with ghosts, and
  // per level the transposed V-cycle's u bar (two), f bar and a temporary
  double* adj_ubar = nullptr;
  std::vector<double*> adj_u, adj_v, adj_f, adj_w;
  double* adj_psi = nullptr;    // [npix_s] psi_SHT bar
  double* adj_psi_priv = nullptr;  // [adj_ncopy][npix_s] per-block copies of psi_SHT bar
  double* adj_rrows = nullptr;  // reciprocal row table, laid out like coef
  int adj_ncopy = 1;
  double* adj_ks = nullptr;     // [npix_s] kappa_SHT bar
  double* adj_alm = nullptr;    // [nalm] complex

  std::vector<Slot> slots;

  // the distances, curvature and plane of the latest ray update, for the
  // galaxy step of the shell the rays have just reached
  std::vector<double> ray_chi;
  double ray_K = 0.0;
  int ray_plane = -1;

  // per-stage timing (off unless enabled); a non-empty filter restricts it
  // to the stages named there
  bool timing = false;
  std::vector<std::string> timing_only;
  bool timed_stage(const char* name) const {
    if (timing_only.empty()) return true;
    for (const auto& t : timing_only)
      if (t == name) return true;
    return false;
  }
  std::vector<std::string> stage_names;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  int stage_id(const char* name);
  hipEvent_t take_event();

  ~Plan();
};

// Brackets one kernel launch with timing events when timing is enabled.
struct TimedLaunch {
  Plan* p;
  hipStream_t s;
  int stage = -1;
  hipEvent_t a = nullptr;
  TimedLaunch(Plan* p_, hipStream_t s_, const char* name) : p(p_), s(s_) {
    if (!p->timing || !p->timed_stage(name)) return;
    stage = p->stage_id(name);
    a = p->take_event();
    if (a) (void)hipEventRecord(a, s);
  }
  ~TimedLaunch() {
    if (!p->timing || !a) return;
    hipEvent_t b = p->take_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    p->recs.push_back({stage, a, b});
  }
};
#define CLM_TIMED(p, s, name) ::clm::TimedLaunch clm_timed_##__LINE__(p, s, name)

#define CLM_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      p->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return CLM_EHIP;                                                       \
    }                                                                        \
  } while (0)

#define CLM_HIP_P(plan, call)                                               \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      (plan)->err = std::string(#call) + ": " + hipGetErrorString(e_);       \
      return CLM_EHIP;                                                       \
    }                                                                        \
  } while (0)

#define CLM_LAUNCH_CHECK()                                                   \
  do {                                                                       \
    hipError_t e_ = hipGetLastError();                                       \
    if (e_ != hipSuccess) {                                                  \
      p->err = std::string("kernel launch: ") + hipGetErrorString(e_);       \
      return CLM_EHIP;                                                       \
    }                                                                        \
  } while (0)

inline clm_status fail(Plan* p, clm_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

// Dynamic LDS above 64 KiB needs an explicit opt-in per kernel.  A plan asks
// once per kernel and size, so later calls (and calls under stream capture)
// make no attribute call.
inline clm_status lds_opt_in(Plan* p, const void* fn, size_t bytes) {
  if (bytes <= 65536) return CLM_OK;
  for (const auto& e : p->lds_set)
    if (e.first == fn && e.second >= bytes) return CLM_OK;
  CLM_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  p->lds_set.emplace_back(fn, bytes);
  return CLM_OK;
}

// lambda_mm(theta) of the north rings (rt: ring table, H rings), mantissa
// and scale exponent [lmax+1][H] (sht.hip; launched at plan creation).
__global__ void k_lambda_mm(const double* rt, int H, int lmax, double* mant, int* scale);

// ---- stage launchers (each returns CLM_OK or an error recorded in p->err)
clm_status build_tables(Plan* p);                       // plan.hip
// psi_map = false: stop at psi_lm (the pure-SHT ray tracing, which needs
// only the derivative fields)
clm_status sht_solve(Plan* p, const void* kappa, int kappa_fp64, int slot,
                     hipStream_t s, bool psi_map = true);  // sht.hip
clm_status plane_mean(Plan* p, const void* kappa, int kappa_fp64,
                      hipStream_t s);                   // sht.hip: red[1023] = mean
clm_status ring_plan(Plan* p);                          // sht.hip
clm_status sht_solve_batch(Plan* p, const void* kappa, int kappa_fp64, int first_slot,
                           int nplanes, hipStream_t s, bool psi_map = true);  // sht.hip
clm_status sht_plane_fields(Plan* p, int slot, hipStream_t s);  // sht.hip: into p->deriv
clm_status sht_batch_fields(Plan* p, int k, hipStream_t s);     // sht.hip: into p->deriv
clm_status sht_adjoint(Plan* p, const double* psibar, double* alm, double* ksbar,
                       hipStream_t s);                   // sht.hip
clm_status shear_adjoint(Plan* p, const double* th, const double* ph, int64_t npts,
                         const double* gbar, const double* hbar,
                         hipStream_t s);                 // adjoint.hip
clm_status poisson_adjoint(Plan* p, double* dkappa, hipStream_t s);
clm_status adjoint_tables(Plan* p);                      // adjoint.hip
// One grid's share of a persistent matrix-core launch: plan, first slot and
// number of planes (the plan's Fb / Gb hold their ring sums).
struct MfmaGroup {
  Plan* p;
  int first_slot, P;
};
int mfma_ring_blocks(int H);                             // sht_mfma.hip
clm_status mfma_autotune(Plan* p);
clm_status mfma_analysis_multi(const MfmaGroup* gs, int ng, hipStream_t s);
clm_status mfma_synthesis_multi(const MfmaGroup* gs, int ng, hipStream_t s);
clm_status sht_solve_multi(Plan* const* ps, int n, const void* const* kappa,
                           const int32_t* kappa_fp64, const int32_t* nplanes,
                           hipStream_t s);                // sht.hip
clm_status mfma_tables(Plan* p, hipStream_t s);
clm_status mfma_analysis(Plan* p, int first_slot, int P, hipStream_t s);
clm_status mfma_synthesis(Plan* p, int first_slot, int P, hipStream_t s);
int mfma_deriv_planes();                                 // planes per derivative synthesis
clm_status mfma_deriv_synthesis(Plan* p, int first_slot, int P, hipStream_t s);
clm_status jacobian_fields(Plan* p, const clm_rays* r, double* out,
                           hipStream_t s);  // rays.hip: [4][npix_s] RING maps
clm_status sht_jacobian_spectra(Plan* p, const clm_rays* rays, double* alm, double* cl,
                                hipStream_t s);  // sht.hip
clm_status sht_pixel_derivs_batch(Plan* p, int first_slot, int nplanes, int order,
                                  int out_fp64, void* grad, void* hess,
                                  hipStream_t s);  // sht.hip
clm_status sht_pixel_derivs(Plan* p, int slot, int order, int out_fp64,
                            void* grad, void* hess, hipStream_t s);  // sht.hip
// kappa = nullptr with particles: the source is the particles' deposition
// on the patch cells
clm_status mg_solve(Plan* p, const void* kappa, int kappa_fp64, int slot,
                    hipStream_t s, const clm_particles* parts = nullptr);  // mg.hip
clm_status patch_deposit(Plan* p, const clm_particles* parts, hipStream_t s);  // deposit.hip
clm_status deposit_map(const clm_particles* parts, int64_t nside, double* map,
                       hipStream_t s);                  // deposit.hip: adds into a RING map
int64_t setup_tiles(const Plan* p);                     // mg.hip: patch-setup tiles
int setup_ring_pad(int nside);                          // mg.hip: pad_s / pad_f of a grid
clm_status setup_tables(Plan* p, hipStream_t s);        // mg.hip: fills setup_meta
clm_status mg_patch_potential(Plan* p, int slot, int64_t first, int64_t np,
                              double* out, hipStream_t s);  // mg.hip
clm_status eval_points(Plan* p, int slot, const double* th, const double* ph,
                       int64_t npts, int order, int out_fp64, void* grad,
                       void* hess, hipStream_t s);      // eval.hip
clm_status rays_init(Plan* p, const clm_rays* r, hipStream_t s);  // rays.hip
clm_status ray_update(Plan* p, int slot, const double* chi, int nchi, int m,
                      double K, const clm_rays* r, hipStream_t s);   // rays.hip
clm_status galaxies_shell(Plan* p, const double* chi, int nchi, int k, double K,
                          const clm_rays* r, const clm_galaxies* g,
                          hipStream_t s);               // rays.hip
clm_status galaxy_images(Plan* p, const double* chi, int nchi, int k, double K,
                         const clm_rays* r, const clm_galaxies* g, double radius,
                         double* th_img, double* ph_img, int* found,
                         hipStream_t s);                // rays.hip

inline int ilog2(int64_t v) {
  int k = 0;
  while ((int64_t(1) << (k + 1)) <= v) ++k;
  return k;
}

}  // namespace clm

struct clm_plan_s : clm::Plan {};
