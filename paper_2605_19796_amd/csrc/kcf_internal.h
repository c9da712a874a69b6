// Internal declarations shared by the HIP kernels and the C-ABI layer of libkcf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kcf {

constexpr int kMaxR = 12;                 // largest stencil radius on the GPU
constexpr int kMaxTaps = 2 * kMaxR + 1;
constexpr int kNStat = 40;                // FP64 sums per filter width

// Slots of the per-width FP64 sums.
enum StatSlot {
  S_N = 0, S_RHO = 1, S_KE = 2, S_PI = 3, S_PIGM = 4, S_PI2 = 5, S_PIGM2 = 6, S_PIPIGM = 7,
  S_TAU = 8, S_TGM = 14, S_TAU2 = 20, S_TGM2 = 26, S_TAUTGM = 32, S_NONFINITE = 38,
  S_PISM = 39
};

struct WidthArgs {          // outputs, closure constants and statistics of one width
  float* rho_bar;
  float* ut;
  float* tau;
  float* grad;
  float* tau_gm;
  float* tau_smag;
  float* k_sgs;
  float* nu_t;
  float* omega_t;
  float* q_crit;
  float gm_coef;          // C2 of the gradient model
  float smag_coef;        // (C_s Delta)^2
  float cnu_delta;        // C_nu Delta
  float inv_theta;        // 1 / theta
  float nu_mol;           // molecular viscosity of the clip
  float half_dt;          // dt / 2 of the shifted rate
  int gm_form;            // 0: G G^T, 1: G^T G
  int ksgs_rho_ref;       // 0: rho_bar, 1: 1
  int exact_stats;        // box kernels with FP64 sums: exact FP64 statistics contributions
  double* partials;       // [records][kNStat] FP64 partial sums (one record per wave), or NULL
};

struct FilterArgs {
  const float* rho;
  const float* u;
  int nx, ny, nz;
  int64_t ntot;
  float inv2h;
  int ntx, nty, ntiles;   // output tiles in x, y and their product
  int nzc, zlen;          // z chunks per column and their length
  int tiles_per_xcd;      // tiles of one XCD's contiguous band
  int strip_w;            // tile numbering: strips of strip_w tiles, or plain rows when 0
  WidthArgs wa;
};

struct ClosureArgs {        // standalone gradient/closure pass from stored fields
  const float* rho_bar;
  const float* ut;
  const float* tau;
  int nx, ny, nz;
  int64_t ntot;
  float inv2h;
  WidthArgs wa;
};

struct TapArgs {           // general-tap filter (kcf_taps.hip)
  const float* rho;
  const float* u;
  int nx, ny, nz;
  int64_t ntot;
  int ntx, nty;            // tiles of the x-y pass (taps_tile_x, taps_tile_y)
  int zb, nbuf;            // slab buffer: planes zb .. zb + nbuf - 1 (mod nz)
  int zo0, zo1;            // output planes of the z pass
  void* xy;                // slab buffer [10][nbuf][ny][nx], float or double
  float w[kMaxTaps];       // taps w_{-R..R}
  double wd[kMaxTaps];
  float* rho_bar;          // outputs, each may be NULL
  float* ut;
  float* tau;
};

struct InputStatArgs {
  const float* rho;
  const float* u;
  int nx, ny, nz;
  int64_t ntot;
  double inv60h;
  double* partials;       // [records][4]
};

// launchers (kcf_filter.hip)
int64_t grad_closure_records(const ClosureArgs& a);  // per-wave partial records
hipError_t launch_grad_closure(const ClosureArgs& a, hipStream_t s);
int64_t input_stats_records(const InputStatArgs& a);  // per-wave partial records
hipError_t launch_input_stats(const InputStatArgs& a, hipStream_t s);
// Sums of nparts records of nstat (<= kNStat) doubles into out; scratch holds
// kRedBlocks * nstat doubles of chunk totals.
constexpr int kRedBlocks = 256;
hipError_t launch_reduce(const double* partials, int nparts, int nstat, double* out,
                         double* scratch, hipStream_t s);
hipError_t launch_reduce_check(const float* a, const float* b, int64_t n, double* partials,
                               int nblocks, hipStream_t s);
hipError_t launch_stream_probe(const float* in, int nin, float* out, int nout, int64_t n,
                               hipStream_t s);

// general-tap kernels (kcf_taps.hip)
constexpr size_t kTapBufferCap = (size_t)8 << 30;  // bytes of x-y filtered planes held at once
constexpr size_t kTapBufferMax = (size_t)48 << 30;  // the same for filter_favre, memory permitting
int taps_tile_x(int fp64);
int taps_tile_y();
int taps_z_planes(int fp64);
hipError_t launch_taps(const TapArgs& a, int R, int fp64, hipStream_t s);

// Filtered monomials of rho u (and rho theta): the SGS carrier of the D3Q27 lattice and the
// third-order SGS moment (kcf_monomials.hip)
constexpr int kSetCarrier = 0, kSetMoment3 = 1, kSetKcMp = 2;
constexpr int kCStat = 9;   // FP64 sums of the carrier
enum CarrierSlot { C_N = 0, C_F2 = 1, C_ERR2 = 2, C_HERM = 3, C_NONFINITE = 8 };
constexpr int kM3Stat = 23;  // FP64 sums of the third-order moment
enum Moment3Slot { M3_N = 0, M3_SUM = 1, M3_SQ = 11, M3_THETA = 21, M3_NONFINITE = 22 };
constexpr int kKcStat = 40;  // FP64 sums of the KC-MP evaluation
enum KcSlot {
  KC_N = 0, KC_M = 1, KC_T = 7, KC_M2 = 13, KC_T2 = 19, KC_MT = 25, KC_ERR2 = 31, KC_TAU2 = 32,
  KC_K = 33, KC_KE = 34, KC_OM = 35, KC_OME = 36, KC_CLIP = 37, KC_CLIPE = 38, KC_NONFINITE = 39
};

struct MonoArgs {
  const float* rho;
  const float* u;
  const float* theta;      // temperature (third-order set only), or NULL
  int nx, ny, nz;
  int64_t ntot;
  int ntx, nty, ntiles;    // output tiles of the x-y pass
  int zs, nzs;             // z slab: planes zs .. zs + nzs - 1
  int nq;                  // quantities kept in the slab buffer
  void* zbuf;              // z-filtered quantities [nzs][nq][ny][nx], float or double
  float w[kMaxTaps];       // taps w_{-R..R}
  double wd[kMaxTaps];
  float* f_sgs;            // carrier: [27][N], or NULL
  float* f_h2;             // carrier: [27][N], or NULL
  float* m3;               // third-order moment: [10][N], or NULL
  float* theta_t;          // Favre temperature: [N], or NULL
  // KC-MP evaluation
  const float* ext;        // stored filtered fields: rho_bar [N], tau [6N], G [9N]
  float* m_sgs;            // [6][N], or NULL
  float* m_ce;             // [6][N], or NULL
  float* k_sgs;            // [N], or NULL
  float* nu_t_eff;         // [N], or NULL
  float* omega_sgs;        // [N], or NULL
  float inv2h;             // 1 / (2 h)
  float kc_coef;           // 2 theta tau_hat
  float nu;                // molecular viscosity
  float inv_theta;         // 1 / theta
  float half_dt;           // dt / 2
  float cnu_delta;         // C_nu Delta
  int rho_ref_one;         // k_sgs with rho_0 = 1 (1) or rho_bar (0)
  double* partials;        // [mono_records][statistics] records of the slab, or NULL
};
int mono_tile_x(int R);             // the x-y tile for radius R
int mono_tile_y(int R);
int mono_z_planes(int fp64);        // planes per thread of the z pass
int64_t mono_xy_records(const MonoArgs& a);  // x-y workgroups of one slab
int mono_records_per_block(int set);         // statistics records per x-y workgroup
hipError_t launch_mono_z(const MonoArgs& a, int set, int R, int fp64, hipStream_t s);
hipError_t launch_mono_xy(const MonoArgs& a, int set, int R, int fp64, hipStream_t s);

// D3Q27 lattice-Boltzmann step (kcf_lbm.hip)
constexpr int kLbmBgk = 0, kLbmKcrb = 1, kLbmKcrbRaw = 2, kLbmKcmp = 3, kLbmKcrr = 4;
constexpr int kLbmStat = 8;  // FP64 sums: rho, rho u (3), rho |u|^2 / 2, omega_sgs, clipped, k_sgs
struct LbmArgs {
  const float* fin;        // populations [27][N] at time t
  float* fout;             // populations [27][N] at time t + 1 (distinct from fin)
  int nx, ny, nz;
  int64_t ntot;
  int ntx, nty, ntiles;    // tiles of colliding columns
  int nzc, zlen;           // z chunks and their length
  int items_per_xcd;       // (z-chunk, tile) items of one XCD's band
  float omega;             // shifted molecular rate (nu / theta + 1/2)^-1
  float tau_hat;           // 1 / omega
  float nu;                // molecular viscosity (lattice units)
  float c_nu;              // closure constant C_nu (Delta = 1)
  int model;               // kLbm*
  double* partials;        // [records][kLbmStat] or NULL
};
int lbm_tile_x();
int lbm_tile_y();
int lbm_records_per_block();
hipError_t launch_lbm_step(const LbmArgs& a, int nblocks, hipStream_t s);
hipError_t launch_lbm_equilibrium(const float* rho, const float* u, float* f, int64_t n,
                                  hipStream_t s);

// box kernels (kcf_box.hip)
struct BoxGeom {
  int tile_x, tile_y;  // output columns of a tile
  int threads;         // threads per workgroup
  int stat_waves;      // per-wave statistics records per (tile, z-chunk) item
  int blocks_per_cu;   // resident workgroups per CU
  int strip_w;         // tile numbering (FilterArgs::strip_w)
};
bool box_supported(int R, int fp64);
BoxGeom box_geometry(int R, int fp64);
hipError_t launch_box(const FilterArgs& a, int R, int fp64, int nblocks, hipStream_t s);

}  // namespace kcf
