// C-ABI layer of libkcf: argument checks, filter taps, launch geometry, FP64 statistics.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kcf.h"
#include "kcf_internal.h"

using namespace kcf;

struct kcf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double* d_part = nullptr;   // FP64 partial sums of the kernels
  size_t part_cap = 0;        // doubles
  double* d_sums = nullptr;   // reduced sums (device)
  double* d_red = nullptr;    // chunk totals of the reductions (kRedBlocks x kNStat)
  double* h_sums = nullptr;   // reduced sums (pinned host)
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop) of timed launches
  size_t ev_used = 0;
  void* d_xy = nullptr;        // slab buffer of the general-tap filter
  size_t xy_cap = 0;           // bytes
  float* d_fld = nullptr;      // Favre fields the caller did not ask for (10 N floats)
  size_t fld_cap = 0;          // bytes
  float* d_kc = nullptr;       // rho_bar, tau and G for the KC-MP evaluation (16 N floats)
  size_t kc_cap = 0;           // bytes
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  // every KCF_ENOMEM follows a failed device allocation, whose error HIP would otherwise
  // report again at the next launch check of this thread
  if (code == KCF_ENOMEM) (void)hipGetLastError();
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(KCF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define KCF_HIP(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr int kSumCap = 4 * kNStat;

int ensure_partials(kcf_ctx* c, size_t n) {
  if (n <= c->part_cap) return KCF_OK;
  if (c->d_part) {
    hipStreamSynchronize(c->stream);
    hipFree(c->d_part);
    c->d_part = nullptr;
    c->part_cap = 0;
  }
  if (hipMalloc(&c->d_part, n * sizeof(double)) != hipSuccess)
    return fail(KCF_ENOMEM, "cannot allocate FP64 partial sums");
  c->part_cap = n;
  return KCF_OK;
}

// Device buffers that only grow; the stream is drained before one is replaced.
template <typename P>
int ensure_buffer(kcf_ctx* c, P*& ptr, size_t& cap, size_t bytes, const char* what) {
  if (bytes <= cap) return KCF_OK;
  if (ptr) {
    hipStreamSynchronize(c->stream);
    hipFree(ptr);
    ptr = nullptr;
    cap = 0;
  }
  if (hipMalloc((void**)&ptr, bytes) != hipSuccess) return fail(KCF_ENOMEM, what);
  cap = bytes;
  return KCF_OK;
}

int check_grid(const kcf_grid* g) {
  if (!g) return fail(KCF_EINVAL, "grid is NULL");
  if (g->nx < 3 || g->ny < 3 || g->nz < 3) return fail(KCF_EINVAL, "grid needs n >= 3 per direction");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(KCF_EINVAL, "grid spacing must be > 0");
  if ((int64_t)g->nx * g->ny > (int64_t)1 << 30) return fail(KCF_EUNSUPPORTED, "plane too large");
  return KCF_OK;
}

struct Taps {
  double wd[2 * 64 + 1];
  int R;
  double m2;
};

// Taps in double: box = trapezoidal top-hat of width n h, gauss = exp(-6 m^2/n^2) on
// |m| <= ceil(1.5 n) normalised to unit sum; M2 = sum w_m (m h)^2.
int compute_taps(int kind, int n, double h, Taps& t) {
  if (!(h > 0.0)) return fail(KCF_EINVAL, "grid spacing must be > 0");
  int R;
  if (kind == KCF_BOX) {
    if (n < 2 || (n & 1)) return fail(KCF_EINVAL, "box filter needs an even width >= 2 (in h)");
    R = n / 2;
    if (2 * R + 1 > 129) return fail(KCF_EUNSUPPORTED, "filter too wide");
    for (int m = -R; m <= R; ++m) t.wd[m + R] = (m == -R || m == R) ? 0.5 / n : 1.0 / n;
  } else if (kind == KCF_GAUSS) {
    if (n < 1) return fail(KCF_EINVAL, "gaussian filter needs a width >= 1 (in h)");
    R = (int)std::ceil(1.5 * n);
    if (2 * R + 1 > 129) return fail(KCF_EUNSUPPORTED, "filter too wide");
    double s = 0;
    for (int m = -R; m <= R; ++m) {
      t.wd[m + R] = std::exp(-6.0 * (double)m * m / ((double)n * n));
      s += t.wd[m + R];
    }
    for (int m = -R; m <= R; ++m) t.wd[m + R] /= s;
  } else {
    return fail(KCF_EINVAL, "unknown filter kind");
  }
  t.R = R;
  double mm = 0;
  for (int m = -R; m <= R; ++m) mm += t.wd[m + R] * (m * h) * (m * h);
  t.m2 = mm;
  return KCF_OK;
}

void set_closure(WidthArgs& W, const kcf_closure_params* cp, double delta, double m2) {
  kcf_closure_params d{0.11, 0.02, 1.0, 0.0, 0.0, 0, 0, 0};
  if (cp) d = *cp;
  W.gm_coef = (float)(d.m2_mode == 1 ? delta * delta / 12.0 : m2);
  W.smag_coef = (float)((d.c_s * delta) * (d.c_s * delta));
  W.cnu_delta = (float)(d.c_nu * delta);
  W.inv_theta = (float)(1.0 / d.theta);
  W.nu_mol = (float)d.nu_mol;
  W.half_dt = (float)(0.5 * d.dt);
  W.gm_form = d.gm_form;
  W.ksgs_rho_ref = d.ksgs_rho_ref;
}

int check_closure(const kcf_closure_params* cp) {
  if (!cp) return KCF_OK;
  if (!(cp->theta > 0)) return fail(KCF_EINVAL, "theta must be > 0");
  if (cp->nu_mol < 0 || cp->dt < 0 || cp->c_s < 0 || cp->c_nu < 0)
    return fail(KCF_EINVAL, "closure constants must be >= 0");
  if ((cp->gm_form != 0 && cp->gm_form != 1) || (cp->m2_mode != 0 && cp->m2_mode != 1) ||
      (cp->ksgs_rho_ref != 0 && cp->ksgs_rho_ref != 1))
    return fail(KCF_EINVAL, "closure flags must be 0 or 1");
  return KCF_OK;
}

void set_outputs(WidthArgs& W, const kcf_outputs* o) {
  W.rho_bar = o->rho_bar;
  W.ut = o->ut;
  W.tau = o->tau;
  W.grad = o->grad;
  W.tau_gm = o->tau_gm;
  W.tau_smag = o->tau_smag;
  W.k_sgs = o->k_sgs;
  W.nu_t = o->nu_t;
  W.omega_t = o->omega_t;
  W.q_crit = o->q_crit;
}

// Statistics of one width from its 40 FP64 sums.
void derive_stats(const double* raw, double delta, double m2, kcf_width_stats* s) {
  std::memset(s, 0, sizeof(*s));
  std::memcpy(s->raw, raw, sizeof(double) * kNStat);
  s->delta = delta;
  s->m2 = m2;
  const double n = raw[S_N];
  s->n_points = (int64_t)llround(n);
  s->n_nonfinite = (int64_t)llround(raw[S_NONFINITE]);
  if (n <= 0) return;
  s->mean_rho_bar = raw[S_RHO] / n;
  s->ke_resolved = raw[S_KE] / n;
  s->pi = raw[S_PI] / n;
  s->pi_gm = raw[S_PIGM] / n;
  s->pi_smag = raw[S_PISM] / n;
  auto corr = [n](double sa, double sb, double saa, double sbb, double sab) {
    const double cov = sab - sa * sb / n;
    const double va = saa - sa * sa / n;
    const double vb = sbb - sb * sb / n;
    return (va > 0 && vb > 0) ? cov / std::sqrt(va * vb) : NAN;
  };
  for (int c = 0; c < 6; ++c) {
    s->mean_tau[c] = raw[S_TAU + c] / n;
    s->corr_tau_gm[c] = corr(raw[S_TAU + c], raw[S_TGM + c], raw[S_TAU2 + c], raw[S_TGM2 + c],
                             raw[S_TAUTGM + c]);
  }
  s->corr_pi = corr(raw[S_PI], raw[S_PIGM], raw[S_PI2], raw[S_PIGM2], raw[S_PIPIGM]);
}

int reduce_to_host(kcf_ctx* c, int nparts, int nstat, int slot) {
  hipError_t e = launch_reduce(c->d_part, nparts, nstat, c->d_sums + slot * kNStat, c->d_red,
                               c->stream);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  return KCF_OK;
}

int timed_begin(kcf_ctx* c) {
  if (!c->timing) return KCF_OK;
  if (c->ev_used + 2 > c->ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      KCF_HIP(hipEventCreate(&e), "hipEventCreate");
      c->ev.push_back(e);
    }
  }
  KCF_HIP(hipEventRecord(c->ev[c->ev_used], c->stream), "hipEventRecord");
  return KCF_OK;
}

int timed_end(kcf_ctx* c) {
  if (!c->timing) return KCF_OK;
  KCF_HIP(hipEventRecord(c->ev[c->ev_used + 1], c->stream), "hipEventRecord");
  c->ev_used += 2;
  return KCF_OK;
}

// Number of z chunks: enough workgroups to fill the chip, balanced against the 2R+2 planes
// each chunk spends filling its window.
int choose_zchunks(int64_t items_per_chunk, int nz, int R, int blocks_per_cu) {
  const double cus = 256.0 * blocks_per_cu;
  double best = -1;
  int best_n = 1;
  for (int n = 1; n <= 16; ++n) {
    const int zlen = (nz + n - 1) / n;
    if (zlen < 4) break;
    const double blocks = (double)items_per_chunk * n;
    const double rounds = std::ceil(blocks / cus);
    const double fill = blocks / (rounds * cus);
    const double eff = fill * zlen / (double)(zlen + 2 * R + 2);
    if (eff > best + 1e-9) {
      best = eff;
      best_n = n;
    }
  }
  return best_n;
}

// The two passes of the monomial filters (kcf_monomials.hip) over z slabs whose filtered
// quantities fit the context buffer; FP64 statistics records reduced into c->d_sums when
// `stats` is set.
int run_monomials(kcf_ctx* c, const kcf_grid* grid, const kcf_filter* filter, int set, int nq,
                  int nstat, MonoArgs& A, bool stats) {
  Taps taps;
  int rc = compute_taps(filter->kind, filter->delta_over_h, grid->h, taps);
  if (rc) return rc;
  const int R = taps.R;
  if (R > kMaxR) return fail(KCF_EUNSUPPORTED, "filter radius above 12 cells");
  if (2 * R + 1 > std::min(grid->nx, std::min(grid->ny, grid->nz)))
    return fail(KCF_EUNSUPPORTED, "filter support 2R+1 exceeds the grid");
  const int p = filter->precision;
  if (p < 0 || p > 2) return fail(KCF_EINVAL, "precision must be 0 (auto), 1 (fp32) or 2 (fp64)");
  const int fp64 = p == 2 || (p == 0 && filter->delta_over_h <= 4);
  if (grid->ny > 65535) return fail(KCF_EUNSUPPORTED, "ny above 65535");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  A.nx = grid->nx;
  A.ny = grid->ny;
  A.nz = grid->nz;
  A.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  A.ntx = (grid->nx + mono_tile_x(R) - 1) / mono_tile_x(R);
  A.nty = (grid->ny + mono_tile_y(R) - 1) / mono_tile_y(R);
  A.ntiles = A.ntx * A.nty;
  A.nq = nq;
  for (int m = 0; m < 2 * R + 1; ++m) {
    A.wd[m] = taps.wd[m];
    A.w[m] = (float)taps.wd[m];
  }
  // z slabs whose filtered quantities fit the buffer cap (the whole field if they can)
  const int64_t plane = (int64_t)grid->nx * grid->ny;
  const size_t per_plane = (size_t)nq * plane * (fp64 ? sizeof(double) : sizeof(float));
  const int zt = mono_z_planes(fp64);
  int slab = grid->nz;
  if (per_plane * (size_t)grid->nz > kTapBufferCap)
    slab = std::max(zt, (int)(kTapBufferCap / per_plane) / zt * zt);
  if ((rc = ensure_buffer(c, c->d_xy, c->xy_cap, per_plane * (size_t)slab,
                          "cannot allocate the monomial slab buffer")))
    return rc;
  A.zbuf = c->d_xy;
  int64_t nrec = 0;  // statistics records of all slabs
  const int rpb = mono_records_per_block(set);
  for (int zs = 0; zs < grid->nz; zs += slab) {
    A.nzs = std::min(slab, grid->nz - zs);
    nrec += mono_xy_records(A) * rpb;
  }
  if (stats) {
    if (nrec > INT32_MAX) return fail(KCF_EUNSUPPORTED, "grid too large for statistics");
    if ((rc = ensure_partials(c, (size_t)nrec * nstat))) return rc;
  }
  int64_t rec0 = 0;
  for (int zs = 0; zs < grid->nz; zs += slab) {
    A.zs = zs;
    A.nzs = std::min(slab, grid->nz - zs);
    A.partials = stats ? c->d_part + (size_t)rec0 * nstat : nullptr;
    rec0 += mono_xy_records(A) * rpb;
    if ((rc = timed_begin(c))) return rc;
    hipError_t e = launch_mono_z(A, set, R, fp64, c->stream);
    if (e != hipSuccess) return hip_fail(e, "z pass launch");
    if ((rc = timed_end(c))) return rc;
    if ((rc = timed_begin(c))) return rc;
    e = launch_mono_xy(A, set, R, fp64, c->stream);
    if (e != hipSuccess) return hip_fail(e, "x-y pass launch");
    if ((rc = timed_end(c))) return rc;
  }
  if (stats) {
    hipError_t e = launch_reduce(c->d_part, (int)nrec, nstat, c->d_sums, c->d_red, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * nstat, hipMemcpyDeviceToHost,
                           c->stream), "stats copy");
    KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  return KCF_OK;
}

// Taps, radius and precision of each width of a filter_favre call, after the argument checks
// both filter_favre entry points share.
struct WidthPlan {
  Taps taps[4];
  int radii[4];
  int fp64[4];
  int use_box[4];  // the sliding-sum box kernel applies
};

int plan_widths(const kcf_grid* grid, const kcf_filter* filters, int nf,
                const kcf_closure_params* cp, WidthPlan& P) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!filters) return fail(KCF_EINVAL, "NULL argument");
  if (nf < 1 || nf > 4) return fail(KCF_EINVAL, "n_filters must be 1..4");
  if ((rc = check_closure(cp))) return rc;
  for (int f = 0; f < nf; ++f) {
    if ((rc = compute_taps(filters[f].kind, filters[f].delta_over_h, grid->h, P.taps[f]))) return rc;
    P.radii[f] = P.taps[f].R;
    if (P.taps[f].R > kMaxR) return fail(KCF_EUNSUPPORTED, "filter radius above 12 cells");
    const int nmin = std::min(grid->nx, std::min(grid->ny, grid->nz));
    if (2 * P.taps[f].R + 1 > nmin)
      return fail(KCF_EUNSUPPORTED, "filter support 2R+1 exceeds the grid");
    const int p = filters[f].precision;
    if (p < 0 || p > 2) return fail(KCF_EINVAL, "precision must be 0 (auto), 1 (fp32) or 2 (fp64)");
    P.fp64[f] = p == 2 || (p == 0 && filters[f].delta_over_h <= 4);
    P.use_box[f] = filters[f].kind == KCF_BOX && box_supported(P.radii[f], P.fp64[f]);
  }
  if (grid->ny > 65535) return fail(KCF_EUNSUPPORTED, "ny above 65535");
  return KCF_OK;
}

// Launch geometry of the box kernel of one width.
void box_args_for(FilterArgs& A, const kcf_grid* grid, const float* rho, const float* u, int R,
                  int fp64) {
  const BoxGeom bg = box_geometry(R, fp64);
  std::memset(&A, 0, sizeof(A));
  A.rho = rho;
  A.u = u;
  A.nx = grid->nx;
  A.ny = grid->ny;
  A.nz = grid->nz;
  A.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  A.inv2h = (float)(1.0 / (2.0 * grid->h));
  A.ntx = (grid->nx + bg.tile_x - 1) / bg.tile_x;
  A.nty = (grid->ny + bg.tile_y - 1) / bg.tile_y;
  A.ntiles = A.ntx * A.nty;
  A.nzc = choose_zchunks(A.ntiles, grid->nz, R, bg.blocks_per_cu);
  A.zlen = (grid->nz + A.nzc - 1) / A.nzc;
  A.nzc = (grid->nz + A.zlen - 1) / A.zlen;
  A.tiles_per_xcd = (A.ntiles * A.nzc + 7) / 8;
  A.strip_w = bg.strip_w;
}

// FP64 statistics records the box kernel of a width writes (one per wave).
int64_t box_records(const FilterArgs& A, int R, int fp64) {
  return (int64_t)A.ntiles * A.nzc * box_geometry(R, fp64).stat_waves;
}

}  // namespace

namespace kcf {
int api_fail(int code, const char* msg) { return fail(code, msg); }
hipStream_t ctx_stream(kcf_ctx* c) { return c->stream; }
int ctx_device(kcf_ctx* c) { return c->device; }
}  // namespace kcf

// ---- scratch of the no-allocation entry point
// Device memory of kcf_filter_favre_noalloc: the reduced sums of up to four widths, the chunk
// totals of the two-pass reduction and the per-wave FP64 records of one width (the widths are
// reduced one after the other, so they reuse the record area). Each GPU the library runs on
// holds its own copy for the life of the process.
constexpr size_t kNoAllocSums = 4 * kNStat;
constexpr size_t kNoAllocRed = (size_t)kRedBlocks * kNStat;
constexpr size_t kNoAllocDoubles = (size_t)2 << 20;  // 16 MiB
constexpr size_t kNoAllocRecords = (kNoAllocDoubles - kNoAllocSums - kNoAllocRed) / kNStat;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current when called), looked up once per device.
// Host code must use this address: the name itself is a host-side stand-in.
int scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(KCF_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return KCF_OK;
}
}  // namespace

extern "C" {

int kcf_version(void) { return 100; }

const char* kcf_last_error(void) { return g_err.c_str(); }

int kcf_ctx_create(kcf_ctx** out, int device, void* stream) {
  if (!out) return fail(KCF_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  KCF_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(KCF_EINVAL, "no such device");
  KCF_HIP(hipSetDevice(device), "hipSetDevice");
  kcf_ctx* c = new kcf_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipMalloc(&c->d_sums, kSumCap * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_red, (size_t)kRedBlocks * kNStat * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&c->h_sums, kSumCap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    kcf_ctx_destroy(c);
    return fail(KCF_ENOMEM, "cannot allocate statistics buffers");
  }
  *out = c;
  return KCF_OK;
}

int kcf_ctx_set_stream(kcf_ctx* c, void* stream) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  c->stream = (hipStream_t)stream;
  return KCF_OK;
}

void kcf_ctx_destroy(kcf_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  if (c->d_part) hipFree(c->d_part);
  if (c->d_xy) hipFree(c->d_xy);
  if (c->d_fld) hipFree(c->d_fld);
  if (c->d_kc) hipFree(c->d_kc);
  if (c->d_sums) hipFree(c->d_sums);
  if (c->d_red) hipFree(c->d_red);
  if (c->h_sums) hipHostFree(c->h_sums);
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  delete c;
}

int kcf_ctx_enable_timing(kcf_ctx* c, int on) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  c->timing = on != 0;
  c->ev_used = 0;
  return KCF_OK;
}

int kcf_ctx_kernel_times(kcf_ctx* c, float* ms, int cap, int* launches) {
  if (!c || !ms || !launches) return fail(KCF_EINVAL, "NULL argument");
  const int n = (int)(c->ev_used / 2);
  if (n > cap) return fail(KCF_EINVAL, "ms holds fewer entries than timed launches");
  KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (int i = 0; i < n; ++i)
    KCF_HIP(hipEventElapsedTime(&ms[i], c->ev[2 * i], c->ev[2 * i + 1]), "hipEventElapsedTime");
  *launches = n;
  c->ev_used = 0;
  return KCF_OK;
}

int kcf_ctx_kernel_ms(kcf_ctx* c, double* ms, int* launches) {
  if (!c || !ms) return fail(KCF_EINVAL, "NULL argument");
  KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  double t = 0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float m = 0;
    KCF_HIP(hipEventElapsedTime(&m, c->ev[i], c->ev[i + 1]), "hipEventElapsedTime");
    t += m;
  }
  *ms = t;
  if (launches) *launches = (int)(c->ev_used / 2);
  c->ev_used = 0;
  return KCF_OK;
}

int kcf_filter_taps(int kind, int n, double h, float* w, int cap, int* radius, double* m2) {
  if (!w || !radius) return fail(KCF_EINVAL, "NULL argument");
  Taps t;
  int rc = compute_taps(kind, n, h, t);
  if (rc) return rc;
  *radius = t.R;
  if (2 * t.R + 1 > cap) return fail(KCF_EINVAL, "tap buffer too small");
  for (int m = 0; m < 2 * t.R + 1; ++m) w[m] = (float)t.wd[m];
  if (m2) *m2 = t.m2;
  return KCF_OK;
}

int kcf_filter_favre(kcf_ctx* c, const kcf_grid* grid, const kcf_filter* filters, int nf,
                     const float* rho, const float* u, const kcf_outputs* outs,
                     const kcf_closure_params* cp, kcf_width_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  WidthPlan P;
  int rc = plan_widths(grid, filters, nf, cp, P);
  if (rc) return rc;
  if (!outs || !rho || !u) return fail(KCF_EINVAL, "NULL argument");
  const Taps* taps = P.taps;
  const int* radii = P.radii;
  const int* fp64 = P.fp64;
  const int* use_box = P.use_box;
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  // kernel per width: the sliding-sum box kernel where it applies, the general-tap filter
  // followed by the gradient/closure pass otherwise
  const int64_t ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  const int64_t plane = (int64_t)grid->nx * grid->ny;
  auto box_args = [&](FilterArgs& A, int f) { box_args_for(A, grid, rho, u, radii[f], fp64[f]); };
  ClosureArgs CG;  // geometry of the gradient/closure pass (same for every width)
  std::memset(&CG, 0, sizeof(CG));
  CG.nx = grid->nx;
  CG.ny = grid->ny;
  CG.nz = grid->nz;
  CG.ntot = ntot;
  CG.inv2h = (float)(1.0 / (2.0 * grid->h));
  // partial sums: [width][records][kNStat]
  size_t part_off[4];
  int nparts[4];
  {
    size_t off = 0;
    for (int f = 0; f < nf; ++f) {
      if (use_box[f]) {
        FilterArgs G;
        box_args(G, f);
        nparts[f] = (int)box_records(G, radii[f], fp64[f]);
      } else {
        nparts[f] = (int)grad_closure_records(CG);
      }
      part_off[f] = off;
      off += (size_t)nparts[f] * kNStat;
    }
    if (stats && (rc = ensure_partials(c, off))) return rc;
  }
  auto fill_width = [&](WidthArgs& W, int f) {
    std::memset(&W, 0, sizeof(W));
    set_outputs(W, &outs[f]);
    set_closure(W, cp, filters[f].delta_over_h * grid->h, taps[f].m2);
    W.partials = stats ? c->d_part + part_off[f] : nullptr;
    W.exact_stats = filters[f].precision == 2;
  };
  for (int f = 0; f < nf; ++f) {
    if (use_box[f]) {
      FilterArgs A;
      box_args(A, f);
      fill_width(A.wa, f);
      if ((rc = timed_begin(c))) return rc;
      hipError_t e = launch_box(A, radii[f], fp64[f], 8 * A.tiles_per_xcd, c->stream);
      if (e != hipSuccess) return hip_fail(e, "box filter launch");
      if ((rc = timed_end(c))) return rc;
      continue;
    }
    // general taps: x-y pass into a z-slab buffer, z pass with Favre division, then the
    // gradient/closure pass on the stored fields when anything needs the gradient
    WidthArgs W;
    fill_width(W, f);
    const bool grad_pass = stats || W.grad || W.tau_gm || W.tau_smag || W.k_sgs || W.nu_t ||
                           W.omega_t || W.q_crit;
    float* fb = W.rho_bar;
    float* fu = W.ut;
    float* ft = W.tau;
    if (grad_pass && (!fb || !fu || !ft)) {
      if ((rc = ensure_buffer(c, c->d_fld, c->fld_cap, sizeof(float) * 10 * (size_t)ntot,
                              "cannot allocate Favre field scratch")))
        return rc;
      if (!fb) fb = c->d_fld;
      if (!fu) fu = c->d_fld + ntot;
      if (!ft) ft = c->d_fld + 4 * ntot;
    }
    TapArgs T;
    std::memset(&T, 0, sizeof(T));
    T.rho = rho;
    T.u = u;
    T.nx = grid->nx;
    T.ny = grid->ny;
    T.nz = grid->nz;
    T.ntot = ntot;
    T.ntx = (grid->nx + taps_tile_x(fp64[f]) - 1) / taps_tile_x(fp64[f]);
    T.nty = (grid->ny + taps_tile_y() - 1) / taps_tile_y();
    const int R = radii[f];
    for (int m = 0; m < 2 * R + 1; ++m) {
      T.wd[m] = taps[f].wd[m];
      T.w[m] = (float)taps[f].wd[m];
    }
    T.rho_bar = fb;
    T.ut = fu;
    T.tau = ft;
    // slab of planes whose x-y filtered products fit the buffer cap (the whole field if it can)
    const size_t esize = fp64[f] ? sizeof(double) : sizeof(float);
    const size_t per_plane = 10 * (size_t)plane * esize;
    const int zt = taps_z_planes(fp64[f]);
    // buffer cap: 8 GiB, raised up to 48 GiB while that leaves half of the free device memory
    // (with what the context's buffer already holds) to the caller; the slab count does not
    // change any output, only how many halo planes the x-y pass filters twice
    size_t cap = kTapBufferCap;
    {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess)
        cap = std::max(cap, std::min(kTapBufferMax, (fr + c->xy_cap) / 2));
    }
    int slab = grid->nz;
    if (per_plane * (size_t)grid->nz > cap) {
      slab = (int)(cap / per_plane) - 2 * R;
      slab = std::max(zt, slab / zt * zt);
      if (slab + 2 * R >= grid->nz) slab = grid->nz;
    }
    const int nbuf_max = slab == grid->nz ? grid->nz : slab + 2 * R;
    if ((rc = ensure_buffer(c, c->d_xy, c->xy_cap, per_plane * (size_t)nbuf_max,
                            "cannot allocate the filter slab buffer")))
      return rc;
    T.xy = c->d_xy;
    if ((rc = timed_begin(c))) return rc;
    for (int z0 = 0; z0 < grid->nz; z0 += slab) {
      const int z1 = std::min(z0 + slab, grid->nz);
      T.zo0 = z0;
      T.zo1 = z1;
      if (slab == grid->nz) {
        T.zb = 0;
        T.nbuf = grid->nz;
      } else {
        T.zb = z0 - R;
        T.nbuf = (z1 - z0) + 2 * R;
      }
      hipError_t e = launch_taps(T, R, fp64[f], c->stream);
      if (e != hipSuccess) return hip_fail(e, "general-tap filter launch");
    }
    if (grad_pass) {
      ClosureArgs C = CG;
      C.rho_bar = fb;
      C.ut = fu;
      C.tau = ft;
      C.wa = W;
      hipError_t e = launch_grad_closure(C, c->stream);
      if (e != hipSuccess) return hip_fail(e, "closure launch");
    }
    if ((rc = timed_end(c))) return rc;
  }
  if (stats) {
    for (int f = 0; f < nf; ++f) {
      hipError_t e = launch_reduce(c->d_part + part_off[f], nparts[f], kNStat,
                                   c->d_sums + f * kNStat, c->d_red, c->stream);
      if (e != hipSuccess) return hip_fail(e, "reduce launch");
    }
    KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * kNStat * nf,
                           hipMemcpyDeviceToHost, c->stream), "stats copy");
    KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    for (int f = 0; f < nf; ++f)
      derive_stats(c->h_sums + f * kNStat, filters[f].delta_over_h * grid->h, taps[f].m2,
                   &stats[f]);
  }
  return KCF_OK;
}

int kcf_filter_favre_noalloc(const kcf_grid* grid, const kcf_filter* filters, int nf,
                             const float* rho, const float* u, const kcf_outputs* outs,
                             const kcf_closure_params* cp, kcf_width_stats* stats, int device,
                             void* stream) {
  WidthPlan P;
  int rc = plan_widths(grid, filters, nf, cp, P);
  if (rc) return rc;
  if (!outs || !rho || !u) return fail(KCF_EINVAL, "NULL argument");
  for (int f = 0; f < nf; ++f)
    if (!P.use_box[f])
      return fail(KCF_EUNSUPPORTED, "the no-allocation entry point runs box filters up to 16h "
                                    "(FP32) or 8h (FP64) only");
  int ndev = 0;
  KCF_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(KCF_EINVAL, "no such device");
  KCF_HIP(hipSetDevice(device), "hipSetDevice");
  const hipStream_t st = (hipStream_t)stream;
  FilterArgs A[4];
  for (int f = 0; f < nf; ++f) {
    box_args_for(A[f], grid, rho, u, P.radii[f], P.fp64[f]);
    if (stats && (size_t)box_records(A[f], P.radii[f], P.fp64[f]) > kNoAllocRecords)
      return fail(KCF_EUNSUPPORTED,
                  "grid too large for the statistics scratch of the no-allocation entry point ("
                  + std::to_string(box_records(A[f], P.radii[f], P.fp64[f])) + " records, " +
                  std::to_string(kNoAllocRecords) + " available)");
  }
  double* scr = nullptr;
  if (stats && (rc = scratch_address(device, &scr))) return rc;
  double* d_sums = scr;
  double* d_red = scr ? scr + kNoAllocSums : nullptr;
  double* d_part = scr ? scr + kNoAllocSums + kNoAllocRed : nullptr;
  for (int f = 0; f < nf; ++f) {
    std::memset(&A[f].wa, 0, sizeof(WidthArgs));
    set_outputs(A[f].wa, &outs[f]);
    set_closure(A[f].wa, cp, filters[f].delta_over_h * grid->h, P.taps[f].m2);
    A[f].wa.partials = d_part;  // every wave writes its record: nothing to clear
    A[f].wa.exact_stats = filters[f].precision == 2;
    hipError_t e = launch_box(A[f], P.radii[f], P.fp64[f], 8 * A[f].tiles_per_xcd, st);
    if (e != hipSuccess) return hip_fail(e, "box filter launch");
    if (stats) {  // reduce before the next width overwrites the records (same stream)
      e = launch_reduce(d_part, (int)box_records(A[f], P.radii[f], P.fp64[f]), kNStat,
                        d_sums + f * kNStat, d_red, st);
      if (e != hipSuccess) return hip_fail(e, "reduce launch");
    }
  }
  if (stats) {
    double h_sums[kNoAllocSums];
    KCF_HIP(hipMemcpyAsync(h_sums, d_sums, sizeof(double) * kNStat * nf, hipMemcpyDeviceToHost,
                           st), "stats copy");
    KCF_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (int f = 0; f < nf; ++f)
      derive_stats(h_sums + f * kNStat, filters[f].delta_over_h * grid->h, P.taps[f].m2,
                   &stats[f]);
  }
  return KCF_OK;
}

int kcf_lbm_equilibrium(kcf_ctx* c, const kcf_grid* grid, const float* rho, const float* u,
                        float* f_out) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!rho || !u || !f_out) return fail(KCF_EINVAL, "NULL argument");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
  hipError_t e = launch_lbm_equilibrium(rho, u, f_out, n, c->stream);
  if (e != hipSuccess) return hip_fail(e, "equilibrium launch");
  return KCF_OK;
}

int kcf_lbm_step(kcf_ctx* c, const kcf_grid* grid, const kcf_lbm_params* p, const float* f_in,
                 float* f_out, kcf_lbm_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!p || !f_in || !f_out) return fail(KCF_EINVAL, "NULL argument");
  if (f_in == f_out) return fail(KCF_EINVAL, "f_in and f_out must be distinct buffers");
  if (p->model < KCF_LBM_BGK || p->model > KCF_LBM_KCRR) return fail(KCF_EINVAL, "unknown model");
  if (!(p->nu > 0.0) || !std::isfinite(p->nu)) return fail(KCF_EINVAL, "nu must be > 0");
  if (!(p->c_nu >= 0.0) || !std::isfinite(p->c_nu)) return fail(KCF_EINVAL, "c_nu must be >= 0");
  const int64_t ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  LbmArgs A;
  std::memset(&A, 0, sizeof(A));
  A.fin = f_in;
  A.fout = f_out;
  A.nx = grid->nx;
  A.ny = grid->ny;
  A.nz = grid->nz;
  A.ntot = ntot;
  A.ntx = (grid->nx + lbm_tile_x() - 1) / lbm_tile_x();
  A.nty = (grid->ny + lbm_tile_y() - 1) / lbm_tile_y();
  A.ntiles = A.ntx * A.nty;
  A.nzc = choose_zchunks(A.ntiles, grid->nz, 0, 1);  // one 512-thread workgroup per CU
  A.zlen = (grid->nz + A.nzc - 1) / A.nzc;
  A.nzc = (grid->nz + A.zlen - 1) / A.zlen;
  A.items_per_xcd = (A.ntiles * A.nzc + 7) / 8;
  const double tau_hat = p->nu * 3.0 + 0.5;  // nu / theta_R + dt / 2, theta_R = 1/3
  A.tau_hat = (float)tau_hat;
  A.omega = (float)(1.0 / tau_hat);
  A.nu = (float)p->nu;
  A.c_nu = (float)p->c_nu;
  A.model = p->model;
  const int64_t nrec = (int64_t)A.ntiles * A.nzc * lbm_records_per_block();
  if (stats) {
    if (nrec > INT32_MAX) return fail(KCF_EUNSUPPORTED, "grid too large for statistics");
    if ((rc = ensure_partials(c, (size_t)nrec * kLbmStat))) return rc;
    A.partials = c->d_part;
  }
  if ((rc = timed_begin(c))) return rc;
  hipError_t e = launch_lbm_step(A, 8 * A.items_per_xcd, c->stream);
  if (e != hipSuccess) return hip_fail(e, "lattice-Boltzmann step launch");
  if ((rc = timed_end(c))) return rc;
  if (stats) {
    e = launch_reduce(c->d_part, (int)nrec, kLbmStat, c->d_sums, c->d_red, c->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * kLbmStat,
                           hipMemcpyDeviceToHost, c->stream), "stats copy");
    KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    const double* raw = c->h_sums;
    std::memset(stats, 0, sizeof(*stats));
    std::memcpy(stats->raw, raw, sizeof(double) * kLbmStat);
    stats->n_nodes = ntot;
    stats->mass = raw[0];
    for (int a = 0; a < 3; ++a) stats->momentum[a] = raw[1 + a];
    stats->kinetic_energy = raw[4];
    stats->mean_omega_sgs = raw[5] / (double)ntot;
    stats->clip_fraction = raw[6] / (double)ntot;
    stats->mean_k_sgs = raw[7] / (double)ntot;
  }
  return KCF_OK;
}

int kcf_sgs_carrier(kcf_ctx* c, const kcf_grid* grid, const kcf_filter* filter, const float* rho,
                    const float* u, float* f_sgs, float* f_h2, kcf_carrier_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!filter || !rho || !u) return fail(KCF_EINVAL, "NULL argument");
  if (!f_sgs && !f_h2 && !stats) return fail(KCF_EINVAL, "nothing requested");
  MonoArgs A;
  std::memset(&A, 0, sizeof(A));
  A.rho = rho;
  A.u = u;
  A.f_sgs = f_sgs;
  A.f_h2 = f_h2;
  if ((rc = run_monomials(c, grid, filter, kSetCarrier, 27, kCStat, A, stats != nullptr)))
    return rc;
  if (stats) {
    const double* raw = c->h_sums;
    std::memset(stats, 0, sizeof(*stats));
    std::memcpy(stats->raw, raw, sizeof(double) * kCStat);
    const double n = raw[C_N];
    stats->n_points = (int64_t)llround(n);
    stats->n_nonfinite = (int64_t)llround(raw[C_NONFINITE]);
    if (n > 0) {
      stats->sgs_l2 = raw[C_F2] / n;
      stats->err_l2 = raw[C_ERR2] / n;
      stats->rel_err = raw[C_F2] > 0 ? std::sqrt(raw[C_ERR2] / raw[C_F2]) : 0.0;
      for (int k = 0; k < 5; ++k) stats->hermite[k] = raw[C_HERM + k] / n;
    }
  }
  return KCF_OK;
}

int kcf_sgs_moment3(kcf_ctx* c, const kcf_grid* grid, const kcf_filter* filter, const float* rho,
                    const float* u, const float* theta, float* m3, float* theta_t,
                    kcf_moment3_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!filter || !rho || !u) return fail(KCF_EINVAL, "NULL argument");
  if (!m3 && !theta_t && !stats) return fail(KCF_EINVAL, "nothing requested");
  if (theta_t && !theta) return fail(KCF_EINVAL, "theta_t needs a temperature field");
  MonoArgs A;
  std::memset(&A, 0, sizeof(A));
  A.rho = rho;
  A.u = u;
  A.theta = theta;
  A.m3 = m3;
  A.theta_t = theta_t;
  if ((rc = run_monomials(c, grid, filter, kSetMoment3, theta ? 15 : 14, kM3Stat, A,
                          stats != nullptr)))
    return rc;
  if (stats) {
    const double* raw = c->h_sums;
    std::memset(stats, 0, sizeof(*stats));
    std::memcpy(stats->raw, raw, sizeof(double) * kM3Stat);
    const double n = raw[M3_N];
    stats->n_points = (int64_t)llround(n);
    stats->n_nonfinite = (int64_t)llround(raw[M3_NONFINITE]);
    if (n > 0) {
      for (int k = 0; k < 10; ++k) {
        stats->mean_m3[k] = raw[M3_SUM + k] / n;
        stats->rms_m3[k] = std::sqrt(raw[M3_SQ + k] / n);
      }
      stats->mean_theta_t = raw[M3_THETA] / n;
    }
  }
  return KCF_OK;
}

int kcf_kc_mp(kcf_ctx* c, const kcf_grid* grid, const kcf_filter* filter, const float* rho,
              const float* u, const kcf_kc_params* kp, float* m_sgs, float* m_ce, float* k_sgs,
              float* nu_t_eff, float* omega_sgs, kcf_kc_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!filter || !rho || !u || !kp) return fail(KCF_EINVAL, "NULL argument");
  if (!m_sgs && !m_ce && !k_sgs && !nu_t_eff && !omega_sgs && !stats)
    return fail(KCF_EINVAL, "nothing requested");
  if (!(kp->nu >= 0) || !(kp->dt >= 0) || !(kp->theta > 0) || !(kp->c_nu >= 0) ||
      (kp->rho_ref_one != 0 && kp->rho_ref_one != 1))
    return fail(KCF_EINVAL, "KC parameters: nu, dt, c_nu >= 0, theta > 0, rho_ref_one 0 or 1");
  const int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  // rho_bar, tau and G of the filter path, held by the context
  if ((rc = ensure_buffer(c, c->d_kc, c->kc_cap, sizeof(float) * 16 * (size_t)N,
                          "cannot allocate the KC field scratch")))
    return rc;
  kcf_outputs o;
  std::memset(&o, 0, sizeof(o));
  o.rho_bar = c->d_kc;
  o.tau = c->d_kc + N;
  o.grad = c->d_kc + 7 * N;
  if ((rc = kcf_filter_favre(c, grid, filter, 1, rho, u, &o, nullptr, nullptr))) return rc;
  MonoArgs A;
  std::memset(&A, 0, sizeof(A));
  A.rho = rho;
  A.u = u;
  A.ext = c->d_kc;
  A.m_sgs = m_sgs;
  A.m_ce = m_ce;
  A.k_sgs = k_sgs;
  A.nu_t_eff = nu_t_eff;
  A.omega_sgs = omega_sgs;
  const double tau_hat = kp->nu / kp->theta + 0.5 * kp->dt;
  A.inv2h = (float)(1.0 / (2.0 * grid->h));
  A.kc_coef = (float)(2.0 * kp->theta * tau_hat);
  A.nu = (float)kp->nu;
  A.inv_theta = (float)(1.0 / kp->theta);
  A.half_dt = (float)(0.5 * kp->dt);
  A.cnu_delta = (float)(kp->c_nu * filter->delta_over_h * grid->h);
  A.rho_ref_one = kp->rho_ref_one;
  if ((rc = run_monomials(c, grid, filter, kSetKcMp, 6, kKcStat, A, stats != nullptr))) return rc;
  if (stats) {
    const double* raw = c->h_sums;
    std::memset(stats, 0, sizeof(*stats));
    std::memcpy(stats->raw, raw, sizeof(double) * kKcStat);
    const double n = raw[KC_N];
    stats->n_points = (int64_t)llround(n);
    stats->n_nonfinite = (int64_t)llround(raw[KC_NONFINITE]);
    if (n > 0) {
      for (int k = 0; k < 6; ++k) {
        const double sm = raw[KC_M + k], st = raw[KC_T + k];
        const double cov = raw[KC_MT + k] - sm * st / n;
        const double vm = raw[KC_M2 + k] - sm * sm / n, vt = raw[KC_T2 + k] - st * st / n;
        stats->corr[k] = (vm > 0 && vt > 0) ? cov / std::sqrt(vm * vt) : NAN;
        stats->mean_m[k] = sm / n;
        stats->mean_tau[k] = st / n;
      }
      stats->rel_err = raw[KC_TAU2] > 0 ? std::sqrt(raw[KC_ERR2] / raw[KC_TAU2]) : NAN;
      stats->mean_k = raw[KC_K] / n;
      stats->mean_k_exact = raw[KC_KE] / n;
      stats->mean_omega = raw[KC_OM] / n;
      stats->mean_omega_exact = raw[KC_OME] / n;
      stats->clip = raw[KC_CLIP] / n;
      stats->clip_exact = raw[KC_CLIPE] / n;
    }
  }
  return KCF_OK;
}

int kcf_grad_closure(kcf_ctx* c, const kcf_grid* grid, const float* rho_bar, const float* ut,
                     const float* tau, double delta, double m2, const kcf_closure_params* cp,
                     const kcf_outputs* outs, kcf_width_stats* stats) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!rho_bar || !ut || !outs) return fail(KCF_EINVAL, "NULL argument");
  if (!(delta > 0) || !(m2 >= 0)) return fail(KCF_EINVAL, "delta must be > 0 and m2 >= 0");
  if ((rc = check_closure(cp))) return rc;
  if (!tau && (outs->k_sgs || outs->nu_t || outs->omega_t || stats))
    return fail(KCF_EINVAL, "k_sgs, nu_t, omega_t and statistics need tau");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  ClosureArgs C;
  std::memset(&C, 0, sizeof(C));
  C.rho_bar = rho_bar;
  C.ut = ut;
  C.tau = tau;
  C.nx = grid->nx;
  C.ny = grid->ny;
  C.nz = grid->nz;
  C.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  C.inv2h = (float)(1.0 / (2.0 * grid->h));
  set_outputs(C.wa, outs);
  set_closure(C.wa, cp, delta, m2);
  if (grid->ny > 65535) return fail(KCF_EUNSUPPORTED, "ny above 65535");
  const int64_t nrec = grad_closure_records(C);
  if (stats) {
    if ((rc = ensure_partials(c, (size_t)nrec * kNStat))) return rc;
    C.wa.partials = c->d_part;
  }
  hipError_t e = launch_grad_closure(C, c->stream);
  if (e != hipSuccess) return hip_fail(e, "closure launch");
  if (stats) {
    if ((rc = reduce_to_host(c, (int)nrec, kNStat, 0))) return rc;
    KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * kNStat, hipMemcpyDeviceToHost,
                           c->stream), "stats copy");
    KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    derive_stats(c->h_sums, delta, m2, stats);
  }
  return KCF_OK;
}

int kcf_input_stats(kcf_ctx* c, const kcf_grid* grid, const float* rho, const float* u,
                    kcf_input_summary* out) {
  if (!c) return fail(KCF_EINVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!rho || !u || !out) return fail(KCF_EINVAL, "NULL argument");
  if (grid->nx < 7 || grid->ny < 7 || grid->nz < 7)
    return fail(KCF_EUNSUPPORTED, "sixth-order vorticity needs n >= 7");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  InputStatArgs S;
  S.rho = rho;
  S.u = u;
  S.nx = grid->nx;
  S.ny = grid->ny;
  S.nz = grid->nz;
  S.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  S.inv60h = 1.0 / (60.0 * grid->h);
  if (grid->ny > 65535) return fail(KCF_EUNSUPPORTED, "ny above 65535");
  const int64_t nrec = input_stats_records(S);
  if ((rc = ensure_partials(c, (size_t)nrec * 4))) return rc;
  S.partials = c->d_part;
  hipError_t e = launch_input_stats(S, c->stream);
  if (e != hipSuccess) return hip_fail(e, "input stats launch");
  e = launch_reduce(c->d_part, (int)nrec, 4, c->d_sums, c->d_red, c->stream);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * 4, hipMemcpyDeviceToHost,
                         c->stream), "stats copy");
  KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  const double n = (double)S.ntot - c->h_sums[3];
  out->mean_rho = c->h_sums[0] / n;
  out->ek = c->h_sums[1] / n;
  out->enstrophy = c->h_sums[2] / n;
  out->n_nonfinite = (int64_t)llround(c->h_sums[3]);
  return KCF_OK;
}

int kcf_reduce_check(kcf_ctx* c, const float* a, const float* b, int64_t n, double* out) {
  if (!c || !a || !out) return fail(KCF_EINVAL, "NULL argument");
  if (n < 1) return fail(KCF_EINVAL, "n must be >= 1");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  int rc = ensure_partials(c, (size_t)nb * 4 * 3);
  if (rc) return rc;
  hipError_t e = launch_reduce_check(a, b, n, c->d_part, (int)nb, c->stream);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  e = launch_reduce(c->d_part, (int)nb * 4, 3, c->d_sums, c->d_red, c->stream);
  if (e != hipSuccess) return hip_fail(e, "reduce launch");
  KCF_HIP(hipMemcpyAsync(c->h_sums, c->d_sums, sizeof(double) * 3, hipMemcpyDeviceToHost,
                         c->stream), "copy");
  KCF_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  std::memcpy(out, c->h_sums, sizeof(double) * 3);
  return KCF_OK;
}

int kcf_stream_probe(kcf_ctx* c, const float* in, int nin, float* out, int nout, int64_t n) {
  if (!c || !in || !out) return fail(KCF_EINVAL, "NULL argument");
  if (nin < 1 || nin > 8 || nout < 1 || nout > 64 || n < 1)
    return fail(KCF_EINVAL, "need 1 <= nin <= 8, 1 <= nout <= 64, n >= 1");
  KCF_HIP(hipSetDevice(c->device), "hipSetDevice");
  int rc = timed_begin(c);
  if (rc) return rc;
  hipError_t e = launch_stream_probe(in, nin, out, nout, n, c->stream);
  if (e != hipSuccess) return hip_fail(e, "stream probe launch");
  return timed_end(c);
}

}  // extern "C"
