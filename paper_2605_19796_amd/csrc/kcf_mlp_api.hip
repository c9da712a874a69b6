// C-ABI layer of the learned closure: parameter state, normalisation, training steps,
// gradient export, inference over a field, checkpoints.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kcf.h"
#include "kcf_checkpoint.h"
#include "kcf_internal.h"
#include "kcf_mlp_internal.h"

using namespace kcf::mlp;

namespace kcf {
int api_fail(int code, const char* msg);
hipStream_t ctx_stream(kcf_ctx* c);
int ctx_device(kcf_ctx* c);
}  // namespace kcf

struct kcf_mlp {
  kcf_ctx* ctx = nullptr;
  float* d_params = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  __bf16* d_packed = nullptr;
  float* d_norm = nullptr;  // x_mu 14, x_sd 14, y_mu 6, y_sd 6, x_lo 14, x_hi 14
  float h_norm[68];
  int64_t step = 0;
  int cap = 0;  // batch capacity of the training scratch
  int nw_cap = 0;  // weight-gradient partials the scratch holds (batch / wgrad_chunk(batch))
  __bf16* d_act = nullptr;
  __bf16* d_dz = nullptr;
  float* d_db_part = nullptr;
  double* d_loss_part = nullptr;
  float* d_w_part = nullptr;
  float* d_grad = nullptr;
  int64_t* d_fb_part = nullptr;
  int fb_cap = 0;
  double* d_colpart = nullptr;
  int colpart_cap = 0;
};

namespace {

constexpr int kNormFloats = 68;
static_assert(kNormFloats == kcf::ckpt::kCkNorm && kNParams == kcf::ckpt::kCkParams, "checkpoint layout");
constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;

int fail(int code, const char* msg) { return kcf::api_fail(code, msg); }

int hipfail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return kcf::api_fail(KCF_EHIP, m.c_str());
}

#define MLP_HIP(call, what)                          \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hipfail(e_, what);  \
  } while (0)

MlpArgs args_of(kcf_mlp* m) {
  MlpArgs a;
  a.params = m->d_params;
  a.m = m->d_m;
  a.v = m->d_v;
  a.packed = m->d_packed;
  a.x_mu = m->d_norm;
  a.x_sd = m->d_norm + 14;
  a.y_mu = m->d_norm + 28;
  a.y_sd = m->d_norm + 34;
  a.x_lo = m->d_norm + 40;
  a.x_hi = m->d_norm + 54;
  return a;
}

// The split-K pass of a smaller batch can have more partials than that of a larger one (its
// chunk is the largest power of two dividing the batch), so both capacities are checked.
int ensure_train(kcf_mlp* m, int batch) {
  const int nw_req = batch / wgrad_chunk(batch);
  if (batch <= m->cap && nw_req <= m->nw_cap) return KCF_OK;
  batch = std::max(batch, m->cap);
  hipStream_t s = kcf::ctx_stream(m->ctx);
  hipStreamSynchronize(s);
  // freed and cleared together, so that a failed allocation below leaves nothing to free twice
  for (void** q : {(void**)&m->d_act, (void**)&m->d_dz, (void**)&m->d_db_part,
                   (void**)&m->d_loss_part, (void**)&m->d_w_part}) {
    hipFree(*q);
    *q = nullptr;
  }
  m->cap = 0;
  const size_t rows = 16 + 3 * 64;
  const int fb = fwdbwd_blocks(batch);
  const int nw = std::max({nw_req, batch / wgrad_chunk(batch), m->nw_cap});
  m->nw_cap = 0;
  if (hipMalloc(&m->d_act, rows * batch * sizeof(__bf16)) != hipSuccess ||
      hipMalloc(&m->d_dz, rows * batch * sizeof(__bf16)) != hipSuccess ||
      hipMalloc(&m->d_db_part, (size_t)fb * 198 * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_loss_part, (size_t)fb * sizeof(double)) != hipSuccess ||
      hipMalloc(&m->d_w_part, (size_t)nw * kNParams * sizeof(float)) != hipSuccess)
    return fail(KCF_ENOMEM, "cannot allocate training scratch");
  m->cap = batch;
  m->nw_cap = nw;
  return KCF_OK;
}

TrainArgs train_args(kcf_mlp* m, const float* x, const float* y, int64_t n, const int32_t* idx,
                     int batch) {
  TrainArgs t;
  t.x = x;
  t.y = y;
  t.idx = idx;
  t.n_rows = n;
  t.batch = batch;
  t.act0 = m->d_act;
  for (int l = 0; l < 3; ++l) t.act[l] = m->d_act + (size_t)(16 + 64 * l) * batch;
  for (int l = 0; l < 3; ++l) t.dz[l] = m->d_dz + (size_t)64 * l * batch;
  t.dz4 = m->d_dz + (size_t)192 * batch;
  t.db_part = m->d_db_part;
  t.loss_part = m->d_loss_part;
  t.w_part = m->d_w_part;
  return t;
}

int check_batch(const float* x, const float* y, int64_t n, const int32_t* idx, int batch) {
  if (!x || !y) return fail(KCF_EINVAL, "NULL dataset");
  if (n < 1) return fail(KCF_EINVAL, "dataset needs n >= 1 rows");
  if (!idx && batch > n) return fail(KCF_EINVAL, "batch larger than the dataset");
  if (batch < 32 || batch % 32 || batch > (1 << 22))
    return fail(KCF_EINVAL, "batch must be a multiple of 32 in [32, 4194304]");
  return KCF_OK;
}

// Forward/backward and weight-gradient passes; then, with adam NULL, the gradient into
// m->d_grad, else the gradient reduction and the Adam step (and the loss into loss_dev) in
// one launch.
int forward_backward(kcf_mlp* m, const float* x, const float* y, int64_t n, const int32_t* idx,
                     int batch, int* nfb, const AdamArgs* adam = nullptr,
                     float* loss_dev = nullptr) {
  int rc = ensure_train(m, batch);
  if (rc) return rc;
  hipStream_t s = kcf::ctx_stream(m->ctx);
  TrainArgs t = train_args(m, x, y, n, idx, batch);
  int nw = 0;
  MLP_HIP(launch_train_passes(args_of(m), t, nfb, &nw, s), "training pass launch");
  if (adam) {
    MLP_HIP(launch_grad_adam(t, nw, *nfb, args_of(m), *adam, m->d_loss_part, *nfb, loss_dev,
                             m->d_packed, s),
            "gradient and Adam launch");
  } else {
    MLP_HIP(launch_grad_reduce(t, nw, *nfb, m->d_grad, s), "gradient reduce launch");
  }
  return KCF_OK;
}


}  // namespace

extern "C" {

int kcf_mlp_create(kcf_ctx* ctx, kcf_mlp** out) {
  if (!ctx || !out) return fail(KCF_EINVAL, "NULL argument");
  *out = nullptr;
  MLP_HIP(hipSetDevice(kcf::ctx_device(ctx)), "hipSetDevice");
  kcf_mlp* m = new kcf_mlp();
  m->ctx = ctx;
  if (hipMalloc(&m->d_params, kNParams * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_m, kNParams * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_v, kNParams * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_grad, kNParams * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_packed, kPackTotal * sizeof(__bf16)) != hipSuccess ||
      hipMalloc(&m->d_norm, kNormFloats * sizeof(float)) != hipSuccess) {
    kcf_mlp_destroy(m);
    return fail(KCF_ENOMEM, "cannot allocate network state");
  }
  hipStream_t s = kcf::ctx_stream(ctx);
  MLP_HIP(hipMemsetAsync(m->d_params, 0, kNParams * sizeof(float), s), "memset");
  MLP_HIP(hipMemsetAsync(m->d_m, 0, kNParams * sizeof(float), s), "memset");
  MLP_HIP(hipMemsetAsync(m->d_v, 0, kNParams * sizeof(float), s), "memset");
  for (int i = 0; i < kNormFloats; ++i) m->h_norm[i] = 0.f;
  for (int i = 0; i < 14; ++i) {
    m->h_norm[14 + i] = 1.f;
    m->h_norm[40 + i] = -INFINITY;
    m->h_norm[54 + i] = INFINITY;
  }
  for (int i = 0; i < 6; ++i) m->h_norm[34 + i] = 1.f;
  MLP_HIP(hipMemcpyAsync(m->d_norm, m->h_norm, sizeof(m->h_norm), hipMemcpyHostToDevice, s),
          "norm copy");
  MLP_HIP(launch_pack(m->d_params, m->d_packed, s), "pack launch");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  *out = m;
  return KCF_OK;
}

void kcf_mlp_destroy(kcf_mlp* m) {
  if (!m) return;
  hipStreamSynchronize(kcf::ctx_stream(m->ctx));
  hipFree(m->d_params);
  hipFree(m->d_m);
  hipFree(m->d_v);
  hipFree(m->d_grad);
  hipFree(m->d_packed);
  hipFree(m->d_norm);
  hipFree(m->d_act);
  hipFree(m->d_dz);
  hipFree(m->d_db_part);
  hipFree(m->d_loss_part);
  hipFree(m->d_w_part);
  hipFree(m->d_fb_part);
  hipFree(m->d_colpart);
  delete m;
}

int kcf_mlp_set_params(kcf_mlp* m, const float* params) {
  if (!m || !params) return fail(KCF_EINVAL, "NULL argument");
  for (int i = 0; i < kNParams; ++i)
    if (!std::isfinite(params[i])) return fail(KCF_EINVAL, "parameters must be finite");
  hipStream_t s = kcf::ctx_stream(m->ctx);
  MLP_HIP(hipMemcpyAsync(m->d_params, params, kNParams * sizeof(float), hipMemcpyHostToDevice, s),
          "param copy");
  MLP_HIP(hipMemsetAsync(m->d_m, 0, kNParams * sizeof(float), s), "memset");
  MLP_HIP(hipMemsetAsync(m->d_v, 0, kNParams * sizeof(float), s), "memset");
  MLP_HIP(launch_pack(m->d_params, m->d_packed, s), "pack launch");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  m->step = 0;
  return KCF_OK;
}

int kcf_mlp_get_params(kcf_mlp* m, float* params) {
  if (!m || !params) return fail(KCF_EINVAL, "NULL argument");
  hipStream_t s = kcf::ctx_stream(m->ctx);
  MLP_HIP(hipMemcpyAsync(params, m->d_params, kNParams * sizeof(float), hipMemcpyDeviceToHost, s),
          "param copy");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  return KCF_OK;
}

int kcf_mlp_set_norm(kcf_mlp* m, const float* norm) {
  if (!m || !norm) return fail(KCF_EINVAL, "NULL argument");
  if (const char* why = kcf::ckpt::check_norm(norm)) return fail(KCF_EINVAL, why);
  std::memcpy(m->h_norm, norm, sizeof(m->h_norm));
  hipStream_t s = kcf::ctx_stream(m->ctx);
  MLP_HIP(hipMemcpyAsync(m->d_norm, m->h_norm, sizeof(m->h_norm), hipMemcpyHostToDevice, s),
          "norm copy");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  return KCF_OK;
}

int kcf_mlp_get_norm(kcf_mlp* m, float* norm) {
  if (!m || !norm) return fail(KCF_EINVAL, "NULL argument");
  std::memcpy(norm, m->h_norm, sizeof(m->h_norm));
  return KCF_OK;
}

int kcf_mlp_features(kcf_ctx* ctx, const kcf_grid* grid, const float* rho_bar, const float* ut,
                     const float* tau, double delta, float* x_out, float* y_out) {
  if (!ctx || !grid || !rho_bar || !ut || !x_out) return fail(KCF_EINVAL, "NULL argument");
  if (y_out && !tau) return fail(KCF_EINVAL, "targets need tau");
  if (grid->nx < 3 || grid->ny < 3 || grid->nz < 3 || !(grid->h > 0))
    return fail(KCF_EINVAL, "bad grid");
  if (!(delta > 0)) return fail(KCF_EINVAL, "delta must be > 0");
  FeatArgs A;
  A.rho_bar = rho_bar;
  A.ut = ut;
  A.tau = tau;
  A.nx = grid->nx;
  A.ny = grid->ny;
  A.nz = grid->nz;
  A.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  A.inv2h = (float)(1.0 / (2.0 * grid->h));
  A.delta = (float)delta;
  A.x = x_out;
  A.y = y_out;
  MLP_HIP(launch_features(A, kcf::ctx_stream(ctx)), "features launch");
  return KCF_OK;
}

int kcf_mlp_column_stats(kcf_ctx* ctx, const float* X, int64_t n, int ncol, double* sum,
                         double* sumsq, double* mn, double* mx) {
  if (!ctx || !X || !sum || !sumsq || !mn || !mx) return fail(KCF_EINVAL, "NULL argument");
  if (n < 1 || ncol < 1 || ncol > 32) return fail(KCF_EINVAL, "need n >= 1 and 1 <= ncol <= 32");
  hipStream_t s = kcf::ctx_stream(ctx);
  int blocks = (int)std::min<int64_t>(1024, (n + 4095) / 4096);
  if (blocks < 1) blocks = 1;
  double* part = nullptr;
  MLP_HIP(hipMallocAsync((void**)&part, (size_t)blocks * ncol * 4 * sizeof(double), s), "alloc");
  MLP_HIP(launch_colstats(X, n, ncol, part, blocks, s), "colstats launch");
  std::vector<double> h((size_t)blocks * ncol * 4);
  MLP_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
  MLP_HIP(hipFreeAsync(part, s), "free");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  for (int c = 0; c < ncol; ++c) {
    double S = 0, S2 = 0, MN = INFINITY, MX = -INFINITY;
    for (int b = 0; b < blocks; ++b) {
      const double* o = &h[((size_t)b * ncol + c) * 4];
      S += o[0];
      S2 += o[1];
      MN = std::fmin(MN, o[2]);
      MX = std::fmax(MX, o[3]);
    }
    sum[c] = S;
    sumsq[c] = S2;
    mn[c] = MN;
    mx[c] = MX;
  }
  return KCF_OK;
}

int kcf_mlp_fit_norm(kcf_mlp* m, const float* X, const float* Y, int64_t n) {
  if (!m || !X || !Y) return fail(KCF_EINVAL, "NULL argument");
  double s[14], s2[14], mn[14], mx[14], t[6], t2[6], tmn[6], tmx[6];
  int rc = kcf_mlp_column_stats(m->ctx, X, n, 14, s, s2, mn, mx);
  if (rc) return rc;
  if ((rc = kcf_mlp_column_stats(m->ctx, Y, n, 6, t, t2, tmn, tmx))) return rc;
  float norm[kNormFloats];
  for (int c = 0; c < 14; ++c) {
    const double mu = s[c] / n;
    const double var = std::fmax(s2[c] / n - mu * mu, 0.0);
    const double sd = var > 0 ? std::sqrt(var) : 1.0;
    norm[c] = (float)mu;
    norm[14 + c] = (float)sd;
    norm[40 + c] = (float)((mn[c] - mu) / sd);
    norm[54 + c] = (float)((mx[c] - mu) / sd);
  }
  for (int c = 0; c < 6; ++c) {
    const double mu = t[c] / n;
    const double var = std::fmax(t2[c] / n - mu * mu, 0.0);
    norm[28 + c] = (float)mu;
    norm[34 + c] = (float)(var > 0 ? std::sqrt(var) : 1.0);
  }
  return kcf_mlp_set_norm(m, norm);
}

int kcf_mlp_grads(kcf_mlp* m, const float* x, const float* y, int64_t n, const int32_t* idx,
                  int batch, float* grads, double* loss) {
  if (!m || !grads) return fail(KCF_EINVAL, "NULL argument");
  int rc = check_batch(x, y, n, idx, batch);
  if (rc) return rc;
  int nfb = 0;
  if ((rc = forward_backward(m, x, y, n, idx, batch, &nfb))) return rc;
  hipStream_t s = kcf::ctx_stream(m->ctx);
  MLP_HIP(hipMemcpyAsync(grads, m->d_grad, kNParams * sizeof(float), hipMemcpyDeviceToHost, s),
          "grad copy");
  std::vector<double> lp(nfb);
  MLP_HIP(hipMemcpyAsync(lp.data(), m->d_loss_part, nfb * sizeof(double), hipMemcpyDeviceToHost, s),
          "loss copy");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  if (loss) {
    double t = 0;
    for (double v : lp) t += v;
    *loss = t / ((double)batch * 6.0);
  }
  return KCF_OK;
}

int kcf_mlp_train_step(kcf_mlp* m, const float* x, const float* y, int64_t n, const int32_t* idx,
                       int batch, float lr, float* loss_dev) {
  if (!m) return fail(KCF_EINVAL, "NULL argument");
  int rc = check_batch(x, y, n, idx, batch);
  if (rc) return rc;
  if (!(lr > 0) || !std::isfinite(lr)) return fail(KCF_EINVAL, "learning rate must be > 0");
  const int64_t step = m->step + 1;
  AdamArgs A;
  A.lr = lr;
  A.b1 = kB1;
  A.b2 = kB2;
  A.eps = kEps;
  A.c1 = (float)(1.0 / (1.0 - std::pow((double)kB1, (double)step)));
  A.c2 = (float)(1.0 / (1.0 - std::pow((double)kB2, (double)step)));
  A.loss_den = (double)batch * 6.0;
  int nfb = 0;
  if ((rc = forward_backward(m, x, y, n, idx, batch, &nfb, &A, loss_dev))) return rc;
  m->step = step;  // the launch also rewrote the BF16 operands of the updated weights
  return KCF_OK;
}

int kcf_mlp_step_count(kcf_mlp* m, int64_t* step) {
  if (!m || !step) return fail(KCF_EINVAL, "NULL argument");
  *step = m->step;
  return KCF_OK;
}

int kcf_mlp_predict(kcf_mlp* m, const float* x, int64_t n, float* y_std) {
  if (!m || !x || !y_std) return fail(KCF_EINVAL, "NULL argument");
  if (n < 1) return fail(KCF_EINVAL, "n must be >= 1");
  MLP_HIP(launch_predict(args_of(m), x, n, y_std, kcf::ctx_stream(m->ctx)), "predict launch");
  return KCF_OK;
}

int kcf_mlp_infer_field(kcf_mlp* m, const kcf_grid* grid, const float* rho_bar, const float* ut,
                        double delta, double m2, float* tau, uint16_t* mask, int64_t* n_fallback) {
  if (!m || !grid || !rho_bar || !ut || !tau) return fail(KCF_EINVAL, "NULL argument");
  if (grid->nx < 3 || grid->ny < 3 || grid->nz < 3 || !(grid->h > 0))
    return fail(KCF_EINVAL, "bad grid");
  if (!(delta > 0) || !(m2 >= 0)) return fail(KCF_EINVAL, "delta must be > 0 and m2 >= 0");
  hipStream_t s = kcf::ctx_stream(m->ctx);
  InferArgs I;
  I.rho_bar = rho_bar;
  I.ut = ut;
  I.nx = grid->nx;
  I.ny = grid->ny;
  I.nz = grid->nz;
  I.ntot = (int64_t)grid->nx * grid->ny * grid->nz;
  I.inv2h = (float)(1.0 / (2.0 * grid->h));
  I.delta = (float)delta;
  I.gm_coef = (float)m2;
  I.tau = tau;
  I.mask = mask;
  const int64_t chunks = (I.ntot + 63) / 64;  // one wave per 64 points, four waves a block
  int blocks = (int)std::min<int64_t>(4096, (chunks + 3) / 4);
  I.fallback_part = nullptr;
  if (n_fallback) {
    if (m->fb_cap < blocks * 4) {
      hipStreamSynchronize(s);
      hipFree(m->d_fb_part);
      m->d_fb_part = nullptr;
      m->fb_cap = 0;
      if (hipMalloc(&m->d_fb_part, (size_t)blocks * 4 * sizeof(int64_t)) != hipSuccess)
        return fail(KCF_ENOMEM, "cannot allocate fallback counters");
      m->fb_cap = blocks * 4;
    }
    I.fallback_part = m->d_fb_part;
  }
  MLP_HIP(launch_infer(args_of(m), I, blocks, s), "infer launch");
  if (n_fallback) {
    std::vector<int64_t> h((size_t)blocks * 4);
    MLP_HIP(hipMemcpyAsync(h.data(), m->d_fb_part, h.size() * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s), "copy");
    MLP_HIP(hipStreamSynchronize(s), "sync");
    int64_t t = 0;
    for (int64_t v : h) t += v;
    *n_fallback = t;
  }
  return KCF_OK;
}

// Checkpoint: "KCFMLP01", int64 step, params, m, v (float32 x 9670 each), norm (68 floats),
// then an FNV-1a 64-bit checksum of everything before it.
int kcf_mlp_save(kcf_mlp* m, const char* path) {
  if (!m || !path) return fail(KCF_EINVAL, "NULL argument");
  std::vector<float> buf(3 * kNParams);
  hipStream_t s = kcf::ctx_stream(m->ctx);
  MLP_HIP(hipMemcpyAsync(buf.data(), m->d_params, kNParams * 4, hipMemcpyDeviceToHost, s), "copy");
  MLP_HIP(hipMemcpyAsync(buf.data() + kNParams, m->d_m, kNParams * 4, hipMemcpyDeviceToHost, s), "copy");
  MLP_HIP(hipMemcpyAsync(buf.data() + 2 * kNParams, m->d_v, kNParams * 4, hipMemcpyDeviceToHost, s), "copy");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  const std::vector<unsigned char> out = kcf::ckpt::encode(m->step, buf.data(), m->h_norm);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(KCF_EIO, "cannot open checkpoint for writing");
  const size_t w = std::fwrite(out.data(), 1, out.size(), f);
  const int c = std::fclose(f);
  if (w != out.size() || c != 0) return fail(KCF_EIO, "short write of checkpoint");
  return KCF_OK;
}

int kcf_mlp_load(kcf_mlp* m, const char* path) {
  if (!m || !path) return fail(KCF_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(KCF_EIO, "cannot open checkpoint");
  std::vector<unsigned char> in;
  unsigned char tmp[65536];
  size_t r;
  // read at most one byte past a checkpoint: enough to tell that a file is too long
  while (in.size() <= kcf::ckpt::kSize && (r = std::fread(tmp, 1, sizeof(tmp), f)) > 0)
    in.insert(in.end(), tmp, tmp + r);
  std::fclose(f);
  int64_t step;
  std::vector<float> pmv(3 * kNParams);
  float norm[kNormFloats];
  if (const char* why = kcf::ckpt::decode(in.data(), in.size(), &step, pmv.data(), norm))
    return fail(KCF_EIO, why);
  int rc = kcf_mlp_set_norm(m, norm);
  if (rc) return rc;
  hipStream_t s = kcf::ctx_stream(m->ctx);
  const float* p = pmv.data();
  MLP_HIP(hipMemcpyAsync(m->d_params, p, kNParams * 4, hipMemcpyHostToDevice, s), "copy");
  MLP_HIP(hipMemcpyAsync(m->d_m, p + kNParams, kNParams * 4, hipMemcpyHostToDevice, s), "copy");
  MLP_HIP(hipMemcpyAsync(m->d_v, p + 2 * kNParams, kNParams * 4, hipMemcpyHostToDevice, s), "copy");
  MLP_HIP(launch_pack(m->d_params, m->d_packed, s), "pack launch");
  MLP_HIP(hipStreamSynchronize(s), "sync");
  m->step = step;
  return KCF_OK;
}

}  // extern "C"
