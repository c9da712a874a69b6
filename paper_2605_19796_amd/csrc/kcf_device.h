// Device helpers shared by the filtering kernels: per-point closures, FP64 statistics with a
// fixed-order wave reduction, output stores and the XCD-aware block mapping.
#pragma once

#include "kcf_internal.h"

namespace kcf {
namespace dev {

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------- per-point closures + stats
struct PointOut {
  float G[3][3];
  float tgm[6];
  float tsm[6];
  float ksgs, nut, omt;
};

__device__ __forceinline__ void point_closures(const WidthArgs& W, float rb, const float (&tau)[6],
                                               PointOut& P) {
  const float(&G)[3][3] = P.G;
  float c = W.gm_coef * rb;
  const int ii[6] = {0, 0, 0, 1, 1, 2};
  const int jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = ii[s], j = jj[s];
    float a;
    if (W.gm_form == 0)
      a = G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2];
    else
      a = G[0][i] * G[0][j] + G[1][i] * G[1][j] + G[2][i] * G[2][j];
    P.tgm[s] = c * a;
  }
  float S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = 0.5f * (G[i][j] + G[j][i]);
  float ss = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) ss += S[i][j] * S[i][j];
  const float smag = sqrtf(2.f * ss);
  const float trs = (S[0][0] + S[1][1] + S[2][2]) * (1.f / 3.f);
  const float cs = -2.f * rb * W.smag_coef * smag;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = ii[s], j = jj[s];
    P.tsm[s] = cs * (S[i][j] - (i == j ? trs : 0.f));
  }
  const float rref = W.ksgs_rho_ref ? 1.f : rb;
  P.ksgs = fabsf(tau[0] + tau[3] + tau[5]) / (2.f * rref);
  P.nut = W.cnu_delta * sqrtf(P.ksgs);
  P.omt = 1.f / (fmaxf(W.nu_mol, P.nut) * W.inv_theta + W.half_dt);
}

// Contribution of one point to FP64 sum slot s. Products of two float32 values are exact
// in double, so every contribution is computed in double from the stored float outputs.
struct StatIn {
  float rb, tau[6], tgm[6];
  double ke, pi, pigm, pism;
  bool use, bad;
};

__device__ __forceinline__ void stat_inputs(float rb, const float (&u)[3], const float (&tau)[6],
                                            const PointOut& P, bool valid, StatIn& I) {
  const int ii[6] = {0, 0, 0, 1, 1, 2};
  const int jj[6] = {0, 1, 2, 1, 2, 2};
  double pi = 0, pigm = 0, pism = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const double S = 0.5 * ((double)P.G[ii[s]][jj[s]] + (double)P.G[jj[s]][ii[s]]);
    const double m = (ii[s] == jj[s]) ? S : 2.0 * S;
    pi -= (double)tau[s] * m;
    pigm -= (double)P.tgm[s] * m;
    pism -= (double)P.tsm[s] * m;
  }
  const double ke = 0.5 * (double)rb *
                    ((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
  bool fin = isfinite(pi) && isfinite(pigm) && isfinite(pism) && isfinite(ke) && isfinite(rb);
#pragma unroll
  for (int s = 0; s < 6; ++s) fin = fin && isfinite(tau[s]) && isfinite(P.tgm[s]);
  I.bad = valid && !fin;
  I.use = valid && fin;
  I.rb = rb;
  I.ke = ke;
  I.pi = pi;
  I.pigm = pigm;
  I.pism = pism;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    I.tau[s] = tau[s];
    I.tgm[s] = P.tgm[s];
  }
}

__device__ __forceinline__ double stat_raw(const StatIn& I, int s) {
  if (s == S_N) return 1.0;
  if (s == S_RHO) return (double)I.rb;
  if (s == S_KE) return I.ke;
  if (s == S_PI) return I.pi;
  if (s == S_PIGM) return I.pigm;
  if (s == S_PI2) return I.pi * I.pi;
  if (s == S_PIGM2) return I.pigm * I.pigm;
  if (s == S_PIPIGM) return I.pi * I.pigm;
  if (s >= S_TAU && s < S_TAU + 6) return (double)I.tau[s - S_TAU];
  if (s >= S_TGM && s < S_TGM + 6) return (double)I.tgm[s - S_TGM];
  if (s >= S_TAU2 && s < S_TAU2 + 6) return (double)I.tau[s - S_TAU2] * (double)I.tau[s - S_TAU2];
  if (s >= S_TGM2 && s < S_TGM2 + 6) return (double)I.tgm[s - S_TGM2] * (double)I.tgm[s - S_TGM2];
  if (s >= S_TAUTGM && s < S_TAUTGM + 6)
    return (double)I.tau[s - S_TAUTGM] * (double)I.tgm[s - S_TAUTGM];
  return I.pism;  // S_PISM
}

__device__ __forceinline__ double stat_value(const StatIn& I, int s) {
  if (s == S_NONFINITE) return I.bad ? 1.0 : 0.0;
  return I.use ? stat_raw(I, s) : 0.0;
}

// Reduce 8 per-lane values over the wave: afterwards every lane holds the wave total of
// slot (lane >> 3). Fixed order: the result does not depend on timing.
__device__ __forceinline__ double wave_reduce8(double (&v)[8]) {
  const int lane = __lane_id();
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double send = b5 ? v[s] : v[s + 4];
    const double keep = b5 ? v[s + 4] : v[s];
    v[s] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double send = b4 ? v[s] : v[s + 2];
    const double keep = b4 ? v[s + 2] : v[s];
    v[s] = keep + __shfl_xor(send, 16);
  }
  {
    const double send = b3 ? v[0] : v[1];
    const double keep = b3 ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 8);
  }
  double r = v[0];
  r += __shfl_xor(r, 4);
  r += __shfl_xor(r, 2);
  r += __shfl_xor(r, 1);
  return r;
}

__device__ __forceinline__ void accumulate_stats(const StatIn& I, double (&acc)[5]) {
#pragma unroll
  for (int g = 0; g < 5; ++g) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = stat_value(I, g * 8 + j);
    acc[g] += wave_reduce8(v);
  }
}

__device__ __forceinline__ void write_stats(double* part, const double (&acc)[5]) {
  const int lane = __lane_id();
  if ((lane & 7) == 0) {
#pragma unroll
    for (int g = 0; g < 5; ++g) part[g * 8 + (lane >> 3)] = acc[g];
  }
}

__device__ __forceinline__ void store_point(const WidthArgs& W, int64_t g, int64_t ntot,
                                            const PointOut& P) {
  if (W.grad) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) W.grad[(i * 3 + j) * ntot + g] = P.G[i][j];
  }
  if (W.tau_gm) {
#pragma unroll
    for (int s = 0; s < 6; ++s) W.tau_gm[s * ntot + g] = P.tgm[s];
  }
  if (W.tau_smag) {
#pragma unroll
    for (int s = 0; s < 6; ++s) W.tau_smag[s * ntot + g] = P.tsm[s];
  }
  if (W.k_sgs) W.k_sgs[g] = P.ksgs;
  if (W.nu_t) W.nu_t[g] = P.nut;
  if (W.omega_t) W.omega_t[g] = P.omt;
}

// XCD-aware block mapping: consecutive block ids go to different XCDs, so block L is
// placed on XCD L % 8. Every XCD gets a contiguous band of (z-chunk, tile) items, and
// within the band the widths of one item are adjacent, so the input planes they share
// are read through one L2.
__device__ __forceinline__ bool map_block(const FilterArgs& A, int& widx, int& item) {
  const int L = blockIdx.x;
  const int xcd = L & 7;
  const int r = L >> 3;
  widx = r % A.nw;
  const int j = r / A.nw;
  item = xcd * A.tiles_per_xcd + j;
  return j < A.tiles_per_xcd && item < A.ntiles * A.nzc;
}

}  // namespace dev
}  // namespace kcf
