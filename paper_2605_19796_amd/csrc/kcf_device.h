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

// XCD bands for a 1-D grid of 8 * ceil(nitems / 8) workgroups: the hardware hands workgroup L
// to XCD L % 8, so giving it item (L % 8) * per + L / 8 lets each XCD work through one
// contiguous range of items, and neighbouring items (which read each other's rows or halos)
// meet in one L2. False for the padding workgroups past the last item.
__device__ __forceinline__ bool xcd_band_item(int64_t nitems, int64_t& item) {
  const int64_t per = (nitems + 7) / 8;
  const int64_t j = blockIdx.x >> 3;
  item = (int64_t)(blockIdx.x & 7) * per + j;
  return j < per && item < nitems;
}

// sum_m w_m v[c + m], m = -R..R, with w symmetric: w_0 v_c + sum_{m>0} w_m (v_{c+m} + v_{c-m}).
template <int R, typename T>
__device__ __forceinline__ T tap_sum(const T* w, const T* v, int c) {
  T s = w[R] * v[c];
#pragma unroll
  for (int m = 1; m <= R; ++m) s = fma(w[R + m], v[c + m] + v[c - m], s);
  return s;
}

// ---------------------------------------------------------------- per-point closures + stats
struct PointOut {
  float G[3][3];
  float tgm[6];
  float tsm[6];
  float ksgs, nut, omt;
};

// Gradient model rho_bar C M2 (G G^T)_ij (gm_form 0) or the transposed contraction
// (G^T G)_ij (gm_form 1); gm_coef holds C M2.
// The closures spell out every fused multiply-add and allow no other contraction, so that a
// point gets the same bits in every kernel instance, whatever the compiler shares between
// them and the other per-point expressions of that instance.
__device__ __forceinline__ void gm_closure(const WidthArgs& W, float rb, PointOut& P) {
#pragma clang fp contract(off)
  const float(&G)[3][3] = P.G;
  float c = W.gm_coef * rb;
  const int ii[6] = {0, 0, 0, 1, 1, 2};
  const int jj[6] = {0, 1, 2, 1, 2, 2};
  // one contraction or the other (uniform): the empty asm keeps the compiler from
  // evaluating both and selecting
  if (W.gm_form == 0) {
    __asm__ volatile("");
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = ii[s], j = jj[s];
      P.tgm[s] = c * fmaf(G[i][0], G[j][0], fmaf(G[i][1], G[j][1], G[i][2] * G[j][2]));
    }
  } else {
    __asm__ volatile("");
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = ii[s], j = jj[s];
      P.tgm[s] = c * fmaf(G[0][i], G[0][j], fmaf(G[1][i], G[1][j], G[2][i] * G[2][j]));
    }
  }
}

// Smagorinsky -2 rho_bar (C_s Delta)^2 |S| S^d; smag_coef holds (C_s Delta)^2.
__device__ __forceinline__ void smag_closure(const WidthArgs& W, float rb, PointOut& P) {
#pragma clang fp contract(off)  // as in gm_closure
  const float(&G)[3][3] = P.G;
  const int ii[6] = {0, 0, 0, 1, 1, 2};
  const int jj[6] = {0, 1, 2, 1, 2, 2};
  float S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = 0.5f * (G[i][j] + G[j][i]);
  float ss = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) ss = fmaf(S[i][j], S[i][j], ss);
  // the hardware square root (within 1 ulp): a correctly rounded one costs about ten more
  // instructions per point, far below the closure's own accuracy
  const float smag = __builtin_amdgcn_sqrtf(2.f * ss);
  const float trs = (S[0][0] + S[1][1] + S[2][2]) * (1.f / 3.f);
  const float cs = -2.f * rb * W.smag_coef * smag;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int i = ii[s], j = jj[s];
    P.tsm[s] = cs * (S[i][j] - (i == j ? trs : 0.f));
  }
}

// Closures of one point from its gradient (in P.G), filtered density and tau. Only what is
// stored or reduced is evaluated; the rest is left at zero.
// exact_stats: the statistics take the exact FP64 path (stat_inputs), which contracts the
// Smagorinsky tensor; the float32 path (stat_point) needs only its dissipation, which
// smag_dissipation forms without the tensor. Both need the gradient-model tensor.
__device__ __forceinline__ void point_closures(const WidthArgs& W, float rb, const float (&tau)[6],
                                               PointOut& P, bool exact_stats = false) {
  const bool stats = W.partials != nullptr;
#pragma unroll
  for (int s = 0; s < 6; ++s) P.tgm[s] = P.tsm[s] = 0.f;
  P.ksgs = P.nut = P.omt = 0.f;
  if (stats || W.tau_gm) {  // uniform
    gm_closure(W, rb, P);
  }
  if (W.tau_smag || (stats && exact_stats)) {  // uniform
    smag_closure(W, rb, P);
  }
  if (W.k_sgs || W.nu_t || W.omega_t) {  // uniform; only stored, never reduced
    const float rref = W.ksgs_rho_ref ? 1.f : rb;
    P.ksgs = fabsf(tau[0] + tau[3] + tau[5]) / (2.f * rref);
    P.nut = W.cnu_delta * sqrtf(P.ksgs);
    P.omt = 1.f / fmaf(fmaxf(W.nu_mol, P.nut), W.inv_theta, W.half_dt);
  }
}

// What one point contributes to the FP64 sums of the exact path (kernels whose filter sums
// are FP64). Products of two float32 values are exact in double, so every contribution is
// formed in double from the stored float outputs. Points
// outside the interior or with a non-finite value (use false) contribute nothing: the lane
// fold replaces their inputs by zero before any product is formed, the per-lane sums skip
// them, so no NaN reaches a sum.
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
    // S_ij counted for (i,j) and (j,i): G_ii on the diagonal, G_ij + G_ji off it (exact)
    const double m = (ii[s] == jj[s]) ? (double)P.G[ii[s]][ii[s]]
                                      : (double)P.G[ii[s]][jj[s]] + (double)P.G[jj[s]][ii[s]];
    pi -= (double)tau[s] * m;
    pigm -= (double)P.tgm[s] * m;
    pism -= (double)P.tsm[s] * m;
  }
  const double ke = 0.5 * (double)rb *
                    ((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
  // Every input reaches one of these four sums through a product (a NaN or an infinity stays
  // non-finite, also when multiplied by zero), and sums of products of float32 values cannot
  // overflow in double, so one test on their total covers the point.
  const bool fin = isfinite(pi + pigm + pism + ke);
  const bool use = valid && fin;
  I.bad = valid && !fin;
  I.use = use;
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

// The inputs of a point that is not used replaced by zero.
__device__ __forceinline__ StatIn stat_masked(const StatIn& I) {
  StatIn J = I;
  const bool use = I.use;
  J.rb = use ? I.rb : 0.f;
  J.ke = use ? I.ke : 0.0;
  J.pi = use ? I.pi : 0.0;
  J.pigm = use ? I.pigm : 0.0;
  J.pism = use ? I.pism : 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    J.tau[s] = use ? I.tau[s] : 0.f;
    J.tgm[s] = use ? I.tgm[s] : 0.f;
  }
  return J;
}

// Contribution to slot s (s is a compile-time constant after unrolling).
__device__ __forceinline__ double stat_val(const StatIn& I, int s) {
  if (s == S_N) return I.use ? 1.0 : 0.0;
  if (s == S_NONFINITE) return I.bad ? 1.0 : 0.0;
  if (s == S_RHO) return (double)I.rb;
  if (s == S_KE) return I.ke;
  if (s == S_PI) return I.pi;
  if (s == S_PIGM) return I.pigm;
  if (s == S_PISM) return I.pism;
  if (s == S_PI2) return I.pi * I.pi;
  if (s == S_PIGM2) return I.pigm * I.pigm;
  if (s == S_PIPIGM) return I.pi * I.pigm;
  if (s >= S_TAU && s < S_TAU + 6) return (double)I.tau[s - S_TAU];
  if (s >= S_TGM && s < S_TGM + 6) return (double)I.tgm[s - S_TGM];
  if (s >= S_TAU2 && s < S_TAU2 + 6) {
    const double t = I.tau[s - S_TAU2];
    return t * t;
  }
  if (s >= S_TGM2 && s < S_TGM2 + 6) {
    const double g = I.tgm[s - S_TGM2];
    return g * g;
  }
  const double t = I.tau[s - S_TAUTGM], g = I.tgm[s - S_TAUTGM];
  return t * g;  // S_TAUTGM
}

// Smagorinsky dissipation -tau^SM_ij S_ij of a point without forming tau^SM: with
// tau^SM = -2 rho_bar c |S| S^d and S^d : S = S : S - (tr S)^2 / 3 it is
// 2 rho_bar c |S| (S : S - (tr S)^2 / 3), |S| = sqrt(2 S : S); smag_coef holds c = (C_s Delta)^2.
__device__ __forceinline__ float smag_dissipation(const WidthArgs& W, float rb,
                                                  const float (&G)[3][3]) {
  // no implicit multiply-add contraction: the rounding must not depend on what the compiler
  // fuses in the surrounding kernel (the statistics of every kernel instance agree bit for bit)
#pragma clang fp contract(off)
  const float sxy = 0.5f * (G[0][1] + G[1][0]), sxz = 0.5f * (G[0][2] + G[2][0]);
  const float syz = 0.5f * (G[1][2] + G[2][1]);
  const float tr = G[0][0] + G[1][1] + G[2][2];
  float ss = G[0][0] * G[0][0] + G[1][1] * G[1][1] + G[2][2] * G[2][2];
  ss = fmaf(2.f * sxy, sxy, fmaf(2.f * sxz, sxz, fmaf(2.f * syz, syz, ss)));
  const float smag = __builtin_amdgcn_sqrtf(2.f * ss);
  return 2.f * rb * W.smag_coef * smag * fmaf(-(1.f / 3.f) * tr, tr, ss);
}

// ---- statistics of the gradient epilogue: float32 sums per lane, FP64 per wave
//
// A point's 40 contributions (slots of StatSlot) are formed in float32 and added to the
// thread's float32 partial sums. Every kStatFlush points the partials of the whole wave are
// folded in a fixed order into one FP64 total per slot, which one lane of the wave adds to
// its FP64 accumulator; the partials start again from zero. So FP64 is used only where sums
// run over many points, and a partial holds at most kStatFlush points: its rounding error is
// below (kStatFlush + 2) 2^-24 times the sum of the magnitudes of its contributions (the
// products of two float32 values are rounded once, the additions once each). Points that are
// not used contribute nothing; a point with a non-finite contribution (a NaN or infinite
// input, or a product beyond the float32 range) is counted in S_NONFINITE and left out.
constexpr int kStatFlush = 16;

struct StatPart {
  float s[kNStat];
};

__device__ __forceinline__ void stat_zero(StatPart& a) {
#pragma unroll
  for (int k = 0; k < kNStat; ++k) a.s[k] = 0.f;
}

// Adds one point: filtered density rb, Favre velocity u, tau and tau^GM (xx xy xz yy yz zz),
// the gradient G and the Smagorinsky dissipation pism.
__device__ __forceinline__ void stat_point(float rb, const float (&u)[3], const float (&tau)[6],
                                           const float (&G)[3][3], const float (&tgm)[6],
                                           float pism, bool valid, StatPart& a) {
#pragma clang fp contract(off)  // as in smag_dissipation
  // S_ij counted for (i, j) and (j, i): G_ii on the diagonal, G_ij + G_ji off it
  const float m[6] = {G[0][0], G[0][1] + G[1][0], G[0][2] + G[2][0],
                      G[1][1], G[1][2] + G[2][1], G[2][2]};
  float pi = 0.f, pigm = 0.f, t2 = 0.f, g2 = 0.f;
  float tt[6], gg[6], tg[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    pi = fmaf(-tau[s], m[s], pi);
    pigm = fmaf(-tgm[s], m[s], pigm);
    tt[s] = tau[s] * tau[s];
    gg[s] = tgm[s] * tgm[s];
    tg[s] = tau[s] * tgm[s];
    t2 += tt[s];
    g2 += gg[s];
  }
  const float ke = 0.5f * rb * fmaf(u[0], u[0], fmaf(u[1], u[1], u[2] * u[2]));
  // every input reaches one of these through a product, and the squares cover the products
  // of the correlation sums, so one test on the total covers the point
  const bool fin = isfinite(pi + pigm + pism + ke + t2 + g2 + pi * pi + pigm * pigm);
  if (valid && fin) {
    a.s[S_N] += 1.f;
    a.s[S_RHO] += rb;
    a.s[S_KE] += ke;
    a.s[S_PI] += pi;
    a.s[S_PIGM] += pigm;
    a.s[S_PISM] += pism;
    a.s[S_PI2] = fmaf(pi, pi, a.s[S_PI2]);
    a.s[S_PIGM2] = fmaf(pigm, pigm, a.s[S_PIGM2]);
    a.s[S_PIPIGM] = fmaf(pi, pigm, a.s[S_PIPIGM]);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      a.s[S_TAU + s] += tau[s];
      a.s[S_TGM + s] += tgm[s];
      a.s[S_TAU2 + s] += tt[s];
      a.s[S_TGM2 + s] += gg[s];
      a.s[S_TAUTGM + s] += tg[s];
    }
  } else if (valid) {
    a.s[S_NONFINITE] += 1.f;
  }
}

// ---- FP64 statistics folded over the wave with lane swaps
//
// Per-lane values of 40 slots are reduced over the wave in two swap-and-add steps that use
// the row-swap permutes of gfx950 (lanes L and L ^ 32, then L and L ^ 16): afterwards lane
// L holds the 4-lane sums of slots 10 * (2 * b5 + b4) + k, k < 10, where b5 and b4 are bits
// 5 and 4 of L. These ten values are accumulated per lane across every point the thread
// visits, and the remaining 16-lane reduction runs once, when the block writes its record.
// The order of every addition is fixed, so the totals do not depend on timing. All 64 lanes
// of the wave must be active wherever these helpers run.

struct StatAcc {
  double s[10];
};

__device__ __forceinline__ void stat_zero(StatAcc& a) {
#pragma unroll
  for (int k = 0; k < 10; ++k) a.s[k] = 0.0;
}

// x from this lane and the partner's copy of the value it does not keep: lanes in the lower
// half of each pair keep x (their own plus the partner's x), the upper half keep y.
template <int Span>
__device__ __forceinline__ double swap_add(double x, double y) {
  const unsigned long long xb = __double_as_longlong(x), yb = __double_as_longlong(y);
  const unsigned xl = (unsigned)xb, xh = (unsigned)(xb >> 32);
  const unsigned yl = (unsigned)yb, yh = (unsigned)(yb >> 32);
  unsigned nxl, nxh, nyl, nyh;
  if constexpr (Span == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    nxl = lo[0], nyl = lo[1], nxh = hi[0], nyh = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    nxl = lo[0], nyl = lo[1], nxh = hi[0], nyh = hi[1];
  }
  const double nx = __longlong_as_double((long long)(((unsigned long long)nxh << 32) | nxl));
  const double ny = __longlong_as_double((long long)(((unsigned long long)nyh << 32) | nyl));
  return nx + ny;
}

// Slots are folded in the order k, k + 20 (first swap) and k, k + 10 (second swap), one
// accumulator at a time, so that only a few contributions are live at once. val(s) gives
// slot s (0..39) of the lane's point.
template <class V>
__device__ __forceinline__ void stat_fold(const V& val, StatAcc& a) {
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const double lo = swap_add<32>(val(k), val(k + 20));
    const double hi = swap_add<32>(val(k + 10), val(k + 30));
    a.s[k] += swap_add<16>(lo, hi);
  }
}

__device__ __forceinline__ void stat_add(const StatIn& I, StatAcc& a) {
  const StatIn J = stat_masked(I);  // every lane takes part in the fold
  stat_fold([&](int s) { return stat_val(J, s); }, a);
}

// Wave totals: the 16-lane reduction of every accumulator, then lanes 0, 16, 32 and 48
// write their ten slots of the wave's 40-slot record.
__device__ __forceinline__ void write_stats(double* part, const StatAcc& a) {
  const int lane = __lane_id();
  double t[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    double r = a.s[k];
    r += __shfl_xor(r, 8);
    r += __shfl_xor(r, 4);
    r += __shfl_xor(r, 2);
    r += __shfl_xor(r, 1);
    t[k] = r;
  }
  if ((lane & 15) == 0) {
    const int g = 2 * (lane >> 5) + ((lane >> 4) & 1);
#pragma unroll
    for (int k = 0; k < 10; ++k) part[10 * g + k] = t[k];
  }
}

// ---- float32 statistics folded over the wave per point (kernels short of registers)
//
// The same float32 contributions as stat_point, folded over the wave at every point with the
// two lane swaps of stat_fold (in float32: one permute and one add per swap), into ten float32
// sums per lane (lane L then holds 4-lane sums of slots 10 * (2 b5 + b4) + k); every
// kStatFlush points these are added to the lane's ten FP64 sums (StatAcc) and cleared, and
// write_stats finishes the reduction once per block. A float32 sum then spans at most
// 4 kStatFlush contributions: (2 + kStatFlush + 7) 2^-24 of the sum of its terms' magnitudes.
// Costs 30 registers per lane where stat_point's sums cost 42, and about 2.5 times fewer
// instructions per point than the exact FP64 fold. All 64 lanes must be active.
struct StatFold32 {
  float s[10];
};

__device__ __forceinline__ void stat_zero(StatFold32& a) {
#pragma unroll
  for (int k = 0; k < 10; ++k) a.s[k] = 0.f;
}

template <int Span>
__device__ __forceinline__ float swap_add32(float x, float y) {
  const unsigned xb = __float_as_uint(x), yb = __float_as_uint(y);
  unsigned nx, ny;
  if constexpr (Span == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(xb, yb, false, false);
    nx = r[0], ny = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(xb, yb, false, false);
    nx = r[0], ny = r[1];
  }
  return __uint_as_float(nx) + __uint_as_float(ny);
}

__device__ __forceinline__ void stat_point_fold(float rb, const float (&u)[3], const float (&tau)[6],
                                                const float (&G)[3][3], const float (&tgm)[6],
                                                float pism, bool valid, StatFold32& a) {
#pragma clang fp contract(off)  // as in smag_dissipation
  const float m0[6] = {G[0][0], G[0][1] + G[1][0], G[0][2] + G[2][0],
                       G[1][1], G[1][2] + G[2][1], G[2][2]};
  float pi = 0.f, pigm = 0.f, t2 = 0.f, g2 = 0.f;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    pi = fmaf(-tau[s], m0[s], pi);
    pigm = fmaf(-tgm[s], m0[s], pigm);
    t2 = fmaf(tau[s], tau[s], t2);
    g2 = fmaf(tgm[s], tgm[s], g2);
  }
  const float ke0 = 0.5f * rb * fmaf(u[0], u[0], fmaf(u[1], u[1], u[2] * u[2]));
  const bool fin = isfinite(pi + pigm + pism + ke0 + t2 + g2 + pi * pi + pigm * pigm);
  const bool use = valid && fin;
  // the inputs of a point that is not used become zero, so that all its sums are zero
  const float r = use ? rb : 0.f;
  const float ke = use ? ke0 : 0.f, ps = use ? pism : 0.f, p1 = use ? pi : 0.f;
  const float p2 = use ? pigm : 0.f;
  float t[6], g[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    t[s] = use ? tau[s] : 0.f;
    g[s] = use ? tgm[s] : 0.f;
  }
  auto val = [&](int k) -> float {
    if (k == S_N) return use ? 1.f : 0.f;
    if (k == S_NONFINITE) return (valid && !fin) ? 1.f : 0.f;
    if (k == S_RHO) return r;
    if (k == S_KE) return ke;
    if (k == S_PI) return p1;
    if (k == S_PIGM) return p2;
    if (k == S_PISM) return ps;
    if (k == S_PI2) return p1 * p1;
    if (k == S_PIGM2) return p2 * p2;
    if (k == S_PIPIGM) return p1 * p2;
    if (k >= S_TAU && k < S_TAU + 6) return t[k - S_TAU];
    if (k >= S_TGM && k < S_TGM + 6) return g[k - S_TGM];
    if (k >= S_TAU2 && k < S_TAU2 + 6) return t[k - S_TAU2] * t[k - S_TAU2];
    if (k >= S_TGM2 && k < S_TGM2 + 6) return g[k - S_TGM2] * g[k - S_TGM2];
    return t[k - S_TAUTGM] * g[k - S_TAUTGM];  // S_TAUTGM
  };
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const float lo = swap_add32<32>(val(k), val(k + 20));
    const float hi = swap_add32<32>(val(k + 10), val(k + 30));
    a.s[k] += swap_add32<16>(lo, hi);
  }
}

// Adds the ten float32 lane sums to the FP64 ones and clears them.
__device__ __forceinline__ void stat_flush32(StatFold32& a, StatAcc& acc) {
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    acc.s[k] += (double)a.s[k];
    a.s[k] = 0.f;
  }
}

// Slot whose wave total lane `lane` holds after stat_flush, or -1 (24 lanes hold none).
__device__ __forceinline__ int stat_lane_slot(int lane) {
  const int g = 2 * ((lane >> 5) & 1) + ((lane >> 4) & 1);
  const int base = (lane & 8) ? 5 : 0;
  const int b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
  const int pos = b2 ? (b1 ? -1 : 3 + b0) : (b1 ? (b0 ? -1 : 2) : b0);
  return pos < 0 ? -1 : 10 * g + base + pos;
}

// Folds the float32 partials of the wave into one FP64 total per slot and adds it to the
// FP64 accumulator of the lane stat_lane_slot assigns to that slot; clears the partials.
// The fold: lane swaps across the halves and rows of the wave as in stat_fold (lane L then
// holds ten 4-lane sums), then within each 16-lane row four exchanges that each halve the
// values a lane keeps (10 -> 5 -> 3 -> 2 -> 1; a lane that keeps an odd count pads with zero).
// The order of every addition is fixed. All 64 lanes of the wave must be active.
__device__ __forceinline__ void stat_flush(StatPart& a, double& acc) {
  const int lane = __lane_id();
  double t[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const double lo = swap_add<32>((double)a.s[k], (double)a.s[k + 20]);
    const double hi = swap_add<32>((double)a.s[k + 10], (double)a.s[k + 30]);
    t[k] = swap_add<16>(lo, hi);
  }
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  double v5[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double keep = b3 ? t[i + 5] : t[i];
    const double send = b3 ? t[i] : t[i + 5];
    v5[i] = keep + __shfl_xor(send, 8);
  }
  double v3[3];
  v3[0] = (b2 ? v5[3] : v5[0]) + __shfl_xor(b2 ? v5[0] : v5[3], 4);
  v3[1] = (b2 ? v5[4] : v5[1]) + __shfl_xor(b2 ? v5[1] : v5[4], 4);
  v3[2] = (b2 ? 0.0 : v5[2]) + __shfl_xor(b2 ? v5[2] : 0.0, 4);
  double v2[2];
  v2[0] = (b1 ? v3[2] : v3[0]) + __shfl_xor(b1 ? v3[0] : v3[2], 2);
  v2[1] = (b1 ? 0.0 : v3[1]) + __shfl_xor(b1 ? v3[1] : 0.0, 2);
  acc += (b0 ? v2[1] : v2[0]) + __shfl_xor(b0 ? v2[0] : v2[1], 1);
  stat_zero(a);
}

// The wave's 40-slot record from the lane accumulators of stat_flush.
__device__ __forceinline__ void write_stat_record(double* part, double acc) {
  const int slot = stat_lane_slot(__lane_id());
  if (slot >= 0) part[slot] = acc;
}

// Whether the gradient epilogue has anything to produce (uniform over the launch).
__device__ __forceinline__ bool needs_gradient(const WidthArgs& W) {
  return W.partials || W.grad || W.tau_gm || W.tau_smag || W.k_sgs || W.nu_t || W.omega_t ||
         W.q_crit;
}

// Stores of one point's requested outputs; at(base, c) gives the address of component c of
// the point in the field that starts at base.
template <class At>
__device__ __forceinline__ void store_point_at(const WidthArgs& W, const PointOut& P, At&& at) {
  if (W.grad) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) *at(W.grad, i * 3 + j) = P.G[i][j];
  }
  if (W.tau_gm) {
#pragma unroll
    for (int s = 0; s < 6; ++s) *at(W.tau_gm, s) = P.tgm[s];
  }
  if (W.tau_smag) {
#pragma unroll
    for (int s = 0; s < 6; ++s) *at(W.tau_smag, s) = P.tsm[s];
  }
  if (W.k_sgs) *at(W.k_sgs, 0) = P.ksgs;
  if (W.nu_t) *at(W.nu_t, 0) = P.nut;
  if (W.omega_t) *at(W.omega_t, 0) = P.omt;
  if (W.q_crit) {  // (|W|^2 - |S|^2) / 2 = -G_ij G_ji / 2
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) q = fmaf(P.G[i][j], P.G[j][i], q);
    *at(W.q_crit, 0) = -0.5f * q;
  }
}

__device__ __forceinline__ void store_point(const WidthArgs& W, int64_t g, int64_t ntot,
                                            const PointOut& P) {
  store_point_at(W, P, [&](float* base, int c) { return base + c * ntot + g; });
}

// Address of component c of a point in the field at base: plane offset zb (elements, uniform)
// plus the point's byte offset o within the plane (below 2^32), the form that compiles to a
// scalar base and a 32-bit vector offset. The component's offset is made opaque so that the
// compiler does not share one 64-bit vector address between components.
__device__ __forceinline__ float* plane_addr(float* base, int c, int64_t ntot, int64_t zb,
                                             uint32_t o) {
  int64_t off = (c * ntot + zb) * (int64_t)sizeof(float);
  __asm__ volatile("" : "+s"(off));
  return reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off + o);
}

// Tile t of a z-chunk -> tile coordinates. With strip_w > 0 tiles are numbered in vertical
// strips strip_w tiles wide, row by row inside a strip, so that the workgroups an XCD runs at
// the same time cover a compact patch and share their halos in L2 (tall tiles); otherwise in
// plain rows.
__device__ __forceinline__ void tile_coords(const FilterArgs& A, int t, int& tx, int& ty) {
  const int sw = A.strip_w;
  if (sw <= 0 || sw >= A.ntx) {
    tx = t % A.ntx;
    ty = t / A.ntx;
    return;
  }
  const int full = A.ntx / sw;  // strips of full width
  const int per_strip = sw * A.nty;
  if (t < full * per_strip) {
    const int s = t / per_strip, r = t % per_strip;
    tx = s * sw + r % sw;
    ty = r / sw;
  } else {
    const int w = A.ntx - full * sw;  // the last, narrower strip
    const int r = t - full * per_strip;
    tx = full * sw + r % w;
    ty = r / w;
  }
}

// XCD-aware block mapping: consecutive block ids go to different XCDs, so block L is
// placed on XCD L % 8. Every XCD gets a contiguous band of (z-chunk, tile) items, so the
// input planes that neighbouring tiles share are read through one L2.
__device__ __forceinline__ bool map_block(const FilterArgs& A, int& item) {
  const int L = blockIdx.x;
  const int xcd = L & 7;
  const int j = L >> 3;
  item = xcd * A.tiles_per_xcd + j;
  return j < A.tiles_per_xcd && item < A.ntiles * A.nzc;
}

}  // namespace dev
}  // namespace kcf
