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
__device__ __forceinline__ void gm_closure(const WidthArgs& W, float rb, PointOut& P) {
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
      P.tgm[s] = c * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
    }
  } else {
    __asm__ volatile("");
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int i = ii[s], j = jj[s];
      P.tgm[s] = c * (G[0][i] * G[0][j] + G[1][i] * G[1][j] + G[2][i] * G[2][j]);
    }
  }
}

// Smagorinsky -2 rho_bar (C_s Delta)^2 |S| S^d; smag_coef holds (C_s Delta)^2.
__device__ __forceinline__ void smag_closure(const WidthArgs& W, float rb, PointOut& P) {
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
    for (int j = 0; j < 3; ++j) ss += S[i][j] * S[i][j];
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
__device__ __forceinline__ void point_closures(const WidthArgs& W, float rb, const float (&tau)[6],
                                               PointOut& P) {
  const bool stats = W.partials != nullptr;  // the statistics need both closures
#pragma unroll
  for (int s = 0; s < 6; ++s) P.tgm[s] = P.tsm[s] = 0.f;
  P.ksgs = P.nut = P.omt = 0.f;
  if (stats || W.tau_gm) {  // uniform
    gm_closure(W, rb, P);
  }
  if (stats || W.tau_smag) {  // uniform
    smag_closure(W, rb, P);
  }
  if (W.k_sgs || W.nu_t || W.omega_t) {  // uniform; only stored, never reduced
    const float rref = W.ksgs_rho_ref ? 1.f : rb;
    P.ksgs = fabsf(tau[0] + tau[3] + tau[5]) / (2.f * rref);
    P.nut = W.cnu_delta * sqrtf(P.ksgs);
    P.omt = 1.f / (fmaxf(W.nu_mol, P.nut) * W.inv_theta + W.half_dt);
  }
}

// What one point contributes to the FP64 sums. Products of two float32 values are exact in
// double, so every contribution is formed in double from the stored float outputs. Points
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

// ---- FP64 statistics: per-point contributions folded over the wave with lane swaps
//
// A point's 40 contributions are reduced over the wave in two swap-and-add steps that use
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

// Per-lane sums of all 40 slots, with no lane swaps per point: for kernels whose register
// budget has room for them (80 registers). The wave reduction at the end applies the same
// fixed-order fold to the lane sums.
struct StatLane {
  double s[kNStat];
};

__device__ __forceinline__ void stat_zero(StatLane& a) {
#pragma unroll
  for (int k = 0; k < kNStat; ++k) a.s[k] = 0.0;
}

__device__ __forceinline__ void stat_add(const StatIn& I, StatLane& a) {
  if (I.use) {  // lanes of points not used skip the additions
#pragma unroll
    for (int k = 0; k < kNStat; ++k)
      if (k != S_NONFINITE) a.s[k] += stat_val(I, k);
  }
  if (I.bad) a.s[S_NONFINITE] += 1.0;
}

__device__ __forceinline__ void write_stats(double* part, const StatLane& a) {
  StatAcc f;
  stat_zero(f);
  stat_fold([&](int s) { return a.s[s]; }, f);
  write_stats(part, f);
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
