// Filtered monomials rho u_x^a u_y^b u_z^c (and rho theta, rho S_ij) and the SGS quantities
// built from them, as two streaming kernels per z slab shared by three quantity sets:
//
//   carrier  the a priori SGS carrier of the D3Q27 lattice, f_sgs,i = bar(f0_i(rho, u)) -
//            f0_i(rho_bar, ut) (eqs. f0bar and fsgs_def) with the product equilibrium of
//            eq. discrete_equilibrium, and the second-order Hermite reconstruction of the KC-MP
//            closure from tau (eq. f_sgs_KCMP);
//   moment3  the third-order SGS moment m3_ijk = bar(rho u_i u_j u_k) - rho_bar ut_i ut_j ut_k
//            (the order-3 term of eq. f_sgs_hermite) and the Favre temperature
//            bar(rho theta) / rho_bar (definition after eq. f0resolved);
//   kc-mp    bar(rho S_ij) of the input strain, for the a priori KC-MP estimate of the SGS
//            second moment and the KC relaxation-rate field (App. "Operational
//            implementation of KC-MP", eq. omega_sgs_operational).
//
// Carrier. With velocities in units of sqrt(theta_R) and xh = xi / sqrt(theta_R) in
// {0, +-sqrt3}, the equilibrium is w_i rho prod_a (P_0 + P_1(xh_ia) u_a + P_2(xh_ia) u_a^2)
// with the D1Q3 Hermite polynomials P_0 = 1, P_1 = xh, P_2 = (xh^2 - 1)/2. The filter is
// linear, hence
//   f_sgs,i = w_i sum_abc P_a(xh_ix) P_b(xh_iy) P_c(xh_iz) D_abc,
//   D_abc   = bar(rho u_x^a u_y^b u_z^c) - rho_bar ut_x^a ut_y^b ut_z^c,     a, b, c in 0..2:
// 27 filtered monomials replace 27 filtered populations, and the subtraction happens where
// the cancellation is smallest. D vanishes at total degree <= 1 (definition of ut); the
// degree-2 D are tau, whose terms alone form the reconstruction f_h2. The total degree is the
// Hermite order of a term (eq. f_sgs_hermite on the tensor-product lattice).
//
//   k_*_z   one thread per (x, y) column and ZT planes: the set's products of the input,
//           one group of up to nine at a time (k_kc_z: the six rho S_ij, with the x and y
//           neighbours of each point), filtered along z over a register window of the input
//           planes and written to the slab buffer [planes][quantities][ny][nx] (the
//           quantities of a plane together: an x-y tile then reads one compact region);
//   k_*_xy  one workgroup per (tile of 256 points, run of eight planes), XCD-banded: per plane,
//           the quantities of the tile and its halo staged in LDS G at a time, filtered along
//           x and y in place, each thread keeping its point's filtered values; then the set's
//           epilogue (stores and statistics: a point's values in FP32, their sums over points
//           in FP64; one record per workgroup, or per wave for the 40 folded KC-MP sums).
// T is the type of the products, of both filter passes and of the slab buffer (double for
// narrow widths, as in the Favre path); the differences against the Favre fields are formed
// in T, what follows them in FP32.
#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

constexpr int kZB = 256;  // threads of the z kernels
constexpr int kXT = 256;  // threads of the x-y kernels (one per tile point)
constexpr int kLook = 3;  // input planes in flight ahead of the FMAs in the z kernels
constexpr int kXZ = 8;    // planes per workgroup of the x-y kernels

template <typename T>
constexpr int cz_planes() { return sizeof(T) == 8 ? 8 : 16; }

template <typename T>
__device__ __forceinline__ const T* cweights(const MonoArgs& A);
template <>
__device__ __forceinline__ const float* cweights<float>(const MonoArgs& A) { return A.w; }
template <>
__device__ __forceinline__ const double* cweights<double>(const MonoArgs& A) { return A.wd; }

// Statistics of the carrier and third-order sets: NS FP64 sums per thread over its points,
// reduced over the wave and the workgroup in a fixed order into one record per workgroup.
template <int NS>
struct ArrayAcc {
  double v[NS];
  static constexpr int kRecords = 1;
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = 0.0;
  }
  // every thread of the workgroup calls this
  __device__ void write(double* part, double* smem, int item) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v[k] += __shfl_xor(v[k], d);
    }
    if (__lane_id() == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) smem[(tid >> 6) * NS + k] = v[k];
    }
    __syncthreads();
    if (tid < NS) {
      double a = 0;
#pragma unroll
      for (int wv = 0; wv < kXT / 64; ++wv) a += smem[wv * NS + tid];
      part[(int64_t)item * NS + tid] = a;
    }
  }
};

// ---------------------------------------------------------------- the SGS carrier
// Monomial m = a + 3 b + 9 c stands for rho u_x^a u_y^b u_z^c.
__host__ __device__ constexpr int mono_deg(int m) { return m % 3 + (m / 3) % 3 + m / 9; }
// weighted norm n_a n_b n_c of the basis term, n = (1, 1, 1/2)
__host__ __device__ constexpr double mono_norm(int m) {
  return (m % 3 == 2 ? 0.5 : 1.0) * ((m / 3) % 3 == 2 ? 0.5 : 1.0) * (m / 9 == 2 ? 0.5 : 1.0);
}

// One direction of the Hermite synthesis, in place: coefficients (d_0, d_1, d_2) of P_0, P_1,
// P_2 to the values at xh = -sqrt3, 0, +sqrt3, times the D1Q3 weights 1/6, 2/3, 1/6.
__device__ __forceinline__ void synth1(float& v0, float& v1, float& v2) {
  const float s = v0 + v2;
  const float t = 1.7320508075688772f * v1;
  const float mid = v0 - 0.5f * v2;
  v0 = (s - t) * (float)(1.0 / 6.0);
  v1 = mid * (float)(2.0 / 3.0);
  v2 = (s + t) * (float)(1.0 / 6.0);
}

// d[a + 3 b + 9 c] = D_abc in, d[ix + 3 iy + 9 iz] = f of the population (ix - 1, iy - 1,
// iz - 1) out: z, then y, then x.
__device__ __forceinline__ void synth(float (&d)[27]) {
#pragma unroll
  for (int ab = 0; ab < 9; ++ab) synth1(d[ab], d[ab + 9], d[ab + 18]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int iz = 0; iz < 3; ++iz) synth1(d[a + 9 * iz], d[a + 3 + 9 * iz], d[a + 6 + 9 * iz]);
#pragma unroll
  for (int yz = 0; yz < 9; ++yz) synth1(d[3 * yz], d[3 * yz + 1], d[3 * yz + 2]);
}

struct CarrierSet {
  static constexpr int kQ = 27;      // quantities: monomial m = a + 3 b + 9 c
  static constexpr int kGroups = 3;  // z-pass groups: one power c of u_z each
  static constexpr int kGS = 9;      // products per group
  static constexpr int kStat = kCStat;
  static constexpr bool kStaticGroups = false;  // one code copy, group index at run time
  static constexpr bool kOptionalLast = false;  // every quantity always filtered

  // products of group g: p[a + 3 b] = rho u_z^g u_y^b u_x^a
  template <int GRP, typename T>
  __device__ static void products(int g, T r, T vx, T vy, T vz, T, T (&p)[kGS]) {
    T b0 = r;
    if (g >= 1) b0 = b0 * vz;
    if (g == 2) b0 = b0 * vz;
    T yb = b0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (b > 0) yb = yb * vy;
      p[3 * b] = yb;
      p[3 * b + 1] = yb * vx;
      p[3 * b + 2] = p[3 * b + 1] * vx;
    }
  }

  using Acc = ArrayAcc<kStat>;

  template <typename T>
  __device__ static void epilogue(const MonoArgs& A, const T (&M)[kQ], bool valid, int64_t g,
                                  Acc& acc) {
    const T rb = M[0];
    const T ri = (T)1 / rb;
    const T uv[3] = {M[1] * ri, M[3] * ri, M[9] * ri};
    float D[27];
    float herm[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // weighted energies of Hermite orders 2..6
#pragma unroll
    for (int m = 0; m < 27; ++m) {
      if (mono_deg(m) <= 1) {
        D[m] = 0.f;
        continue;
      }
      T p = rb;
      const int e[3] = {m % 3, (m / 3) % 3, m / 9};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (e[a] >= 1) p = p * uv[a];
        if (e[a] >= 2) p = p * uv[a];
      }
      D[m] = (float)(M[m] - p);
      herm[mono_deg(m) - 2] = fmaf((float)mono_norm(m) * D[m], D[m], herm[mono_deg(m) - 2]);
    }
    // tau = degree-2 D: xx xy xz yy yz zz
    const float txx = D[2], txy = D[4], txz = D[10], tyy = D[6], tyz = D[12], tzz = D[18];
    synth(D);
    float sf2 = 0.f, serr = 0.f;
    // population i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1)
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
#pragma unroll
      for (int iy = 0; iy < 3; ++iy) {
#pragma unroll
        for (int iz = 0; iz < 3; ++iz) {
          const int cx = ix - 1, cy = iy - 1, cz = iz - 1;
          // f_h2 = w_i (sum_a P_2(xh_a) tau_aa + sum_{a<b} xh_a xh_b tau_ab),
          // xh_a xh_b = 3 c_a c_b
          float h = (cx ? 1.f : -0.5f) * txx + (cy ? 1.f : -0.5f) * tyy +
                    (cz ? 1.f : -0.5f) * tzz;
          if (cx && cy) h += (float)(3 * cx * cy) * txy;
          if (cx && cz) h += (float)(3 * cx * cz) * txz;
          if (cy && cz) h += (float)(3 * cy * cz) * tyz;
          const float wi = (float)((cx ? 1.0 / 6.0 : 2.0 / 3.0) * (cy ? 1.0 / 6.0 : 2.0 / 3.0) *
                                   (cz ? 1.0 / 6.0 : 2.0 / 3.0));
          const float fh = wi * h;
          const float fs = D[ix + 3 * iy + 9 * iz];
          const int i = 9 * ix + 3 * iy + iz;
          if (valid) {
            if (A.f_sgs) A.f_sgs[(int64_t)i * A.ntot + g] = fs;
            if (A.f_h2) A.f_h2[(int64_t)i * A.ntot + g] = fh;
          }
          const float e = fs - fh;
          sf2 = fmaf(fs, fs, sf2);
          serr = fmaf(e, e, serr);
        }
      }
    }
    const bool finite = isfinite(sf2 + serr + herm[0] + herm[1] + herm[2] + herm[3] + herm[4]);
    const bool use = valid && finite;
    acc.v[C_N] += use ? 1.0 : 0.0;
    acc.v[C_F2] += use ? (double)sf2 : 0.0;
    acc.v[C_ERR2] += use ? (double)serr : 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) acc.v[C_HERM + k] += use ? (double)herm[k] : 0.0;
    acc.v[C_NONFINITE] += valid && !finite ? 1.0 : 0.0;
  }
};

// ---------------------------------------------------------------- third-order moment
// Quantities: 0 rho, 1..3 rho u_x, rho u_y, rho u_z, 4..13 rho u_i u_j u_k in the order
// xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz, 14 rho theta (filtered only with a temperature).
struct Moment3Set {
  static constexpr int kQ = 15;
  static constexpr int kGroups = 2;
  static constexpr int kGS = 8;  // groups of eight (the last slot of the second is unused)
  static constexpr int kStat = kM3Stat;
  static constexpr bool kStaticGroups = true;  // a code copy per group
  static constexpr bool kOptionalLast = true;  // rho theta only with a temperature

  template <int GRP, typename T>
  __device__ static void products(int, T r, T vx, T vy, T vz, T th, T (&p)[kGS]) {
    const T rx = r * vx, ry = r * vy, rz = r * vz;
    if constexpr (GRP == 0) {
      const T rxx = rx * vx;
      p[0] = r;
      p[1] = rx;
      p[2] = ry;
      p[3] = rz;
      p[4] = rxx * vx;        // xxx
      p[5] = rxx * vy;        // xxy
      p[6] = rxx * vz;        // xxz
      p[7] = (rx * vy) * vy;  // xyy
    } else {
      const T ryy = ry * vy, rzz = rz * vz;
      p[0] = (rx * vy) * vz;  // xyz
      p[1] = rx * vz * vz;    // xzz
      p[2] = ryy * vy;        // yyy
      p[3] = ryy * vz;        // yyz
      p[4] = ry * vz * vz;    // yzz
      p[5] = rzz * vz;        // zzz
      p[6] = r * th;          // rho theta
      p[7] = (T)0;
    }
  }

  using Acc = ArrayAcc<kStat>;

  template <typename T>
  __device__ static void epilogue(const MonoArgs& A, const T (&M)[kQ], bool valid, int64_t g,
                                  Acc& acc) {
    const T rb = M[0];
    const T ri = (T)1 / rb;
    const T uv[3] = {M[1] * ri, M[2] * ri, M[3] * ri};
    constexpr int ia[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2};
    constexpr int ja[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2};
    constexpr int ka[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
    float m3[10];
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 10; ++c) {
      m3[c] = (float)(M[4 + c] - ((rb * uv[ia[c]]) * uv[ja[c]]) * uv[ka[c]]);
      s += m3[c];
    }
    const float tt = A.theta ? (float)(M[14] * ri) : 1.f;
    if (valid) {
      if (A.m3) {
#pragma unroll
        for (int c = 0; c < 10; ++c) A.m3[(int64_t)c * A.ntot + g] = m3[c];
      }
      if (A.theta_t) A.theta_t[g] = tt;
    }
    const bool finite = isfinite(s + tt);
    const bool use = valid && finite;
    acc.v[M3_N] += use ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < 10; ++c) {
      acc.v[M3_SUM + c] += use ? (double)m3[c] : 0.0;
      acc.v[M3_SQ + c] += use ? (double)(m3[c] * m3[c]) : 0.0;
    }
    acc.v[M3_THETA] += use ? (double)tt : 0.0;
    acc.v[M3_NONFINITE] += valid && !finite ? 1.0 : 0.0;
  }
};

// ---------------------------------------------------------------- a priori KC-MP
// Quantities: rho S_ij of the input (S from central differences, stored order xx xy xz yy yz
// zz). The z pass is k_kc_z (it needs the neighbours of each point); the epilogue reads the
// stored rho_bar, tau and G of the filter path at its point and forms
//   m_sgs = tau - 2 theta tau_hat (bar(rho S) - rho_bar S_t),   S_t = (G + G^T) / 2,
// the KC-MP estimate of the SGS second moment when the fine-grained state carries its
// Chapman-Enskog part (m_cneq - m_CE, eqs. m_ce_reference and kcmp_operational_msgstrace),
// and the rates of eq. omega_sgs_operational from it and from the exact tau.
struct KcSet {
  static constexpr int kQ = 6;
  static constexpr int kStat = kKcStat;
  static constexpr bool kOptionalLast = false;

  // 40 FP64 sums folded over the wave (the filter path's statistics scheme), one record per
  // wave
  struct Acc {
    StatAcc a;
    static constexpr int kRecords = kXT / 64;
    __device__ void zero() { stat_zero(a); }
    __device__ void write(double* part, double*, int item) {
      write_stats(part + ((int64_t)item * kRecords + (threadIdx.x >> 6)) * kKcStat, a);
    }
  };

  __device__ static void rates(const MonoArgs& A, float tr, float rb, float& k, float& nue,
                               float& om, bool& clip) {
    k = fabsf(tr) / (2.f * (A.rho_ref_one ? 1.f : rb));
    const float nut = A.cnu_delta * sqrtf(k);
    clip = !(nut > A.nu);
    nue = clip ? A.nu : nut;
    om = 1.f / (nue * A.inv_theta + A.half_dt);
  }

  template <typename T>
  __device__ static void epilogue(const MonoArgs& A, const T (&M)[kQ], bool valid, int64_t g,
                                  Acc& acc) {
    const int64_t N = A.ntot;
    const int64_t gc = valid ? g : 0;  // points past the grid edge read a valid point
    const float rb = A.ext[gc];
    float tau[6], G[9];
#pragma unroll
    for (int c = 0; c < 6; ++c) tau[c] = A.ext[(1 + c) * N + gc];
#pragma unroll
    for (int c = 0; c < 9; ++c) G[c] = A.ext[(7 + c) * N + gc];
    const float St[6] = {G[0], 0.5f * (G[1] + G[3]), 0.5f * (G[2] + G[6]), G[4],
                         0.5f * (G[5] + G[7]), G[8]};
    float m[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float d = (float)(M[c] - (T)rb * (T)St[c]);  // bar(rho S) - rho_bar S_t
      m[c] = fmaf(-A.kc_coef, d, tau[c]);
    }
    float k, nue, om, ke, nuee, ome;
    bool clip, clipe;
    rates(A, m[0] + m[3] + m[5], rb, k, nue, om, clip);
    rates(A, tau[0] + tau[3] + tau[5], rb, ke, nuee, ome, clipe);
    if (valid) {
      if (A.m_sgs) {
#pragma unroll
        for (int c = 0; c < 6; ++c) A.m_sgs[c * N + g] = m[c];
      }
      if (A.m_ce) {  // -2 rho_bar theta tau_hat S_t
#pragma unroll
        for (int c = 0; c < 6; ++c) A.m_ce[c * N + g] = -A.kc_coef * rb * St[c];
      }
      if (A.k_sgs) A.k_sgs[g] = k;
      if (A.nu_t_eff) A.nu_t_eff[g] = nue;
      if (A.omega_sgs) A.omega_sgs[g] = om;
    }
    float err = 0.f, nrm = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float wgt = (c == 0 || c == 3 || c == 5) ? 1.f : 2.f;  // off-diagonal pairs twice
      const float e = m[c] - tau[c];
      err = fmaf(wgt * e, e, err);
      nrm = fmaf(wgt * tau[c], tau[c], nrm);
    }
    const bool finite = isfinite(err + nrm + k + om + ke + ome);
    const bool use = valid && finite;
    auto val = [&](int s) -> double {
      if (s == KC_NONFINITE) return valid && !finite ? 1.0 : 0.0;
      if (!use) return 0.0;
      if (s == KC_N) return 1.0;
      if (s >= KC_M && s < KC_M + 6) return (double)m[s - KC_M];
      if (s >= KC_T && s < KC_T + 6) return (double)tau[s - KC_T];
      if (s >= KC_M2 && s < KC_M2 + 6) return (double)m[s - KC_M2] * (double)m[s - KC_M2];
      if (s >= KC_T2 && s < KC_T2 + 6) return (double)tau[s - KC_T2] * (double)tau[s - KC_T2];
      if (s >= KC_MT && s < KC_MT + 6) return (double)m[s - KC_MT] * (double)tau[s - KC_MT];
      if (s == KC_ERR2) return (double)err;
      if (s == KC_TAU2) return (double)nrm;
      if (s == KC_K) return (double)k;
      if (s == KC_KE) return (double)ke;
      if (s == KC_OM) return (double)om;
      if (s == KC_OME) return (double)ome;
      if (s == KC_CLIP) return clip ? 1.0 : 0.0;
      return clipe ? 1.0 : 0.0;  // KC_CLIPE
    };
    stat_fold(val, acc.a);
  }
};

// ---------------------------------------------------------------- the two passes
// Loads of the input plane zz at the column of byte offset cb (< 2^32 since a plane holds at
// most 2^30 points): uniform plane pointers plus a 32-bit per-lane offset. v[4] is the
// temperature (1 without one).
__device__ __forceinline__ void load_inputs(const MonoArgs& A, int zz, uint32_t cb,
                                            float (&v)[5]) {
  const int64_t zo = (int64_t)zz * A.nx * A.ny;
  const char* pr = reinterpret_cast<const char*>(A.rho + zo);
  const char* pu = reinterpret_cast<const char*>(A.u + zo);
  const int64_t nb = A.ntot * (int64_t)sizeof(float);
  v[0] = *reinterpret_cast<const float*>(pr + cb);
  v[1] = *reinterpret_cast<const float*>(pu + cb);
  v[2] = *reinterpret_cast<const float*>(pu + nb + cb);
  v[3] = *reinterpret_cast<const float*>(pu + 2 * nb + cb);
  v[4] = A.theta ? *reinterpret_cast<const float*>(reinterpret_cast<const char*>(A.theta + zo) + cb)
                 : 1.f;
}

// One group of products (GRP >= 0: fixed at compile time; -1: grp at run time) for the ZT
// planes of one column.
template <class S, int R, typename T, int GRP>
__device__ __forceinline__ void z_group(const MonoArgs& A, int grp, int zl0, int nk,
                                        uint32_t cb, T* out) {
  constexpr int ZT = cz_planes<T>();
  constexpr int NJ = ZT + 2 * R;  // input planes z0 - R .. z0 + ZT + R - 1 of the window
  constexpr int GS = S::kGS;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t qstride = plane;
  const int64_t pstride = (int64_t)A.nq * plane;
  const T* w = cweights<T>(A);
  T acc[GS][ZT];
#pragma unroll
  for (int q = 0; q < GS; ++q)
#pragma unroll
    for (int k = 0; k < ZT; ++k) acc[q][k] = (T)0;
  // first window plane, made opaque per group so that the plane offsets are recomputed (two
  // scalar ops a plane) rather than held for all groups
  int zz = wrapi(A.zs + zl0 - R, A.nz);
  __asm__ volatile("" : "+s"(zz));
  float in[kLook][5];  // planes in flight
#pragma unroll
  for (int j = 0; j < kLook; ++j) {
    load_inputs(A, zz, cb, in[j]);
    zz = zz + 1 == A.nz ? 0 : zz + 1;
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const float(&v)[5] = in[j % kLook];
    const T r = (T)v[0], vx = (T)v[1], vy = (T)v[2], vz = (T)v[3], th = (T)v[4];
    if (j + kLook < NJ) {
      load_inputs(A, zz, cb, in[j % kLook]);
      zz = zz + 1 == A.nz ? 0 : zz + 1;
    }
    // keep the later loads below this point: the window is not held in registers
    __builtin_amdgcn_sched_barrier(0);
    T p[GS];
    S::template products<GRP>(grp, r, vx, vy, vz, th, p);
#pragma unroll
    for (int k = 0; k < ZT; ++k) {
      const int t = j - k;  // tap of plane j for output k
      if (t >= 0 && t <= 2 * R) {
#pragma unroll
        for (int q = 0; q < GS; ++q) acc[q][k] = fma(w[t], p[q], acc[q][k]);
      }
    }
  }
  // strides and count opaque here: the store offsets are formed at the stores instead of
  // being held in scalar registers through the window loop
  int64_t qs = qstride, ps = pstride;
  int nkz = nk;
  __asm__ volatile("" : "+s"(qs), "+s"(ps), "+s"(nkz));
#pragma unroll
  for (int q = 0; q < GS; ++q) {
    const int qq = grp * GS + q;
    if (qq < A.nq) {
      T* o = out + (int64_t)qq * qs;
#pragma unroll
      for (int k = 0; k < ZT; ++k)
        if (k < nkz) o[(int64_t)k * ps] = acc[q][k];
    }
  }
}

// Items of the z kernels: (z-chunk, x-block, row), z-chunks fastest, in XCD bands, so that
// the chunks of one column block run back to back through one L2, which then serves the 2R
// window planes neighbouring chunks share and the window the next group of monomials reads
// again (and, for the KC-MP pass, the neighbouring rows). False past the last item.
template <int ZT>
__device__ __forceinline__ bool z_item(const MonoArgs& A, int& x, int& y, int& zl0) {
  const int nzc = (A.nzs + ZT - 1) / ZT, nxb = (A.nx + kZB - 1) / kZB;
  int64_t item;
  if (!xcd_band_item((int64_t)nzc * nxb * A.ny, item)) return false;
  zl0 = (int)(item % nzc) * ZT;
  const int64_t rest = item / nzc;
  x = (int)(rest % nxb) * kZB + threadIdx.x;
  y = (int)(rest / nxb);
  return x < A.nx;
}

template <class S, int R, typename T>
__device__ __forceinline__ void z_pass(const MonoArgs& A) {
  constexpr int ZT = cz_planes<T>();
  int x, y, zl0;  // zl0: first plane of the thread, relative to the slab
  if (!z_item<ZT>(A, x, y, zl0)) return;
  const int nk = min(ZT, A.nzs - zl0);
  const int64_t plane = (int64_t)A.nx * A.ny;
  const uint32_t cb = (uint32_t)(y * A.nx + x) * (uint32_t)sizeof(float);
  T* out = reinterpret_cast<T*>(A.zbuf) + (int64_t)zl0 * A.nq * plane + (int64_t)y * A.nx + x;
  if constexpr (S::kStaticGroups) {
    static_assert(S::kGroups == 2, "static groups are unrolled for two groups");
    z_group<S, R, T, 0>(A, 0, zl0, nk, cb, out);
    z_group<S, R, T, 1>(A, 1, zl0, nk, cb, out);
  } else {
#pragma unroll 1
    for (int grp = 0; grp < S::kGroups; ++grp) z_group<S, R, T, -1>(A, grp, zl0, nk, cb, out);
  }
}

// z pass of the KC-MP set: rho S_ij at every window plane, S from central differences of
// the input velocity (x and y neighbours read at the plane, z neighbours from the column).
// The values of a plane are loaded two planes ahead of their use.
struct KcPlane {
  float r, c[3], xp[3], xm[3], yp[3], ym[3];  // rho; u at the column and its neighbours
};

template <int R, typename T>
__device__ __forceinline__ void z_pass_kc(const MonoArgs& A) {
  constexpr int ZT = cz_planes<T>();
  constexpr int NJ = ZT + 2 * R;  // window planes z0 - R .. z0 + ZT + R - 1
  int x, y, zl0;
  if (!z_item<ZT>(A, x, y, zl0)) return;
  const int nk = min(ZT, A.nzs - zl0);
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t qstride = plane;
  const int64_t pstride = (int64_t)A.nq * plane;
  const int64_t nb = A.ntot * (int64_t)sizeof(float);
  // byte offsets within a plane (< 2^32): the column and its four neighbours
  const uint32_t c0 = (uint32_t)(y * A.nx + x) * 4u;
  const uint32_t cxm = (uint32_t)(y * A.nx + wrapi(x - 1, A.nx)) * 4u;
  const uint32_t cxp = (uint32_t)(y * A.nx + wrapi(x + 1, A.nx)) * 4u;
  const uint32_t cym = (uint32_t)(wrapi(y - 1, A.ny) * A.nx + x) * 4u;
  const uint32_t cyp = (uint32_t)(wrapi(y + 1, A.ny) * A.nx + x) * 4u;
  const T* w = cweights<T>(A);
  const T i2h = (T)A.inv2h;
  auto load = [&](int zz, KcPlane& P) {
    const char* pr = reinterpret_cast<const char*>(A.rho + (int64_t)zz * plane);
    const char* pu = reinterpret_cast<const char*>(A.u + (int64_t)zz * plane);
    P.r = *reinterpret_cast<const float*>(pr + c0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const char* q = pu + i * nb;
      P.c[i] = *reinterpret_cast<const float*>(q + c0);
      P.xp[i] = *reinterpret_cast<const float*>(q + cxp);
      P.xm[i] = *reinterpret_cast<const float*>(q + cxm);
      P.yp[i] = *reinterpret_cast<const float*>(q + cyp);
      P.ym[i] = *reinterpret_cast<const float*>(q + cym);
    }
  };
  T acc[6][ZT];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int k = 0; k < ZT; ++k) acc[q][k] = (T)0;
  // planes j - 1, j, j + 1 in Pm, P0, Pp (shifted along, so that no array is indexed by j)
  int zz = wrapi(A.zs + zl0 - R - 1, A.nz);
  __asm__ volatile("" : "+s"(zz));
  KcPlane Pm, P0, Pp, Pn;
  load(zz, Pm);
  zz = zz + 1 == A.nz ? 0 : zz + 1;
  load(zz, P0);
  zz = zz + 1 == A.nz ? 0 : zz + 1;
  load(zz, Pp);
  zz = zz + 1 == A.nz ? 0 : zz + 1;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    T G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      G[i][0] = ((T)P0.xp[i] - (T)P0.xm[i]) * i2h;
      G[i][1] = ((T)P0.yp[i] - (T)P0.ym[i]) * i2h;
      G[i][2] = ((T)Pp.c[i] - (T)Pm.c[i]) * i2h;
    }
    const T r = (T)P0.r;
    if (j + 2 <= NJ) {  // plane j + 2
      load(zz, Pn);
      zz = zz + 1 == A.nz ? 0 : zz + 1;
    }
    // keep the later loads below this point: the window is not held in registers
    __builtin_amdgcn_sched_barrier(0);
    const T p[6] = {r * G[0][0], r * ((T)0.5 * (G[0][1] + G[1][0])),
                    r * ((T)0.5 * (G[0][2] + G[2][0])), r * G[1][1],
                    r * ((T)0.5 * (G[1][2] + G[2][1])), r * G[2][2]};
#pragma unroll
    for (int k = 0; k < ZT; ++k) {
      const int t = j - k;
      if (t >= 0 && t <= 2 * R) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          acc[q][k] = fma(w[t], p[q], acc[q][k]);
          // finish this plane's FMAs here: otherwise the products of every plane are kept
          // live to form each output's sum in one chain
          __asm__ volatile("" ::"v"(acc[q][k]));
        }
      }
    }
    Pm = P0;
    P0 = Pp;
    Pp = Pn;
  }
  T* out = reinterpret_cast<T*>(A.zbuf) + (int64_t)zl0 * pstride + (int64_t)y * A.nx + x;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T* o = out + (int64_t)q * qstride;
#pragma unroll
    for (int k = 0; k < ZT; ++k)
      if (k < nk) o[(int64_t)k * pstride] = acc[q][k];
  }
}

// x-y tile of kXT points: 32 x 8 for narrow windows (full 128-byte rows in every store),
// 16 x 16 for wide ones (smaller halo); the x pass works on 16-point row segments.
template <int R>
struct XyTile {
  static constexpr int X = R <= 4 ? 32 : 16;
  static constexpr int Y = kXT / X;
  static constexpr int NH = X / 16;  // row segments
};

template <int R, typename T, int NQ>
struct XyLds {
  static constexpr int HX = XyTile<R>::X + 2 * R;
  static constexpr int HY = XyTile<R>::Y + 2 * R;
  static constexpr int HXP = HX | 1;  // odd row stride
  static constexpr int NRAW = HX * HY;
  static constexpr int QS = HY * HXP;
  // quantities per LDS round: as many as fit in 40 KiB, so that three or four workgroups
  // share a CU (measured faster than fewer, larger rounds)
  static constexpr int G0 = 40960 / (QS * (int)sizeof(T));
  static constexpr int G = G0 < 1 ? 1 : (G0 > NQ ? NQ : G0);
  static constexpr int doubles = (G * QS * (int)sizeof(T) + 7) / 8;
};

template <class S, int R, typename T>
__device__ __forceinline__ void xy_pass(const MonoArgs& A) {
  using L = XyLds<R, T, S::kQ>;
  constexpr int HX = L::HX, HY = L::HY, HXP = L::HXP, QS = L::QS, G = L::G;
  constexpr int kTX = XyTile<R>::X, kTY = XyTile<R>::Y, NH = XyTile<R>::NH;
  // LDS column of tile column x: the second row segment's x outputs sit 2R cells right
  auto lcol = [](int x) { return x + (x >= 16 ? 2 * R : 0); };
  constexpr int NQ = S::kQ;
  constexpr int NS = S::kStat;
  static_assert(4 * NS <= L::doubles, "statistics records do not fit the LDS buffer");
  __shared__ double smem[L::doubles];
  T* buf = reinterpret_cast<T*>(smem);
  // item = (tile, run of kXZ planes); XCD bands: consecutive items (neighbouring tiles, which
  // share halos) on one XCD
  const int nzc = (A.nzs + kXZ - 1) / kXZ;
  const int nb = A.ntiles * nzc;
  const int per = (nb + 7) / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= nb) return;
  const int tile = item % A.ntiles, zc = item / A.ntiles;
  const int x0 = (tile % A.ntx) * kTX, y0 = (tile / A.ntx) * kTY;
  const int tid = threadIdx.x, px = tid % kTX, py = tid / kTX;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t qstride = plane;
  const T* w = cweights<T>(A);
  const bool valid = x0 + px < A.nx && y0 + py < A.ny;
  typename S::Acc acc;  // this thread's FP64 sums over its points
  acc.zero();
  const int z_hi = min((zc + 1) * kXZ, A.nzs);
  for (int zl = zc * kXZ; zl < z_hi; ++zl) {
    const T* zb = reinterpret_cast<const T*>(A.zbuf) + (int64_t)zl * A.nq * plane;
    T M[NQ];
#pragma unroll
    for (int g0 = 0; g0 < NQ; g0 += G) {
      // quantities of this round (uniform; fixed unless the last quantity is optional)
      const int ng = S::kOptionalLast ? min(G, A.nq - g0) : min(G, NQ - g0);
      for (int r = tid; r < L::NRAW; r += kXT) {
        const int hx = r % HX, hy = r / HX;
        const int64_t o = (int64_t)wrapi(y0 - R + hy, A.ny) * A.nx + wrapi(x0 - R + hx, A.nx);
        T* d = buf + hy * HXP + hx;
        // every load of the round is issued before the first store (a load that depends on
        // the run-time count ng would be waited for one at a time); past ng, quantity g0 is
        // read again and not stored
        T v[G];
#pragma unroll
        for (int q = 0; q < G; ++q)
          if (g0 + q < NQ) v[q] = zb[(int64_t)(g0 + (q < ng ? q : 0)) * qstride + o];
#pragma unroll
        for (int q = 0; q < G; ++q)
          if (g0 + q < NQ && q < ng) d[q * QS] = v[q];
      }
      __syncthreads();
      // x, in place: one (quantity, row, 16-point segment) per task; the second segment's
      // outputs go 2R cells to the right, clear of the first segment's inputs
      for (int t = tid; t < ng * HY * NH; t += kXT) {
        const int h = t % NH;
        T* v = buf + (t / NH) * HXP + h * 16;
        T vr[16 + 2 * R];
#pragma unroll
        for (int i = 0; i < 16 + 2 * R; ++i) vr[i] = v[i];
        T* vo = v + h * 2 * R;
#pragma unroll
        for (int o = 0; o < 16; ++o) vo[o] = tap_sum<R, T>(w, vr, o + R);
      }
      __syncthreads();
      // y, in place: one (quantity, column) per task, outputs to rows 0 .. kTY - 1
      for (int t = tid; t < ng * kTX; t += kXT) {
        T* v = buf + (t / kTX) * QS + lcol(t % kTX);
        T vr[HY];
#pragma unroll
        for (int i = 0; i < HY; ++i) vr[i] = v[i * HXP];
#pragma unroll
        for (int o = 0; o < kTY; ++o) v[o * HXP] = tap_sum<R, T>(w, vr, o + R);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (g0 + q < NQ) M[g0 + q] = q < ng ? buf[q * QS + py * HXP + lcol(px)] : (T)0;
      __syncthreads();
    }
    const int64_t g = (int64_t)(A.zs + zl) * plane + (int64_t)(y0 + py) * A.nx + x0 + px;
    S::epilogue(A, M, valid, g, acc);
  }
  if (A.partials) acc.write(A.partials, smem, item);
}

// Two waves per SIMD for the z kernels: the register budget then bounds how far the
// scheduler hoists the window loads ahead of their FMAs.
template <int R, typename T>
__global__ void __launch_bounds__(kZB) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_carrier_z(MonoArgs A) {
  z_pass<CarrierSet, R, T>(A);
}

template <int R, typename T>
__global__ void __launch_bounds__(kXT) k_carrier_xy(MonoArgs A) {
  xy_pass<CarrierSet, R, T>(A);
}

template <int R, typename T>
__global__ void __launch_bounds__(kZB) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_moment3_z(MonoArgs A) {
  z_pass<Moment3Set, R, T>(A);
}

template <int R, typename T>
__global__ void __launch_bounds__(kXT) k_moment3_xy(MonoArgs A) {
  xy_pass<Moment3Set, R, T>(A);
}

template <int R, typename T>
__global__ void __launch_bounds__(kZB) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_kc_z(MonoArgs A) {
  z_pass_kc<R, T>(A);
}

template <int R, typename T>
__global__ void __launch_bounds__(kXT) k_kc_xy(MonoArgs A) {
  xy_pass<KcSet, R, T>(A);
}

// ---------------------------------------------------------------- launches
template <int R>
hipError_t launch_z_of(const MonoArgs& a, int set, int fp64, hipStream_t s) {
  const int zt = fp64 ? cz_planes<double>() : cz_planes<float>();
  const int64_t items = (int64_t)((a.nzs + zt - 1) / zt) * ((a.nx + kZB - 1) / kZB) * a.ny;
  if (8 * ((items + 7) / 8) > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(8 * ((items + 7) / 8)));
  if (set == kSetCarrier) {
    if (fp64)
      hipLaunchKernelGGL((k_carrier_z<R, double>), grid, dim3(kZB), 0, s, a);
    else
      hipLaunchKernelGGL((k_carrier_z<R, float>), grid, dim3(kZB), 0, s, a);
  } else if (set == kSetKcMp) {
    if (fp64)
      hipLaunchKernelGGL((k_kc_z<R, double>), grid, dim3(kZB), 0, s, a);
    else
      hipLaunchKernelGGL((k_kc_z<R, float>), grid, dim3(kZB), 0, s, a);
  } else {
    if (fp64)
      hipLaunchKernelGGL((k_moment3_z<R, double>), grid, dim3(kZB), 0, s, a);
    else
      hipLaunchKernelGGL((k_moment3_z<R, float>), grid, dim3(kZB), 0, s, a);
  }
  return hipGetLastError();
}

template <int R>
hipError_t launch_xy_of(const MonoArgs& a, int set, int fp64, hipStream_t s) {
  const int64_t nb = mono_xy_records(a);
  const dim3 grid((unsigned)(8 * ((nb + 7) / 8)));
  if (set == kSetCarrier) {
    if (fp64)
      hipLaunchKernelGGL((k_carrier_xy<R, double>), grid, dim3(kXT), 0, s, a);
    else
      hipLaunchKernelGGL((k_carrier_xy<R, float>), grid, dim3(kXT), 0, s, a);
  } else if (set == kSetKcMp) {
    if (fp64)
      hipLaunchKernelGGL((k_kc_xy<R, double>), grid, dim3(kXT), 0, s, a);
    else
      hipLaunchKernelGGL((k_kc_xy<R, float>), grid, dim3(kXT), 0, s, a);
  } else {
    if (fp64)
      hipLaunchKernelGGL((k_moment3_xy<R, double>), grid, dim3(kXT), 0, s, a);
    else
      hipLaunchKernelGGL((k_moment3_xy<R, float>), grid, dim3(kXT), 0, s, a);
  }
  return hipGetLastError();
}

template <template <int> class F, typename... Args>
hipError_t dispatch_r(int R, Args... args) {
  switch (R) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
struct RunZ {
  static hipError_t run(const MonoArgs& a, int set, int fp64, hipStream_t s) {
    return launch_z_of<R>(a, set, fp64, s);
  }
};
template <int R>
struct RunXY {
  static hipError_t run(const MonoArgs& a, int set, int fp64, hipStream_t s) {
    return launch_xy_of<R>(a, set, fp64, s);
  }
};

}  // namespace

int mono_tile_x(int R) { return R <= 4 ? XyTile<1>::X : XyTile<kMaxR>::X; }
int mono_tile_y(int R) { return kXT / mono_tile_x(R); }
int mono_z_planes(int fp64) { return fp64 ? cz_planes<double>() : cz_planes<float>(); }
int64_t mono_xy_records(const MonoArgs& a) {
  return (int64_t)a.ntiles * ((a.nzs + kXZ - 1) / kXZ);
}
int mono_records_per_block(int set) {
  return set == kSetKcMp ? KcSet::Acc::kRecords : 1;
}

hipError_t launch_mono_z(const MonoArgs& a, int set, int R, int fp64, hipStream_t s) {
  if (a.ny > 65535) return hipErrorInvalidValue;
  return dispatch_r<RunZ>(R, a, set, fp64, s);
}

hipError_t launch_mono_xy(const MonoArgs& a, int set, int R, int fp64, hipStream_t s) {
  return dispatch_r<RunXY>(R, a, set, fp64, s);
}

}  // namespace kcf
