// Box-filter kernels (gfx950): trapezoidal top-hat of width 2R h, all ten filtered quantities
// of a column in one thread, sliding sums along x and y, a running window sum along z.
//
// A workgroup owns a tile of columns (the output columns plus the one-cell halo of the
// central-difference gradient) and marches along z: short tiles (18x14 columns, 256 threads,
// three workgroups per CU) for R = 1, R = 3 and FP64 products at R = 4, tall tiles (18x28,
// 512 threads, one per CU) otherwise. At step k the plane za = za0 + k arrives:
//   * staging: the inputs of plane za and of plane za - 2R (the one leaving the window: kept
//     in registers since it arrived where they allow, R = 1 and tall tiles up to R = 4,
//     otherwise read a second time, from cache), loaded during the previous step, are turned
//     into the differences d = P(za) - P(za - 2R) of the ten products P = rho, rho u_i,
//     rho u_i u_j;
//   * x pass and y pass through LDS: each task slides a trapezoid window over one row
//     (column) of one quantity in registers, three operations per output (the window is the
//     sum of two boxcars, unscaled: each pass multiplies by 2n); the y pass works in place in
//     short tiles and writes a separate buffer in tall ones;
//   * z: since the x-y filter is linear, the filtered d is the change of the 2R-plane boxcar
//     sum B of the filtered products; B is kept per column thread in FP64, and the trapezoid
//     of plane za - R is the mean of two consecutive boxcars, (B_{k-1} + B_k) / (2n), and
//     the factors of the x and y passes are divided out with it;
//   * epilogue A: Favre velocity and tau from the FP64 window sums, stored (tall tiles: at
//     the end of the step), the velocity and rho_bar, tau kept in LDS rings;
//   * epilogue B: gradient, closures and statistics of a plane one (short tiles) or two (tall
//     tiles) planes behind, from the rings.
// T is the type of the products and of the x-y passes: double for narrow widths, where tau
// is a small difference of large filtered products, float otherwise. Outputs are float32.
#include <type_traits>

#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

constexpr int kBX = 18;       // computed columns of a tile along x (16 outputs + halo)
constexpr int kBOX = kBX - 2;
constexpr int kLdsPerCU = 160 * 1024;

// Tile and workgroup shape. Narrow windows use short tiles (18x14 columns, 256 threads) so
// that three workgroups share a CU; wide windows use tall tiles (18x28, 512 threads), where
// the 2R-cell halo of a short tile would cost more than the lost occupancy. R = 2 and float
// products at R = 4 take tall tiles too: at two waves per SIMD their registers hold the
// inputs of the last 2R planes, which was measured faster than three waves of short tiles
// that read the leaving plane again (FP64 products at R = 4 exceed the LDS in tall tiles).
template <int BY_, int BT_, int WAVES_, int STRIP_>
struct BoxCfg {
  static constexpr int BY = BY_;         // computed rows
  static constexpr int BOY = BY - 2;     // output rows
  static constexpr int BN = kBX * BY;    // column threads
  static constexpr int BT = BT_;         // threads per workgroup
  static constexpr int WAVES = WAVES_;   // waves per SIMD the register budget allows
  static constexpr int YP = BT >= 512 ? 2 : 1;  // y-pass tasks per (quantity, column)
  static constexpr int BYP = BY / YP;    // rows per y-pass task
  static constexpr int STRIP = STRIP_;   // tile numbering in strips this wide (0: rows)
  static_assert(BN <= BT && BY % YP == 0 && BT % 64 == 0, "tile does not fit the workgroup");
};
using ShortTile = BoxCfg<14, 256, 3, 0>;
using TallTile = BoxCfg<28, 512, 2, 8>;
template <int R, typename T>
using TileFor = typename std::conditional<(R == 1 || R == 3 || (R == 4 && sizeof(T) == 8)),
                                          ShortTile, TallTile>::type;

// Waves per SIMD of a (radius, precision) pair: the tile's, except double products with
// R >= 3, whose LDS buffer leaves room for two workgroups per CU and whose x-y windows need
// more than the 168 registers of three waves.
template <int R, typename T>
constexpr int box_waves() {
  return sizeof(T) == 8 && R >= 3 ? 2 : TileFor<R, T>::WAVES;
}

// One buffer of 10 planes of HY rows with an odd row stride (conflict-free row-per-lane
// access): products, then x-filtered rows (first kBX entries), then y-filtered rows.
// Tall tiles have the LDS to spare for a separate y output and deeper rings, which removes
// two of the five barriers of a step: the y pass no longer works in place, and the gradient
// epilogue runs two planes behind the window instead of one, on planes written in earlier
// steps.
template <int R, typename T, class C = TileFor<R, T>>
struct BoxLds {
  static constexpr int HX = kBX + 2 * R;
  static constexpr int HY = C::BY + 2 * R;
  static constexpr int HXP = HX | 1;
  static constexpr int NRAW = HX * HY;
  static constexpr int prod = (10 * HY * HXP * (int)sizeof(T) + 15) / 16 * 16;
  static constexpr int NI = kBOX * C::BOY;  // interior (output) columns
  static constexpr bool split = C::BT >= 512;
  static constexpr int D = split ? 2 : 1;       // planes between the window and the gradient
  static constexpr int NSU = D + 2;             // planes of ut kept for the gradient
  static constexpr int NLG = D + 1;             // planes of rho_bar and tau kept for it
  static constexpr int yout = split ? (10 * C::BY * kBX * (int)sizeof(T) + 15) / 16 * 16 : 0;
  // ut of NSU planes, then rho_bar and tau of the interior columns of NLG planes
  static constexpr int su = (NSU * 3 * C::BN + NLG * 7 * NI) * 4;
  static constexpr int bytes = prod + yout + su;
  static constexpr int doubles = (bytes + 7) / 8;
  // resident workgroups per CU: the smaller of the register and the LDS limit
  static constexpr int by_waves = box_waves<R, T>() * 4 / (C::BT / 64);
  static constexpr int by_lds = kLdsPerCU / bytes;
  static constexpr int blocks_per_cu = by_waves < by_lds ? by_waves : by_lds;
};

// Trapezoid windows over v[o .. o + 2R], o = 0 .. NO - 1, each scaled by 2n = 4R: with
// S_o = v[o] + ... + v[o + 2R - 1] the 2R-point boxcar, 2n times the trapezoid (ends 1/(2n),
// interior 1/n) is S_o + S_{o+1}. Three operations per output; the factor 2n of each pass
// is divided out once, in double, after the z sum.
template <int R, int NO, typename T, class St>
__device__ __forceinline__ void trap_row(const T* v, St&& store) {
  T S = v[0];
#pragma unroll
  for (int i = 1; i < 2 * R; ++i) S += v[i];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const T Sn = S + (v[o + 2 * R] - v[o]);
    store(o, S + Sn);
    S = Sn;
  }
}

template <typename T>
__device__ __forceinline__ void products(const float (&f)[4], T (&p)[10]) {
  const T r = (T)f[0], ux = (T)f[1], uy = (T)f[2], uz = (T)f[3];
  const T mx = r * ux, my = r * uy, mz = r * uz;
  p[0] = r;
  p[1] = mx;
  p[2] = my;
  p[3] = mz;
  p[4] = mx * ux;
  p[5] = mx * uy;
  p[6] = mx * uz;
  p[7] = my * uy;
  p[8] = my * uz;
  p[9] = mz * uz;
}

// kX: exact FP64 statistics contributions (FP64 filter sums only). kRingOK: the registers
// allow the ring of arriving inputs below (not at the all-outputs level, which would spill)
template <int R, typename T, bool kX, bool kRingOK>
__device__ __forceinline__ void box_body(const FilterArgs& A, const WidthArgs& W, int item,
                                         unsigned char* smem) {
  static_assert(!kX || sizeof(T) == 8, "exact statistics need FP64 filter sums");
  using L = BoxLds<R, T>;
  using C = TileFor<R, T>;
  constexpr int kBT = C::BT, kBN = C::BN, kBOY = C::BOY, kYP = C::YP, kBYP = C::BYP;
  constexpr int HX = L::HX;
  constexpr int HY = L::HY;
  constexpr int HXP = L::HXP;
  constexpr int NRAW = L::NRAW;
  constexpr int NPF = (NRAW + kBT - 1) / kBT;
  constexpr int QS = HY * HXP;  // stride of one quantity in the buffer
  T* buf = reinterpret_cast<T*>(smem);
  constexpr int NI = L::NI;
  constexpr bool kSplit = L::split;
  constexpr int D = L::D, NSU = L::NSU, NLG = L::NLG;
  T* yb = reinterpret_cast<T*>(smem + L::prod);                     // split: 10 x BY x kBX
  float* su = reinterpret_cast<float*>(smem + L::prod + L::yout);  // NSU planes x 3 x kBN
  float* lagb = su + NSU * 3 * kBN;                                 // NLG planes x 7 x NI
  // the mean of two z boxcars, and the factor 4R of each of the x and y passes
  const double inv_2n = 1.0 / ((4.0 * R) * (4.0 * R) * (4.0 * R));

  const int tid = threadIdx.x;
  const int tile = item % A.ntiles;
  const int zc = item / A.ntiles;
  int tx, ty;
  tile_coords(A, tile, tx, ty);
  const int x0 = tx * kBOX - 1, y0 = ty * kBOY - 1;  // global coordinates of column (0, 0)
  const int z0 = zc * A.zlen;
  const int z1 = min(z0 + A.zlen, A.nz);
  const int nfilt = (z1 - z0) + 2 * R + 2;  // steps that bring in a plane
  const int nsteps = nfilt + D - 1;         // and those that only finish the gradient
  const int za0 = z0 - 1 - R;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t ntot = A.ntot;

  // raw points of this thread: byte offsets within a plane (below 2^32: a plane holds at
  // most 2^30 points) and LDS offsets; only the last round can hold threads without a point
  uint32_t pfoff[NPF];
  int ldoff[NPF];
  bool has[NPF];
#pragma unroll
  for (int i = 0; i < NPF; ++i) {
    const int p = tid + i * kBT;
    has[i] = (i + 1) * kBT <= NRAW || p < NRAW;
    if (has[i]) {
      const int hx = p % HX, hy = p / HX;
      pfoff[i] = (uint32_t)(wrapi(y0 - R + hy, A.ny) * A.nx + wrapi(x0 - R + hx, A.nx)) * 4u;
      ldoff[i] = hy * HXP + hx;
    } else {
      pfoff[i] = 0;
      ldoff[i] = 0;
    }
  }
  // inputs of the arriving plane (pn) and of the plane leaving the window (po), raw-point
  // groups i0 .. i1 - 1; the plane's base addresses are uniform, so each load is a scalar
  // base plus this thread's offset
  float pn[NPF][4], po[NPF][4];
  // the inputs of the last 2R arriving planes stay in registers (rg[0] the oldest) where the
  // registers allow, so that the plane leaving the window is not read again: R = 1, and tall
  // tiles (two waves per SIMD) up to R = 4 (wider windows have no registers left for their
  // 2R planes)
  constexpr int kRing = (R == 1 || (R <= 4 && L::split)) && kRingOK ? 2 * R : 0;
  float rg[kRing > 0 ? kRing : 1][NPF][4];
  auto load = [&](float (&pf)[NPF][4], int za, int i0, int i1) {
    // za lies in [z0 - 1 - R, z1 + R] and the grid holds the support (nz >= 2R + 1), so one
    // period brings it into range (no integer division in the loop)
    const int zw = za < 0 ? za + A.nz : (za >= A.nz ? za - A.nz : za);
    const int64_t zoff = (int64_t)zw * plane;
    const char* b0 = reinterpret_cast<const char*>(A.rho + zoff);
    const char* b1 = reinterpret_cast<const char*>(A.u + zoff);
    const char* b2 = reinterpret_cast<const char*>(A.u + ntot + zoff);
    const char* b3 = reinterpret_cast<const char*>(A.u + 2 * ntot + zoff);
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      if (i >= i0 && i < i1 && has[i]) {
        // opaque here, so that the 32-bit offset is not widened once outside the loop
        // (which would cost a 64-bit address add per load instead of the scalar-base form)
        uint32_t o = pfoff[i];
        __asm__ volatile("" : "+v"(o));
        pf[i][0] = *reinterpret_cast<const float*>(b0 + o);
        pf[i][1] = *reinterpret_cast<const float*>(b1 + o);
        pf[i][2] = *reinterpret_cast<const float*>(b2 + o);
        pf[i][3] = *reinterpret_cast<const float*>(b3 + o);
      }
    }
  };
  load(pn, za0, 0, NPF);

  const bool col_thread = tid < kBN;
  const int col = col_thread ? tid : 0;
  const int cx = col % kBX, cy = col / kBX;
  const int gx = x0 + cx, gy = y0 + cy;
  const bool interior = col_thread && cx >= 1 && cx <= kBOX && cy >= 1 && cy <= kBOY &&
                        gx < A.nx && gy < A.ny;
  const int ycol = cy * HXP + cx;  // this column's entry in a y-filtered plane
  const uint32_t cofs = interior ? (uint32_t)(gy * A.nx + gx) * 4u : 0u;  // bytes in a plane

  double B[10];  // boxcar sums of the 2R planes za - 2R + 1 .. za
#pragma unroll
  for (int q = 0; q < 10; ++q) B[q] = 0.0;
  // Statistics, in one of three forms:
  //  - exact (kX): every contribution an exact FP64 product, folded over the wave per point
  //    into ten FP64 sums per lane;
  //  - FP64 filter sums otherwise: float32 contributions folded over the wave per point into
  //    ten float32 sums per lane, added to the FP64 ones every kStatFlush points (these
  //    kernels hold three waves per SIMD, which leaves no room for per-lane sums of all 40
  //    slots, and the float32 fold takes about 2.5 times fewer instructions than the exact one);
  //  - float32 filter sums: float32 contributions summed per lane over all 40 slots and folded
  //    into FP64 every kStatFlush points.
  constexpr bool kFold = sizeof(T) == 8;  // the first two forms
  StatAcc xacc;      // wave-fold forms: the lane's ten 4-lane FP64 sums
  stat_zero(xacc);
  StatFold32 fold;   // float32 fold: the lane's ten 4-lane float32 sums since the last flush
  stat_zero(fold);
  StatPart part;     // per-lane form: statistics of the points since the last flush
  stat_zero(part);
  double acc = 0.0;  // per-lane form: this lane's slot of the wave's FP64 record
  int npart = 0;     // points since the last flush (the same in every lane of a wave)
  const bool need_grad = needs_gradient(W);

  for (int k = 0; k < nsteps; ++k) {
    const int za = za0 + k;
    const int zo = za - R;
    const int us = (k - 2 * R + NSU) % NSU;  // ut slot of plane zo
    // tall tiles store the Favre fields of plane zo at the end of the step, after the
    // gradient epilogue, when the vector memory path is idle (its loads and these stores
    // are the CU's busiest shared resource); short tiles store them at once
    bool st_do = false;
    float st_rb = 0.f, st_u[3] = {0.f, 0.f, 0.f}, st_tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto store_fields = [&](bool on, float rb_v, const float (&u_v)[3], const float (&t_v)[6]) {
      if (!on) return;
      const int64_t zb = (int64_t)zo * plane;
      uint32_t o = cofs;
      __asm__ volatile("" : "+v"(o));  // keeps the scalar-base store form (see load)
      if (W.rho_bar) *plane_addr(W.rho_bar, 0, ntot, zb, o) = rb_v;
      if (W.ut) {
#pragma unroll
        for (int i = 0; i < 3; ++i) *plane_addr(W.ut, i, ntot, zb, o) = u_v[i];
      }
      if (W.tau) {
#pragma unroll
        for (int s = 0; s < 6; ++s) *plane_addr(W.tau, s, ntot, zb, o) = t_v[s];
      }
    };
    if (k < nfilt) {  // uniform
      const bool leaving = k >= 2 * R;  // uniform: plane za - 2R is inside the window
      // ---- staging: product differences of plane za
#pragma unroll
      for (int i = 0; i < NPF; ++i) {
        if (has[i]) {
          T d[10];
          products<T>(pn[i], d);
          if (leaving) {
            T o[10];
            if constexpr (kRing > 0)
              products<T>(rg[0][i], o);
            else
              products<T>(po[i], o);
#pragma unroll
            for (int q = 0; q < 10; ++q) d[q] -= o[q];
          }
#pragma unroll
          for (int q = 0; q < 10; ++q) buf[q * QS + ldoff[i]] = d[q];
        }
      }
      if constexpr (kRing > 0) {  // before the next plane's inputs replace pn
#pragma unroll
        for (int j = 0; j + 1 < kRing; ++j)
#pragma unroll
          for (int i = 0; i < NPF; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) rg[j][i][c] = rg[j + 1][i][c];
#pragma unroll
        for (int i = 0; i < NPF; ++i)
#pragma unroll
          for (int c = 0; c < 4; ++c) rg[kRing - 1][i][c] = pn[i][c];
      }
      __syncthreads();
      // ---- x pass, in place: one (quantity, row) per task
      for (int t = tid; t < 10 * HY; t += kBT) {
        T* v = buf + t * HXP;
        T vr[HX];
#pragma unroll
        for (int i = 0; i < HX; ++i) vr[i] = v[i];
        trap_row<R, kBX>(vr, [&](int o, T x) { v[o] = x; });
      }
      // The next step's inputs are requested in parts between the phases of this step: the
      // loads of all waves of the CU queue in one vector memory unit, and a burst of them
      // right after a barrier holds every wave up behind it (a sixth of the time at R = 8).
      if (k + 1 < nfilt) load(pn, za + 1, 0, 2);
      __syncthreads();
      // ---- y pass: one (quantity, column, half of the rows) per task. In place (short tiles):
      // all reads are done before the barrier, all writes after it; tall tiles write to yb.
      {
        constexpr int NYT = 10 * kYP * kBX;
        constexpr int NYI = (NYT + kBT - 1) / kBT;
        T vr[NYI][kBYP + 2 * R];
#pragma unroll
        for (int j = 0; j < NYI; ++j) {
          const int t = tid + j * kBT;
          if (t < NYT) {
            const int x = t % kBX, part = (t / kBX) % kYP, q = t / (kYP * kBX);
            const T* src = buf + q * QS + part * kBYP * HXP + x;
#pragma unroll
            for (int i = 0; i < kBYP + 2 * R; ++i) vr[j][i] = src[i * HXP];
          }
        }
        if (!kSplit) __syncthreads();
#pragma unroll
        for (int j = 0; j < NYI; ++j) {
          const int t = tid + j * kBT;
          if (t < NYT) {
            const int x = t % kBX, part = (t / kBX) % kYP, q = t / (kYP * kBX);
            if (kSplit) {
              T* dst = yb + (q * C::BY + part * kBYP) * kBX + x;
              trap_row<R, kBYP>(vr[j], [&](int o, T x) { dst[o * kBX] = x; });
            } else {
              T* dst = buf + q * QS + part * kBYP * HXP + x;
              trap_row<R, kBYP>(vr[j], [&](int o, T x) { dst[o * HXP] = x; });
            }
          }
        }
      }
      if (k + 1 < nfilt) load(pn, za + 1, 2, NPF);
      __syncthreads();
      // ---- z: advance the boxcars; the trapezoid of plane zo = za - R is their mean
      const bool full = k >= 2 * R;
      double qb[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        const double prev = B[q];
        B[q] = prev + (double)(kSplit ? yb[q * kBN + col] : buf[q * QS + ycol]);
        qb[q] = (prev + B[q]) * inv_2n;
      }
      if (full) {  // uniform
        // 1 / rho_bar from the hardware estimate and two Newton steps (within an ulp of
        // double; the quotient itself is correctly rounded only to float32 in the outputs)
        double rinv = __builtin_amdgcn_rcp(qb[0]);
        rinv = fma(rinv, fma(-qb[0], rinv, 1.0), rinv);
        rinv = fma(rinv, fma(-qb[0], rinv, 1.0), rinv);
        const double uT[3] = {qb[1] * rinv, qb[2] * rinv, qb[3] * rinv};
        const float cur_rb = (float)qb[0];
        float cur_tau[6];
        // tau_ij = bar(rho u_i u_j) - bar(rho u_i) ut_j
        cur_tau[0] = (float)fma(-qb[1], uT[0], qb[4]);
        cur_tau[1] = (float)fma(-qb[1], uT[1], qb[5]);
        cur_tau[2] = (float)fma(-qb[1], uT[2], qb[6]);
        cur_tau[3] = (float)fma(-qb[2], uT[1], qb[7]);
        cur_tau[4] = (float)fma(-qb[2], uT[2], qb[8]);
        cur_tau[5] = (float)fma(-qb[3], uT[2], qb[9]);
        if (col_thread) {
#pragma unroll
          for (int i = 0; i < 3; ++i) su[(us * 3 + i) * kBN + col] = (float)uT[i];
        }
        if (interior) {  // for the gradient epilogue D steps later
          float* lg = lagb + (k % NLG) * 7 * NI + (cy - 1) * kBOX + (cx - 1);
          lg[0] = cur_rb;
#pragma unroll
          for (int s = 0; s < 6; ++s) lg[(1 + s) * NI] = cur_tau[s];
        }
        const bool on = interior && zo >= z0 && zo < z1;
        const float cur_u[3] = {(float)uT[0], (float)uT[1], (float)uT[2]};
        if (kSplit) {
          st_do = on;
          st_rb = cur_rb;
#pragma unroll
          for (int i = 0; i < 3; ++i) st_u[i] = cur_u[i];
#pragma unroll
          for (int s = 0; s < 6; ++s) st_tau[s] = cur_tau[s];
        } else {
          store_fields(on, cur_rb, cur_u, cur_tau);
        }
      }
    }
    if (kRing == 0 && k + 1 < nfilt && k + 1 >= 2 * R) load(po, za + 1 - 2 * R, 0, NPF);
    // Short tiles, every step: the reads of the y-filtered plane are done before the next
    // staging overwrites it, and the velocity of plane zo is in LDS before the gradient
    // reads it. Tall tiles read only planes of earlier steps here, behind the three barriers
    // of this step, or behind this one in a step that brings in no plane.
    if (!kSplit || k >= nfilt) __syncthreads();
    const int zg = zo - D;
    // ---- epilogue B: gradient, closures, statistics of plane zg, one interior column per
    // thread (the waves past the NI interior columns have nothing to do)
    if (need_grad && k >= 2 * R + D && zg >= z0 && zg < z1 && (tid & ~63) < NI) {  // uniform
      // ut slots of planes zg - 1, zg, zg + 1
      const int sm = (us - D - 1 + 2 * NSU) % NSU, sg = (us - D + NSU) % NSU;
      const int sp = (us - D + 1 + NSU) % NSU;
      const int t = tid < NI ? tid : 0;
      const int ex = 1 + t % kBOX, ey = 1 + t / kBOX;
      const int ecol = ey * kBX + ex;
      const int egx = x0 + ex, egy = y0 + ey;
      const bool valid = tid < NI && egx < A.nx && egy < A.ny;
      const float* lg = lagb + ((k - D) % NLG) * 7 * NI + t;
      const float rb = lg[0];
      float tau[6];
#pragma unroll
      for (int s = 0; s < 6; ++s) tau[s] = lg[(1 + s) * NI];
      PointOut P;
      float u[3];
      const float* uc = su + sg * 3 * kBN;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float* ui = uc + i * kBN;
        P.G[i][0] = (ui[ecol + 1] - ui[ecol - 1]) * A.inv2h;
        P.G[i][1] = (ui[ecol + kBX] - ui[ecol - kBX]) * A.inv2h;
        P.G[i][2] = (su[(sp * 3 + i) * kBN + ecol] - su[(sm * 3 + i) * kBN + ecol]) * A.inv2h;
        u[i] = ui[ecol];
      }
      point_closures(W, rb, tau, P, kX);
      if (valid) {
        const int64_t zb = (int64_t)zg * plane;
        uint32_t o = (uint32_t)(egy * A.nx + egx) * 4u;
        __asm__ volatile("" : "+v"(o));
        store_point_at(W, P, [&](float* b, int c) { return plane_addr(b, c, ntot, zb, o); });
      }
      if (W.partials) {  // uniform
        if constexpr (kX) {
          StatIn I;
          stat_inputs(rb, u, tau, P, valid, I);
          stat_add(I, xacc);
        } else if constexpr (kFold) {
          stat_point_fold(rb, u, tau, P.G, P.tgm, smag_dissipation(W, rb, P.G), valid, fold);
          if (++npart == kStatFlush) {  // uniform
            stat_flush32(fold, xacc);
            npart = 0;
          }
        } else {
          stat_point(rb, u, tau, P.G, P.tgm, smag_dissipation(W, rb, P.G), valid, part);
          if (++npart == kStatFlush) {  // uniform
            stat_flush(part, acc);
            npart = 0;
          }
        }
      }
    }
    if (kSplit) store_fields(st_do, st_rb, st_u, st_tau);
  }
  if (W.partials) {
    double* rec = W.partials + ((int64_t)item * (kBT / 64) + (tid >> 6)) * kNStat;
    if constexpr (kFold) {
      if (!kX && npart > 0) stat_flush32(fold, xacc);  // uniform
      write_stats(rec, xacc);
    } else {
      if (npart > 0) stat_flush(part, acc);  // uniform
      write_stat_record(rec, acc);
    }
  }
}

// kOut: which optional gradient-epilogue outputs the call can store (0: none, 1: the gradient
// and Q only, 2: any); the others, their stores and (below 2) the KC scalars compile away,
// which also keeps the kernel's scalar registers from spilling
template <int R, typename T, int kOut>
__global__ void __launch_bounds__((TileFor<R, T>::BT))
    __attribute__((amdgpu_waves_per_eu(box_waves<R, T>(), box_waves<R, T>())))
    k_box1(FilterArgs A) {
  __shared__ double smem[BoxLds<R, T>::doubles];
  int item;
  if (!map_block(A, item)) return;
  WidthArgs W = A.wa;
  if constexpr (kOut < 2) W.tau_gm = W.tau_smag = W.k_sgs = W.nu_t = W.omega_t = nullptr;
  if constexpr (kOut < 1) W.grad = W.q_crit = nullptr;
  box_body<R, T, false, (kOut < 2)>(A, W, item, reinterpret_cast<unsigned char*>(smem));
}

// Exact statistics (FP64 filter sums): one instance per radius, with every output the call
// may store.
template <int R>
__global__ void __launch_bounds__((TileFor<R, double>::BT))
    __attribute__((amdgpu_waves_per_eu(box_waves<R, double>(), box_waves<R, double>())))
    k_box1_exact(FilterArgs A) {
  __shared__ double smem[BoxLds<R, double>::doubles];
  int item;
  if (!map_block(A, item)) return;
  box_body<R, double, true, true>(A, A.wa, item, reinterpret_cast<unsigned char*>(smem));
}

template <int R, typename T>
BoxGeom geom_of() {
  using C = TileFor<R, T>;
  return BoxGeom{kBOX, C::BOY, C::BT, C::BT / 64, BoxLds<R, T>::blocks_per_cu, C::STRIP};
}

template <int R, typename T>
hipError_t launch_of(const FilterArgs& a, int nblocks, hipStream_t s) {
  const WidthArgs& w = a.wa;
  if constexpr (sizeof(T) == 8) {
    if (w.partials && w.exact_stats) {
      hipLaunchKernelGGL((k_box1_exact<R>), dim3(nblocks), dim3(TileFor<R, double>::BT), 0, s, a);
      return hipGetLastError();
    }
  }
  if (w.tau_gm || w.tau_smag || w.k_sgs || w.nu_t || w.omega_t)
    hipLaunchKernelGGL((k_box1<R, T, 2>), dim3(nblocks), dim3(TileFor<R, T>::BT), 0, s, a);
  else if (w.grad || w.q_crit)
    hipLaunchKernelGGL((k_box1<R, T, 1>), dim3(nblocks), dim3(TileFor<R, T>::BT), 0, s, a);
  else
    hipLaunchKernelGGL((k_box1<R, T, 0>), dim3(nblocks), dim3(TileFor<R, T>::BT), 0, s, a);
  return hipGetLastError();
}

// Calls f.template operator()<R, T>() for a supported (radius, precision) pair.
template <class F>
bool dispatch(int R, int fp64, F&& f) {
  if (fp64) {
    switch (R) {
      case 1: f.template operator()<1, double>(); return true;
      case 2: f.template operator()<2, double>(); return true;
      case 3: f.template operator()<3, double>(); return true;
      case 4: f.template operator()<4, double>(); return true;
      default: return false;
    }
  }
  switch (R) {
    case 1: f.template operator()<1, float>(); return true;
    case 2: f.template operator()<2, float>(); return true;
    case 3: f.template operator()<3, float>(); return true;
    case 4: f.template operator()<4, float>(); return true;
    case 5: f.template operator()<5, float>(); return true;
    case 6: f.template operator()<6, float>(); return true;
    case 7: f.template operator()<7, float>(); return true;
    case 8: f.template operator()<8, float>(); return true;
    default: return false;
  }
}

}  // namespace

bool box_supported(int R, int fp64) { return R >= 1 && (fp64 ? R <= 4 : R <= 8); }

BoxGeom box_geometry(int R, int fp64) {
  BoxGeom g{};
  dispatch(R, fp64, [&]<int RR, typename T>() { g = geom_of<RR, T>(); });
  return g;
}

hipError_t launch_box(const FilterArgs& a, int R, int fp64, int nblocks, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  dispatch(R, fp64, [&]<int RR, typename T>() { e = launch_of<RR, T>(a, nblocks, s); });
  return e;
}

}  // namespace kcf
