// Box-filter kernels (gfx950): trapezoidal top-hat of width 2R h, all ten filtered quantities
// of a column in one thread, sliding sums along x, y and z.
//
// A workgroup of 512 threads owns an 18x28 column tile (16x26 output columns plus the
// one-cell halo of the central-difference gradient) and marches along z:
//   * staging: each arriving plane (with an R-cell halo) is read once from HBM (prefetched one
//     plane ahead) and turned into the ten products rho, rho u_i, rho u_i u_j in LDS;
//   * x pass and y pass: every task slides a trapezoid window over one row (column) of one
//     quantity in registers, about four operations per output instead of 2R+1 taps;
//   * z pass: every column thread keeps the last 2R x-y filtered planes of its ten quantities
//     in register rings indexed by a uniform slot (indexed moves, no rotation) and updates a
//     running window sum, re-seeded from the ring every 2R planes;
//   * epilogue: Favre velocity and tau in registers; the velocity of three planes goes to LDS
//     for the gradient, which is evaluated one plane behind together with the closures and
//     the FP64 statistics.
// T is the accumulation type: double for narrow widths, where tau is a small difference of
// large filtered products, float otherwise. Outputs are float32.
#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

constexpr int kBX = 18, kBY = 28;            // computed columns of a tile
constexpr int kBOX = kBX - 2, kBOY = kBY - 2;  // output columns
constexpr int kBN = kBX * kBY;               // 504 column threads
constexpr int kBT = 512;                     // threads per workgroup (8 full waves)
constexpr int kBYP = kBY / 2;                // rows per y-pass task

template <int R, typename T>
struct BoxLds {
  static constexpr int HX = kBX + 2 * R;
  static constexpr int HY = kBY + 2 * R;
  static constexpr int NRAW = HX * HY;
  static constexpr int prod = 10 * NRAW * (int)sizeof(T);     // products, then y-filtered planes
  static constexpr int yf = 10 * kBN * (int)sizeof(T);
  static constexpr int p0 = ((prod > yf ? prod : yf) + 15) / 16 * 16;
  static constexpr int xf = 10 * HY * kBX * (int)sizeof(T);
  static constexpr int su = 9 * kBN * 4;                       // ut of three planes
  static constexpr int bytes = p0 + xf + su;
  static constexpr int doubles = (bytes + 7) / 8;
};

// Trapezoid window over v[o .. o + 2R]: (1/n)(sum of the interior + half the two ends).
// J holds v[o+1] + ... + v[o+2R] on entry and is advanced to the next output.
template <int R, typename T>
__device__ __forceinline__ T trap_slide(const T* v, int o, T& J, T inv_n) {
  const T out = inv_n * (J + (T)0.5 * (v[o] - v[o + 2 * R]));
  J += v[o + 2 * R + 1] - v[o + 1];
  return out;
}

template <int R, typename T>
__device__ __forceinline__ T trap_last(const T* v, int o, T J, T inv_n) {
  return inv_n * (J + (T)0.5 * (v[o] - v[o + 2 * R]));
}

// One ring of the last 2R planes of one quantity (a plain array, so that the compiler keeps
// it in VGPRs and indexes it with the uniform slot); J is the sum of the 2R planes
// z_o - R + 1 .. z_o + R of the current window.
template <int R, typename T>
__device__ __forceinline__ T ring_push(T (&r)[2 * R], T& J, T v, int slot, T inv_n) {
  const T old = r[slot];
  r[slot] = v;
  J += v - old;
  return inv_n * (J + (T)0.5 * (old - v));
}

template <int R, typename T>
__device__ __forceinline__ void ring_reseed(const T (&r)[2 * R], T& J) {
  T s = 0;
#pragma unroll
  for (int t = 0; t < 2 * R; ++t) s += r[t];
  J = s;
}

template <int R, typename T>
__device__ __forceinline__ void box_body(const FilterArgs& A, const WidthArgs& W, int item,
                                         unsigned char* smem) {
  using L = BoxLds<R, T>;
  constexpr int HX = L::HX;
  constexpr int HY = L::HY;
  constexpr int NRAW = L::NRAW;
  constexpr int NPF = (NRAW + kBT - 1) / kBT;
  T* prod = reinterpret_cast<T*>(smem);                   // 10 x HY x HX
  T* yf = prod;                                           // 10 x kBN (after the x pass)
  T* xf = reinterpret_cast<T*>(smem + L::p0);             // 10 x HY x kBX
  float* su = reinterpret_cast<float*>(smem + L::p0 + L::xf);  // 3 planes x 3 x kBN
  const T inv_n = (T)1 / (T)(2 * R);

  const int tid = threadIdx.x;
  const int tile = item % A.ntiles;
  const int zc = item / A.ntiles;
  const int tx = tile % A.ntx, ty = tile / A.ntx;
  const int x0 = tx * kBOX - 1, y0 = ty * kBOY - 1;  // global coordinates of column (0, 0)
  const int z0 = zc * A.zlen;
  const int z1 = min(z0 + A.zlen, A.nz);
  const int nsteps = (z1 - z0) + 2 * R + 2;
  const int za0 = z0 - 1 - R;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t ntot = A.ntot;

  int pfoff[NPF];
#pragma unroll
  for (int i = 0; i < NPF; ++i) {
    const int p = tid + i * kBT;
    if (p < NRAW) {
      const int hx = p % HX, hy = p / HX;
      pfoff[i] = wrapi(y0 - R + hy, A.ny) * A.nx + wrapi(x0 - R + hx, A.nx);
    } else {
      pfoff[i] = -1;
    }
  }
  float pf[NPF][4];
  auto load_plane = [&](int za) {
    const int64_t zoff = (int64_t)wrapi(za, A.nz) * plane;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      if (pfoff[i] >= 0) {
        const int64_t g = zoff + pfoff[i];
        pf[i][0] = A.rho[g];
        pf[i][1] = A.u[g];
        pf[i][2] = A.u[g + ntot];
        pf[i][3] = A.u[g + 2 * ntot];
      }
    }
  };
  load_plane(za0);

  const bool col_thread = tid < kBN;
  const int col = col_thread ? tid : 0;
  const int cx = col % kBX, cy = col / kBX;
  const int gx = x0 + cx, gy = y0 + cy;
  const bool interior = col_thread && cx >= 1 && cx <= kBOX && cy >= 1 && cy <= kBOY &&
                        gx < A.nx && gy < A.ny;

  T r0[2 * R], r1[2 * R], r2[2 * R], r3[2 * R], r4[2 * R], r5[2 * R], r6[2 * R], r7[2 * R],
      r8[2 * R], r9[2 * R];
#pragma unroll
  for (int t = 0; t < 2 * R; ++t)
    r0[t] = r1[t] = r2[t] = r3[t] = r4[t] = r5[t] = r6[t] = r7[t] = r8[t] = r9[t] = 0;
  T Jz[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) Jz[q] = 0;
  float lag_rb = 1.f, lag_tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  double acc[5] = {0, 0, 0, 0, 0};

  for (int k = 0; k < nsteps; ++k) {
    const int za = za0 + k;
    // ---- stage plane za as the ten products
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      if (pfoff[i] >= 0) {
        const int p = tid + i * kBT;
        const T r = (T)pf[i][0];
        const T ux = (T)pf[i][1], uy = (T)pf[i][2], uz = (T)pf[i][3];
        const T mx = r * ux, my = r * uy, mz = r * uz;
        prod[p] = r;
        prod[NRAW + p] = mx;
        prod[2 * NRAW + p] = my;
        prod[3 * NRAW + p] = mz;
        prod[4 * NRAW + p] = mx * ux;
        prod[5 * NRAW + p] = mx * uy;
        prod[6 * NRAW + p] = mx * uz;
        prod[7 * NRAW + p] = my * uy;
        prod[8 * NRAW + p] = my * uz;
        prod[9 * NRAW + p] = mz * uz;
      }
    }
    __syncthreads();
    if (k + 1 < nsteps) load_plane(za + 1);
    // ---- x pass: one (quantity, row) per task
    for (int t = tid; t < 10 * HY; t += kBT) {
      const T* v = prod + t * HX;
      T vr[HX];
#pragma unroll
      for (int i = 0; i < HX; ++i) vr[i] = v[i];
      T J = 0;
#pragma unroll
      for (int i = 1; i <= 2 * R; ++i) J += vr[i];
      T* dst = xf + t * kBX;
#pragma unroll
      for (int o = 0; o < kBX - 1; ++o) dst[o] = trap_slide<R, T>(vr, o, J, inv_n);
      dst[kBX - 1] = trap_last<R, T>(vr, kBX - 1, J, inv_n);
    }
    __syncthreads();
    // ---- y pass: one (quantity, column, half of the rows) per task
    for (int t = tid; t < 20 * kBX; t += kBT) {
      const int x = t % kBX;
      const int part = (t / kBX) & 1;
      const int q = t / (2 * kBX);
      const T* src = xf + (q * HY + part * kBYP) * kBX + x;
      T vr[kBYP + 2 * R];
#pragma unroll
      for (int i = 0; i < kBYP + 2 * R; ++i) vr[i] = src[i * kBX];
      T J = 0;
#pragma unroll
      for (int i = 1; i <= 2 * R; ++i) J += vr[i];
      T* dst = yf + q * kBN + part * kBYP * kBX + x;
#pragma unroll
      for (int o = 0; o < kBYP - 1; ++o) dst[o * kBX] = trap_slide<R, T>(vr, o, J, inv_n);
      dst[(kBYP - 1) * kBX] = trap_last<R, T>(vr, kBYP - 1, J, inv_n);
    }
    __syncthreads();
    // ---- z pass and epilogue A (column threads)
    const int slot = k % (2 * R);
    const bool full = k >= 2 * R;
    T qb[10];
    qb[0] = ring_push<R, T>(r0, Jz[0], yf[0 * kBN + col], slot, inv_n);
    qb[1] = ring_push<R, T>(r1, Jz[1], yf[1 * kBN + col], slot, inv_n);
    qb[2] = ring_push<R, T>(r2, Jz[2], yf[2 * kBN + col], slot, inv_n);
    qb[3] = ring_push<R, T>(r3, Jz[3], yf[3 * kBN + col], slot, inv_n);
    qb[4] = ring_push<R, T>(r4, Jz[4], yf[4 * kBN + col], slot, inv_n);
    qb[5] = ring_push<R, T>(r5, Jz[5], yf[5 * kBN + col], slot, inv_n);
    qb[6] = ring_push<R, T>(r6, Jz[6], yf[6 * kBN + col], slot, inv_n);
    qb[7] = ring_push<R, T>(r7, Jz[7], yf[7 * kBN + col], slot, inv_n);
    qb[8] = ring_push<R, T>(r8, Jz[8], yf[8 * kBN + col], slot, inv_n);
    qb[9] = ring_push<R, T>(r9, Jz[9], yf[9 * kBN + col], slot, inv_n);
    if (slot == 2 * R - 1) {
      ring_reseed<R, T>(r0, Jz[0]);
      ring_reseed<R, T>(r1, Jz[1]);
      ring_reseed<R, T>(r2, Jz[2]);
      ring_reseed<R, T>(r3, Jz[3]);
      ring_reseed<R, T>(r4, Jz[4]);
      ring_reseed<R, T>(r5, Jz[5]);
      ring_reseed<R, T>(r6, Jz[6]);
      ring_reseed<R, T>(r7, Jz[7]);
      ring_reseed<R, T>(r8, Jz[8]);
      ring_reseed<R, T>(r9, Jz[9]);
    }
    const int zo = za - R;
    const int us = (k - 2 * R + 3) % 3;
    float cur_rb = 1.f, cur_tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (full) {  // uniform
      const T rinv = (T)1 / qb[0];
      const T uT[3] = {qb[1] * rinv, qb[2] * rinv, qb[3] * rinv};
      cur_rb = (float)qb[0];
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
      if (interior && zo >= z0 && zo < z1) {
        const int64_t g = (int64_t)zo * plane + (int64_t)gy * A.nx + gx;
        if (W.rho_bar) W.rho_bar[g] = cur_rb;
        if (W.ut) {
#pragma unroll
          for (int i = 0; i < 3; ++i) W.ut[i * ntot + g] = (float)uT[i];
        }
        if (W.tau) {
#pragma unroll
          for (int s = 0; s < 6; ++s) W.tau[s * ntot + g] = cur_tau[s];
        }
      }
    }
    // every step: the ring reads of yf are done before the next staging overwrites it, and
    // the velocity of plane zo is in LDS before the gradient reads it
    __syncthreads();
    const int zg = zo - 1;
    if (k >= 2 * R + 1 && zg >= z0 && zg < z1) {  // uniform
      // ---- epilogue B: gradient, closures, statistics of plane zg
      const int sg = (us + 2) % 3, sm = (us + 1) % 3, sp = us;
      PointOut P;
      float u[3] = {0.f, 0.f, 0.f};
      if (interior) {
        const float* uc = su + sg * 3 * kBN;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float* ui = uc + i * kBN;
          P.G[i][0] = (ui[col + 1] - ui[col - 1]) * A.inv2h;
          P.G[i][1] = (ui[col + kBX] - ui[col - kBX]) * A.inv2h;
          P.G[i][2] = (su[(sp * 3 + i) * kBN + col] - su[(sm * 3 + i) * kBN + col]) * A.inv2h;
          u[i] = ui[col];
        }
        point_closures(W, lag_rb, lag_tau, P);
        const int64_t g = (int64_t)zg * plane + (int64_t)gy * A.nx + gx;
        store_point(W, g, ntot, P);
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) P.G[i][j] = 0.f;
#pragma unroll
        for (int s = 0; s < 6; ++s) P.tgm[s] = P.tsm[s] = 0.f;
        P.ksgs = P.nut = P.omt = 0.f;
      }
      StatIn I;
      stat_inputs(lag_rb, u, lag_tau, P, interior, I);
      accumulate_stats(I, acc);
    }
    if (full) {
      lag_rb = cur_rb;
#pragma unroll
      for (int s = 0; s < 6; ++s) lag_tau[s] = cur_tau[s];
    }
  }
  write_stats(W.partials + ((int64_t)item * (kBT / 64) + (tid >> 6)) * kNStat, acc);
}

template <int R, typename T>
__global__ void __launch_bounds__(kBT) k_box1(FilterArgs A) {
  __shared__ double smem[BoxLds<R, T>::doubles];
  int widx, item;
  if (!map_block(A, widx, item)) return;
  box_body<R, T>(A, A.wa[widx], item, reinterpret_cast<unsigned char*>(smem));
}

constexpr int bmax(int a, int b) { return a > b ? a : b; }

// Box widths 2h, 4h, 8h, 16h in one launch: FP64 sums for the two narrow widths.
__global__ void __launch_bounds__(kBT) k_box4(FilterArgs A) {
  __shared__ double smem[bmax(bmax(BoxLds<1, double>::doubles, BoxLds<2, double>::doubles),
                              bmax(BoxLds<4, float>::doubles, BoxLds<8, float>::doubles))];
  int widx, item;
  if (!map_block(A, widx, item)) return;
  unsigned char* s = reinterpret_cast<unsigned char*>(smem);
  switch (widx) {
    case 0: box_body<1, double>(A, A.wa[0], item, s); break;
    case 1: box_body<2, double>(A, A.wa[1], item, s); break;
    case 2: box_body<4, float>(A, A.wa[2], item, s); break;
    default: box_body<8, float>(A, A.wa[3], item, s); break;
  }
}

}  // namespace

int box_tile_x() { return kBOX; }
int box_tile_y() { return kBOY; }
int box_stat_waves() { return kBT / 64; }
bool box_supported(int R, int fp64) { return R >= 1 && (fp64 ? R <= 4 : R <= 8); }

hipError_t launch_box(const FilterArgs& a, const int* radii, const int* fp64, int nblocks,
                      hipStream_t s) {
  const dim3 block(kBT), grid(nblocks);
  if (a.nw == 4) {
    if (!(radii[0] == 1 && radii[1] == 2 && radii[2] == 4 && radii[3] == 8 && fp64[0] &&
          fp64[1] && !fp64[2] && !fp64[3]))
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_box4, grid, block, 0, s, a);
    return hipGetLastError();
  }
  if (a.nw != 1) return hipErrorInvalidValue;
  if (fp64[0]) {
    switch (radii[0]) {
      case 1: hipLaunchKernelGGL((k_box1<1, double>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_box1<2, double>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_box1<3, double>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_box1<4, double>), grid, block, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (radii[0]) {
      case 1: hipLaunchKernelGGL((k_box1<1, float>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_box1<2, float>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_box1<3, float>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_box1<4, float>), grid, block, 0, s, a); break;
      case 5: hipLaunchKernelGGL((k_box1<5, float>), grid, block, 0, s, a); break;
      case 6: hipLaunchKernelGGL((k_box1<6, float>), grid, block, 0, s, a); break;
      case 7: hipLaunchKernelGGL((k_box1<7, float>), grid, block, 0, s, a); break;
      case 8: hipLaunchKernelGGL((k_box1<8, float>), grid, block, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace kcf
