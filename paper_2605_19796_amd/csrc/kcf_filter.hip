// HIP kernels (gfx950) of the filtering path: products -> separable periodic filter ->
// Favre division and SGS tensor -> central-difference gradient -> closures -> FP64 sums.
//
// One workgroup owns an 18x14 column tile of the x-y plane (16x12 output columns plus a
// one-cell halo for the gradient) and marches along z:
//   * every arriving plane is staged into LDS with a halo of R cells (rho, u and a plane of
//     ones, so each filtered quantity is rho * A * B with A, B in {1, u_x, u_y, u_z});
//   * the x and y passes run from LDS into LDS, each thread filtering a register strip;
//   * the z pass keeps the last 2R+1 x-y filtered planes of each column in registers
//     (two threads per column, five quantities each) and indexes the ring with
//     compile-time slots, so no register moves are needed as the window slides;
//   * the epilogue forms rho_bar, ut, tau for plane z-R, keeps ut of three planes in LDS and
//     evaluates the gradient, closures and statistics one plane behind.
// Statistics are accumulated in FP64 with a fixed-order wave reduction, so repeated runs
// give identical bits.
#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

// Filtered quantity q = rho * F[a(q)] * F[b(q)], F planes 0 rho, 1 u_x, 2 u_y, 3 u_z, 4 one.
// q: 0 rho, 1..3 rho u_i, 4..9 rho u_i u_j with ij = xx xy xz yy yz zz.
constexpr unsigned long long kQA = 0x3221113214ull;  // nibble q -> plane a
constexpr unsigned long long kQB = 0x3323214444ull;  // nibble q -> plane b
__device__ __forceinline__ int qa(int q) { return (int)((kQA >> (4 * q)) & 15ull); }
__device__ __forceinline__ int qb(int q) { return (int)((kQB >> (4 * q)) & 15ull); }

// LDS layout of one width: raw planes (float), x-filtered and x-y filtered quantities
// (accumulation type T), Favre velocity of three planes and the lagged rho_bar/tau (float).
template <int R, typename T>
struct Lds {
  static constexpr int HX = kCX + 2 * R;
  static constexpr int HY = kCY + 2 * R;
  static constexpr int NRAW = HX * HY;
  static constexpr int raw = ((5 * NRAW * 4) + 7) / 8 * 8;
  static constexpr int sx = 10 * HY * kCX * (int)sizeof(T);
  static constexpr int sy = 10 * kNCol * (int)sizeof(T);
  static constexpr int su = 9 * kNCol * 4;
  static constexpr int slag = 14 * kNCol * 4;
  static constexpr int bytes = raw + sx + sy + su + slag;
  static constexpr int doubles = (bytes + 7) / 8;
};


// ---------------------------------------------------------------- z ring (compile-time slots)
template <int D, int S, typename T, typename WT>
__device__ __forceinline__ void ring_step(T (&ring)[5][D], const T (&val)[5], T (&out)[5],
                                          const WT* __restrict__ w) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    ring[j][S] = val[j];
    T s = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) s = fma((T)w[t], ring[j][(S + 1 + t) % D], s);
    out[j] = s;
  }
}

template <int D, int S = 0, typename T, typename WT>
__device__ __forceinline__ void ring_dispatch(int slot, T (&ring)[5][D], const T (&val)[5],
                                              T (&out)[5], const WT* __restrict__ w) {
  if constexpr (S < D) {
    if (slot == S)
      ring_step<D, S>(ring, val, out, w);
    else
      ring_dispatch<D, S + 1>(slot, ring, val, out, w);
  }
}

template <typename T>
__device__ __forceinline__ const T* taps(const WidthArgs& W);
template <>
__device__ __forceinline__ const float* taps<float>(const WidthArgs& W) { return W.w; }
template <>
__device__ __forceinline__ const double* taps<double>(const WidthArgs& W) { return W.wd; }

// ---------------------------------------------------------------- the z-marching body
template <int R, typename T>
__device__ __forceinline__ void filter_body(const FilterArgs& A, const WidthArgs& W, int item,
                                            unsigned char* smem) {
  using L = Lds<R, T>;
  constexpr int D = 2 * R + 1;
  constexpr int HX = L::HX;
  constexpr int HY = L::HY;
  constexpr int NRAW = L::NRAW;
  constexpr int NPF = (NRAW + kNT - 1) / kNT;
  float* sraw = reinterpret_cast<float*>(smem);                           // 5 x HY x HX
  T* sx = reinterpret_cast<T*>(smem + L::raw);                             // 10 x HY x CX
  T* sy = reinterpret_cast<T*>(smem + L::raw + L::sx);                     // 10 x NCol
  float* su = reinterpret_cast<float*>(smem + L::raw + L::sx + L::sy);     // 3 x 3 x NCol
  float* slag = su + 9 * kNCol;                                            // 2 x 7 x NCol
  const T* w = taps<T>(W);

  const int tid = threadIdx.x;
  const int tile = item % A.ntiles;
  const int zc = item / A.ntiles;
  int tx, ty;
  tile_coords(A, tile, tx, ty);
  const int x0 = tx * kOX - 1, y0 = ty * kOY - 1;  // global coordinates of column (0, 0)
  const int z0 = zc * A.zlen;
  const int z1 = min(z0 + A.zlen, A.nz);
  const int nsteps = (z1 - z0) + 2 * R + 2;
  const int za0 = z0 - 1 - R;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t ntot = A.ntot;

  for (int p = tid; p < NRAW; p += kNT) sraw[4 * NRAW + p] = 1.0f;

  int pfoff[NPF];
#pragma unroll
  for (int i = 0; i < NPF; ++i) {
    const int p = tid + i * kNT;
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

  const int half = tid >= kNCol ? 1 : 0;
  const int col = half ? tid - kNCol : tid;
  const int cx = col % kCX, cy = col / kCX;
  const int qbase = 5 * half;
  const int gx = x0 + cx, gy = y0 + cy;
  const bool interior = (cx >= 1) && (cx <= kOX) && (cy >= 1) && (cy <= kOY) && (gx < A.nx) &&
                        (gy < A.ny);
  const bool stat_wave = (tid >> 6) < kStatWaves;
  const bool need_grad = needs_gradient(W);

  T ring[5][D];
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int t = 0; t < D; ++t) ring[j][t] = 0;
  StatAcc acc;
  stat_zero(acc);

  for (int k = 0; k < nsteps; ++k) {
    const int za = za0 + k;
    // ---- stage plane za
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      if (pfoff[i] >= 0) {
        const int p = tid + i * kNT;
        sraw[p] = pf[i][0];
        sraw[NRAW + p] = pf[i][1];
        sraw[2 * NRAW + p] = pf[i][2];
        sraw[3 * NRAW + p] = pf[i][3];
      }
    }
    __syncthreads();
    if (k + 1 < nsteps) load_plane(za + 1);
    // ---- x pass: task (q, row) filters one row of CX outputs
    for (int t = tid; t < 10 * HY; t += kNT) {
      const int q = t / HY, row = t - (t / HY) * HY;
      const float* r0 = sraw + row * HX;
      const float* ra = sraw + qa(q) * NRAW + row * HX;
      const float* rb = sraw + qb(q) * NRAW + row * HX;
      T v[HX];
#pragma unroll
      for (int i = 0; i < HX; ++i) v[i] = ((T)r0[i] * (T)ra[i]) * (T)rb[i];
      T* dst = sx + (q * HY + row) * kCX;
#pragma unroll
      for (int o = 0; o < kCX; ++o) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) s = fma(w[m], v[o + m], s);
        dst[o] = s;
      }
    }
    __syncthreads();
    // ---- y pass: task (q, x, part) filters kYP outputs of one column
    for (int t = tid; t < 20 * kCX; t += kNT) {
      const int x = t % kCX;
      const int part = (t / kCX) & 1;
      const int q = t / (2 * kCX);
      const T* src = sx + q * HY * kCX + part * kYP * kCX + x;
      T v[kYP + 2 * R];
#pragma unroll
      for (int i = 0; i < kYP + 2 * R; ++i) v[i] = src[i * kCX];
      T* dst = sy + q * kNCol + part * kYP * kCX + x;
#pragma unroll
      for (int o = 0; o < kYP; ++o) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) s = fma(w[m], v[o + m], s);
        dst[o * kCX] = s;
      }
    }
    __syncthreads();
    // ---- z pass
    {
      T val[5], out[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) val[j] = sy[(qbase + j) * kNCol + col];
      ring_dispatch<D>(k % D, ring, val, out, w);
      if (k < 2 * R) continue;  // ring not full yet (uniform)
#pragma unroll
      for (int j = 0; j < 5; ++j) sy[(qbase + j) * kNCol + col] = out[j];
    }
    __syncthreads();
    // ---- epilogue A: rho_bar, ut, tau of plane zo
    const int zo = za - R;
    const int us = (k - 2 * R) % 3;
    const int ls = (k - 2 * R) & 1;
    const bool store_o = interior && zo >= z0 && zo < z1;
    {
      const T rbT = sy[col];
      const T m[3] = {sy[kNCol + col], sy[2 * kNCol + col], sy[3 * kNCol + col]};
      T uT[3];
      float u[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        uT[i] = m[i] / rbT;
        u[i] = (float)uT[i];
      }
      const float rb = (float)rbT;
      const int64_t g = (int64_t)zo * plane + (int64_t)gy * A.nx + gx;
      // tau_ij = bar(rho u_i u_j) - bar(rho u_i) ut_j; half 0: xx xy xz, half 1: yy yz zz
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int s = half * 3 + c;  // stored component
        const int i = (s < 3) ? 0 : (s < 5 ? 1 : 2);
        const int j = (s == 0) ? 0 : (s == 1 || s == 3) ? 1 : 2;
        const T tq = sy[(4 + s) * kNCol + col];
        const float tv = (float)fma(-m[i], uT[j], tq);
        slag[(ls * 7 + 1 + s) * kNCol + col] = tv;
        if (store_o && W.tau) W.tau[s * ntot + g] = tv;
      }
      if (half == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) su[(us * 3 + i) * kNCol + col] = u[i];
        slag[(ls * 7) * kNCol + col] = rb;
        if (store_o) {
          if (W.rho_bar) W.rho_bar[g] = rb;
          if (W.ut) {
#pragma unroll
            for (int i = 0; i < 3; ++i) W.ut[i * ntot + g] = u[i];
          }
        }
      }
    }
    if (k < 2 * R + 1 || !need_grad) continue;  // the gradient needs the plane above (uniform)
    const int zg = zo - 1;
    if (zg < z0 || zg >= z1) continue;  // uniform
    __syncthreads();
    // ---- epilogue B: gradient, closures and statistics of plane zg
    if (half == 0 || stat_wave) {
      const int sg = (us + 2) % 3, sm = (us + 1) % 3, sp = us;
      const int lg = ls ^ 1;
      PointOut P;
      float rb = 1.f, u[3] = {0.f, 0.f, 0.f}, tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const bool valid = (half == 0) && interior;
      if (valid) {
        const float* uc = su + sg * 3 * kNCol;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float* ui = uc + i * kNCol;
          P.G[i][0] = (ui[col + 1] - ui[col - 1]) * A.inv2h;
          P.G[i][1] = (ui[col + kCX] - ui[col - kCX]) * A.inv2h;
          P.G[i][2] = (su[(sp * 3 + i) * kNCol + col] - su[(sm * 3 + i) * kNCol + col]) * A.inv2h;
          u[i] = ui[col];
        }
        rb = slag[(lg * 7) * kNCol + col];
#pragma unroll
        for (int s = 0; s < 6; ++s) tau[s] = slag[(lg * 7 + 1 + s) * kNCol + col];
        point_closures(W, rb, tau, P);
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
      if (stat_wave && W.partials) {
        StatIn I;
        stat_inputs(rb, u, tau, P, valid, I);
        stat_add(I, acc);
      }
    }
  }
  if (stat_wave && W.partials) {
    write_stats(W.partials + ((int64_t)item * kStatWaves + (tid >> 6)) * kNStat, acc);
  }
}

template <int R, typename T>
__global__ void __launch_bounds__(kNT) k_filter1(FilterArgs A) {
  __shared__ double smem[Lds<R, T>::doubles];
  int widx, item;
  if (!map_block(A, widx, item)) return;
  filter_body<R, T>(A, A.wa[widx], item, reinterpret_cast<unsigned char*>(smem));
}

// ---------------------------------------------------------------- standalone closure pass
constexpr int kCT = 256;

__global__ void __launch_bounds__(kCT) k_grad_closure(ClosureArgs C) {
  const WidthArgs& W = C.wa;
  StatAcc acc;
  stat_zero(acc);
  const int64_t plane = (int64_t)C.nx * C.ny;
  const int64_t stride = (int64_t)gridDim.x * kCT;
  // all lanes run the same trip count so the wave reductions stay converged
  const int64_t trips = (C.ntot + stride - 1) / stride;
  for (int64_t it = 0; it < trips; ++it) {
    const int64_t g = it * stride + (int64_t)blockIdx.x * kCT + threadIdx.x;
    const bool valid = g < C.ntot;
    PointOut P;
    float rb = 1.f, u[3] = {0.f, 0.f, 0.f}, tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid) {
      const int x = (int)(g % C.nx);
      const int y = (int)((g / C.nx) % C.ny);
      const int z = (int)(g / plane);
      const int64_t base = (int64_t)z * plane + (int64_t)y * C.nx;
      const int64_t xp = base + (x + 1 == C.nx ? 0 : x + 1), xm = base + (x == 0 ? C.nx - 1 : x - 1);
      const int64_t yb = (int64_t)z * plane + x;
      const int64_t yp = yb + (int64_t)(y + 1 == C.ny ? 0 : y + 1) * C.nx;
      const int64_t ym = yb + (int64_t)(y == 0 ? C.ny - 1 : y - 1) * C.nx;
      const int64_t zb = (int64_t)y * C.nx + x;
      const int64_t zp = zb + (int64_t)(z + 1 == C.nz ? 0 : z + 1) * plane;
      const int64_t zm = zb + (int64_t)(z == 0 ? C.nz - 1 : z - 1) * plane;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float* ui = C.ut + i * C.ntot;
        P.G[i][0] = (ui[xp] - ui[xm]) * C.inv2h;
        P.G[i][1] = (ui[yp] - ui[ym]) * C.inv2h;
        P.G[i][2] = (ui[zp] - ui[zm]) * C.inv2h;
        u[i] = ui[g];
      }
      rb = C.rho_bar[g];
      if (C.tau) {
#pragma unroll
        for (int s = 0; s < 6; ++s) tau[s] = C.tau[s * C.ntot + g];
      }
      point_closures(W, rb, tau, P);
      store_point(W, g, C.ntot, P);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P.G[i][j] = 0.f;
#pragma unroll
      for (int s = 0; s < 6; ++s) P.tgm[s] = P.tsm[s] = 0.f;
      P.ksgs = P.nut = P.omt = 0.f;
    }
    if (W.partials) {
      StatIn I;
      stat_inputs(rb, u, tau, P, valid, I);
      stat_add(I, acc);
    }
  }
  if (W.partials)
    write_stats(W.partials + ((int64_t)blockIdx.x * (kCT / 64) + (threadIdx.x >> 6)) * kNStat, acc);
}

// ---------------------------------------------------------------- input statistics
// E_k, enstrophy (sixth-order central vorticity) and <rho> of the unfiltered input. A block
// owns kIX consecutive points of one x-row and kIZ planes; each thread marches along z with
// the seven planes of u_x and u_y that the z-derivatives need held in registers, and reads
// the x and y neighbours of its plane through the caches.
constexpr int kIX = 128, kIZ = 16;

__device__ __forceinline__ double d6(float p1, float p2, float p3, float m1, float m2, float m3) {
  return 45.0 * ((double)p1 - (double)m1) - 9.0 * ((double)p2 - (double)m2) +
         ((double)p3 - (double)m3);
}

__global__ void __launch_bounds__(kIX) k_input_stats(InputStatArgs S) {
  const int x = blockIdx.x * kIX + threadIdx.x;
  const int y = blockIdx.y;
  const int z0 = blockIdx.z * kIZ;
  const int z1 = min(z0 + kIZ, S.nz);
  const bool valid = x < S.nx;
  const int xc = valid ? x : 0;
  const int64_t plane = (int64_t)S.nx * S.ny;
  const int64_t row = (int64_t)y * S.nx;
  const float* ux = S.u;
  const float* uy = S.u + S.ntot;
  const float* uz = S.u + 2 * S.ntot;
  int xo[6];      // x + 1, x + 2, x + 3, x - 1, x - 2, x - 3 (periodic)
  int64_t yo[6];  // the same rows, as offsets
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    xo[m] = wrapi(xc + m + 1, S.nx);
    xo[m + 3] = wrapi(xc - m - 1, S.nx);
    yo[m] = (int64_t)wrapi(y + m + 1, S.ny) * S.nx;
    yo[m + 3] = (int64_t)wrapi(y - m - 1, S.ny) * S.nx;
  }
  float wx[7], wy[7];  // u_x, u_y at planes z - 3 .. z + 3
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int64_t g = (int64_t)wrapi(z0 - 3 + m, S.nz) * plane + row + xc;
    wx[m] = ux[g];
    wy[m] = uy[g];
  }
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int z = z0; z < z1; ++z) {
    const int64_t gp = (int64_t)wrapi(z + 3, S.nz) * plane + row + xc;
    wx[6] = ux[gp];
    wy[6] = uy[gp];
    const int64_t base = (int64_t)z * plane;
    const int64_t g = base + row + xc;
    const float* pyy = uy + base + row;
    const float* pzx = uz + base + row;
    const float* pxb = ux + base + xc;
    const float* pzb = uz + base + xc;
    const double dy_uz = d6(pzb[yo[0]], pzb[yo[1]], pzb[yo[2]], pzb[yo[3]], pzb[yo[4]], pzb[yo[5]]);
    const double dy_ux = d6(pxb[yo[0]], pxb[yo[1]], pxb[yo[2]], pxb[yo[3]], pxb[yo[4]], pxb[yo[5]]);
    const double dx_uz = d6(pzx[xo[0]], pzx[xo[1]], pzx[xo[2]], pzx[xo[3]], pzx[xo[4]], pzx[xo[5]]);
    const double dx_uy = d6(pyy[xo[0]], pyy[xo[1]], pyy[xo[2]], pyy[xo[3]], pyy[xo[4]], pyy[xo[5]]);
    const double dz_uy = d6(wy[4], wy[5], wy[6], wy[2], wy[1], wy[0]);
    const double dz_ux = d6(wx[4], wx[5], wx[6], wx[2], wx[1], wx[0]);
    const double ox = (dy_uz - dz_uy) * S.inv60h;
    const double oy = (dz_ux - dx_uz) * S.inv60h;
    const double oz = (dx_uy - dy_ux) * S.inv60h;
    const double r = S.rho[g];
    const double vx = wx[3], vy = wy[3], vz = uz[g];
    const double ek = 0.5 * r * (vx * vx + vy * vy + vz * vz);
    const double en = 0.5 * (ox * ox + oy * oy + oz * oz);
    if (valid) {
      if (isfinite(ek + en + r)) {
        a0 += r;
        a1 += ek;
        a2 += en;
      } else {
        a3 += 1.0;
      }
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      wx[m] = wx[m + 1];
      wy[m] = wy[m + 1];
    }
  }
  // fixed-order wave reduction, then one partial per wave
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a0 += __shfl_xor(a0, d);
    a1 += __shfl_xor(a1, d);
    a2 += __shfl_xor(a2, d);
    a3 += __shfl_xor(a3, d);
  }
  if (__lane_id() == 0) {
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    double* p = S.partials + (blk * (kIX / 64) + (threadIdx.x >> 6)) * 4;
    p[0] = a0;
    p[1] = a1;
    p[2] = a2;
    p[3] = a3;
  }
}

// ---------------------------------------------------------------- FP64 partial sums
__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ part, int nparts,
                                                int nstat, double* __restrict__ out) {
  __shared__ double sh[256];
  const int s = blockIdx.x;
  double a = 0;
  for (int p = threadIdx.x; p < nparts; p += 256) a += part[(int64_t)p * nstat + s];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = sh[0];
}

__global__ void __launch_bounds__(kCT) k_reduce_check(const float* __restrict__ a,
                                                      const float* __restrict__ b, int64_t n,
                                                      double* __restrict__ part) {
  double s0 = 0, s1 = 0, s2 = 0;
  const int64_t stride = (int64_t)gridDim.x * kCT;
  for (int64_t i = (int64_t)blockIdx.x * kCT + threadIdx.x; i < n; i += stride) {
    const double x = a[i];
    s0 += x;
    s1 += x * x;
    if (b) s2 += x * (double)b[i];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    s0 += __shfl_xor(s0, d);
    s1 += __shfl_xor(s1, d);
    s2 += __shfl_xor(s2, d);
  }
  if (__lane_id() == 0) {
    double* p = part + ((int64_t)blockIdx.x * (kCT / 64) + (threadIdx.x >> 6)) * 3;
    p[0] = s0;
    p[1] = s1;
    p[2] = s2;
  }
}

}  // namespace

int kernel_radius_for(int r) {
  const int inst[] = {1, 2, 3, 4, 6, 8, 12};
  for (int v : inst)
    if (r <= v) return v;
  return -1;
}

bool fp64_supported(int kr) { return kr <= 8; }

hipError_t launch_filter(const FilterArgs& a, const int* radii, const int* fp64, int nblocks,
                         hipStream_t s) {
  const dim3 block(kNT);
  const dim3 grid(nblocks);
  if (a.nw != 1) return hipErrorInvalidValue;
#define KCF_CASE(RR)                                                              \
  case RR:                                                                        \
    if (fp64[0]) hipLaunchKernelGGL((k_filter1<RR, double>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_filter1<RR, float>), grid, block, 0, s, a);        \
    break;
  switch (radii[0]) {
    KCF_CASE(1)
    KCF_CASE(2)
    KCF_CASE(3)
    KCF_CASE(4)
    KCF_CASE(6)
    KCF_CASE(8)
    case 12:
      if (fp64[0]) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_filter1<12, float>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
#undef KCF_CASE
  return hipGetLastError();
}

int grad_closure_blocks(int64_t ntot) {
  int64_t b = (ntot + kCT - 1) / kCT;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_grad_closure(const ClosureArgs& a, int* nblocks, hipStream_t s) {
  *nblocks = grad_closure_blocks(a.ntot);
  hipLaunchKernelGGL(k_grad_closure, dim3(*nblocks), dim3(kCT), 0, s, a);
  return hipGetLastError();
}

int64_t input_stats_records(const InputStatArgs& a) {
  return (int64_t)((a.nx + kIX - 1) / kIX) * a.ny * ((a.nz + kIZ - 1) / kIZ) * (kIX / 64);
}

hipError_t launch_input_stats(const InputStatArgs& a, hipStream_t s) {
  const dim3 grid((a.nx + kIX - 1) / kIX, a.ny, (a.nz + kIZ - 1) / kIZ);
  hipLaunchKernelGGL(k_input_stats, grid, dim3(kIX), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int nstat, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nstat), dim3(256), 0, s, partials, nparts, nstat, out);
  return hipGetLastError();
}

hipError_t launch_reduce_check(const float* a, const float* b, int64_t n, double* partials,
                               int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_check, dim3(nblocks), dim3(kCT), 0, s, a, b, n, partials);
  return hipGetLastError();
}

}  // namespace kcf
