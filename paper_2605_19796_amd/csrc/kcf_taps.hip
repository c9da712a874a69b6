// Separable periodic filter with arbitrary symmetric taps w_{-R..R} (the Gaussian kernel, and
// box widths the sliding-sum kernel does not cover), as two streaming kernels:
//
//   k_taps_xy  one workgroup per (tile, 8 consecutive planes, group of quantities): per
//              plane the products rho, rho u_i, rho u_i u_j of the group over the tile and its
//              R-cell halo are staged in LDS (odd row stride), filtered along both directions
//              and written to a z-slab buffer [10][planes][ny][nx]; the next plane's inputs are
//              requested right after the staging, so their latency passes under the filter
//              passes (one plane per workgroup left ~25 % of the kernel waiting on them). FP32 takes 64x16 tiles and two groups of five
//              quantities, filtered along y first (each task holds one column in registers),
//              then along x (16-point row segments, back to LDS) and copied out along the
//              rows: the y pass runs over the halo columns only once per 64 outputs, which
//              cuts the taps per output by a third against a square tile at R = 12. FP64
//              (narrow widths, small R) takes 16x16 tiles with all ten quantities, x first
//              (whole rows in registers), then y with lanes along x writing the slab buffer:
//              there the taps are cheap, and one staging of the inputs and no second LDS
//              round trip are worth more;
//   k_taps_z   one thread per (x, y) column and 16 (FP32) or 8 (FP64) consecutive output
//              planes: the z taps over a register window of the slab buffer, then the Favre
//              velocity and tau, written to the caller's fields.
//
// Gradient, closures and statistics then run as the standalone closure pass on the stored
// fields. T is the type of the products, of both passes and of the slab buffer: double for
// narrow widths, where tau is a small difference of large filtered products, float otherwise.
#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

// Shape of k_taps_xy per precision: tile width, quantities per workgroup, threads. FP32: 64x16,
// five (71 KB of LDS at R = 12, two workgroups per CU), 512. FP64: 16x16, ten (131 KB at
// R = 12, 65 KB at R = 6), 256.
template <typename T>
constexpr int tile_x() { return sizeof(T) == 8 ? 16 : 64; }
constexpr int kTY = 16;
template <typename T>
constexpr int xy_groups() { return sizeof(T) == 8 ? 1 : 2; }
template <typename T>
constexpr int xy_threads() { return sizeof(T) == 8 ? 256 : 512; }
constexpr int kSeg = 16;           // outputs of one x-pass task
constexpr int kXyPlanes = 8;       // planes of one k_taps_xy workgroup
constexpr int kZB = 256;           // threads of k_taps_z

template <int R, typename T>
struct TapLds {
  static constexpr int HX = tile_x<T>() + 2 * R;
  static constexpr int HY = kTY + 2 * R;
  static constexpr int HXP = HX | 1;
  static constexpr int NRAW = HX * HY;
  static constexpr int QS = HY * HXP;
  static constexpr int QG = 10 / xy_groups<T>();
  static constexpr int doubles = (QG * QS * (int)sizeof(T) + 7) / 8;
};

template <typename T>
__device__ __forceinline__ const T* tap_weights(const TapArgs& A);
template <>
__device__ __forceinline__ const float* tap_weights<float>(const TapArgs& A) { return A.w; }
template <>
__device__ __forceinline__ const double* tap_weights<double>(const TapArgs& A) { return A.wd; }

template <int R, typename T>
__global__ void __launch_bounds__(xy_threads<T>()) k_taps_xy(TapArgs A) {
  using L = TapLds<R, T>;
  constexpr int kTX = tile_x<T>(), kTT = xy_threads<T>();
  constexpr int HX = L::HX, HY = L::HY, HXP = L::HXP, QS = L::QS, kQG = L::QG;
  constexpr int NIT = (L::NRAW + kTT - 1) / kTT;  // staged points per thread
  __shared__ double smem[L::doubles];
  T* buf = reinterpret_cast<T*>(smem);
  const T* w = tap_weights<T>(A);
  const int tid = threadIdx.x;
  // items (group fastest, then tile, then run of planes) in XCD bands: both groups of a tile
  // and its neighbouring tiles run close together on one XCD, whose L2 then serves the
  // inputs the second group and the overlapping halos read again
  constexpr int NG = xy_groups<T>();
  const int ntiles = A.ntx * A.nty;
  int64_t item;
  if (!xcd_band_item((int64_t)NG * ntiles * ((A.nbuf + kXyPlanes - 1) / kXyPlanes), item)) return;
  const int grp = (int)(item % NG);  // quantities kQG grp .. kQG grp + kQG - 1
  const int tile = (int)(item / NG % ntiles);
  const int p0 = (int)(item / NG / ntiles) * kXyPlanes;  // first buffer plane of this workgroup
  const int np = min(kXyPlanes, A.nbuf - p0);
  const int tx = tile % A.ntx, ty = tile / A.ntx;
  const int x0 = tx * kTX, y0 = ty * kTY;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t bplane = (int64_t)A.nbuf * plane;
  // in-plane offsets of this thread's staged points (the same on every plane)
  uint32_t off[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int r = min(tid + it * kTT, L::NRAW - 1);
    const int hx = r % HX, hy = r / HX;
    off[it] = (uint32_t)(wrapi(y0 - R + hy, A.ny) * A.nx + wrapi(x0 - R + hx, A.nx));
  }
  // inputs of the next plane to stage, requested before the passes of the current one
  float raw[NIT][4];
  auto fetch = [&](int p) {
    const int64_t zoff = (int64_t)wrapi(A.zb + p, A.nz) * plane;
    const float* rz = A.rho + zoff;
    const float* uv = A.u + zoff;  // u_x of the plane; u_y, u_z follow at ntot strides
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      if (tid + it * kTT < L::NRAW) {
        raw[it][0] = rz[off[it]];
        raw[it][1] = uv[off[it]];
        raw[it][2] = uv[off[it] + A.ntot];
        raw[it][3] = uv[off[it] + 2 * A.ntot];
      }
    }
  };
  fetch(p0);
  for (int k = 0; k < np; ++k) {
    const int p = p0 + k;  // buffer plane
    if (k > 0) __syncthreads();  // the previous plane's passes are done with the LDS
    // ---- products of the group, tile and halo
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int r = tid + it * kTT;
      if (r >= L::NRAW) continue;
      const int hx = r % HX, hy = r / HX;
      const T rho = (T)raw[it][0];
      const T ux = (T)raw[it][1], uy = (T)raw[it][2], uz = (T)raw[it][3];
      const T mx = rho * ux, my = rho * uy, mz = rho * uz;
      T* d = buf + hy * HXP + hx;
      if constexpr (kQG == 10) {
        d[0] = rho;
        d[QS] = mx;
        d[2 * QS] = my;
        d[3 * QS] = mz;
        d[4 * QS] = mx * ux;
        d[5 * QS] = mx * uy;
        d[6 * QS] = mx * uz;
        d[7 * QS] = my * uy;
        d[8 * QS] = my * uz;
        d[9 * QS] = mz * uz;
      } else if (grp == 0) {  // uniform
        d[0] = rho;
        d[QS] = mx;
        d[2 * QS] = my;
        d[3 * QS] = mz;
        d[4 * QS] = mx * ux;
      } else {
        d[0] = mx * uy;
        d[QS] = mx * uz;
        d[2 * QS] = my * uy;
        d[3 * QS] = my * uz;
        d[4 * QS] = mz * uz;
      }
    }
    __syncthreads();
    if (k + 1 < np) fetch(p + 1);
    if constexpr (kQG == 10) {
      // square FP64 tile: x first, in place, one (quantity, row) per task; then y, one
      // (quantity, column) per task with consecutive lanes on consecutive columns, straight to
      // the slab buffer
      for (int t = tid; t < 10 * HY; t += kTT) {
        T* v = buf + t * HXP;  // row t % HY of quantity t / HY
        T vr[HX];
#pragma unroll
        for (int i = 0; i < HX; ++i) vr[i] = v[i];
#pragma unroll
        for (int o = 0; o < kTX; ++o) v[o] = tap_sum<R, T>(w, vr, o + R);
      }
      __syncthreads();
      T* out = reinterpret_cast<T*>(A.xy) + (int64_t)p * plane;
      for (int t = tid; t < 10 * kTX; t += kTT) {
        const int x = t % kTX, qq = t / kTX;
        const T* src = buf + qq * QS + x;
        T vr[HY];
#pragma unroll
        for (int i = 0; i < HY; ++i) vr[i] = src[i * HXP];
        if (x0 + x < A.nx) {
          T* dst = out + qq * bplane + x0 + x;
#pragma unroll
          for (int o = 0; o < kTY; ++o)
            if (y0 + o < A.ny) dst[(int64_t)(y0 + o) * A.nx] = tap_sum<R, T>(w, vr, o + R);
        }
      }
      continue;
    }
    // ---- y first, in place: one (quantity, column) per task, the tile's rows to rows 0..kTY-1
    for (int t = tid; t < kQG * HX; t += kTT) {
      T* col = buf + (t / HX) * QS + t % HX;
      T vr[HY];
#pragma unroll
      for (int i = 0; i < HY; ++i) vr[i] = col[i * HXP];
#pragma unroll
      for (int o = 0; o < kTY; ++o) col[o * HXP] = tap_sum<R, T>(w, vr, o + R);
    }
    __syncthreads();
    // ---- x: one (quantity, row, 16-point segment) per thread; the results go back to the
    // row's first kTX slots once every window is read
    constexpr int NSEG = kTX / kSeg, NXT = kQG * kTY * NSEG;
    static_assert(NXT <= kTT, "one x-pass task per thread");
    const int sg = tid % NSEG, o = (tid / NSEG) % kTY, q = tid / (NSEG * kTY);
    T res[kSeg];
    if (tid < NXT) {
      const T* src = buf + q * QS + o * HXP + sg * kSeg;
      T vr[kSeg + 2 * R];
#pragma unroll
      for (int i = 0; i < kSeg + 2 * R; ++i) vr[i] = src[i];
#pragma unroll
      for (int j = 0; j < kSeg; ++j) res[j] = tap_sum<R, T>(w, vr, j + R);
    }
    __syncthreads();
    if (tid < NXT) {
      T* dst = buf + q * QS + o * HXP + sg * kSeg;
#pragma unroll
      for (int j = 0; j < kSeg; ++j) dst[j] = res[j];
    }
    __syncthreads();
    // ---- copy-out along x: consecutive lanes take consecutive 16-byte pieces of a tile row
    constexpr int V = 16 / (int)sizeof(T), NV = kTX / V;
    const bool vec = A.nx % V == 0;  // rows start on 16-byte boundaries
    T* out = reinterpret_cast<T*>(A.xy) + (int64_t)kQG * grp * bplane + (int64_t)p * plane;
    for (int e = tid; e < kQG * kTY * NV; e += kTT) {
      const int xv = e % NV, oo = (e / NV) % kTY, qq = e / (NV * kTY);
      const int gx = x0 + xv * V, gy = y0 + oo;
      if (gy >= A.ny || gx >= A.nx) continue;
      const T* src = buf + qq * QS + oo * HXP + xv * V;
      T* dst = out + (int64_t)qq * bplane + (int64_t)gy * A.nx + gx;
      if (vec) {  // gx and nx are multiples of V: the piece lies wholly inside the row
        if constexpr (sizeof(T) == 4)
          *reinterpret_cast<float4*>(dst) = make_float4(src[0], src[1], src[2], src[3]);
        else
          *reinterpret_cast<double2*>(dst) = make_double2(src[0], src[1]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (gx + v < A.nx) dst[v] = src[v];
      }
    }
  }
}

// z taps of one quantity for kZT planes from the slab buffer.
template <int R, typename T, int ZT>
__device__ __forceinline__ void z_taps(const TapArgs& A, const T* w, int q, int64_t col, int z0,
                                       T (&f)[ZT]) {
  const int64_t plane = (int64_t)A.nx * A.ny;
  const T* src = reinterpret_cast<const T*>(A.xy) + (int64_t)q * A.nbuf * plane + col;
  T win[ZT + 2 * R];
#pragma unroll
  for (int i = 0; i < ZT + 2 * R; ++i) {
    // buffer plane of global plane z0 - R + i; past the last output plane of a partial chunk
    // the window is clamped to the buffer (those outputs are not stored)
    const int bi = min(wrapi(z0 - R + i - A.zb, A.nz), A.nbuf - 1);
    win[i] = src[(int64_t)bi * plane];
  }
#pragma unroll
  for (int k = 0; k < ZT; ++k) f[k] = tap_sum<R, T>(w, win, k + R);
}

template <typename T>
constexpr int z_planes() { return sizeof(T) == 8 ? 8 : 16; }

template <int R, typename T>
__global__ void __launch_bounds__(kZB) k_taps_z(TapArgs A) {
  constexpr int ZT = z_planes<T>();
  // items (z-chunk fastest, then x-block, then row y) in contiguous bands per XCD (block L
  // runs on XCD L % 8): the z-chunks of one column block run back to back through one L2,
  // which then serves the 2R window planes neighbouring chunks share
  const int nzc = (A.zo1 - A.zo0 + ZT - 1) / ZT, nxb = (A.nx + kZB - 1) / kZB;
  const int64_t nitems = (int64_t)nzc * nxb * A.ny;
  const int64_t per_xcd = (nitems + 7) / 8;
  const int64_t j = blockIdx.x >> 3;
  const int64_t item = (int64_t)(blockIdx.x & 7) * per_xcd + j;
  if (j >= per_xcd || item >= nitems) return;
  const int zc = (int)(item % nzc);
  const int64_t rest = item / nzc;
  const int x = (int)(rest % nxb) * kZB + threadIdx.x;
  if (x >= A.nx) return;
  const int y = (int)(rest / nxb);
  const int z0 = A.zo0 + zc * ZT;
  const int nk = min(ZT, A.zo1 - z0);
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t col = (int64_t)y * A.nx + x;
  const T* w = tap_weights<T>(A);
  T rinv[ZT], m[3][ZT], f[ZT];  // 1/rho_bar and bar(rho u_i)
  z_taps<R, T, ZT>(A, w, 0, col, z0, f);
#pragma unroll
  for (int k = 0; k < ZT; ++k) {
    rinv[k] = (T)1 / f[k];
    if (k < nk && A.rho_bar) A.rho_bar[(int64_t)(z0 + k) * plane + col] = (float)f[k];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    z_taps<R, T, ZT>(A, w, 1 + i, col, z0, m[i]);
    if (A.ut) {
#pragma unroll
      for (int k = 0; k < ZT; ++k)
        if (k < nk) A.ut[i * A.ntot + (int64_t)(z0 + k) * plane + col] = (float)(m[i][k] * rinv[k]);
    }
  }
  if (!A.tau) return;
  // tau_ij = bar(rho u_i u_j) - bar(rho u_i) ut_j
  const int ii[6] = {0, 0, 0, 1, 1, 2};
  const int jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    z_taps<R, T, ZT>(A, w, 4 + s, col, z0, f);
#pragma unroll
    for (int k = 0; k < ZT; ++k) {
      if (k < nk) {
        const int64_t g = (int64_t)(z0 + k) * plane + col;
        A.tau[s * A.ntot + g] = (float)fma(-m[ii[s]][k], m[jj[s]][k] * rinv[k], f[k]);
      }
    }
  }
}

template <int R, typename T>
hipError_t launch_taps_of(const TapArgs& a, hipStream_t s) {
  const int64_t xy_items =
      (int64_t)xy_groups<T>() * a.ntx * a.nty * ((a.nbuf + kXyPlanes - 1) / kXyPlanes);
  if (8 * ((xy_items + 7) / 8) > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_taps_xy<R, T>), dim3((unsigned)(8 * ((xy_items + 7) / 8))),
                     dim3(xy_threads<T>()), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int ZT = z_planes<T>();
  const int64_t nitems = (int64_t)((a.nx + kZB - 1) / kZB) * a.ny * ((a.zo1 - a.zo0 + ZT - 1) / ZT);
  const int64_t nblocks = 8 * ((nitems + 7) / 8);
  if (nblocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_taps_z<R, T>), dim3((unsigned)nblocks), dim3(kZB), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int taps_tile_x(int fp64) { return fp64 ? tile_x<double>() : tile_x<float>(); }
int taps_tile_y() { return kTY; }
int taps_z_planes(int fp64) { return fp64 ? z_planes<double>() : z_planes<float>(); }

hipError_t launch_taps(const TapArgs& a, int R, int fp64, hipStream_t s) {
#define KCF_TAPS(RR)                                                                  \
  case RR:                                                                            \
    return fp64 ? launch_taps_of<RR, double>(a, s) : launch_taps_of<RR, float>(a, s);
  switch (R) {
    KCF_TAPS(1)
    KCF_TAPS(2)
    KCF_TAPS(3)
    KCF_TAPS(4)
    KCF_TAPS(5)
    KCF_TAPS(6)
    KCF_TAPS(7)
    KCF_TAPS(8)
    KCF_TAPS(9)
    KCF_TAPS(10)
    KCF_TAPS(11)
    KCF_TAPS(12)
    default: return hipErrorInvalidValue;
  }
#undef KCF_TAPS
}

}  // namespace kcf
