// Separable periodic filter with arbitrary symmetric taps w_{-R..R} (the Gaussian kernel, and
// box widths the sliding-sum kernel does not cover), as two streaming kernels:
//
//   k_taps_xy  one workgroup per (16x16 tile, plane): the ten products rho, rho u_i,
//              rho u_i u_j of the tile and its R-cell halo are staged in LDS (odd row stride),
//              filtered along x in place (each task holds one row in registers), then
//              along y, and written to a z-slab buffer [10][planes][ny][nx];
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

constexpr int kTX = 16, kTY = 16;  // output tile of k_taps_xy
constexpr int kTT = 256;           // threads of k_taps_xy
constexpr int kZB = 256;           // threads of k_taps_z

template <int R, typename T>
struct TapLds {
  static constexpr int HX = kTX + 2 * R;
  static constexpr int HY = kTY + 2 * R;
  static constexpr int HXP = HX | 1;
  static constexpr int NRAW = HX * HY;
  static constexpr int QS = HY * HXP;
  static constexpr int doubles = (10 * QS * (int)sizeof(T) + 7) / 8;
};

template <typename T>
__device__ __forceinline__ const T* tap_weights(const TapArgs& A);
template <>
__device__ __forceinline__ const float* tap_weights<float>(const TapArgs& A) { return A.w; }
template <>
__device__ __forceinline__ const double* tap_weights<double>(const TapArgs& A) { return A.wd; }

template <int R, typename T>
__global__ void __launch_bounds__(kTT) k_taps_xy(TapArgs A) {
  using L = TapLds<R, T>;
  constexpr int HX = L::HX, HY = L::HY, HXP = L::HXP, QS = L::QS;
  __shared__ double smem[L::doubles];
  T* buf = reinterpret_cast<T*>(smem);
  const T* w = tap_weights<T>(A);
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int p = blockIdx.y;  // buffer plane
  const int tx = tile % A.ntx, ty = tile / A.ntx;
  const int x0 = tx * kTX, y0 = ty * kTY;
  const int64_t plane = (int64_t)A.nx * A.ny;
  const int64_t zoff = (int64_t)wrapi(A.zb + p, A.nz) * plane;
  // ---- products of the tile and its halo
  for (int r = tid; r < L::NRAW; r += kTT) {
    const int hx = r % HX, hy = r / HX;
    const int64_t g = zoff + (int64_t)wrapi(y0 - R + hy, A.ny) * A.nx + wrapi(x0 - R + hx, A.nx);
    const T rho = (T)A.rho[g];
    const T ux = (T)A.u[g], uy = (T)A.u[g + A.ntot], uz = (T)A.u[g + 2 * A.ntot];
    const T mx = rho * ux, my = rho * uy, mz = rho * uz;
    T* d = buf + hy * HXP + hx;
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
  }
  __syncthreads();
  // ---- x, in place: one (quantity, row) per task
  for (int t = tid; t < 10 * HY; t += kTT) {
    T* v = buf + t * HXP;
    T vr[HX];
#pragma unroll
    for (int i = 0; i < HX; ++i) vr[i] = v[i];
#pragma unroll
    for (int o = 0; o < kTX; ++o) v[o] = tap_sum<R, T>(w, vr, o + R);
  }
  __syncthreads();
  // ---- y: one (quantity, column) per task, straight to the slab buffer
  const int64_t bplane = (int64_t)A.nbuf * plane;
  T* out = reinterpret_cast<T*>(A.xy);
  for (int t = tid; t < 10 * kTX; t += kTT) {
    const int x = t % kTX, q = t / kTX;
    const T* src = buf + q * QS + x;
    T vr[HY];
#pragma unroll
    for (int i = 0; i < HY; ++i) vr[i] = src[i * HXP];
    if (x0 + x < A.nx) {
      T* dst = out + q * bplane + (int64_t)p * plane + x0 + x;
#pragma unroll
      for (int o = 0; o < kTY; ++o)
        if (y0 + o < A.ny) dst[(int64_t)(y0 + o) * A.nx] = tap_sum<R, T>(w, vr, o + R);
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
  const int x = blockIdx.x * kZB + threadIdx.x;
  if (x >= A.nx) return;
  const int y = blockIdx.y;
  const int z0 = A.zo0 + blockIdx.z * ZT;
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
  hipLaunchKernelGGL((k_taps_xy<R, T>), dim3(a.ntx * a.nty, a.nbuf), dim3(kTT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int ZT = z_planes<T>();
  const dim3 gz((a.nx + kZB - 1) / kZB, a.ny, (a.zo1 - a.zo0 + ZT - 1) / ZT);
  hipLaunchKernelGGL((k_taps_z<R, T>), gz, dim3(kZB), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int taps_tile_x() { return kTX; }
int taps_tile_y() { return kTY; }
int taps_z_planes(int fp64) { return fp64 ? z_planes<double>() : z_planes<float>(); }

hipError_t launch_taps(const TapArgs& a, int R, int fp64, hipStream_t s) {
  if (a.ny > 65535 || a.nbuf > 65535) return hipErrorInvalidValue;
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
