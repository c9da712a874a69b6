// HIP kernels (gfx950) that work on stored fields: the gradient/closure pass (gradient,
// plain closures and FP64 statistics from rho_bar, ut, tau), the statistics of the unfiltered
// input (E_k, enstrophy, <rho>), and the FP64 reductions of per-wave partial sums.
// Statistics are folded in a fixed order, so repeated runs give identical bits.
#include "kcf_device.h"

namespace kcf {

namespace {

using namespace dev;

// ---------------------------------------------------------------- standalone closure pass
// Gradient, closures and statistics from stored rho_bar, ut (and tau). A block owns kGX
// consecutive points of one x-row and kGZ planes; each thread marches along z with the three
// planes of ut that the z-derivative needs held in registers, and reads its x and y
// neighbours through the caches (items in XCD bands, x-blocks fastest, then rows: the rows
// y +- 1 a block reads are those its neighbours in the band load). Every lane stays active
// to the end (the statistics are folded across the full wave).
constexpr int kGX = 128, kGZ = 16;

__global__ void __launch_bounds__(kGX) k_grad_closure(ClosureArgs C) {
  const WidthArgs& W = C.wa;
  const int nxb = (C.nx + kGX - 1) / kGX;
  int64_t item;
  if (!xcd_band_item((int64_t)nxb * C.ny * ((C.nz + kGZ - 1) / kGZ), item)) return;
  const int x = (int)(item % nxb) * kGX + threadIdx.x;
  const int y = (int)(item / nxb % C.ny);
  const int z0 = (int)(item / nxb / C.ny) * kGZ;
  const int z1 = min(z0 + kGZ, C.nz);
  const bool valid = x < C.nx;
  const int xc = valid ? x : 0;
  const int64_t plane = (int64_t)C.nx * C.ny;
  const int64_t row = (int64_t)y * C.nx;
  const int xp = xc + 1 == C.nx ? 0 : xc + 1;
  const int xm = xc == 0 ? C.nx - 1 : xc - 1;
  const int64_t yp = (int64_t)(y + 1 == C.ny ? 0 : y + 1) * C.nx;
  const int64_t ym = (int64_t)(y == 0 ? C.ny - 1 : y - 1) * C.nx;
  float w[3][3];  // ut_i at planes z - 1, z, z + 1
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float* ui = C.ut + i * C.ntot;
    w[i][0] = ui[(int64_t)wrapi(z0 - 1, C.nz) * plane + row + xc];
    w[i][1] = ui[(int64_t)z0 * plane + row + xc];
  }
  static_assert(kGZ <= kStatFlush, "one flush of the statistics per thread");
  StatPart part;
  stat_zero(part);
  for (int z = z0; z < z1; ++z) {
    const int64_t base = (int64_t)z * plane;
    const int64_t zpb = (int64_t)(z + 1 == C.nz ? 0 : z + 1) * plane;
    const int64_t g = base + row + xc;
    PointOut P;
    float u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float* ui = C.ut + i * C.ntot;
      w[i][2] = ui[zpb + row + xc];
      P.G[i][0] = (ui[base + row + xp] - ui[base + row + xm]) * C.inv2h;
      P.G[i][1] = (ui[base + yp + xc] - ui[base + ym + xc]) * C.inv2h;
      P.G[i][2] = (w[i][2] - w[i][0]) * C.inv2h;
      u[i] = w[i][1];
    }
    const float rb = C.rho_bar[g];
    float tau[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (C.tau) {
#pragma unroll
      for (int s = 0; s < 6; ++s) tau[s] = C.tau[s * C.ntot + g];
    }
    point_closures(W, rb, tau, P);
    if (valid) store_point(W, g, C.ntot, P);
    if (W.partials) {  // uniform
      stat_point(rb, u, tau, P.G, P.tgm, smag_dissipation(W, rb, P.G), valid, part);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      w[i][0] = w[i][1];
      w[i][1] = w[i][2];
    }
  }
  if (W.partials) {
    double acc = 0.0;
    stat_flush(part, acc);
    write_stat_record(W.partials + (item * (kGX / 64) + (threadIdx.x >> 6)) * kNStat, acc);
  }
}

// ---------------------------------------------------------------- input statistics
// E_k, enstrophy (sixth-order central vorticity) and <rho> of the unfiltered input. A block
// owns kIX consecutive points of one x-row and kIZ planes; each thread marches along z with
// the seven planes of u_x and u_y that the z-derivatives need held in registers, reads the y
// neighbours of its plane through the caches, one plane ahead of their use, as a uniform
// plane base plus 32-bit offsets, and takes the x neighbours from the block's row of u_z and
// u_y in LDS (its own values plus a three-point halo on each side, loaded by six threads), so
// that the vector memory path carries 18 loads per point instead of 28. Items in XCD bands,
// x-blocks fastest, then rows.
constexpr int kIX = 128, kIZ = 16;

__device__ __forceinline__ double d6(float p1, float p2, float p3, float m1, float m2, float m3) {
  return 45.0 * ((double)p1 - (double)m1) - 9.0 * ((double)p2 - (double)m2) +
         ((double)p3 - (double)m3);
}

__global__ void __launch_bounds__(kIX) k_input_stats(InputStatArgs S) {
  const int nxb = (S.nx + kIX - 1) / kIX;
  int64_t item;
  if (!xcd_band_item((int64_t)nxb * S.ny * ((S.nz + kIZ - 1) / kIZ), item)) return;
  const int xb0 = (int)(item % nxb) * kIX;  // first column of the block
  const int x = xb0 + threadIdx.x;
  const int y = (int)(item / nxb % S.ny);
  const int z0 = (int)(item / nxb / S.ny) * kIZ;
  const int z1 = min(z0 + kIZ, S.nz);
  const bool valid = x < S.nx;
  const int tid = threadIdx.x;
  const int nvalid = min(kIX, S.nx - xb0);  // columns of the block inside the grid
  // the row of u_z and u_y of the current plane in LDS (two buffers by plane parity): the
  // block's columns at 3 .. 3 + nvalid - 1, three periodic neighbours on each side
  __shared__ float srow[2][2][kIX + 6];
  const int xc = valid ? x : 0;
  const int64_t plane = (int64_t)S.nx * S.ny;
  // byte offsets within a plane (below 2^32): the column, its y neighbours y +- 1..3 and its
  // x neighbours x +- 1..3 (periodic)
  const uint32_t own = (uint32_t)(y * S.nx + xc) * 4u;
  uint32_t oy[6];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    oy[m] = (uint32_t)(wrapi(y + m + 1, S.ny) * S.nx + xc) * 4u;
    oy[m + 3] = (uint32_t)(wrapi(y - m - 1, S.ny) * S.nx + xc) * 4u;
  }
  // threads 0..5 also bring in the halo: columns xb0 - 3 .. xb0 - 1 and the three after the
  // block's last column, into LDS slots 0..2 and 3 + nvalid .. 5 + nvalid
  const bool halo = tid < 6;
  const int hslot = tid < 3 ? tid : 3 + nvalid + (tid - 3);
  const int hx = tid < 3 ? wrapi(xb0 - 3 + tid, S.nx) : wrapi(xb0 + nvalid + (tid - 3), S.nx);
  const uint32_t oh = (uint32_t)(y * S.nx + hx) * 4u;
  const float* ux = S.u;
  const float* uy = S.u + S.ntot;
  const float* uz = S.u + 2 * S.ntot;
  auto at = [](const float* base, int64_t zoff, uint32_t o) {
    __asm__ volatile("" : "+v"(o));  // keeps the 32-bit offset form of the load
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base + zoff) + o);
  };
  float wx[7], wy[7];  // u_x, u_y at planes z - 3 .. z + 3
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int64_t zoff = (int64_t)wrapi(z0 - 3 + m, S.nz) * plane;
    wx[m] = at(ux, zoff, own);
    wy[m] = at(uy, zoff, own);
  }
  // values of one plane: z-window entry, y and x neighbours, rho and u_z of the column
  struct Pl { float wx6, wy6, zy[6], xy[6], hz, hy, r, vz; };
  auto fetch = [&](int z, Pl& P) {
    const int64_t zp = (int64_t)wrapi(z + 3, S.nz) * plane;
    P.wx6 = at(ux, zp, own);
    P.wy6 = at(uy, zp, own);
    const int64_t zb = (int64_t)z * plane;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      P.zy[m] = at(uz, zb, oy[m]);
      P.xy[m] = at(ux, zb, oy[m]);
    }
    P.hz = P.hy = 0.f;
    if (halo) {  // wave 0 only
      P.hz = at(uz, zb, oh);
      P.hy = at(uy, zb, oh);
    }
    P.r = at(S.rho, zb, own);
    P.vz = at(uz, zb, own);
  };
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  Pl P;
  Pl Q;
  if (z0 < z1) fetch(z0, Q);
  for (int z = z0; z < z1; ++z) {
    P = Q;
    if (z + 1 < z1) fetch(z + 1, Q);
    wx[6] = P.wx6;
    wy[6] = P.wy6;
    // x neighbours of u_z and u_y through the LDS row (one barrier per plane: a buffer is
    // written again two planes later, after every thread has passed the next barrier)
    float (*row)[kIX + 6] = srow[(z - z0) & 1];
    if (tid < nvalid) {
      row[0][3 + tid] = P.vz;
      row[1][3 + tid] = wy[3];
    }
    if (halo) {
      row[0][hslot] = P.hz;
      row[1][hslot] = P.hy;
    }
    __syncthreads();
    float zx[6], yx[6];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      zx[m] = row[0][3 + tid + m + 1];
      zx[m + 3] = row[0][3 + tid - m - 1];
      yx[m] = row[1][3 + tid + m + 1];
      yx[m + 3] = row[1][3 + tid - m - 1];
    }
    const double dy_uz = d6(P.zy[0], P.zy[1], P.zy[2], P.zy[3], P.zy[4], P.zy[5]);
    const double dy_ux = d6(P.xy[0], P.xy[1], P.xy[2], P.xy[3], P.xy[4], P.xy[5]);
    const double dx_uz = d6(zx[0], zx[1], zx[2], zx[3], zx[4], zx[5]);
    const double dx_uy = d6(yx[0], yx[1], yx[2], yx[3], yx[4], yx[5]);
    const double dz_uy = d6(wy[4], wy[5], wy[6], wy[2], wy[1], wy[0]);
    const double dz_ux = d6(wx[4], wx[5], wx[6], wx[2], wx[1], wx[0]);
    const double ox_ = (dy_uz - dz_uy) * S.inv60h;
    const double oy_ = (dz_ux - dx_uz) * S.inv60h;
    const double oz_ = (dx_uy - dy_ux) * S.inv60h;
    const double r = P.r;
    const double vx = wx[3], vy = wy[3], vz = P.vz;
    const double ek = 0.5 * r * (vx * vx + vy * vy + vz * vz);
    const double en = 0.5 * (ox_ * ox_ + oy_ * oy_ + oz_ * oz_);
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
    double* p = S.partials + (item * (kIX / 64) + (threadIdx.x >> 6)) * 4;
    p[0] = a0;
    p[1] = a1;
    p[2] = a2;
    p[3] = a3;
  }
}

// ---------------------------------------------------------------- FP64 partial sums
// Records of nstat sums, reduced in two fixed-order passes (deterministic): each of up to
// kRedBlocks workgroups sums a contiguous chunk of records, 256 / nstat threads per sum
// reading neighbouring statistics of a record together; one workgroup then sums the chunk
// totals in chunk order.
__global__ void __launch_bounds__(256) k_reduce_part(const double* __restrict__ part, int nparts,
                                                     int nstat, int chunk,
                                                     double* __restrict__ red) {
  __shared__ double sh[256];
  const int G = 256 / nstat;  // threads per statistic
  const int t = threadIdx.x, s = t % nstat, g = t / nstat;
  const int r0 = blockIdx.x * chunk, r1 = min(r0 + chunk, nparts);
  double a = 0;
  if (g < G)
    for (int r = r0 + g; r < r1; r += G) a += part[(int64_t)r * nstat + s];
  sh[t] = a;
  __syncthreads();
  if (t < nstat) {
    double b = 0;
    for (int k = 0; k < G; ++k) b += sh[k * nstat + t];
    red[(int64_t)blockIdx.x * nstat + t] = b;
  }
}

// One thread per chunk brings its totals into LDS in one round of loads; then one thread per
// statistic adds them up in chunk order.
__global__ void __launch_bounds__(kRedBlocks) k_reduce_final(const double* __restrict__ red,
                                                             int nblocks, int nstat,
                                                             double* __restrict__ out) {
  __shared__ double sh[kNStat * kRedBlocks];
  const int t = threadIdx.x;
  if (t < nblocks)
    for (int s = 0; s < nstat; ++s) sh[s * kRedBlocks + t] = red[(int64_t)t * nstat + s];
  __syncthreads();
  if (t < nstat) {
    double b = 0;
    for (int k = 0; k < nblocks; ++k) b += sh[t * kRedBlocks + k];
    out[t] = b;
  }
}

constexpr int kCT = 256;  // threads of the reduction-check kernel

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

int64_t grad_closure_records(const ClosureArgs& a) {
  return (int64_t)((a.nx + kGX - 1) / kGX) * a.ny * ((a.nz + kGZ - 1) / kGZ) * (kGX / 64);
}

// 1-D grids of 8 * ceil(items / 8) workgroups (XCD bands)
static int64_t banded_blocks(int64_t items) { return 8 * ((items + 7) / 8); }

hipError_t launch_grad_closure(const ClosureArgs& a, hipStream_t s) {
  const int64_t nb = banded_blocks((int64_t)((a.nx + kGX - 1) / kGX) * a.ny * ((a.nz + kGZ - 1) / kGZ));
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad_closure, dim3((unsigned)nb), dim3(kGX), 0, s, a);
  return hipGetLastError();
}

int64_t input_stats_records(const InputStatArgs& a) {
  return (int64_t)((a.nx + kIX - 1) / kIX) * a.ny * ((a.nz + kIZ - 1) / kIZ) * (kIX / 64);
}

hipError_t launch_input_stats(const InputStatArgs& a, hipStream_t s) {
  const int64_t nb = banded_blocks((int64_t)((a.nx + kIX - 1) / kIX) * a.ny * ((a.nz + kIZ - 1) / kIZ));
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_input_stats, dim3((unsigned)nb), dim3(kIX), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int nstat, double* out,
                         double* scratch, hipStream_t s) {
  if (nstat < 1 || nstat > kNStat || nparts < 0) return hipErrorInvalidValue;
  int nb = (nparts + 63) / 64;
  nb = nb < 1 ? 1 : (nb > kRedBlocks ? kRedBlocks : nb);
  const int chunk = (nparts + nb - 1) / nb;
  hipLaunchKernelGGL(k_reduce_part, dim3(nb), dim3(256), 0, s, partials, nparts, nstat, chunk,
                     scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlocks), 0, s, scratch, nb, nstat, out);
  return hipGetLastError();
}

// Streaming reference: out block j = in block (j mod nin) times (j + 1), element by element;
// nin fields read once and nout fields written once, with the access pattern of the filter
// path's inputs and outputs and no other work.
__global__ void __launch_bounds__(256) k_stream_probe(const float* __restrict__ in, int nin,
                                                      float* __restrict__ out, int nout,
                                                      int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < nin) v[k] = in[(int64_t)k * n + p];
    for (int j = 0; j < nout; ++j) {
      int k = j % nin;
      float x = v[0];
#pragma unroll
      for (int q = 1; q < 8; ++q)
        if (q == k) x = v[q];
      out[(int64_t)j * n + p] = x * (float)(j + 1);
    }
  }
}

hipError_t launch_stream_probe(const float* in, int nin, float* out, int nout, int64_t n,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_stream_probe, dim3(8192), dim3(256), 0, s, in, nin, out, nout, n);
  return hipGetLastError();
}

hipError_t launch_reduce_check(const float* a, const float* b, int64_t n, double* partials,
                               int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_check, dim3(nblocks), dim3(kCT), 0, s, a, b, n, partials);
  return hipGetLastError();
}

}  // namespace kcf
