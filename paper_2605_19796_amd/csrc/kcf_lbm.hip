// D3Q27 lattice-Boltzmann collide-and-stream with the kinetic closures (gfx950).
//
// One launch performs one time step on a periodic lattice of FP32 populations stored as 27
// blocks of N values (population i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1), node i + nx (j +
// ny k)). A workgroup owns a 34 x 15 tile of node columns (the 32 x 13 inner ones collide and
// start on a 128-byte row boundary; the ring of one column around them only supplies
// velocities to the central differences) and marches along z:
//   * the 27 populations of the arriving plane are read once (coalesced rows) and kept in
//     registers for one step; their density and velocity go to LDS (three plane slots, one
//     barrier per step), so the plane behind has all six face neighbours' velocities;
//   * the plane behind collides in place: f_neq = f - f0(rho, u) in population space (the
//     product equilibrium), then its 27 Hermite coefficients by three 3-point transforms (D1Q3
//     basis 1, xi, xi^2 - theta along each axis); the closure relaxes the coefficients (the
//     second-order block holds m_cneq; the 17 higher-order components of the tensor-product
//     basis are the rest; density and momentum belong to f0), and the relaxed coefficients go
//     back through the inverse transforms and are added to f0, so every small population keeps
//     its relative precision and 27 registers hold the whole node;
//   * each post-collision population is pushed along its link to the output lattice.
// Closures act on the coefficients as follows (omega = shifted molecular rate, omega_s the SGS
// rate from the trace, m_CE = -2 rho theta tau_hat S):
//   second order, every KC closure : d2' = d2 - omega_s d2 + (omega_s - omega) m_CE
//   higher orders, KC-MP            : dh' = (1 - omega) dh
//                  KC-RB            : dh' = (1 - omega_s) dh
//                  KC-RR            : dh' = (1 - omega) a_rr + (1 - omega_s)(dh - a_rr)
//   KC-RB with the raw xi xi first-order part also changes the density by
//   (omega - omega_s) rho tau_hat tr S; BGK relaxes every non-conserved coefficient by omega.
#include <math.h>

#include "kcf_internal.h"

namespace kcf {

namespace {

constexpr float kTh = 1.0f / 3.0f;
constexpr int kLX = 34, kLY = 15, kLT = kLX * kLY;  // thread columns of a tile (510)
constexpr int kIX = kLX - 2, kIY = kLY - 2;         // colliding columns of a tile
constexpr int kBT = 512;                            // threads: the columns and 2 spare
constexpr int kWaves = kBT / 64;                    // waves of a workgroup

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Three-point transforms along one axis of a 27-array indexed 9 x + 3 y + z. In a forward
// pass the slot along the axis turns from the position (xi = -1, 0, +1) into the degree of
// the D1Q3 polynomial (1, xi, xi^2 - theta); the inverse pass takes coefficients scaled by
// the inverse norms (1, 1/theta, 1/(2 theta^2)) and multiplies by the D1Q3 weights.
template <int Stride>
__device__ __forceinline__ void fwd3(float* v, int b) {
  const float m = v[b], c = v[b + Stride], p = v[b + 2 * Stride];
  const float s = m + p;
  const float d0 = s + c;
  v[b] = d0;
  v[b + Stride] = p - m;
  v[b + 2 * Stride] = fmaf(-kTh, d0, s);
}

template <int Stride>
__device__ __forceinline__ void inv3(float* v, int b) {
  const float e0 = v[b], e1 = v[b + Stride] * 3.0f, e2 = v[b + 2 * Stride] * 4.5f;
  const float side = fmaf(2.0f / 3.0f, e2, e0);  // e0 + (1 - theta) e2
  v[b] = (side - e1) * (1.0f / 6.0f);
  v[b + Stride] = fmaf(-kTh, e2, e0) * (2.0f / 3.0f);
  v[b + 2 * Stride] = (side + e1) * (1.0f / 6.0f);
}

__device__ __forceinline__ void forward(float* v) {
#pragma unroll
  for (int b = 0; b < 9; ++b) fwd3<1>(v, 3 * b);  // z
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int z = 0; z < 3; ++z) fwd3<3>(v, 9 * x + z);  // y
#pragma unroll
  for (int b = 0; b < 9; ++b) fwd3<9>(v, b);  // x
}

__device__ __forceinline__ void inverse(float* v) {
#pragma unroll
  for (int b = 0; b < 9; ++b) inv3<9>(v, b);
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int z = 0; z < 3; ++z) inv3<3>(v, 9 * x + z);
#pragma unroll
  for (int b = 0; b < 9; ++b) inv3<1>(v, 3 * b);
}

__device__ __forceinline__ float upow(const float (&u)[3], const float (&u2)[3], int a, int n) {
  return n == 0 ? 1.0f : (n == 1 ? u[a] : u2[a]);
}

struct NodeStat {  // FP64 sums per lane
  double s[kLbmStat];
};

// One node, in place: populations f, density, velocity and the strain S of the central
// differences. Accumulates the node's statistics when `use`.
template <int M>
__device__ __forceinline__ void collide_node(float (&f)[27], float rho, const float (&u)[3],
                                             const float (&S)[3][3], const LbmArgs& A,
                                             NodeStat& st, bool use) {
  // equilibrium by directions: F[a][p] = 1 + xi u/theta + (xi^2 - theta) u^2 / (2 theta^2)
  float F[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float q = 4.5f * u[a] * u[a];  // u^2 / (2 theta^2)
    const float l = 3.0f * u[a];         // u / theta
    F[a][1] = fmaf(-kTh, q, 1.0f);
    const float side = fmaf(2.0f / 3.0f, q, 1.0f);
    F[a][0] = side - l;
    F[a][2] = side + l;
  }
  const float W1[3] = {1.0f / 6.0f, 2.0f / 3.0f, 1.0f / 6.0f};
  auto f0 = [&](int px, int py, int pz) {
    return rho * (W1[px] * W1[py] * W1[pz]) * F[0][px] * F[1][py] * F[2][pz];
  };
#pragma unroll
  for (int px = 0; px < 3; ++px)
#pragma unroll
    for (int py = 0; py < 3; ++py)
#pragma unroll
      for (int pz = 0; pz < 3; ++pz) f[9 * px + 3 * py + pz] -= f0(px, py, pz);
  float* d = f;
  forward(d);  // Hermite coefficients of f_neq; index 9 ax + 3 ay + az by degree
  const float tau_hat = A.tau_hat, om = A.omega;
  const int i2[6] = {18, 6, 2, 12, 10, 4};   // xx yy zz xy xz yz
  const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
  float oms = om, ksgs = 0.0f, clip = 1.0f;
  // density and momentum belong to f0: their coefficients of f_neq are rounding residue
  d[0] = d[1] = d[3] = d[9] = 0.0f;
  if constexpr (M == kLbmBgk) {  // every coefficient of degree >= 2 relaxes with omega
#pragma unroll
    for (int i = 0; i < 27; ++i) d[i] *= 1.0f - om;
  } else {
    float mce[6];
    const float cce = -2.0f * rho * kTh * tau_hat;
#pragma unroll
    for (int s = 0; s < 6; ++s) mce[s] = cce * S[pa[s]][pb[s]];
    const float trS = S[0][0] + S[1][1] + S[2][2];
    float tr = (d[18] + d[6] + d[2]) - (mce[0] + mce[1] + mce[2]);
    if constexpr (M == kLbmKcrbRaw) tr = fmaf(rho * tau_hat, trS, tr);
    ksgs = 0.5f * fabsf(tr);
    const float nut = A.c_nu * __builtin_amdgcn_sqrtf(ksgs);
    const float nue = fmaxf(A.nu, nut);
    clip = nut <= A.nu ? 1.0f : 0.0f;
    oms = 1.0f / fmaf(3.0f, nue, 0.5f);
    const float dr = oms - om;
    // second order: (1 - omega) m_CE + (1 - omega_s)(m_cneq - m_CE)
#pragma unroll
    for (int s = 0; s < 6; ++s) d[i2[s]] = fmaf(dr, mce[s], (1.0f - oms) * d[i2[s]]);
    // the raw xi xi first-order part moves density: (omega - omega_s) rho tau_hat tr S
    if constexpr (M == kLbmKcrbRaw) d[0] = -dr * rho * tau_hat * trS;
    // higher orders: every index with at least three letters (17 of them)
    float u2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u2[a] = u[a] * u[a];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int az = 0; az < 3; ++az) {
          const int n = ax + ay + az;
          if (n < 3) continue;
          const int i = 9 * ax + 3 * ay + az;
          if constexpr (M == kLbmKcmp) {
            d[i] *= 1.0f - om;
          } else if constexpr (M == kLbmKcrb || M == kLbmKcrbRaw) {
            d[i] *= 1.0f - oms;
          } else {
            // RR reference of eq. kcrr_rr with the seed m_CE: a sum over the pairs of letters,
            // the pair carrying m_CE and the other letters a velocity each
            const int c[3] = {ax, ay, az};
            float rr = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              if (c[a] == 2) {
                float p = mce[a];
#pragma unroll
                for (int b = 0; b < 3; ++b)
                  if (b != a) p *= upow(u, u2, b, c[b]);
                rr += p;
              }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b = a + 1; b < 3; ++b) {
                if (c[a] >= 1 && c[b] >= 1) {
                  const int s = a == 0 ? (b == 1 ? 3 : 4) : 5;
                  const int g = 3 - a - b;
                  float p = (float)(c[a] * c[b]) * mce[s] * upow(u, u2, a, c[a] - 1) *
                            upow(u, u2, b, c[b] - 1) * upow(u, u2, g, c[g]);
                  rr += p;
                }
              }
            // (1 - omega) a_rr + (1 - omega_s)(d - a_rr)
            d[i] = fmaf(dr, rr, (1.0f - oms) * d[i]);
          }
        }
  }
  inverse(d);
#pragma unroll
  for (int px = 0; px < 3; ++px)
#pragma unroll
    for (int py = 0; py < 3; ++py)
#pragma unroll
      for (int pz = 0; pz < 3; ++pz) f[9 * px + 3 * py + pz] += f0(px, py, pz);
  if (use) {
    st.s[0] += (double)rho;
    st.s[1] += (double)(rho * u[0]);
    st.s[2] += (double)(rho * u[1]);
    st.s[3] += (double)(rho * u[2]);
    st.s[4] += 0.5 * (double)rho * ((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
    st.s[5] += (double)oms;
    st.s[6] += (double)clip;
    st.s[7] += (double)ksgs;
  }
}

__device__ __forceinline__ void moments(const float (&f)[27], float& rho, float (&u)[3]) {
  // sums over the planes of constant c_x, c_y and c_z
  float sx[3] = {0.f, 0.f, 0.f}, sy[3] = {0.f, 0.f, 0.f}, sz[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int px = 0; px < 3; ++px)
#pragma unroll
    for (int py = 0; py < 3; ++py) {
      const float a = f[9 * px + 3 * py], b = f[9 * px + 3 * py + 1], c = f[9 * px + 3 * py + 2];
      const float t = a + b + c;
      sx[px] += t;
      sy[py] += t;
      sz[0] += a;
      sz[2] += c;
    }
  rho = sx[0] + sx[1] + sx[2];
  const float ir = 1.0f / rho;
  u[0] = (sx[2] - sx[0]) * ir;
  u[1] = (sy[2] - sy[0]) * ir;
  u[2] = (sz[2] - sz[0]) * ir;
}

// Barrier for LDS hand-offs only: the fences cover the local address space, so loads and
// stores of global memory in flight (the next plane's populations, the pushed outputs) are
// not waited for at the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// XCD-aware block mapping (as for the filter kernels): XCD L % 8 gets a contiguous band of
// (z-chunk, tile) items.
__device__ __forceinline__ bool lbm_block(const LbmArgs& A, int& item) {
  const int L = blockIdx.x;
  const int j = L >> 3;
  item = (L & 7) * A.items_per_xcd + j;
  return j < A.items_per_xcd && item < A.ntiles * A.nzc;
}

template <int M>
__global__ void __launch_bounds__(kBT) k_lbm_step(LbmArgs A) {
  __shared__ float su[3][3][kBT];  // velocity of three planes (spare threads write their own slot)
  int item;
  if (!lbm_block(A, item)) return;
  const int tile = item % A.ntiles, zc = item / A.ntiles;
  const int tx = tile % A.ntx, ty = tile / A.ntx;
  // threads past the 34 x 15 columns (cy == 15) load a wrapped column and never collide
  const int tid = threadIdx.x, cx = tid % kLX, cy = tid / kLX;
  const int x0 = tx * kIX - 1, y0 = ty * kIY - 1;  // column (0, 0): one left of the inner ones
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int gx = wrapi(x0 + cx, nx), gy = wrapi(y0 + cy, ny);
  const bool interior = cx >= 1 && cx <= kIX && cy >= 1 && cy <= kIY && x0 + cx < nx &&
                        y0 + cy < ny;
  const int z0 = zc * A.zlen;
  const int z1 = min(z0 + A.zlen, nz);
  const int nk = (z1 - z0) + 2;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t ntot = A.ntot;
  const uint32_t col = (uint32_t)(gy * nx + gx);
  // push targets within a plane for the links' x and y steps
  uint32_t off_xy[9];
#pragma unroll
  for (int py = 0; py < 3; ++py)
#pragma unroll
    for (int px = 0; px < 3; ++px)
      off_xy[3 * px + py] = (uint32_t)(wrapi(gy + py - 1, ny) * nx + wrapi(gx + px - 1, nx));

  auto load_plane = [&](float (&f)[27], int z) {
    const int64_t zb = (int64_t)wrapi(z, nz) * plane + col;
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = A.fin[(int64_t)i * ntot + zb];
  };

  // populations of three planes per thread: the one behind (collides), the arriving one
  // (moments) and the next one, requested a step ahead
  float fc[27], fp[27], fn[27];
  float rho_p = 1.0f, up[3] = {0.f, 0.f, 0.f}, upp[3] = {0.f, 0.f, 0.f};
  load_plane(fc, z0 - 1);
  NodeStat st;
#pragma unroll
  for (int s = 0; s < kLbmStat; ++s) st.s[s] = 0.0;

  for (int k = 0; k < nk; ++k) {
    const int zl = z0 - 1 + k;
    float rho_c, uc[3];
    moments(fc, rho_c, uc);
    float* slot = &su[k % 3][0][0];
#pragma unroll
    for (int a = 0; a < 3; ++a) slot[a * kBT + tid] = uc[a];
    if (k + 1 < nk) load_plane(fn, zl + 1);
    lds_barrier();
    if (k >= 2 && interior) {
      // plane zl - 1: x and y neighbours from the LDS slot of the previous step, z neighbours
      // from registers (plane zl - 2) and this step (plane zl)
      const float* sp = &su[(k + 2) % 3][0][0];
      float G[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float* ua = sp + a * kBT;
        G[a][0] = 0.5f * (ua[tid + 1] - ua[tid - 1]);
        G[a][1] = 0.5f * (ua[tid + kLX] - ua[tid - kLX]);
        G[a][2] = 0.5f * (uc[a] - upp[a]);
      }
      float S[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = 0.5f * (G[a][b] + G[b][a]);
      collide_node<M>(fp, rho_p, up, S, A, st, true);
      const int zc0 = zl - 1;
      int64_t zoff[3];
#pragma unroll
      for (int pz = 0; pz < 3; ++pz) zoff[pz] = (int64_t)wrapi(zc0 + pz - 1, nz) * plane;
#pragma unroll
      for (int px = 0; px < 3; ++px)
#pragma unroll
        for (int py = 0; py < 3; ++py)
#pragma unroll
          for (int pz = 0; pz < 3; ++pz) {
            const int i = 9 * px + 3 * py + pz;
            A.fout[(int64_t)i * ntot + zoff[pz] + off_xy[3 * px + py]] = fp[i];
          }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      upp[a] = up[a];
      up[a] = uc[a];
    }
    rho_p = rho_c;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      fp[i] = fc[i];
      fc[i] = fn[i];
    }
  }
  if (A.partials) {  // per-wave record: fixed-order wave reduction of the lane sums
    double* rec = A.partials + ((int64_t)item * kWaves + (tid >> 6)) * kLbmStat;
#pragma unroll
    for (int s = 0; s < kLbmStat; ++s) {
      double r = st.s[s];
      r += __shfl_xor(r, 32);
      r += __shfl_xor(r, 16);
      r += __shfl_xor(r, 8);
      r += __shfl_xor(r, 4);
      r += __shfl_xor(r, 2);
      r += __shfl_xor(r, 1);
      if ((tid & 63) == 0) rec[s] = r;
    }
  }
}

// Equilibrium populations of density and velocity fields (eq. discrete_equilibrium).
__global__ void __launch_bounds__(256) k_lbm_equilibrium(const float* rho, const float* u,
                                                          float* f, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float r = rho[p];
  float F[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float v = u[(int64_t)a * n + p];
    const float q = 4.5f * v * v;
    const float l = 3.0f * v;
    F[a][1] = fmaf(-kTh, q, 1.0f);
    const float side = fmaf(2.0f / 3.0f, q, 1.0f);
    F[a][0] = side - l;
    F[a][2] = side + l;
  }
  const float W1[3] = {1.0f / 6.0f, 2.0f / 3.0f, 1.0f / 6.0f};
#pragma unroll
  for (int px = 0; px < 3; ++px)
#pragma unroll
    for (int py = 0; py < 3; ++py)
#pragma unroll
      for (int pz = 0; pz < 3; ++pz)
        f[(int64_t)(9 * px + 3 * py + pz) * n + p] =
            r * (W1[px] * W1[py] * W1[pz]) * F[0][px] * F[1][py] * F[2][pz];
}

}  // namespace

int lbm_tile_x() { return kIX; }
int lbm_tile_y() { return kIY; }
int lbm_records_per_block() { return kWaves; }

hipError_t launch_lbm_step(const LbmArgs& a, int nblocks, hipStream_t s) {
  switch (a.model) {
    case kLbmBgk: hipLaunchKernelGGL(k_lbm_step<kLbmBgk>, dim3(nblocks), dim3(kBT), 0, s, a); break;
    case kLbmKcrb: hipLaunchKernelGGL(k_lbm_step<kLbmKcrb>, dim3(nblocks), dim3(kBT), 0, s, a); break;
    case kLbmKcrbRaw:
      hipLaunchKernelGGL(k_lbm_step<kLbmKcrbRaw>, dim3(nblocks), dim3(kBT), 0, s, a);
      break;
    case kLbmKcmp: hipLaunchKernelGGL(k_lbm_step<kLbmKcmp>, dim3(nblocks), dim3(kBT), 0, s, a); break;
    case kLbmKcrr: hipLaunchKernelGGL(k_lbm_step<kLbmKcrr>, dim3(nblocks), dim3(kBT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lbm_equilibrium(const float* rho, const float* u, float* f, int64_t n,
                                  hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_lbm_equilibrium, dim3((unsigned)nb), dim3(256), 0, s, rho, u, f, n);
  return hipGetLastError();
}

}  // namespace kcf
