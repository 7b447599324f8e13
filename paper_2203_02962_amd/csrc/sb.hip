// Strain-based scheme with the finite-element Green operator (Sec. 7.1, eq.
// projection_chceme): CG on the quadrature-point strain field eps for
// Gamma0 C eps = -Gamma0 C e, Gamma0 = D (D^T W Cref D)^+ D^T W.  The
// pseudo-inverse is the displacement scheme's FFT preconditioner; the
// kernels here are the quadrature-point parts: C times a field and its
// weighted divergence (element forces, summed at the nodes by
// launch_gather_nodes), the gradient of a nodal field at the 8 Gauss points
// of every voxel, the Cref- or C-weighted inner products, and the CG vector
// updates.  3D trilinear hexahedra, fields [6][8][N] (Mandel component,
// Gauss point q = qx + 2 qy + 4 qz, voxel).
#include "fh_internal.h"

namespace fh {
namespace {

constexpr int kSbThreads = 256;
constexpr double kGl = 0.21132486540518711775, kGh = 0.78867513459481288225;  // 1/2 -+ 1/(2 sqrt 3)
constexpr double kIs2 = 0.70710678118654752440;                                // 1/sqrt 2

__device__ __forceinline__ int wraps(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// gradient of corner a's shape function at Gauss point q (physical units)
__device__ __forceinline__ void hex_dN(int q, int a, const double ih[3], double d[3]) {
  const double x0 = (q & 1) ? kGh : kGl, x1 = ((q >> 1) & 1) ? kGh : kGl,
               x2 = ((q >> 2) & 1) ? kGh : kGl;
  const int c0 = a & 1, c1 = (a >> 1) & 1, c2 = (a >> 2) & 1;
  const double L0 = c0 ? x0 : 1.0 - x0, L1 = c1 ? x1 : 1.0 - x1, L2 = c2 ? x2 : 1.0 - x2;
  d[0] = (c0 ? 1.0 : -1.0) * L1 * L2 * ih[0];
  d[1] = (c1 ? 1.0 : -1.0) * L0 * L2 * ih[1];
  d[2] = (c2 ? 1.0 : -1.0) * L0 * L1 * ih[2];
}

__device__ __forceinline__ void voxel_xyz(long long e, int nx, int ny, int* x, int* y, int* z) {
  *x = (int)(e % nx);
  *y = (int)((e / nx) % ny);
  *z = (int)(e / ((long long)nx * ny));
}

// fe[a*3+c][e] = sum_q w (B_q^T tau_q)[a, c], tau_q = C_phase (x_q + E)
// (x may be null: tau = C E).
__global__ void __launch_bounds__(kSbThreads)
k_sb_cdiv(Grid g, const uint8_t* __restrict__ phase, const double* __restrict__ C,
          const double* __restrict__ x, Mat6 E, double* __restrict__ fe) {
  const long long N = g.N;
  const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
  const double w = g.h[0] * g.h[1] * g.h[2] * 0.125;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const double* Ce = C + 36 * phase[e];
    double f[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a][0] = f[a][1] = f[a][2] = 0.0;
    // one Gauss point at a time (an unrolled loop over all 8 spills)
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
      double s[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) s[m] = E.v[m] + (x ? x[((long long)m * 8 + q) * N + e] : 0.0);
      double t[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc += Ce[6 * i + j] * s[j];
        t[i] = acc;
      }
      const double S[3][3] = {{t[0], kIs2 * t[5], kIs2 * t[4]},
                              {kIs2 * t[5], t[1], kIs2 * t[3]},
                              {kIs2 * t[4], kIs2 * t[3], t[2]}};
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        double d[3];
        hex_dN(q, a, ih, d);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[a][c] += w * (S[c][0] * d[0] + S[c][1] * d[1] + S[c][2] * d[2]);
      }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) fe[(long long)(a * 3 + c) * N + e] = f[a][c];
  }
}

// out[m][q][e] = (D z) at Gauss point q of voxel e, Mandel component m.
__global__ void __launch_bounds__(kSbThreads)
k_sb_grad(Grid g, const double* __restrict__ z, double* __restrict__ out) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    int x, y, zz;
    voxel_xyz(e, nx, ny, &x, &y, &zz);
    double uc[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const long long I = ((long long)wraps(zz + ((a >> 2) & 1), nz) * ny +
                           wraps(y + ((a >> 1) & 1), ny)) * nx + wraps(x + (a & 1), nx);
#pragma unroll
      for (int c = 0; c < 3; ++c) uc[a][c] = z[c * N + I];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double Gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        double d[3];
        hex_dN(q, a, ih, d);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) Gu[c][k] += uc[a][c] * d[k];
      }
      const double eps[6] = {Gu[0][0], Gu[1][1], Gu[2][2], kIs2 * (Gu[1][2] + Gu[2][1]),
                             kIs2 * (Gu[0][2] + Gu[2][0]), kIs2 * (Gu[0][1] + Gu[1][0])};
#pragma unroll
      for (int m = 0; m < 6; ++m) out[((long long)m * 8 + q) * N + e] = eps[m];
    }
  }
}

// per-block partials of sum_{e,q} w (a_q + Ea)^T M (b_q + Eb), M = Cref
// (Mc) or the voxel's C (C table, when C is not null)
__global__ void __launch_bounds__(kSbThreads)
k_sb_dot(Grid g, const uint8_t* __restrict__ phase, const double* __restrict__ C, Mat6 Mc,
         const double* __restrict__ a, Mat6 Ea, const double* __restrict__ b, Mat6 Eb,
         double* __restrict__ part) {
  __shared__ double sh[kSbThreads];
  const long long N = g.N;
  const double w = g.h[0] * g.h[1] * g.h[2] * 0.125;
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const double* M = C ? C + 36 * phase[e] : Mc.m;
    double ve = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double av[6], bv[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        av[m] = Ea.v[m] + a[((long long)m * 8 + q) * N + e];
        bv[m] = Eb.v[m] + b[((long long)m * 8 + q) * N + e];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) t += M[6 * i + j] * bv[j];
        ve += av[i] * t;
      }
    }
    acc += w * ve;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kSbThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// p = r + beta p
__global__ void k_sb_xpby(double* __restrict__ p, const double* __restrict__ r, double beta,
                          long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

int sb_blocks(long long n) {
  long long b = (n + kSbThreads - 1) / kSbThreads;
  return (int)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

}  // namespace

int sb_dot_partials(const Grid& g) { return sb_blocks(g.N) > 1024 ? 1024 : sb_blocks(g.N); }

hipError_t launch_sb_cdiv(const Grid& g, const uint8_t* phase, const double* C, const double* x,
                          const double* E, double* fe, hipStream_t s) {
  Mat6 Ev{};
  for (int m = 0; m < 6; ++m) Ev.v[m] = E ? E[m] : 0.0;
  hipLaunchKernelGGL(k_sb_cdiv, dim3(sb_blocks(g.N)), dim3(kSbThreads), 0, s, g, phase, C, x, Ev,
                     fe);
  return hipGetLastError();
}

hipError_t launch_sb_grad(const Grid& g, const double* z, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sb_grad, dim3(sb_blocks(g.N)), dim3(kSbThreads), 0, s, g, z, out);
  return hipGetLastError();
}

hipError_t launch_sb_dot(const Grid& g, const uint8_t* phase, const double* C, const double* Mc,
                         const double* a, const double* Ea, const double* b, const double* Eb,
                         double* part, hipStream_t s) {
  Mat6 M{}, A{}, B{};
  if (Mc)
    for (int i = 0; i < 36; ++i) M.m[i] = Mc[i];
  for (int m = 0; m < 6; ++m) {
    A.v[m] = Ea ? Ea[m] : 0.0;
    B.v[m] = Eb ? Eb[m] : 0.0;
  }
  hipLaunchKernelGGL(k_sb_dot, dim3(sb_dot_partials(g)), dim3(kSbThreads), 0, s, g, phase, C, M, a,
                     A, b, B, part);
  return hipGetLastError();
}

hipError_t launch_sb_xpby(double* p, const double* r, double beta, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_sb_xpby, dim3(sb_blocks(n)), dim3(kSbThreads), 0, s, p, r, beta, n);
  return hipGetLastError();
}

}  // namespace fh
