// Material stage and tangent operator of the Newton loop for an elasto-
// plastic material (Sec. 3: eq. non_lin_system, Newton linearisation eq.
// lin_system; Alg. 1).  3D trilinear hexahedra, 2x2x2 Gauss points, w =
// V_p/8, small-strain von Mises plasticity with linear isotropic hardening.
//
// Per quadrature point the material holds the committed internal variables
// of the last load increment (plastic strain eps_p, Mandel, and the
// equivalent plastic strain alpha).  The stress update is the radial return
// (Simo & Hughes, Computational Inelasticity, Sec. 3.3):
//
//   s_tr = 2G (dev eps - eps_p),  f = |s_tr| - sqrt(2/3) (sy0 + H alpha)
//   plastic (f > 0): dg = f / (2G + 2H/3), n = s_tr / |s_tr|,
//     sigma = K tr(eps) 1 + s_tr - 2G dg n
//     C = K 1(x)1 + 2G th P_dev - 2G thb n(x)n,
//     th = 1 - 2G dg / |s_tr|, thb = 1/(1 + H/(3G)) - (1 - th)
//   elastic: sigma = K tr(eps) 1 + s_tr, C = K 1(x)1 + 2G P_dev.
//
// The tangent is kept per point as a = 2G th and v = sqrt(2G thb) n, so
// C eps = K tr(eps) 1 + a dev(eps) - v (v . eps): 7 values per point.
//
// Element-centric passes: one thread per voxel gathers its 8 corner
// displacements, forms the strain at the 8 points, applies the material and
// writes the 24 element forces f_e = sum_q w B_q^T sigma_q to fe[24][N];
// k_gather_nodes then sums the 8 element contributions of every node in a
// fixed order (deterministic, no atomics).
#include "fh_internal.h"

namespace fh {
namespace {

constexpr int kPlThreads = 256;

__device__ __forceinline__ int wrapp(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

struct PlasticArgs {
  Grid g;
  const uint8_t* phase;
  const double* params;  // nphase x {K, G, sy0, H}
  double E[6];           // macroscopic strain (RESIDUAL / COMMIT)
  const double* u;       // [3][N] displacement (or p for TANGENT)
  double* fe;            // [24][N] element forces (null in COMMIT)
  double* eps_p;         // [6][8][N] committed plastic strain (updated in COMMIT)
  double* alpha;         // [8][N]
  double* ta;            // [8][N] tangent a = 2G th
  double* tv;            // [6][8][N] tangent v = sqrt(2G thb) n
  double* part;          // per-block partials (kPlParts doubles each)
};

// partial sums per block: macro stress (6), sum fe^2 (1), sum K (1),
// sum a (1), sum v_i v_j (21, upper triangle row by row), plastic points (1)
constexpr int kPlParts = 31;

enum PlMode { PL_RESIDUAL = 0, PL_TANGENT = 1, PL_COMMIT = 2 };

// Fixed-order block reduction of kPlParts values held by every thread
// (unrolled, so that the values stay in registers).
__device__ __forceinline__ void block_reduce_parts(double* v, double* sh, double* out) {
#pragma unroll
  for (int k = 0; k < kPlParts; ++k) {
    sh[threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kPlThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

template <int MODE>
__global__ void __launch_bounds__(kPlThreads) k_plastic(PlasticArgs A) {
  __shared__ double sh[kPlThreads];
  const Grid& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  const double ih[3] = {1.0 / g.h[0], 1.0 / g.h[1], 1.0 / g.h[2]};
  const double w = g.h[0] * g.h[1] * g.h[2] * 0.125;
  // Gauss points 1/2 -+ 1/(2 sqrt 3) per axis; 1/sqrt 2; sqrt(2/3)
  constexpr double gl = 0.21132486540518711775, gh = 0.78867513459481288225;
  constexpr double is2 = 0.70710678118654752440, sq23 = 0.81649658092772603273;
  double acc[kPlParts];
  for (int k = 0; k < kPlParts; ++k) acc[k] = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(e % nx);
    const int y = (int)((e / nx) % ny);
    const int z = (int)(e / ((long long)nx * ny));
    long long node[8];
    double uc[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      node[a] = ((long long)wrapp(z + az, nz) * ny + wrapp(y + ay, ny)) * nx + wrapp(x + ax, nx);
#pragma unroll
      for (int c = 0; c < 3; ++c) uc[a][c] = A.u[c * N + node[a]];
    }
    const int ph = A.phase[e];
    const double K = A.params[4 * ph + 0], G = A.params[4 * ph + 1];
    const double sy0 = A.params[4 * ph + 2], H = A.params[4 * ph + 3];
    double f[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a][0] = f[a][1] = f[a][2] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double xi[3] = {(q & 1) ? gh : gl, ((q >> 1) & 1) ? gh : gl, ((q >> 2) & 1) ? gh : gl};
      // displacement gradient du_c/dx_k at the point
      double Gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      double dN[8][3];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int c0 = a & 1, c1 = (a >> 1) & 1, c2 = (a >> 2) & 1;
        const double L0 = c0 ? xi[0] : 1.0 - xi[0];
        const double L1 = c1 ? xi[1] : 1.0 - xi[1];
        const double L2 = c2 ? xi[2] : 1.0 - xi[2];
        dN[a][0] = (c0 ? 1.0 : -1.0) * L1 * L2 * ih[0];
        dN[a][1] = (c1 ? 1.0 : -1.0) * L0 * L2 * ih[1];
        dN[a][2] = (c2 ? 1.0 : -1.0) * L0 * L1 * ih[2];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) Gu[c][k] += uc[a][c] * dN[a][k];
      }
      // Mandel strain 11, 22, 33, 23, 13, 12
      double eps[6] = {Gu[0][0], Gu[1][1], Gu[2][2], is2 * (Gu[1][2] + Gu[2][1]),
                       is2 * (Gu[0][2] + Gu[2][0]), is2 * (Gu[0][1] + Gu[1][0])};
      if (MODE != PL_TANGENT)
#pragma unroll
        for (int m = 0; m < 6; ++m) eps[m] += A.E[m];
      const double tr = eps[0] + eps[1] + eps[2];
      double dev[6] = {eps[0] - tr / 3.0, eps[1] - tr / 3.0, eps[2] - tr / 3.0, eps[3], eps[4],
                       eps[5]};
      const long long qi = (long long)q * N + e;
      double sig[6];
      if (MODE == PL_TANGENT) {
        const double a = A.ta[qi];
        double v[6], ve = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          v[m] = A.tv[(long long)m * 8 * N + qi];
          ve += v[m] * eps[m];
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) sig[m] = a * dev[m] - v[m] * ve + (m < 3 ? K * tr : 0.0);
      } else {
        double s[6], ns2 = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          s[m] = 2.0 * G * (dev[m] - A.eps_p[(long long)m * 8 * N + qi]);
          ns2 += s[m] * s[m];
        }
        const double ns = sqrt(ns2);
        const double al = A.alpha[qi];
        const double fy = ns - sq23 * (sy0 + H * al);
        double a = 2.0 * G, gthb = 0.0, nv[6] = {0, 0, 0, 0, 0, 0};
        double dg = 0.0;
        if (fy > 0.0) {
          dg = fy / (2.0 * G + 2.0 * H / 3.0);
#pragma unroll
          for (int m = 0; m < 6; ++m) nv[m] = s[m] / ns;
          const double th = 1.0 - 2.0 * G * dg / ns;
          const double thb = 1.0 / (1.0 + H / (3.0 * G)) - (1.0 - th);
          a = 2.0 * G * th;
          gthb = 2.0 * G * thb;
          acc[30] += 1.0;
        }
#pragma unroll
        for (int m = 0; m < 6; ++m)
          sig[m] = s[m] - 2.0 * G * dg * nv[m] + (m < 3 ? K * tr : 0.0);
        if (MODE == PL_COMMIT) {
#pragma unroll
          for (int m = 0; m < 6; ++m) A.eps_p[(long long)m * 8 * N + qi] += dg * nv[m];
          A.alpha[qi] = al + sq23 * dg;
        } else {
          const double sc = sqrt(gthb);
          A.ta[qi] = a;
#pragma unroll
          for (int m = 0; m < 6; ++m) A.tv[(long long)m * 8 * N + qi] = sc * nv[m];
          // mean tangent sums: K, a, v v^T (upper triangle)
          acc[7] += w * K;
          acc[8] += w * a;
          int t = 9;
#pragma unroll
          for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) acc[t++] += w * gthb * nv[i] * nv[j];
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) acc[m] += w * sig[m];
      }
      if (MODE != PL_COMMIT) {
        // element forces: f_a += w sigma_tensor . grad N_a
        const double S[3][3] = {{sig[0], is2 * sig[5], is2 * sig[4]},
                                {is2 * sig[5], sig[1], is2 * sig[3]},
                                {is2 * sig[4], is2 * sig[3], sig[2]}};
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            f[a][c] += w * (S[c][0] * dN[a][0] + S[c][1] * dN[a][1] + S[c][2] * dN[a][2]);
      }
    }
    if (MODE != PL_COMMIT) {
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          A.fe[(long long)(a * 3 + c) * N + e] = f[a][c];
          if (MODE != PL_TANGENT) acc[6] += f[a][c] * f[a][c];
        }
    }
  }
  if (MODE != PL_TANGENT && A.part)
    block_reduce_parts(acc, sh, A.part + (long long)blockIdx.x * kPlParts);
}

// out[c][I] = sign * sum_a fe[a*3+c][I - corner_a] (fixed order a = 0..7);
// part (optional): per-block sum over nodes and components of dot[c][I] *
// out[c][I] (dot null: out itself, i.e. |out|^2).
__global__ void __launch_bounds__(kPlThreads)
k_gather_nodes(Grid g, const double* __restrict__ fe, double sign, double* __restrict__ out,
               const double* __restrict__ dot, double* __restrict__ part) {
  __shared__ double sh[kPlThreads];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  double acc = 0.0;
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx);
    const int y = (int)((I / nx) % ny);
    const int z = (int)(I / ((long long)nx * ny));
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const long long e =
          ((long long)wrapp(z - az, nz) * ny + wrapp(y - ay, ny)) * nx + wrapp(x - ax, nx);
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] += fe[(long long)(a * 3 + c) * N + e];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = sign * s[c];
      out[c * N + I] = v;
      acc += (dot ? dot[c * N + I] : v) * v;
    }
  }
  if (part) {
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kPlThreads / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
  }
}

}  // namespace

int plastic_parts() { return kPlParts; }

int plastic_blocks(const Grid& g, int max_blocks) {
  long long b = (g.N + kPlThreads - 1) / kPlThreads;
  if (b > max_blocks) b = max_blocks;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_plastic_stage(int mode, const Grid& g, const uint8_t* phase,
                                const double* params, const double* E, const double* u,
                                double* fe, double* eps_p, double* alpha, double* ta, double* tv,
                                double* part, int nblocks, hipStream_t s) {
  PlasticArgs A{};
  A.g = g;
  A.phase = phase;
  A.params = params;
  for (int m = 0; m < 6; ++m) A.E[m] = E ? E[m] : 0.0;
  A.u = u;
  A.fe = fe;
  A.eps_p = eps_p;
  A.alpha = alpha;
  A.ta = ta;
  A.tv = tv;
  A.part = part;
  if (mode == PL_RESIDUAL)
    hipLaunchKernelGGL(k_plastic<PL_RESIDUAL>, dim3(nblocks), dim3(kPlThreads), 0, s, A);
  else if (mode == PL_TANGENT)
    hipLaunchKernelGGL(k_plastic<PL_TANGENT>, dim3(nblocks), dim3(kPlThreads), 0, s, A);
  else
    hipLaunchKernelGGL(k_plastic<PL_COMMIT>, dim3(nblocks), dim3(kPlThreads), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_gather_nodes(const Grid& g, const double* fe, double sign, double* out,
                               const double* dot, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_nodes, dim3(nblocks), dim3(kPlThreads), 0, s, g, fe, sign, out, dot,
                     part);
  return hipGetLastError();
}

}  // namespace fh
