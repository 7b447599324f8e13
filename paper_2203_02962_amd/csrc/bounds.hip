// Guaranteed two-sided bounds on the eigenvalues of the preconditioned
// operator Kref^+ K (Sec. 4.3).
//
// For node I the lower bound is the smallest, the upper bound the largest
// generalized eigenvalue of the pair (C, Cref) over the quadrature points in
// the support of phi^I.  Materials are constant per pixel/voxel here, so one
// eigenvalue pair per material table (or one pair for a unit conductivity,
// scaled by the voxel's k) is enough; the host computes those pairs.  The
// support of a one-node stencil's basis function is the set of the 2^dim
// pixels/voxels that have I as a corner, e = I - c for c in {0,1}^dim.
//
// One thread per node: gather the phase bytes (or conductivities) of those
// voxels, take min/max of the table entries, write the two nodal bounds and
// fold them into per-block min/max partials.  Memory-bound: 2^dim phase
// reads per node that mostly hit in cache, 16 B written per node.
#include "fh_internal.h"

namespace fh {
namespace {

constexpr int kBoundThreads = 256;
constexpr int kBoundMaxBlocks = 512;  // 2 partials each: 1024 doubles

__device__ __forceinline__ int wrapn(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// tab: lo/hi pair per material table (phase fields), or the pair of a unit
// conductivity (kfield != null), scaled by k of each voxel.
__global__ void __launch_bounds__(kBoundThreads)
k_node_bounds(Grid g, const uint8_t* __restrict__ phase, const double* __restrict__ kfield,
              const double* __restrict__ tab, double* __restrict__ lo, double* __restrict__ hi,
              double* __restrict__ part) {
  __shared__ double smin[kBoundThreads], smax[kBoundThreads];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ncorner = g.dim == 3 ? 8 : 4;
  double bmin = __builtin_huge_val(), bmax = -__builtin_huge_val();
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < g.N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx);
    const int y = (int)((I / nx) % ny);
    const int z = (int)(I / ((long long)nx * ny));
    double l = __builtin_huge_val(), h = -__builtin_huge_val();
    for (int a = 0; a < ncorner; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const long long e =
          ((long long)wrapn(z - az, nz) * ny + wrapn(y - ay, ny)) * nx + wrapn(x - ax, nx);
      double el, eh;
      if (kfield) {
        const double k = kfield[e];
        el = k * tab[0];
        eh = k * tab[1];
      } else {
        const int t = phase[e];
        el = tab[2 * t];
        eh = tab[2 * t + 1];
      }
      l = fmin(l, el);
      h = fmax(h, eh);
    }
    if (lo) lo[I] = l;
    if (hi) hi[I] = h;
    bmin = fmin(bmin, l);
    bmax = fmax(bmax, h);
  }
  smin[threadIdx.x] = bmin;
  smax[threadIdx.x] = bmax;
  __syncthreads();
  for (int s = kBoundThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

// out[0] = min of the block minima, out[1] = max of the block maxima
__global__ void __launch_bounds__(kBoundThreads)
k_bounds_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double smin[kBoundThreads], smax[kBoundThreads];
  double a = __builtin_huge_val(), b = -__builtin_huge_val();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    a = fmin(a, part[2 * i]);
    b = fmax(b, part[2 * i + 1]);
  }
  smin[threadIdx.x] = a;
  smax[threadIdx.x] = b;
  __syncthreads();
  for (int s = kBoundThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

}  // namespace

int node_bounds_partials(const Grid& g) {
  long long blocks = (g.N + kBoundThreads - 1) / kBoundThreads;
  return (int)(blocks < kBoundMaxBlocks ? blocks : kBoundMaxBlocks);
}

hipError_t launch_node_bounds(const Grid& g, const uint8_t* phase, const double* kfield,
                              const double* tab, double* lo, double* hi, double* part,
                              double* range, hipStream_t s) {
  const int nb = node_bounds_partials(g);
  hipLaunchKernelGGL(k_node_bounds, dim3(nb), dim3(kBoundThreads), 0, s, g, phase, kfield, tab,
                     lo, hi, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBoundThreads), 0, s, part, nb, range);
  return hipGetLastError();
}

}  // namespace fh
