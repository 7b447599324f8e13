// PCG scalar updates, deterministic reductions and small vector kernels.
//
// Textbook PCG (the method the paper's Alg. 1 calls, Sec. 4.1) keeps its
// scalars on the device: alpha = rho / p.q, beta = rho'/rho and the stopping
// test rho' <= eta^2 rho0, i.e. the Kref^-1-norm of the residual relative to
// its initial value (Sec. 6, termination criteria).  Each finalize kernel is a
// single block per load case that sums per-block partials in a fixed order,
// so every reduction is bitwise reproducible.
#include "fh_internal.h"

namespace fh {

__device__ double block_sum_fixed(double v, double* sh) {
  // blockDim.x == 256
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Thread t adds part[t], part[t + 256], ... in that order.  The reads of 8
// trips are issued before their additions, so a long list costs one memory
// round trip per 8 trips, not one per trip (same sum, same order).
__device__ double sum_parts(const double* part, int nb, double* sh) {
  double v = 0.0;
  for (int base = threadIdx.x; base < nb; base += 8 * 256) {
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = base + k * 256;
      x[k] = i < nb ? part[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (base + k * 256 < nb) v += x[k];
  }
  return block_sum_fixed(v, sh);
}

// rho0 = r0.z0; a load with rho0 == 0 is already solved (zero iterations).
__global__ void k_finalize_init(PcgState* st, const double* part, int nb) {
  __shared__ double sh[256];
  const int ld = blockIdx.x;
  if (st[ld].status != ST_ACTIVE) return;  // load case masked out by the caller
  const double rho = sum_parts(part + (long long)ld * nb, nb, sh);
  if (threadIdx.x == 0) {
    st[ld].rho = rho;
    st[ld].rho0 = rho;
    st[ld].iter = 0;
    st[ld].last = 1.0;
    if (!(rho > 0.0)) {
      st[ld].status = (rho == 0.0) ? ST_CONVERGED : ST_BREAKDOWN;
      st[ld].last = 0.0;
    } else {
      st[ld].status = ST_ACTIVE;
    }
  }
}

// alpha = rho / (p.q); pending states from the previous iteration settle.
__global__ void k_finalize_alpha(PcgState* st, const double* part, int nb) {
  __shared__ double sh[256];
  const int ld = blockIdx.x;
  const int status = st[ld].status;
  if (status == ST_CONVERGED_PENDING) {
    if (threadIdx.x == 0) st[ld].status = ST_CONVERGED;
    return;
  }
  if (status == ST_MAXIT_PENDING) {
    if (threadIdx.x == 0) st[ld].status = ST_MAXIT;
    return;
  }
  if (status != ST_ACTIVE) return;
  const double pq = sum_parts(part + (long long)ld * nb, nb, sh);
  if (threadIdx.x == 0) {
    if (!(pq > 0.0)) {
      st[ld].status = ST_BREAKDOWN;
    } else {
      st[ld].alpha = st[ld].rho / pq;
    }
  }
}

// rho' = r.z, convergence test, beta = rho'/rho.
__global__ void k_finalize_beta(PcgState* st, const double* part, int nb, double* hist,
                                int hist_len) {
  __shared__ double sh[256];
  const int ld = blockIdx.x;
  if (st[ld].status != ST_ACTIVE) return;
  const double rho_new = sum_parts(part + (long long)ld * nb, nb, sh);
  if (threadIdx.x == 0) {
    PcgState s = st[ld];
    s.iter += 1;
    const double rel = rho_new > 0.0 ? sqrt(rho_new / s.rho0) : 0.0;
    s.last = rel;
    if (hist && s.iter <= hist_len) hist[(long long)ld * hist_len + s.iter - 1] = rel;
    if (!(rho_new >= 0.0)) {
      // r.z < 0 (or NaN): the preconditioned residual norm is not defined
      s.status = ST_BREAKDOWN;
    } else if (rho_new <= s.eta2 * s.rho0) {
      s.status = ST_CONVERGED_PENDING;
    } else if (s.iter >= s.itmax) {
      s.status = ST_MAXIT_PENDING;
    } else {
      s.beta = rho_new / s.rho;
      s.rho = rho_new;
    }
    st[ld] = s;
  }
}

hipError_t launch_finalize_init(PcgState* st, const double* part, int nb, int nload,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_init, dim3(nload), dim3(256), 0, s, st, part, nb);
  return hipGetLastError();
}
hipError_t launch_finalize_alpha(PcgState* st, const double* part, int nb, int nload,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_alpha, dim3(nload), dim3(256), 0, s, st, part, nb);
  return hipGetLastError();
}
hipError_t launch_finalize_beta(PcgState* st, const double* part, int nb, int nload,
                                double* hist, int hist_len, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_beta, dim3(nload), dim3(256), 0, s, st, part, nb, hist,
                     hist_len);
  return hipGetLastError();
}

// ------------------------------------------------------------ dots, sums
constexpr int kDotBlocks = 1024;

__global__ void k_dot_partials(const double* a, const double* b, long long n, double* part) {
  __shared__ double sh[256];
  double v = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    v += a[i] * b[i];
  const double s = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_partials(const double* part, int nb, double* out) {
  __shared__ double sh[256];
  const double s = sum_parts(part, nb, sh);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_field_sum(const double* a, long long n, double* part) {
  __shared__ double sh[256];
  double v = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    v += a[i];
  const double s = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_dot_partials(const double* a, const double* b, long long n, double* part,
                               int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, dim3(nb), dim3(256), 0, s, a, b, n, part);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const double* part, int nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, out);
  return hipGetLastError();
}
// x[seg][k] -= mean_k x[seg][k]: per segment nchunk fixed-order partial sums,
// then every thread sums its segment's partials in the same order.
__global__ void k_seg_part(const double* x, long long n, int nchunk, double* part) {
  __shared__ double sh[256];
  const int seg = blockIdx.y, chunk = blockIdx.x;
  const long long len = (n + nchunk - 1) / nchunk;
  const long long k0 = chunk * len, k1 = k0 + len < n ? k0 + len : n;
  double v = 0.0;
  for (long long k = k0 + threadIdx.x; k < k1; k += 256) v += x[(long long)seg * n + k];
  const double s = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) part[(long long)seg * nchunk + chunk] = s;
}
__global__ void k_seg_sub(double* x, long long n, int nchunk, const double* part) {
  const int seg = blockIdx.y;
  double tot = 0.0;
  for (int c = 0; c < nchunk; ++c) tot += part[(long long)seg * nchunk + c];
  const double mean = tot / (double)n;
  for (long long k = blockIdx.x * 256LL + threadIdx.x; k < n; k += (long long)gridDim.x * 256)
    x[(long long)seg * n + k] -= mean;
}
hipError_t launch_remove_mean(double* x, int nseg, long long n, double* part, int nchunk,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_seg_part, dim3(nchunk, nseg), dim3(256), 0, s, x, n, nchunk, part);
  hipLaunchKernelGGL(k_seg_sub, dim3(256, nseg), dim3(256), 0, s, x, n, nchunk, part);
  return hipGetLastError();
}

// flag = 1 if any entry is not a positive finite number (App. A: the
// conductivity of every voxel must be positive)
__global__ void k_flag_nonpositive(const double* a, long long n, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double v = a[i];
    bad |= !(v > 0.0 && v <= 1.7976931348623157e308);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
hipError_t launch_flag_nonpositive(const double* x, long long n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_nonpositive, dim3(1024), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t launch_field_sum(const double* x, long long n, double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_field_sum, dim3(nb), dim3(256), 0, s, x, n, part);
  return hipGetLastError();
}

// All load-pair products within every microstructure of a batch:
// out[ms][i][j] = sum_k A[ms*G+i][k] * B[ms*G+j][k], G <= 8.  Each block
// reads its chunk of the 2G fields once and reduces its G^2 sums with wave
// shuffles and one barrier (a fixed tree, so the result is deterministic);
// chunks are summed in a fixed order by k_pair_dots_sum.
constexpr int kPairMax = 8;
// G is a template argument so that the G x G accumulators stay in registers
// (with a run-time G the array is indexed dynamically and lives in scratch).
template <int G>
__global__ void __launch_bounds__(256) k_pair_dots(const double* A, const double* B, long long F,
                                                   int nchunk, double* part) {
  __shared__ double sh[4][G * G];
  const int ms = blockIdx.y, chunk = blockIdx.x;
  const long long len = (F + nchunk - 1) / nchunk;
  const long long k0 = chunk * len, k1 = k0 + len < F ? k0 + len : F;
  double acc[G * G];
#pragma unroll
  for (int t = 0; t < G * G; ++t) acc[t] = 0.0;
  for (long long k = k0 + threadIdx.x; k < k1; k += 256) {
    double a[G], b[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      a[i] = A[((long long)ms * G + i) * F + k];
      b[i] = B[((long long)ms * G + i) * F + k];
    }
#pragma unroll
    for (int i = 0; i < G; ++i)
#pragma unroll
      for (int j = 0; j < G; ++j) acc[i * G + j] += a[i] * b[j];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < G * G; ++t) {
    double v = acc[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wave][t] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < G * G)
    part[((long long)ms * nchunk + chunk) * G * G + t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
}
// Chunk sums in a fixed order: thread i of a block adds chunks i, i + 256, ...
// of one entry, then the 256 partial sums are added pairwise (fixed tree).
__global__ void k_pair_dots_sum(const double* part, int nchunk, int GG, double* out) {
  __shared__ double sh[256];
  const int ms = blockIdx.y, t = blockIdx.x;
  double v = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) v += part[((long long)ms * nchunk + c) * GG + t];
  const double tot = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) out[(long long)ms * GG + t] = tot;
}
hipError_t launch_pair_dots(const double* A, const double* B, long long F, int G, int nms,
                            int nchunk, double* part, double* out, hipStream_t s) {
  if (G < 1 || G > kPairMax) return hipErrorInvalidValue;
  const dim3 grid(nchunk, nms);
  switch (G) {
    case 1: hipLaunchKernelGGL(k_pair_dots<1>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 2: hipLaunchKernelGGL(k_pair_dots<2>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 3: hipLaunchKernelGGL(k_pair_dots<3>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 4: hipLaunchKernelGGL(k_pair_dots<4>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 5: hipLaunchKernelGGL(k_pair_dots<5>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 6: hipLaunchKernelGGL(k_pair_dots<6>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    case 7: hipLaunchKernelGGL(k_pair_dots<7>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
    default: hipLaunchKernelGGL(k_pair_dots<8>, grid, dim3(256), 0, s, A, B, F, nchunk, part); break;
  }
  hipLaunchKernelGGL(k_pair_dots_sum, dim3(G * G, nms), dim3(256), 0, s, part, nchunk, G * G, out);
  return hipGetLastError();
}

// Phase histogram (integer counts, order independent) and id check.
__global__ void k_phase_count(const uint8_t* phase, long long n, int nphase,
                              unsigned long long* counts, int* bad) {
  __shared__ unsigned int loc[256];
  loc[threadIdx.x] = 0;
  __syncthreads();
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    atomicAdd(&loc[phase[i]], 1u);
  __syncthreads();
  const unsigned int c = loc[threadIdx.x];
  if (c) {
    if ((int)threadIdx.x >= nphase) atomicOr(bad, 1);
    else atomicAdd(&counts[threadIdx.x], (unsigned long long)c);
  }
}

hipError_t launch_phase_count(const uint8_t* phase, long long n, int nphase,
                              unsigned long long* counts, int* bad, hipStream_t s) {
  long long blocks = (n + 256 * 64 - 1) / (256 * 64);
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_phase_count, dim3((unsigned)blocks), dim3(256), 0, s, phase, n, nphase,
                     counts, bad);
  return hipGetLastError();
}

// --------------------------------------------------------- elementwise
template <typename T>
__global__ void k_fill(T* x, T v, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    x[i] = v;
}
__global__ void k_copy(double* d, const double* s, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    d[i] = s[i];
}
__global__ void k_axpy(double* y, double a, const double* x, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    y[i] += a * x[i];
}
__global__ void k_cast_d2f(const double* s, float* d, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    d[i] = (float)s[i];
}
__global__ void k_add_f2d(double* d, const float* s, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    d[i] += (double)s[i];
}
__global__ void k_cast_masked(const double* src, float* dst, long long F, const PcgState* st) {
  // one load case per blockIdx.y; skipped when its state is not active
  const int ld = blockIdx.y;
  if (st && st[ld].status != ST_ACTIVE) return;
  const double* s = src + (long long)ld * F;
  float* d = dst + (long long)ld * F;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < F; i += (long long)gridDim.x * 256)
    d[i] = (float)s[i];
}
__global__ void k_add_masked(double* dst, const float* src, long long F, const int* mask) {
  const int ld = blockIdx.y;
  if (!mask[ld]) return;
  double* d = dst + (long long)ld * F;
  const float* s = src + (long long)ld * F;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < F; i += (long long)gridDim.x * 256)
    d[i] += (double)s[i];
}
__global__ void k_residual(double* r, const double* b, const double* Kx, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    r[i] = b[i] - Kx[i];
}
__global__ void k_impulse(double* f, long long n, long long pos) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    f[i] = (i == pos) ? 1.0 : 0.0;
}

static inline dim3 ew_grid(long long n) {
  long long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

template <typename T>
hipError_t launch_fill(T* x, T v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, ew_grid(n), dim3(256), 0, s, x, v, n);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, double, long long, hipStream_t);
template hipError_t launch_fill<float>(float*, float, long long, hipStream_t);

hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, ew_grid(n), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double* y, double a, const double* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, ew_grid(n), dim3(256), 0, s, y, a, x, n);
  return hipGetLastError();
}
hipError_t launch_cast_d2f(const double* src, float* dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, ew_grid(n), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_add_f2d(double* dst, const float* src, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f2d, ew_grid(n), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_cast_masked(const double* src, float* dst, long long F, int nload,
                              const PcgState* st, hipStream_t s) {
  dim3 g = ew_grid(F);
  g.y = nload;
  hipLaunchKernelGGL(k_cast_masked, g, dim3(256), 0, s, src, dst, F, st);
  return hipGetLastError();
}
hipError_t launch_add_masked(double* dst, const float* src, long long F, int nload,
                             const int* mask, hipStream_t s) {
  dim3 g = ew_grid(F);
  g.y = nload;
  hipLaunchKernelGGL(k_add_masked, g, dim3(256), 0, s, dst, src, F, mask);
  return hipGetLastError();
}
hipError_t launch_residual(double* r, const double* b, const double* Kx, long long n,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_residual, ew_grid(n), dim3(256), 0, s, r, b, Kx, n);
  return hipGetLastError();
}
hipError_t launch_impulse(double* f, long long n, long long pos, hipStream_t s) {
  hipLaunchKernelGGL(k_impulse, ew_grid(n), dim3(256), 0, s, f, n, pos);
  return hipGetLastError();
}

}  // namespace fh
