// Two-node stencil (Fig. tiling c.2, N_n = 2): every pixel carries its
// lowest corner node and its centre node and is cut into four linear
// triangles (centre + one pixel edge), one centroid point each, weight V_p/4.
// Scalar problems: the two node sets are the two fields of a nodal vector,
// u[0][y][x] at the corners, u[1][y][x] at the centres, each a periodic
// pixel grid, so the FFT passes treat them as two components.
//
// The operator K = D^T W C D is applied node by node from per-phase 5 x 5
// element matrices (corners 0..3 with bit 0 = x offset and bit 1 = y offset,
// centre 4; assembled on the host): a corner node sums row a of the four
// pixels that have it as corner a, a centre node row 4 of its own pixel.
//
// The reference symbol (Alg. 2) is a Hermitian 2 x 2 block per frequency,
// complex because the centre sits half a pixel away from the corner, and of
// rank 1 at xi = 0 (the constants over both node sets); its Moore-Penrose
// pseudo-inverse (eq. block_inversion) drops eigenvalues at or below 1e-10
// of the largest eigenvalue over all frequencies.
#include "fh_internal.h"

namespace fh {
namespace {

constexpr int kTnThreads = 256;

__device__ __forceinline__ int wrapt(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <typename T>
__global__ void __launch_bounds__(kTnThreads)
k_kop_tn(Grid g, const T* __restrict__ u, T* __restrict__ q, const uint8_t* __restrict__ phase,
         const T* __restrict__ kfield, const T* __restrict__ ke, long long ustride,
         long long qstride, const PcgState* st, double* pq_part) {
  __shared__ double red[kTnThreads];
  const int ld = blockIdx.y;
  if (st && st[ld].status != ST_ACTIVE) return;
  const int nx = g.nx, ny = g.ny;
  const long long N = g.N;
  const T* __restrict__ u0 = u + (long long)ld * ustride;
  const T* __restrict__ u1 = u0 + N;
  T* __restrict__ q0 = q + (long long)ld * qstride;
  T* __restrict__ q1 = q0 + N;
  double dot = 0.0;
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx), y = (int)(I / nx);
    T acc0 = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int ex = wrapt(x - (a & 1), nx), ey = wrapt(y - (a >> 1), ny);
      const long long e = (long long)ey * nx + ex;
      const T* Ke = phase ? ke + 25 * (size_t)phase[e] : ke;
      const T sc = kfield ? kfield[e] : T(1);
      T s = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long long J = (long long)wrapt(ey + (b >> 1), ny) * nx + wrapt(ex + (b & 1), nx);
        s += Ke[a * 5 + b] * u0[J];
      }
      s += Ke[a * 5 + 4] * u1[e];
      acc0 += sc * s;
    }
    const T* Ki = phase ? ke + 25 * (size_t)phase[I] : ke;
    const T sci = kfield ? kfield[I] : T(1);
    T s1 = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long J = (long long)wrapt(y + (b >> 1), ny) * nx + wrapt(x + (b & 1), nx);
      s1 += Ki[20 + b] * u0[J];
    }
    s1 += Ki[24] * u1[I];
    const T acc1 = sci * s1;
    q0[I] = acc0;
    q1[I] = acc1;
    dot += (double)u0[I] * (double)acc0 + (double)u1[I] * (double)acc1;
  }
  if (pq_part) {
    red[threadIdx.x] = dot;
    __syncthreads();
    for (int s = kTnThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) pq_part[(long long)ld * gridDim.x + blockIdx.x] = red[0];
  }
}

// b[load][0][I] = -sum_a k(e) fe[t(e)][load][a], e = I - corner a;
// b[load][1][I] = -k(I) fe[t(I)][load][4]
__global__ void __launch_bounds__(kTnThreads)
k_rhs_tn(Grid g, const uint8_t* __restrict__ phase, const double* __restrict__ kfield,
         const double* __restrict__ fe, int nload, double* __restrict__ b, long long bstride) {
  const int nx = g.nx, ny = g.ny;
  const long long N = g.N;
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx), y = (int)(I / nx);
    int t[4];
    double sc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const long long e = (long long)wrapt(y - (a >> 1), ny) * nx + wrapt(x - (a & 1), nx);
      t[a] = phase ? phase[e] : 0;
      sc[a] = kfield ? kfield[e] : 1.0;
    }
    const int ti = phase ? phase[I] : 0;
    const double si = kfield ? kfield[I] : 1.0;
    for (int ld = 0; ld < nload; ++ld) {
      // corners in antipodal pairs (0, 3), (1, 2): they cancel exactly in a
      // homogeneous medium
      const double p03 = sc[0] * fe[((size_t)t[0] * nload + ld) * 5 + 0] +
                         sc[3] * fe[((size_t)t[3] * nload + ld) * 5 + 3];
      const double p12 = sc[1] * fe[((size_t)t[1] * nload + ld) * 5 + 1] +
                         sc[2] * fe[((size_t)t[2] * nload + ld) * 5 + 2];
      b[(long long)ld * bstride + I] = -(p03 + p12);
      b[(long long)ld * bstride + N + I] = -si * fe[((size_t)ti * nload + ld) * 5 + 4];
    }
  }
}

struct Herm2 {
  double a, d, br, bi;  // [[a, b], [conj(b), d]], b = br + i bi
};

// K^(xi) from the forward spectra of the impulse responses (B layout,
// spec[beta][alpha]); bad |= 1 where the block is not Hermitian
__device__ __forceinline__ Herm2 tn_block(const Grid& g, const cplx<double>* spec,
                                          long long sstride, long long f, int* bad) {
  const long long cs = (long long)g.nxh * g.ny * g.nz;
  const cplx<double> k00 = spec[f], k10 = spec[cs + f];                  // impulse in field 0
  const cplx<double> k01 = spec[sstride + f], k11 = spec[sstride + cs + f];  // field 1
  const double scale = fabs(k00.re) + fabs(k11.re) + hypot(k01.re, k01.im) + 1e-300;
  if (fabs(k00.im) > 1e-12 * scale || fabs(k11.im) > 1e-12 * scale ||
      fabs(k01.re - k10.re) > 1e-12 * scale || fabs(k01.im + k10.im) > 1e-12 * scale)
    *bad = 1;
  Herm2 h;
  h.a = k00.re;
  h.d = k11.re;
  h.br = 0.5 * (k01.re + k10.re);
  h.bi = 0.5 * (k01.im - k10.im);
  return h;
}

__device__ __forceinline__ void herm2_eig(const Herm2& h, double* lo, double* hi) {
  const double m = 0.5 * (h.a + h.d), r = sqrt(0.25 * (h.a - h.d) * (h.a - h.d) + h.br * h.br +
                                                h.bi * h.bi);
  *lo = m - r;
  *hi = m + r;
}

__global__ void __launch_bounds__(kTnThreads)
k_symbol_tn_max(Grid g, const cplx<double>* spec, long long sstride, double* part, int* bad) {
  __shared__ double red[kTnThreads];
  const long long nf = (long long)g.nxh * g.ny * g.nz;
  double mx = 0.0;
  int b = 0;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nf;
       f += (long long)gridDim.x * blockDim.x) {
    double lo, hi;
    herm2_eig(tn_block(g, spec, sstride, f, &b), &lo, &hi);
    mx = fmax(mx, fmax(fabs(lo), fabs(hi)));
  }
  if (b) *bad = 1;
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kTnThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// kplus[4][nfreq] = {k00, k11, Re k01, Im k01} of K^+ / N
__global__ void __launch_bounds__(kTnThreads)
k_symbol_tn(Grid g, const cplx<double>* spec, long long sstride, const double* part, int nb,
            double* kplus, int* bad) {
  __shared__ double tol_s;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < nb; ++i) mx = fmax(mx, part[i]);
    tol_s = 1e-10 * mx;
  }
  __syncthreads();
  const double tol = tol_s;
  const long long nf = (long long)g.nxh * g.ny * g.nz;
  const double invN = 1.0 / (double)g.N;
  int b = 0;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nf;
       f += (long long)gridDim.x * blockDim.x) {
    const Herm2 h = tn_block(g, spec, sstride, f, &b);
    double lo, hi;
    herm2_eig(h, &lo, &hi);
    double p00 = 0.0, p11 = 0.0, pr = 0.0, pi = 0.0;
    if (lo < -tol) b = 1;  // not positive semi-definite
    if (lo > tol) {
      const double det = h.a * h.d - (h.br * h.br + h.bi * h.bi);
      p00 = h.d / det;
      p11 = h.a / det;
      pr = -h.br / det;
      pi = -h.bi / det;
    } else if (hi > tol) {
      // rank one: the pseudo-inverse is v v^H / hi with v v^H the projector
      // (H - lo I) / (hi - lo) on the eigenvector of hi
      const double s = 1.0 / ((hi - lo) * hi);
      p00 = (h.a - lo) * s;
      p11 = (h.d - lo) * s;
      pr = h.br * s;
      pi = h.bi * s;
    }
    kplus[f] = p00 * invN;
    kplus[nf + f] = p11 * invN;
    kplus[2 * nf + f] = pr * invN;
    kplus[3 * nf + f] = pi * invN;
  }
  if (b) *bad = 1;
}

int tn_blocks(long long n) {
  long long b = (n + kTnThreads - 1) / kTnThreads;
  return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

}  // namespace

template <typename T>
hipError_t launch_kop_tn(const Grid& g, const T* u, T* q, const uint8_t* phase, const T* kfield,
                         const T* ke, int nload, long long ustride, long long qstride,
                         const PcgState* st, double* pq_part, int* nblocks_out, hipStream_t s) {
  const int blocks = kop_nblocks(g, false);
  if (nblocks_out) *nblocks_out = blocks;
  hipLaunchKernelGGL(k_kop_tn<T>, dim3(blocks, nload), dim3(kTnThreads), 0, s, g, u, q, phase,
                     kfield, ke, ustride, qstride, st, pq_part);
  return hipGetLastError();
}
template hipError_t launch_kop_tn<double>(const Grid&, const double*, double*, const uint8_t*,
                                          const double*, const double*, int, long long, long long,
                                          const PcgState*, double*, int*, hipStream_t);
template hipError_t launch_kop_tn<float>(const Grid&, const float*, float*, const uint8_t*,
                                         const float*, const float*, int, long long, long long,
                                         const PcgState*, double*, int*, hipStream_t);

hipError_t launch_rhs_tn(const Grid& g, const uint8_t* phase, const double* kfield,
                         const double* fe, int nload, double* b, long long bstride,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_tn, dim3(tn_blocks(g.N)), dim3(kTnThreads), 0, s, g, phase, kfield, fe,
                     nload, b, bstride);
  return hipGetLastError();
}

hipError_t launch_symbol_tn(const Grid& g, const cplx<double>* spec, long long sstride,
                            double* kplus, int* bad_flag, double* part, hipStream_t s) {
  const long long nf = (long long)g.nxh * g.ny * g.nz;
  const int nb = tn_blocks(nf);
  hipLaunchKernelGGL(k_symbol_tn_max, dim3(nb), dim3(kTnThreads), 0, s, g, spec, sstride, part,
                     bad_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_symbol_tn, dim3(nb), dim3(kTnThreads), 0, s, g, spec, sstride, part, nb,
                     kplus, bad_flag);
  return hipGetLastError();
}

}  // namespace fh
