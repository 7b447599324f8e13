// Real 3D FFT passes, per-frequency block solve and symbol assembly.
//
// Paper Sec. 4.2 (eq. M_inverse): the reference stiffness is block-circulant,
// so F K_ab F^H is diagonal and M^+ r = F^H K^+ F r; Sec. 5.1: F and F^H are
// applied with FFTs; Sec. 5.2-5.3 (Alg. 2, eq. block_inversion): diag K^_ab
// is the FFT of the impulse response of Kref and every frequency block is
// inverted (pseudo-inverted at the zero frequency).
//
// Transform convention: forward X(k) = sum_j x(j) exp(-2 pi i jk/n)
// (unnormalised); the inverse carries no 1/N here -- the 1/N is folded into
// the stored K^+ (kplus = K^+ / N).
//
// Layouts (per load case, per component c < nd):
//   real field        r[c][z][y][x]
//   A (after x pass)  A[c][z][kx][y]     kx < nxh = nx/2+1, y contiguous
//   B (after y pass)  B[c][kx][ky][z]    z contiguous
// Every pass reads whole lines that are contiguous in memory and writes
// transposed tiles of 16 lines, so each global access is a contiguous run of
// at least 16 complex values.  The z pass works in place on B and, in solve
// mode, applies K^+ per frequency between its forward and inverse FFTs and
// accumulates the Parseval form of r.z.
//
// Each block transforms a batch of lines held in LDS with a Stockham
// autosort FFT (mixed radix 4/2/3/5, ping-pong buffers, one barrier per
// stage); twiddles come from a per-length table staged in LDS.
#include "fh_internal.h"

#include <type_traits>

namespace fh {

constexpr int kThreads = 256;
// x passes: KR real rows per block, two per complex line, so KR/2 * nx <=
// 2048 points.  16 rows always fit (nx <= 256).  At nx = 256 a block of 8
// rows already holds 16 KB of FP64 values, and each thread's reads are then
// all issued at once (measured at 256^3: FP64 forward 416 -> 355 us, inverse
// 509 -> 420 us; FP32 inverse 288 -> 245 us, FP32 forward slower).  FP32
// blocks of 16 rows move half the bytes of FP64 ones, and 32 rows
// (nx <= 128) can be chosen by the autotuner.
// Rows per block of the x passes.  FP32 lines up to 128 take 32 rows when
// the batch tuner chose them (g.xrows) and, untuned, in the forward pass
// (128^3: 157 -> 146 us per 6-load launch; the inverse pass is slower that
// way, 172 -> 226 us).
template <typename T>
static int xpass_rows(const Grid& g, bool inverse) {
  if (g.nx >= 256) return (sizeof(T) == 8 || inverse) ? 8 : 16;
  if (sizeof(T) == 4 && g.nx <= 128 && (g.xrows == 32 || (g.xrows == 0 && !inverse))) return 32;
  return 16;
}

template <typename T>
__device__ __forceinline__ cplx<T> conjg(cplx<T> a) { return {a.re, -a.im}; }
// i*a for sign s: s*i*a
template <typename T>
__device__ __forceinline__ cplx<T> muli(cplx<T> a, int s) {
  return s > 0 ? cplx<T>{-a.im, a.re} : cplx<T>{a.im, -a.re};
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* x, int s) {
  if constexpr (R == 2) {
    cplx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cplx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cplx<T> b0 = cadd(x[1], x[3]), b1 = muli(csub(x[1], x[3]), s);
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  } else if constexpr (R == 8) {
    // 8 = 2 x 4: two radix-4 on even/odd samples, twiddles w8^k, radix-2
    const T h = T(0.70710678118654752440084436210485);
    cplx<T> e[4] = {x[0], x[2], x[4], x[6]};
    cplx<T> o[4] = {x[1], x[3], x[5], x[7]};
    dft_small<T, 4>(e, s);
    dft_small<T, 4>(o, s);
    // o[k] *= exp(s 2 pi i k / 8)
    cplx<T> o1 = {h * (o[1].re - s * o[1].im), h * (o[1].im + s * o[1].re)};
    cplx<T> o2 = muli(o[2], s);
    cplx<T> o3 = {h * (-o[3].re - s * o[3].im), h * (-o[3].im + s * o[3].re)};
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
  } else if constexpr (R == 3) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    cplx<T> t1 = cadd(x[1], x[2]), t2 = csub(x[1], x[2]);
    cplx<T> a = {x[0].re - T(0.5) * t1.re, x[0].im - T(0.5) * t1.im};
    cplx<T> b = muli(cplx<T>{h * t2.re, h * t2.im}, s);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(a, b);
    x[2] = csub(a, b);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2pi/5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4pi/5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2pi/5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4pi/5)
    cplx<T> t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    cplx<T> t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    cplx<T> a1 = {x[0].re + c1 * t1.re + c2 * t2.re, x[0].im + c1 * t1.im + c2 * t2.im};
    cplx<T> a2 = {x[0].re + c2 * t1.re + c1 * t2.re, x[0].im + c2 * t1.im + c1 * t2.im};
    cplx<T> b1 = muli(cplx<T>{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im}, s);
    cplx<T> b2 = muli(cplx<T>{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im}, s);
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
  }
}

// In FP64 LDS lines, element e sits at sw<T>(e) = e + e/8 (one pad slot after
// every 8 complex values), so the power-of-two strides of the early Stockham
// writes (8 or 64 elements apart) spread over all banks; lines are
// lds_stride<T>(n) apart, an odd count, so accesses to the same element of
// consecutive lines (the transposed loads and stores of the passes) fall into
// different banks too.
// FP32 lines (8-byte complex values) keep the plain layout, stride n + 1,
// which measured faster for them.
template <typename T>
__host__ __device__ constexpr int sw(int e) {
  return sizeof(T) == 8 ? e + (e >> 3) : e;
}
template <typename T>
__host__ __device__ constexpr int lds_stride(int n) {
  return sizeof(T) == 8 ? ((n + (n >> 3) + 1) | 1) : n + 1;
}

// Streaming (non-temporal) global accesses for data that is read once and
// not again in this iteration, or written now and read only in the next one.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T v, T* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ cplx<double> ld_nt(const cplx<double>* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {v.x, v.y};
}
__device__ __forceinline__ cplx<float> ld_nt(const cplx<float>* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {v.x, v.y};
}
// The x passes move real rows in runs of kXW consecutive values per lane:
// two in FP32, so that each lane still makes 8-byte accesses, one in FP64
// (nx is even, and every row starts at an even element).
template <typename T>
constexpr int kXW = sizeof(T) == 4 ? 2 : 1;
template <typename T>
struct xvec {
  typedef T type __attribute__((ext_vector_type(kXW<T>)));
};

// Quotient by a block-uniform divisor d >= 1 through one 24-bit multiply:
// with M = ceil(2^21 / d), (x M) >> 21 equals x / d whenever x d <= 2^21 and
// x M < 2^32.  (Write M d = 2^21 + e with 0 <= e < d; the excess x e /
// (d 2^21) of x M / 2^21 over x / d is below 1/d, too little to carry the
// fraction (x mod d) / d <= (d - 1) / d across an integer.)  Every use
// divides a block-local index below 4096 by a line length or count of at
// most 256, with quotients below 32 where the index passes 2048, inside both
// bounds; a generic integer division costs about ten instructions per use.
struct UDiv {
  int d;
  unsigned M;
  __device__ __forceinline__ explicit UDiv(int d_)
      : d(d_), M(((1u << 21) + (unsigned)d_ - 1u) / (unsigned)d_) {}
  __device__ __forceinline__ int q(int x) const {
    return (int)(__umul24((unsigned)x, M) >> 21);
  }
  __device__ __forceinline__ int r(int x, int qq) const { return x - __mul24(qq, d); }
};

// One in-place Stockham stage on `nlines` lines of length n (line stride n):
// every thread first reads its butterflies' inputs into registers, the
// block synchronises, then the results are written back.  L = product of the
// radices of the earlier stages.  A block holds at most kMaxPts points, so a
// thread owns at most kMaxPts / (R * 256) butterflies.
constexpr int kMaxPts = 2048;

// src(line, e) gives element e of a line and sink(line, e, v) stores one;
// with in_place false the inputs come from another buffer and the barrier
// between reads and writes is skipped.  In the first stage (L = 1) every
// twiddle is 1 and the table is not read.  NC and LC, when nonzero, are the
// line length and the stride L known at compile time (power-of-two plans):
// every index then comes from shifts and masks and the element offsets of a
// butterfly fold into the addresses.
template <typename T, int R, int NC = 0, int LC = 0, typename Src, typename Sink>
__device__ __forceinline__ void stockham_stage_io(const Src& src, const Sink& sink, bool in_place,
                                                  int n_rt, int nlines, int L_rt,
                                                  const cplx<T>* tw, int sign) {
  constexpr int MAXIT = (kMaxPts / R + kThreads - 1) / kThreads;
  const int n = NC ? NC : n_rt;
  const int L = LC ? LC : L_rt;
  const int m = n / R;
  const int items = nlines * m;
  const int twstep = n / (L * R);
  const UDiv dm(m), dL(L);
  cplx<T> v[MAXIT][R];
  int dst[MAXIT], de[MAXIT];
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const int it = threadIdx.x + k * kThreads;
    dst[k] = -1;
    if (it < items) {
      int line, j, jl, kk;
      if constexpr (NC > 0 && LC > 0) {
        line = it / (NC / R);
        j = it % (NC / R);
        jl = j / LC;
        kk = j % LC;
      } else {
        line = dm.q(it);
        j = dm.r(it, line);
        jl = dL.q(j);
        kk = dL.r(j, jl);
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        cplx<T> a = src(line, j + t * m);
        if (t > 0 && L > 1) {
          // t*kk < R*L, so the index stays below n
          cplx<T> w = tw[(NC > 0 && LC > 0) ? t * kk * (NC / (LC * R)) : t * __mul24(kk, twstep)];
          if (sign > 0) w.im = -w.im;
          a = cmul(a, w);
        }
        v[k][t] = a;
      }
      dst[k] = line;
      de[k] = (NC > 0 && LC > 0) ? jl * (LC * R) + kk : __mul24(jl, L * R) + kk;
    }
  }
  if (in_place) __syncthreads();
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    if (dst[k] >= 0) {
      dft_small<T, R>(v[k], sign);
#pragma unroll
      for (int t = 0; t < R; ++t) sink(dst[k], de[k] + t * L, v[k][t]);
    }
  }
  __syncthreads();
}

template <typename T, int R, typename Src>
__device__ __forceinline__ void stockham_stage_from(const Src& src, bool in_place, cplx<T>* buf,
                                                    int n, int ls, int nlines, int L,
                                                    const cplx<T>* tw, int sign) {
  stockham_stage_io<T, R>(
      src, [&](int line, int e, cplx<T> v) { buf[__mul24(line, ls) + sw<T>(e)] = v; }, in_place, n,
      nlines, L, tw, sign);
}

template <typename T, int R>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int n, int ls, int nlines, int L,
                                               const cplx<T>* tw, int sign) {
  stockham_stage_from<T, R>(
      [&](int line, int e) { return buf[__mul24(line, ls) + sw<T>(e)]; }, true, buf, n, ls, nlines, L,
      tw, sign);
}

// One stage of radix `R` (2, 3, 4 or 8, chosen at run time) with custom
// input and output.
template <typename T, bool P3, typename Src, typename Sink>
__device__ __forceinline__ void stage_io_any(int R, const Src& src, const Sink& sink,
                                             bool in_place, int n, int nlines, int L,
                                             const cplx<T>* tw, int sign) {
  if (R == 8) stockham_stage_io<T, 8>(src, sink, in_place, n, nlines, L, tw, sign);
  else if (R == 4) stockham_stage_io<T, 4>(src, sink, in_place, n, nlines, L, tw, sign);
  else if (R == 2) stockham_stage_io<T, 2>(src, sink, in_place, n, nlines, L, tw, sign);
  else if constexpr (P3) stockham_stage_io<T, 3>(src, sink, in_place, n, nlines, L, tw, sign);
}

// Runs all stages in place on `a` (caller synchronised after filling it);
// returns `a` after a final barrier.
// P3: the length has a factor 3 (radix-3 stages compiled in).  Lengths are
// products of 2 and 3 only.

// Stages [first, last) of the plan, with the radices in plan order or in
// reverse order (a Stockham FFT sorts itself for any order of radices); L0 is
// the product of the radices of the stages before `first`.
template <typename T, bool P3>
__device__ void fft_stages(cplx<T>* a, const AxisPlan& plan, bool reversed, int first, int last,
                           int L0, int nlines, const cplx<T>* tw, int sign) {
  int L = L0;
  const int n = plan.n, ls = lds_stride<T>(n);
  for (int st = first; st < last; ++st) {
    const int R = (plan.code >> (4 * (reversed ? plan.nstage - 1 - st : st))) & 15u;
    if (R == 8) stockham_stage<T, 8>(a, n, ls, nlines, L, tw, sign);
    else if (R == 4) stockham_stage<T, 4>(a, n, ls, nlines, L, tw, sign);
    else if (R == 2) stockham_stage<T, 2>(a, n, ls, nlines, L, tw, sign);
    else if constexpr (P3) stockham_stage<T, 3>(a, n, ls, nlines, L, tw, sign);
    L *= R;
  }
}

template <typename T, bool P3>
__device__ cplx<T>* fft_lines(cplx<T>* a, const AxisPlan& plan, int nlines, const cplx<T>* tw,
                              int sign) {
  fft_stages<T, P3>(a, plan, false, 0, plan.nstage, 1, nlines, tw, sign);
  return a;
}

// Radix plan of a length as the host builds it: radix 8 while it divides,
// then 4, then 2, then 3.
__host__ __device__ constexpr int p2_nstage(int n) {
  int s = 0;
  while (n % 8 == 0) { n /= 8; ++s; }
  while (n % 4 == 0) { n /= 4; ++s; }
  while (n % 2 == 0) { n /= 2; ++s; }
  while (n % 3 == 0) { n /= 3; ++s; }
  return s;
}
__host__ __device__ constexpr int p2_radix(int n, int st) {
  int s = 0;
  while (n % 8 == 0) { if (s++ == st) return 8; n /= 8; }
  while (n % 4 == 0) { if (s++ == st) return 4; n /= 4; }
  while (n % 2 == 0) { if (s++ == st) return 2; n /= 2; }
  while (n % 3 == 0) { if (s++ == st) return 3; n /= 3; }
  return 1;
}
__host__ __device__ constexpr unsigned p2_code(int n) {
  unsigned c = 0;
  for (int st = 0; st < p2_nstage(n); ++st) c |= (unsigned)p2_radix(n, st) << (4 * st);
  return c;
}

// In-place LDS stages [S, SEND) of the compile-time plan of N, radices in
// plan order or reversed; L is the product of the radices before stage S.
template <typename T, int N, int S, int SEND, bool REV, int L>
__device__ __forceinline__ void stages_ct(cplx<T>* a, int nlines, const cplx<T>* tw, int sign) {
  if constexpr (S < SEND) {
    constexpr int NS = p2_nstage(N);
    constexpr int R = p2_radix(N, REV ? NS - 1 - S : S);
    constexpr int ls = lds_stride<T>(N);
    stockham_stage_io<T, R, N, L>(
        [&](int line, int e) { return a[line * ls + sw<T>(e)]; },
        [&](int line, int e, cplx<T> v) { a[line * ls + sw<T>(e)] = v; }, true, N, nlines, L,
        tw, sign);
    stages_ct<T, N, S + 1, SEND, REV, L * R>(a, nlines, tw, sign);
  }
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, const cplx<double>* g, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = {T(g[i].re), T(g[i].im)};
}

__device__ __forceinline__ int load_status(const PcgState* st, int ld) {
  return st ? st[ld].status : ST_ACTIVE;
}

// for (idx = threadIdx.x; idx < n; idx += kThreads) store(idx, load(idx)),
// with the global reads of CH consecutive trips issued before their LDS
// writes: one memory round trip per CH trips instead of one per trip.
template <int CH, typename V, typename Load, typename Store>
__device__ __forceinline__ void staged_fill(int n, Load load, Store store) {
  for (int base = threadIdx.x; base < n; base += CH * kThreads) {
    V v[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = base + k * kThreads;
      if (idx < n) v[k] = load(idx);
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int idx = base + k * kThreads;
      if (idx < n) store(idx, v[k]);
    }
  }
}

// Deterministic block sum (wave shuffles, then waves in order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += sh[w];
  }
  return s;
}

// ------------------------------------------------------------- x forward
// grid (ceil(ny/16), nz, nload*nd).  Optionally r -= alpha q first.
// Five waves per SIMD (at most 96 VGPRs): measured 255 -> 231 us per 6-load
// launch at 128^3 in FP64 (the other passes are slower that way).  FP64 with
// radix-3 stages would spill 27 registers in that budget and keeps four.
template <typename T, bool P3, int kRows, int NX = 0>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 8 && P3 && NX == 0) ? 4 : 5) k_xfwd(Grid g, AxisPlan px, const cplx<double>* twx,
                                                  int mode, T* r, long long rstride, const T* q,
                                                  long long qstride, cplx<T>* A,
                                                  long long sstride, const PcgState* st) {
  const int ld = blockIdx.z / g.nd, c = blockIdx.z % g.nd;
  if (load_status(st, ld) != ST_ACTIVE) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = NX ? NX : g.nx, ny = g.ny, nxh = g.nxh;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* a = tw + nx;
  load_twiddles(tw, twx, nx);
  const int y0 = blockIdx.x * kRows, z = blockIdx.y;
  const long long rbase = (long long)ld * rstride + ((long long)c * g.nz + z) * ny * nx;
  const T alpha = (mode == XF_UPDATE_R) ? T(st[ld].alpha) : T(0);
  const int lsx = lds_stride<T>(nx);
  const T* qb = q ? q + (long long)ld * qstride + ((long long)c * g.nz + z) * ny * nx : nullptr;
  const UDiv dnx(nx);
  constexpr int W = kXW<T>;
  using TV = typename xvec<T>::type;
  staged_fill<8, TV>(
      kRows * nx / W,
      [&](int iv) {
        const int idx = W * iv;
        const int row = dnx.q(idx), x = dnx.r(idx, row), y = y0 + row;
        TV v;
#pragma unroll
        for (int e = 0; e < W; ++e) v[e] = T(0);
        if (y < ny) {
          const long long o = rbase + (long long)y * nx + x;
          v = ld_nt(reinterpret_cast<const TV*>(&r[o]));
          if (mode == XF_UPDATE_R) {
            const TV qv = ld_nt(reinterpret_cast<const TV*>(&qb[(long long)y * nx + x]));
#pragma unroll
            for (int e = 0; e < W; ++e) v[e] -= alpha * qv[e];
            st_nt(v, reinterpret_cast<TV*>(&r[o]));
          }
        }
        return v;
      },
      [&](int iv, TV v) {
        const int idx = W * iv;
        const int row = dnx.q(idx), x = dnx.r(idx, row);
        cplx<T>* d = a + __mul24(row >> 1, lsx);
#pragma unroll
        for (int e = 0; e < W; ++e) {
          if (row & 1) d[sw<T>(x + e)].im = v[e]; else d[sw<T>(x + e)].re = v[e];
        }
      });
  __syncthreads();
  cplx<T>* res = a;
  if constexpr (NX > 0)
    stages_ct<T, NX, 0, p2_nstage(NX), false, 1>(a, kRows / 2, tw, -1);
  else
    res = fft_lines<T, P3>(a, px, kRows / 2, tw, -1);
  const long long abase = (long long)ld * sstride + ((long long)c * g.nz + z) * nxh * ny;
  for (int idx = threadIdx.x; idx < kRows * nxh; idx += blockDim.x) {
    const int yl = idx % kRows, kx = idx / kRows, y = y0 + yl;
    if (y >= ny) continue;
    const cplx<T>* line = res + __mul24(yl >> 1, lsx);
    const cplx<T> ck = line[sw<T>(kx)];
    const cplx<T> cn = line[sw<T>(kx == 0 ? 0 : nx - kx)];
    cplx<T> X;
    if ((yl & 1) == 0) {
      X = {T(0.5) * (ck.re + cn.re), T(0.5) * (ck.im - cn.im)};
    } else {
      // (ck - conj(cn)) / (2i)
      const T dr = ck.re - cn.re, di = ck.im + cn.im;
      X = {T(0.5) * di, -T(0.5) * dr};
    }
    A[abase + (long long)kx * ny + y] = X;
  }
}

// ------------------------------------------------------------- y forward
// grid (ceil(nz/zb), nxh, nload*nd); zb lines per block, zb*ny <= kMaxPts.
// NY > 0: power-of-two length with its compile-time plan (as in k_zpass).
template <typename T, bool P3, int NY = 0>
__global__ void __launch_bounds__(kThreads) k_yfwd(Grid g, AxisPlan py, const cplx<double>* twy,
                                                  int zb, const cplx<T>* A, cplx<T>* B,
                                                  long long sstride, const PcgState* st) {
  const int ld = blockIdx.z / g.nd, c = blockIdx.z % g.nd;
  if (load_status(st, ld) != ST_ACTIVE) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ny = NY ? NY : g.ny, nz = g.nz, nxh = g.nxh;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* a = tw + ny;
  load_twiddles(tw, twy, ny);
  const int z0 = blockIdx.x * zb, kx = blockIdx.y;
  const long long base = (long long)ld * sstride;
  const int ls = lds_stride<T>(ny);
  // the y lines are contiguous in A: the first stage reads them from HBM
  auto gsrc = [&](int zl, int y) -> cplx<T> {
    const int z = z0 + zl;
    cplx<T> v = {T(0), T(0)};
    if (z < nz) v = ld_nt(&A[base + (((long long)c * nz + z) * nxh + kx) * ny + y]);
    return v;
  };
  auto lsink = [&](int l, int y, cplx<T> v) { a[__mul24(l, ls) + sw<T>(y)] = v; };
  cplx<T>* res = a;
  if constexpr (NY > 0) {
    constexpr int NS = p2_nstage(NY), R0c = p2_radix(NY, 0);
    stockham_stage_io<T, R0c, NY, 1>(gsrc, lsink, false, NY, zb, 1, tw, -1);
    stages_ct<T, NY, 1, NS, false, R0c>(a, zb, tw, -1);
  } else if (py.nstage >= 1) {
    const int R0 = py.code & 15u;
    stage_io_any<T, P3>(R0, gsrc, lsink, false, ny, zb, 1, tw, -1);
    fft_stages<T, P3>(a, py, false, 1, py.nstage, R0, zb, tw, -1);
  } else {
    for (int idx = threadIdx.x; idx < zb * ny; idx += blockDim.x)
      lsink(idx / ny, idx % ny, gsrc(idx / ny, idx % ny));
    __syncthreads();
  }
  const long long obase = base + ((long long)c * nxh + kx) * (long long)ny * nz;
  const UDiv dzb(zb);
  for (int idx = threadIdx.x; idx < zb * ny; idx += blockDim.x) {
    const int ky = dzb.q(idx), zl = dzb.r(idx, ky), z = z0 + zl;
    if (z < nz) B[obase + (long long)ky * nz + z] = res[__mul24(zl, ls) + sw<T>(ky)];
  }
}

// z pass, 3 components, plans ending in radix 2 (lengths 16, 128, ...): the
// last forward stage, the per-frequency K^+ solve with its Parseval sum and
// the first stage of the inverse (run with the radices in reverse order, so
// that it starts with radix 2) in one pass through registers.  The forward
// stage leaves X(j) and X(j + n/2) with the thread whose inverse butterfly
// needs exactly those two, so only the three components of a frequency pair
// have to meet in one thread: one LDS round trip and the solve pass are
// saved.
constexpr int kFusedMaxIt = (2048 / 6 + kThreads - 1) / kThreads;  // kyb * n/2 <= 2048 / 6
// PRE: the thread's K^+ entries were loaded into kpre[item][t][0..5] before
// the forward stages (else they are read here and kpre is not touched)
template <typename T, int NC = 0, bool PRE = false>
__device__ double zpass_fused_mid(cplx<T>* a, int n_rt, int ls, int cls, int kyb, int ky0, int ny,
                                  int nz, int kx, const cplx<T>* tw, const T* kplus,
                                  long long nfreq, double wgt,
                                  const T (&kpre)[kFusedMaxIt][2][6]) {
  constexpr int MAXIT = kFusedMaxIt;
  const int n = NC ? NC : n_rt;
  const int m = n / 2;
  const int items = kyb * m;
  const UDiv dm(m);
  cplx<T> v[MAXIT][3][2];
  int jj[MAXIT], kyl_[MAXIT];
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const int it = threadIdx.x + k * kThreads;
    kyl_[k] = -1;
    if (it < items) {
      const int kyl = NC ? it / (NC / 2) : dm.q(it);
      const int j = NC ? it % (NC / 2) : dm.r(it, kyl);
      const cplx<T> w = tw[j];  // forward twiddle of the last stage: L = n/2, t = 1
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<T>* src = a + c * cls + __mul24(kyl, ls);
        const cplx<T> x0 = src[sw<T>(j)];
        const cplx<T> x1 = cmul(src[sw<T>(j + m)], w);
        v[k][c][0] = cadd(x0, x1);
        v[k][c][1] = csub(x0, x1);
      }
      jj[k] = j;
      kyl_[k] = kyl;
    }
  }
  __syncthreads();
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    if (kyl_[k] < 0) continue;
    const int j = jj[k], kyl = kyl_[k], ky = ky0 + kyl;
    if (ky < ny) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // below 6 nxh ny nz < 2^31 for every accepted grid
        const int f = (kx * ny + ky) * nz + j + t * m;
        T kk[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) kk[e] = PRE ? kpre[k][t][e] : kplus[e * nfreq + f];
        const T k00 = kk[0], k11 = kk[1], k22 = kk[2], k12 = kk[3], k02 = kk[4], k01 = kk[5];
        const cplx<T> r0 = v[k][0][t], r1 = v[k][1][t], r2 = v[k][2][t];
        const cplx<T> z0v = {k00 * r0.re + k01 * r1.re + k02 * r2.re,
                             k00 * r0.im + k01 * r1.im + k02 * r2.im};
        const cplx<T> z1v = {k01 * r0.re + k11 * r1.re + k12 * r2.re,
                             k01 * r0.im + k11 * r1.im + k12 * r2.im};
        const cplx<T> z2v = {k02 * r0.re + k12 * r1.re + k22 * r2.re,
                             k02 * r0.im + k12 * r1.im + k22 * r2.im};
        part += wgt * ((double)r0.re * z0v.re + (double)r0.im * z0v.im +
                       (double)r1.re * z1v.re + (double)r1.im * z1v.im +
                       (double)r2.re * z2v.re + (double)r2.im * z2v.im);
        v[k][0][t] = z0v;
        v[k][1][t] = z1v;
        v[k][2][t] = z2v;
      }
    }
    // first inverse stage (radix 2, no twiddle): outputs at 2j and 2j + 1
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cplx<T>* dst = a + c * cls + __mul24(kyl, ls);
      dst[sw<T>(2 * j)] = cadd(v[k][c][0], v[k][c][1]);
      dst[sw<T>(2 * j + 1)] = csub(v[k][c][0], v[k][c][1]);
    }
  }
  __syncthreads();
  return part;
}

// Scalar problems (one component): the same fusion for a last radix R of
// 2, 4 or 8.  The solve is a multiplication per frequency, so the R outputs
// of a forward butterfly are exactly the R inputs of the matching inverse
// butterfly and never leave the thread.
template <int R>
constexpr int fused_scalar_maxit() {
  return (2048 / R + kThreads - 1) / kThreads;  // kyb * n <= 2048
}
// PRE: as for the elastic form, kpre[item][t] holds the item's K^+ entries
template <typename T, int R, bool PRE = false>
__device__ double zpass_fused_mid_scalar(cplx<T>* a, int n, int ls, int kyb, int ky0, int ny,
                                         int nz, int kx, const cplx<T>* tw, const T* kplus,
                                         double wgt, const T (&kpre)[fused_scalar_maxit<R>()][R]) {
  constexpr int MAXIT = fused_scalar_maxit<R>();
  const int m = n / R;
  const int items = kyb * m;
  const UDiv dm(m);
  cplx<T> v[MAXIT][R];
  int jj[MAXIT], kyl_[MAXIT];
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const int it = threadIdx.x + k * kThreads;
    kyl_[k] = -1;
    if (it < items) {
      const int kyl = dm.q(it), j = dm.r(it, kyl);
      const cplx<T>* src = a + __mul24(kyl, ls);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        cplx<T> x = src[sw<T>(j + t * m)];
        if (t > 0) x = cmul(x, tw[t * j]);  // last forward stage: L = n/R
        v[k][t] = x;
      }
      dft_small<T, R>(v[k], -1);  // outputs at j + t m
      jj[k] = j;
      kyl_[k] = kyl;
    }
  }
  __syncthreads();
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    if (kyl_[k] < 0) continue;
    const int j = jj[k], kyl = kyl_[k], ky = ky0 + kyl;
    if (ky < ny) {
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const T kp = PRE ? kpre[k][t] : kplus[(kx * ny + ky) * nz + j + t * m];
        const cplx<T> r = v[k][t];
        part += wgt * (double)kp * ((double)r.re * r.re + (double)r.im * r.im);
        v[k][t] = {kp * r.re, kp * r.im};
      }
    }
    // first inverse stage (radix R, L = 1, no twiddles): outputs at jR + t
    dft_small<T, R>(v[k], +1);
    cplx<T>* dst = a + __mul24(kyl, ls);
#pragma unroll
    for (int t = 0; t < R; ++t) dst[sw<T>(j * R + t)] = v[k][t];
  }
  __syncthreads();
  return part;
}

// ------------------------------------------------ z forward (+ solve + inverse)
// grid (ceil(ny/kyb), nxh, nload).  Dynamic LDS: tw[nz], a/b[nd*kyb*nz].
// Power-of-two lengths run four waves per SIMD (at most 128 VGPRs, 7 spilled
// in FP64): 212 -> 192 us per 6-load launch at 128^3; with radix-3 stages
// that budget would spill 44 registers, so those keep the compiler's choice.
// NZ > 0: the z length, whose plan is p2_code(NZ), known at compile time
// (the solve stages then use the compile-time stage code).
template <typename T, bool P3, int NZ = 0>
__global__ void __launch_bounds__(kThreads, (P3 && NZ == 0) ? 1 : 4) k_zpass(Grid g, AxisPlan pz, const cplx<double>* twz,
                                                   int mode, int kyb, cplx<T>* B,
                                                   long long sstride, const T* kplus,
                                                   const PcgState* st, double* rz_part) {
  // Workgroups go round-robin to the 8 XCDs.  Renumber them so that the load
  // cases of one group of lines run back to back on the same XCD: K^+ of
  // those lines then comes from HBM once and from that XCD's L2 after.
  // The grid is (line groups rounded up to a multiple of 8, 1, loads);
  // padding blocks exit at once.
  const int gx = (g.ny + kyb - 1) / kyb, lg_n = gx * g.nxh;
  const int b = blockIdx.x + gridDim.x * blockIdx.z;
  const int k = b >> 3;
  const int ld = k % gridDim.z;
  const int lg = (k / gridDim.z) * 8 + (b & 7);
  if (lg >= lg_n) return;
  const int bx = lg % gx, by = lg / gx;
  __shared__ double red[16];
  const int active = load_status(st, ld) == ST_ACTIVE;
  if (!active) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ny = g.ny, nz = NZ ? NZ : g.nz, nxh = g.nxh, nd = g.nd;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* a = tw + nz;
  load_twiddles(tw, twz, nz);
  const int ky0 = bx * kyb, kx = by;
  if (kplus) kplus += (ld / g.G) * g.kplus_stride;
  const long long cstride = (long long)nxh * ny * nz;
  const long long base = (long long)ld * sstride + (long long)kx * ny * nz;
  const int per = kyb * nz;
  const int ls = lds_stride<T>(nz);
  const int cls = kyb * ls;  // LDS stride between components
  const int last_radix = (pz.code >> (4 * (pz.nstage - 1))) & 15u;
  const bool fused = mode == Z_SOLVE && pz.nstage >= 2 &&
                     ((nd == 3 && last_radix == 2 && kyb * nz <= 2048 / 3) ||
                      (nd == 1 && (last_radix == 2 || last_radix == 4 || last_radix == 8)));
  // line l = c * kyb + kyl of the block is component c of frequency line ky0 + kyl
  const UDiv dkyb(kyb);
  auto gsrc = [&](int l, int z) -> cplx<T> {
    const int c = dkyb.q(l), ky = ky0 + dkyb.r(l, c);
    cplx<T> v = {T(0), T(0)};
    if (ky < ny) v = ld_nt(&B[base + c * cstride + (long long)ky * nz + z]);
    return v;
  };
  // solve mode: the first forward stage reads the z lines from global memory
  // and the last inverse stage writes them back (their butterflies touch runs
  // of consecutive elements), so no staging pass is needed
  const bool direct = mode == Z_SOLVE && pz.nstage >= 1;  // nz = 1 (2D) has no stage
  auto lsrc = [&](int l, int z) { return a[__mul24(l, ls) + sw<T>(z)]; };
  auto lsink = [&](int l, int z, cplx<T> v) { a[__mul24(l, ls) + sw<T>(z)] = v; };
  auto gsink = [&](int l, int z, cplx<T> v) {
    const int c = dkyb.q(l), ky = ky0 + dkyb.r(l, c);
    if (ky < ny) B[base + c * cstride + (long long)ky * nz + z] = v;
  };
  const int R0 = pz.code & 15u;
  if (!direct) {
    staged_fill<8, cplx<T>>(
        nd * per,
        [&](int idx) {
          const int c = idx / per, rem = idx - c * per, kyl = rem / nz, z = rem - kyl * nz;
          return gsrc(c * kyb + kyl, z);
        },
        [&](int idx, cplx<T> v) {
          const int c = idx / per, rem = idx - c * per, kyl = rem / nz, z = rem - kyl * nz;
          a[c * cls + kyl * ls + sw<T>(z)] = v;
        });
    __syncthreads();
  }
  double part = 0.0;
  cplx<T>* res = a;
  if (fused) {
    const long long nfreq = (long long)nxh * ny * nz;
    const double wgt = (kx == 0 || (2 * kx == g.nx)) ? 1.0 : 2.0;
    if constexpr (NZ > 0) {
      constexpr int NS = p2_nstage(NZ), R0c = p2_radix(NZ, 0), RLc = p2_radix(NZ, NS - 1);
      // K^+ of the frequencies this thread solves, loaded before the forward
      // stages so that its latency overlaps them (same item mapping as the
      // fused solve)
      T kpre[kFusedMaxIt][2][6];
      T kpre1[fused_scalar_maxit<RLc>()][RLc];
      if (nd == 3) {
#pragma unroll
        for (int k = 0; k < kFusedMaxIt; ++k) {
          const int it = threadIdx.x + k * kThreads, kyl = it / (NZ / 2), j = it % (NZ / 2);
          const int ky = ky0 + kyl;
          if (it < kyb * (NZ / 2) && ky < ny) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int f = (kx * ny + ky) * NZ + j + t * (NZ / 2);
#pragma unroll
              for (int e = 0; e < 6; ++e) kpre[k][t][e] = kplus[e * nfreq + f];
            }
          }
        }
      } else {
        constexpr int M = NZ / RLc;
#pragma unroll
        for (int k = 0; k < fused_scalar_maxit<RLc>(); ++k) {
          const int it = threadIdx.x + k * kThreads, kyl = it / M, j = it % M;
          const int ky = ky0 + kyl;
          if (it < kyb * M && ky < ny) {
#pragma unroll
            for (int t = 0; t < RLc; ++t) kpre1[k][t] = kplus[(kx * ny + ky) * NZ + j + t * M];
          }
        }
      }
      stockham_stage_io<T, R0c, NZ, 1>(gsrc, lsink, false, NZ, nd * kyb, 1, tw, -1);
      stages_ct<T, NZ, 1, NS - 1, false, R0c>(a, nd * kyb, tw, -1);
      if (nd == 3)
        part = zpass_fused_mid<T, NZ, true>(a, NZ, ls, cls, kyb, ky0, ny, nz, kx, tw, kplus,
                                            nfreq, wgt, kpre);
      else
        part = zpass_fused_mid_scalar<T, RLc, true>(a, NZ, ls, kyb, ky0, ny, nz, kx, tw, kplus,
                                                    wgt, kpre1);
      stages_ct<T, NZ, 1, NS - 1, true, RLc>(a, nd * kyb, tw, +1);
      stockham_stage_io<T, R0c, NZ, NZ / R0c>(lsrc, gsink, false, NZ, nd * kyb, NZ / R0c, tw,
                                              +1);
    } else {
      stage_io_any<T, P3>(R0, gsrc, lsink, false, nz, nd * kyb, 1, tw, -1);
      fft_stages<T, P3>(a, pz, false, 1, pz.nstage - 1, R0, nd * kyb, tw, -1);
      // run-time plans read K^+ in the fused solve itself (the unused
      // preload arguments are never touched)
      T kpre[kFusedMaxIt][2][6], kp2[fused_scalar_maxit<2>()][2],
          kp4[fused_scalar_maxit<4>()][4], kp8[fused_scalar_maxit<8>()][8];
      if (nd == 3)
        part = zpass_fused_mid<T>(a, nz, ls, cls, kyb, ky0, ny, nz, kx, tw, kplus, nfreq, wgt,
                                  kpre);
      else if (last_radix == 2)
        part = zpass_fused_mid_scalar<T, 2>(a, nz, ls, kyb, ky0, ny, nz, kx, tw, kplus, wgt, kp2);
      else if (last_radix == 4)
        part = zpass_fused_mid_scalar<T, 4>(a, nz, ls, kyb, ky0, ny, nz, kx, tw, kplus, wgt, kp4);
      else
        part = zpass_fused_mid_scalar<T, 8>(a, nz, ls, kyb, ky0, ny, nz, kx, tw, kplus, wgt, kp8);
      fft_stages<T, P3>(a, pz, true, 1, pz.nstage - 1, last_radix, nd * kyb, tw, +1);
      stage_io_any<T, P3>(R0, lsrc, gsink, false, nz, nd * kyb, nz / R0, tw, +1);
    }
  } else if (direct) {
    if constexpr (NZ > 0) {
      constexpr int NS = p2_nstage(NZ), R0c = p2_radix(NZ, 0);
      stockham_stage_io<T, R0c, NZ, 1>(gsrc, lsink, false, NZ, nd * kyb, 1, tw, -1);
      stages_ct<T, NZ, 1, NS, false, R0c>(a, nd * kyb, tw, -1);
    } else {
      stage_io_any<T, P3>(R0, gsrc, lsink, false, nz, nd * kyb, 1, tw, -1);
      fft_stages<T, P3>(a, pz, false, 1, pz.nstage, R0, nd * kyb, tw, -1);
    }
  } else {
    res = fft_lines<T, P3>(a, pz, nd * kyb, tw, -1);
  }
  if (mode == Z_SOLVE && !fused) {
    const long long nfreq = (long long)nxh * ny * nz;
    const double wgt = (kx == 0 || (2 * kx == g.nx)) ? 1.0 : 2.0;
    const UDiv dnz(nz);
    for (int idx0 = threadIdx.x; idx0 < per; idx0 += blockDim.x) {
      const int kyl = NZ ? idx0 / NZ : dnz.q(idx0);
      const int kz = NZ ? idx0 % NZ : dnz.r(idx0, kyl), ky = ky0 + kyl;
      if (ky >= ny) continue;
      const int idx = kyl * ls + sw<T>(kz);
      const long long f = ((long long)kx * ny + ky) * nz + kz;
      if (nd == 3) {
        const T k00 = kplus[f], k11 = kplus[nfreq + f], k22 = kplus[2 * nfreq + f];
        const T k12 = kplus[3 * nfreq + f], k02 = kplus[4 * nfreq + f],
                k01 = kplus[5 * nfreq + f];
        const cplx<T> r0 = res[idx], r1 = res[cls + idx], r2 = res[2 * cls + idx];
        cplx<T> z0v = {k00 * r0.re + k01 * r1.re + k02 * r2.re,
                       k00 * r0.im + k01 * r1.im + k02 * r2.im};
        cplx<T> z1v = {k01 * r0.re + k11 * r1.re + k12 * r2.re,
                       k01 * r0.im + k11 * r1.im + k12 * r2.im};
        cplx<T> z2v = {k02 * r0.re + k12 * r1.re + k22 * r2.re,
                       k02 * r0.im + k12 * r1.im + k22 * r2.im};
        part += wgt * ((double)r0.re * z0v.re + (double)r0.im * z0v.im +
                       (double)r1.re * z1v.re + (double)r1.im * z1v.im +
                       (double)r2.re * z2v.re + (double)r2.im * z2v.im);
        res[idx] = z0v;
        res[cls + idx] = z1v;
        res[2 * cls + idx] = z2v;
      } else if (nd == 2 && g.tn) {
        // two-node stencil: Hermitian block, K^+_01 = kr + i ki
        const T k00 = kplus[f], k11 = kplus[nfreq + f];
        const T kr = kplus[2 * nfreq + f], ki = kplus[3 * nfreq + f];
        const cplx<T> r0 = res[idx], r1 = res[cls + idx];
        cplx<T> z0v = {k00 * r0.re + kr * r1.re - ki * r1.im, k00 * r0.im + kr * r1.im + ki * r1.re};
        cplx<T> z1v = {kr * r0.re + ki * r0.im + k11 * r1.re, kr * r0.im - ki * r0.re + k11 * r1.im};
        part += wgt * ((double)r0.re * z0v.re + (double)r0.im * z0v.im +
                       (double)r1.re * z1v.re + (double)r1.im * z1v.im);
        res[idx] = z0v;
        res[cls + idx] = z1v;
      } else if (nd == 2) {
        const T k00 = kplus[f], k11 = kplus[nfreq + f], k01 = kplus[2 * nfreq + f];
        const cplx<T> r0 = res[idx], r1 = res[cls + idx];
        cplx<T> z0v = {k00 * r0.re + k01 * r1.re, k00 * r0.im + k01 * r1.im};
        cplx<T> z1v = {k01 * r0.re + k11 * r1.re, k01 * r0.im + k11 * r1.im};
        part += wgt * ((double)r0.re * z0v.re + (double)r0.im * z0v.im +
                       (double)r1.re * z1v.re + (double)r1.im * z1v.im);
        res[idx] = z0v;
        res[cls + idx] = z1v;
      } else {
        const T k00 = kplus[f];
        const cplx<T> r0 = res[idx];
        cplx<T> z0v = {k00 * r0.re, k00 * r0.im};
        part += wgt * ((double)r0.re * z0v.re + (double)r0.im * z0v.im);
        res[idx] = z0v;
      }
    }
    __syncthreads();
    if constexpr (NZ > 0) {
      constexpr int NS = p2_nstage(NZ), RLc = p2_radix(NZ, NS - 1);
      stages_ct<T, NZ, 0, NS - 1, false, 1>(a, nd * kyb, tw, +1);
      stockham_stage_io<T, RLc, NZ, NZ / RLc>(lsrc, gsink, false, NZ, nd * kyb, NZ / RLc, tw,
                                              +1);
    } else {
      const int RL = (pz.code >> (4 * (pz.nstage - 1))) & 15u;
      fft_stages<T, P3>(a, pz, false, 0, pz.nstage - 1, 1, nd * kyb, tw, +1);
      stage_io_any<T, P3>(RL, lsrc, gsink, false, nz, nd * kyb, nz / RL, tw, +1);
    }
  }
  if (!direct) {
    for (int idx = threadIdx.x; idx < nd * per; idx += blockDim.x) {
      const int c = idx / per, rem = idx - c * per, kyl = rem / nz, z = rem - kyl * nz;
      const int ky = ky0 + kyl;
      if (ky < ny)
        B[base + c * cstride + (long long)ky * nz + z] = res[c * cls + kyl * ls + sw<T>(z)];
    }
  }
  if (mode == Z_SOLVE && rz_part) {
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) {
      rz_part[(long long)ld * lg_n + lg] = s;
    }
  }
}

// ------------------------------------------------------------- y inverse
template <typename T, bool P3, int NY = 0>
__global__ void __launch_bounds__(kThreads) k_yinv(Grid g, AxisPlan py, const cplx<double>* twy,
                                                  int zb, const cplx<T>* B, cplx<T>* A,
                                                  long long sstride, const PcgState* st) {
  const int ld = blockIdx.z / g.nd, c = blockIdx.z % g.nd;
  if (load_status(st, ld) != ST_ACTIVE) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ny = NY ? NY : g.ny, nz = g.nz, nxh = g.nxh;
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* a = tw + ny;
  load_twiddles(tw, twy, ny);
  const int z0 = blockIdx.x * zb, kx = blockIdx.y;
  const long long base = (long long)ld * sstride;
  const long long ibase = base + ((long long)c * nxh + kx) * (long long)ny * nz;
  const int ls = lds_stride<T>(ny);
  const UDiv dzb(zb);
  staged_fill<8, cplx<T>>(
      zb * ny,
      [&](int idx) {
        const int ky = dzb.q(idx), zl = dzb.r(idx, ky), z = z0 + zl;
        cplx<T> v = {T(0), T(0)};
        if (z < nz) v = ld_nt(&B[ibase + (long long)ky * nz + z]);
        return v;
      },
      [&](int idx, cplx<T> v) {
        const int ky = dzb.q(idx), zl = dzb.r(idx, ky);
        a[__mul24(zl, ls) + sw<T>(ky)] = v;
      });
  __syncthreads();
  // the y lines are contiguous in A: the last stage writes them to HBM
  auto lsrc = [&](int l, int y) { return a[__mul24(l, ls) + sw<T>(y)]; };
  auto gsink = [&](int zl, int y, cplx<T> v) {
    const int z = z0 + zl;
    if (z < nz) A[base + (((long long)c * nz + z) * nxh + kx) * ny + y] = v;
  };
  if constexpr (NY > 0) {
    constexpr int NS = p2_nstage(NY), RLc = p2_radix(NY, NS - 1);
    stages_ct<T, NY, 0, NS - 1, false, 1>(a, zb, tw, +1);
    stockham_stage_io<T, RLc, NY, NY / RLc>(lsrc, gsink, false, NY, zb, NY / RLc, tw, +1);
  } else if (py.nstage >= 1) {
    const int RL = (py.code >> (4 * (py.nstage - 1))) & 15u;
    fft_stages<T, P3>(a, py, false, 0, py.nstage - 1, 1, zb, tw, +1);
    stage_io_any<T, P3>(RL, lsrc, gsink, false, ny, zb, ny / RL, tw, +1);
  } else {
    for (int idx = threadIdx.x; idx < zb * ny; idx += blockDim.x)
      gsink(idx / ny, idx % ny, lsrc(idx / ny, idx % ny));
  }
}

// ------------------------------------------------------------- x inverse
// grid (ceil(ny/16), nz, nload*nd).  LDS: tw[nx], a[8 nx], S[16 nxh].
template <typename T, bool P3, int kRows, int NX = 0>
__global__ void __launch_bounds__(kThreads) k_xinv(Grid g, AxisPlan px, const cplx<double>* twx,
                                                  int mode, const cplx<T>* A, long long sstride,
                                                  T* out, T* x, T* p, long long fstride,
                                                  const PcgState* st) {
  const int ld = blockIdx.z / g.nd, c = blockIdx.z % g.nd;
  const int status = load_status(st, ld);
  const int nx = NX ? NX : g.nx, ny = g.ny, nxh = g.nxh;
  const int y0 = blockIdx.x * kRows, z = blockIdx.y;
  const long long fbase = (long long)ld * fstride + ((long long)c * g.nz + z) * ny * nx;
  const UDiv dnx(nx);
  if (mode == XI_PCG && (status == ST_CONVERGED_PENDING || status == ST_MAXIT_PENDING)) {
    const T alpha = T(st[ld].alpha);
    for (int idx = threadIdx.x; idx < kRows * nx; idx += blockDim.x) {
      const int row = dnx.q(idx), xx = dnx.r(idx, row), y = y0 + row;
      if (y < ny) {
        const long long o = fbase + (long long)y * nx + xx;
        x[o] += alpha * p[o];
      }
    }
    return;
  }
  if (status != ST_ACTIVE) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
  const int lsx = lds_stride<T>(nx);
  cplx<T>* a = tw + nx;
  cplx<T>* S = a + (kRows / 2) * lsx;  // kRows x nxh raw tile, row stride nxh + 1
  load_twiddles(tw, twx, nx);
  // PCG mode: the reads of p and x for the first 8 trips of the output loop
  // are issued here, before the spectrum tile, and land during the FFT
  constexpr int CH = 8;
  constexpr int W = kXW<T>;
  using TV = typename xvec<T>::type;
  const int nout = kRows * nx / W;  // runs of W values
  TV pv0[CH], xv0[CH];
  if (mode == XI_PCG) {
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int iv = threadIdx.x + k * kThreads, idx = W * iv;
      const int row = dnx.q(idx), xx = dnx.r(idx, row), y = y0 + row;
      if (iv < nout && y < ny) {
        const long long o = fbase + (long long)y * nx + xx;
        pv0[k] = ld_nt(reinterpret_cast<const TV*>(&p[o]));
        xv0[k] = ld_nt(reinterpret_cast<const TV*>(&x[o]));
      }
    }
  }
  const long long abase = (long long)ld * sstride + ((long long)c * g.nz + z) * nxh * ny;
  staged_fill<8, cplx<T>>(
      kRows * nxh,
      [&](int idx) {
        const int yl = idx % kRows, kx = idx / kRows, y = y0 + yl;
        cplx<T> v = {T(0), T(0)};
        if (y < ny) v = ld_nt(&A[abase + (long long)kx * ny + y]);
        return v;
      },
      [&](int idx, cplx<T> v) {
        const int yl = idx % kRows, kx = idx / kRows;
        S[__mul24(yl, nxh + 1) + kx] = v;
      });
  __syncthreads();
  // Complex line j carries real rows 2j and 2j+1: X_a + i X_b, with the
  // spectra extended by Hermitian symmetry.  The first Stockham stage reads
  // its inputs this way straight from the tile S (no separate unpack pass).
  const int half = nx / 2;
  auto packed = [&](int j, int k) -> cplx<T> {
    cplx<T> xa, xb;
    const int s0 = __mul24(2 * j, nxh + 1);
    if (k <= half) {
      xa = S[s0 + k];
      xb = S[s0 + nxh + 1 + k];
      if (k == 0 || k == half) {
        xa.im = T(0);
        xb.im = T(0);
      }
    } else {
      xa = conjg(S[s0 + (nx - k)]);
      xb = conjg(S[s0 + nxh + 1 + (nx - k)]);
    }
    return {xa.re - xb.im, xa.im + xb.re};
  };
  if constexpr (NX > 0) {
    constexpr int R0c = p2_radix(NX, 0);
    stockham_stage_io<T, R0c, NX, 1>(
        packed, [&](int line, int e, cplx<T> v) { a[line * lsx + sw<T>(e)] = v; }, false, NX,
        kRows / 2, 1, tw, +1);
    stages_ct<T, NX, 1, p2_nstage(NX), false, R0c>(a, kRows / 2, tw, +1);
  } else {
    const int R0 = px.code & 15u;
    if (R0 == 8) stockham_stage_from<T, 8>(packed, false, a, nx, lsx, kRows / 2, 1, tw, +1);
    else if (R0 == 4) stockham_stage_from<T, 4>(packed, false, a, nx, lsx, kRows / 2, 1, tw, +1);
    else if (R0 == 2) stockham_stage_from<T, 2>(packed, false, a, nx, lsx, kRows / 2, 1, tw, +1);
    else if constexpr (P3) stockham_stage_from<T, 3>(packed, false, a, nx, lsx, kRows / 2, 1, tw, +1);
    fft_stages<T, P3>(a, px, false, 1, px.nstage, R0, kRows / 2, tw, +1);
  }
  cplx<T>* res = a;
  const T alpha = (mode == XI_PCG) ? T(st[ld].alpha) : T(0);
  const T beta = (mode == XI_PCG) ? T(st[ld].beta) : T(0);
  // later trips: the reads of 8 trips are issued before their use
  for (int base = threadIdx.x; base < nout; base += CH * kThreads) {
    TV pv[CH], xv[CH];
    if (mode == XI_PCG && base == (int)threadIdx.x) {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        pv[k] = pv0[k];
        xv[k] = xv0[k];
      }
    } else if (mode == XI_PCG) {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int iv = base + k * kThreads, idx = W * iv;
        const int row = dnx.q(idx), xx = dnx.r(idx, row), y = y0 + row;
        if (iv < nout && y < ny) {
          const long long o = fbase + (long long)y * nx + xx;
          pv[k] = ld_nt(reinterpret_cast<const TV*>(&p[o]));
          xv[k] = ld_nt(reinterpret_cast<const TV*>(&x[o]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int iv = base + k * kThreads, idx = W * iv;
      const int row = dnx.q(idx), xx = dnx.r(idx, row), y = y0 + row;
      if (iv >= nout || y >= ny) continue;
      const cplx<T>* line = res + __mul24(row >> 1, lsx);
      TV zv;
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const cplx<T> v = line[sw<T>(xx + e)];
        zv[e] = (row & 1) ? v.im : v.re;
      }
      const long long o = fbase + (long long)y * nx + xx;
      if (mode == XI_PLAIN) {
        *reinterpret_cast<TV*>(&out[o]) = zv;
      } else if (mode == XI_INIT_P) {
        *reinterpret_cast<TV*>(&p[o]) = zv;
      } else {
        TV xn, pn;
#pragma unroll
        for (int e = 0; e < W; ++e) {
          xn[e] = xv[k][e] + alpha * pv[k][e];
          pn[e] = zv[e] + beta * pv[k][e];
        }
        st_nt(xn, reinterpret_cast<TV*>(&x[o]));
        *reinterpret_cast<TV*>(&p[o]) = pn;
      }
    }
  }
}

// ------------------------------------------------------------- symbol
// K^+(xi)/N from the spectra of the nd impulse responses (Alg. 2).  The
// symbol of a centrosymmetric one-node stencil is real and symmetric: the
// real part is taken and symmetrised.  Zero frequency: the whole block is
// the zero matrix (rigid-body modes), its pseudo-inverse is zero.
__global__ void k_symbol(Grid g, const cplx<double>* spec, long long sstride, double* kplus,
                         int* bad) {
  const long long nfreq = (long long)g.nxh * g.ny * g.nz;
  const long long cstride = nfreq;
  const double invN = 1.0 / (double)g.N;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < nfreq;
       f += (long long)gridDim.x * blockDim.x) {
    auto Kab = [&](int al, int be) -> double {
      return spec[be * sstride + al * cstride + f].re;
    };
    if (g.nd == 3) {
      double a = Kab(0, 0), bb = Kab(1, 1), c = Kab(2, 2);
      double d = 0.5 * (Kab(1, 2) + Kab(2, 1));
      double e = 0.5 * (Kab(0, 2) + Kab(2, 0));
      double ff = 0.5 * (Kab(0, 1) + Kab(1, 0));
      double out[6] = {0, 0, 0, 0, 0, 0};
      if (f != 0) {
        const double c00 = bb * c - d * d, c11 = a * c - e * e, c22 = a * bb - ff * ff;
        const double c12 = e * ff - a * d, c02 = ff * d - bb * e, c01 = d * e - ff * c;
        const double det = a * c00 + ff * c01 + e * c02;
        if (!(a > 0.0 && c22 > 0.0 && det > 0.0)) atomicOr(bad, 1);
        const double s = invN / det;
        out[0] = c00 * s; out[1] = c11 * s; out[2] = c22 * s;
        out[3] = c12 * s; out[4] = c02 * s; out[5] = c01 * s;
      }
      for (int k = 0; k < 6; ++k) kplus[k * nfreq + f] = out[k];
    } else if (g.nd == 2) {
      double a = Kab(0, 0), bb = Kab(1, 1), ff = 0.5 * (Kab(0, 1) + Kab(1, 0));
      double out[3] = {0, 0, 0};
      if (f != 0) {
        const double det = a * bb - ff * ff;
        if (!(a > 0.0 && det > 0.0)) atomicOr(bad, 1);
        const double s = invN / det;
        out[0] = bb * s; out[1] = a * s; out[2] = -ff * s;
      }
      for (int k = 0; k < 3; ++k) kplus[k * nfreq + f] = out[k];
    } else {
      double a = Kab(0, 0);
      double out = 0.0;
      if (f != 0) {
        if (!(a > 0.0)) atomicOr(bad, 1);
        out = invN / a;
      }
      kplus[f] = out;
    }
  }
}

__global__ void k_cast_symbol(long long n, const double* src, float* dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ------------------------------------------------------------ launchers
// The axis of length N runs with the compile-time plan when the host's plan
// is exactly p2_code(N).
template <int N>
static bool ct_plan(const AxisPlan& p, int n) {
  return n == N && p.n == N && p.nstage == p2_nstage(N) && p.code == p2_code(N);
}

template <typename T>
hipError_t launch_xfwd(const Grid& g, const AxisPlan& px, const cplx<double>* twx, int mode,
                       T* r, long long rstride, const T* q, long long qstride, cplx<T>* A,
                       long long sstride, int nload, const PcgState* st, hipStream_t s) {
  const bool P3K = px.n % 3 == 0;
  const int kRows = xpass_rows<T>(g, false);
  dim3 grid((g.ny + kRows - 1) / kRows, g.nz, nload * g.nd);
  size_t lds = sizeof(cplx<T>) * (size_t)(g.nx + (kRows / 2) * lds_stride<T>(g.nx));
  auto go = [&](auto kern) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, g, px, twx, mode, r, rstride, q,
                       qstride, A, sstride, st);
  };
  if (kRows == 32) {
    if (ct_plan<96>(px, g.nx)) go(k_xfwd<T, true, 32, 96>);
    else if (ct_plan<48>(px, g.nx)) go(k_xfwd<T, true, 32, 48>);
    else if (P3K) go(k_xfwd<T, true, 32>);
    else if (ct_plan<128>(px, g.nx)) go(k_xfwd<T, false, 32, 128>);
    else if (ct_plan<64>(px, g.nx)) go(k_xfwd<T, false, 32, 64>);
    else if (ct_plan<32>(px, g.nx)) go(k_xfwd<T, false, 32, 32>);
    else go(k_xfwd<T, false, 32>);
  } else if (kRows == 8) {
    if (P3K) go(k_xfwd<T, true, 8>);
    else if (ct_plan<256>(px, g.nx)) go(k_xfwd<T, false, 8, 256>);
    else go(k_xfwd<T, false, 8>);
  } else {
    if (ct_plan<96>(px, g.nx)) go(k_xfwd<T, true, 16, 96>);
    else if (ct_plan<48>(px, g.nx)) go(k_xfwd<T, true, 16, 48>);
    else if (P3K) go(k_xfwd<T, true, 16>);
    else if (ct_plan<128>(px, g.nx)) go(k_xfwd<T, false, 16, 128>);
    else if (ct_plan<256>(px, g.nx)) go(k_xfwd<T, false, 16, 256>);
    else if (ct_plan<64>(px, g.nx)) go(k_xfwd<T, false, 16, 64>);
    else if (ct_plan<32>(px, g.nx)) go(k_xfwd<T, false, 16, 32>);
    else go(k_xfwd<T, false, 16>);
  }
  return hipGetLastError();
}

static int ypass_zb(const Grid& g) {
  int zb = g.zb > 0 ? g.zb : kMaxPts / g.ny;
  if (zb * g.ny > kMaxPts) zb = kMaxPts / g.ny;
  if (zb > 16) zb = 16;
  if (zb < 1) zb = 1;
  return zb;
}

template <typename T>
hipError_t launch_yfwd(const Grid& g, const AxisPlan& py, const cplx<double>* twy,
                       const cplx<T>* A, cplx<T>* B, long long sstride, int nload,
                       const PcgState* st, hipStream_t s) {
  const bool P3K = py.n % 3 == 0;
  const int zb = ypass_zb(g);
  dim3 grid((g.nz + zb - 1) / zb, g.nxh, nload * g.nd);
  size_t lds = sizeof(cplx<T>) * (size_t)(g.ny + zb * lds_stride<T>(g.ny));
  auto go = [&](auto kern) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, g, py, twy, zb, A, B, sstride, st);
  };
  if (ct_plan<96>(py, g.ny)) go(k_yfwd<T, true, 96>);
  else if (ct_plan<48>(py, g.ny)) go(k_yfwd<T, true, 48>);
  else if (P3K) go(k_yfwd<T, true>);
  else if (ct_plan<128>(py, g.ny)) go(k_yfwd<T, false, 128>);
  else if (ct_plan<64>(py, g.ny)) go(k_yfwd<T, false, 64>);
  else if (ct_plan<256>(py, g.ny)) go(k_yfwd<T, false, 256>);
  else if (ct_plan<32>(py, g.ny)) go(k_yfwd<T, false, 32>);
  else if (ct_plan<16>(py, g.ny)) go(k_yfwd<T, false, 16>);
  else go(k_yfwd<T, false>);
  return hipGetLastError();
}

template <typename T>
static int zpass_kyb(const Grid& g) {
  int kyb = g.kyb > 0 ? g.kyb : kMaxPts / (g.nd * g.nz);
  if (kyb * g.nd * g.nz > kMaxPts) kyb = kMaxPts / (g.nd * g.nz);
  if (kyb > 16) kyb = 16;
  if (kyb < 1) kyb = 1;
  if (kyb > g.ny) kyb = g.ny;
  return kyb;
}

template <typename T>
int zpass_nblocks(const Grid& g) {
  const int kyb = zpass_kyb<T>(g);
  return ((g.ny + kyb - 1) / kyb) * g.nxh;
}
template int zpass_nblocks<double>(const Grid&);
template int zpass_nblocks<float>(const Grid&);

template <typename T>
hipError_t launch_zpass(const Grid& g, const AxisPlan& pz, const cplx<double>* twz, int mode,
                        cplx<T>* B, long long sstride, const T* kplus, int nload,
                        const PcgState* st, double* rz_part, int* nblocks_out, hipStream_t s) {
  const bool P3K = pz.n % 3 == 0;
  const int kyb = zpass_kyb<T>(g);
  const int lg_n = ((g.ny + kyb - 1) / kyb) * g.nxh;
  dim3 grid((lg_n + 7) / 8 * 8, 1, nload);
  if (nblocks_out) *nblocks_out = lg_n;
  size_t lds = sizeof(cplx<T>) * (size_t)(g.nz + g.nd * kyb * lds_stride<T>(g.nz));
  auto go = [&](auto kern) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, g, pz, twz, mode, kyb, B, sstride,
                       kplus, st, rz_part);
  };
  // power-of-two lengths with the host's plan: the compile-time stage code
  auto ct = [&](auto nzc) {
    constexpr int NZ = decltype(nzc)::value;
    return g.nz == NZ && pz.n == NZ && pz.nstage == p2_nstage(NZ) && pz.code == p2_code(NZ);
  };
  if (ct(std::integral_constant<int, 96>{})) go(k_zpass<T, true, 96>);
  else if (ct(std::integral_constant<int, 48>{})) go(k_zpass<T, true, 48>);
  else if (P3K) go(k_zpass<T, true>);
  else if (ct(std::integral_constant<int, 128>{})) go(k_zpass<T, false, 128>);
  else if (ct(std::integral_constant<int, 64>{})) go(k_zpass<T, false, 64>);
  else if (ct(std::integral_constant<int, 256>{})) go(k_zpass<T, false, 256>);
  else if (ct(std::integral_constant<int, 32>{})) go(k_zpass<T, false, 32>);
  else if (ct(std::integral_constant<int, 16>{})) go(k_zpass<T, false, 16>);
  else go(k_zpass<T, false>);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_yinv(const Grid& g, const AxisPlan& py, const cplx<double>* twy,
                       const cplx<T>* B, cplx<T>* A, long long sstride, int nload,
                       const PcgState* st, hipStream_t s) {
  const bool P3K = py.n % 3 == 0;
  const int zb = ypass_zb(g);
  dim3 grid((g.nz + zb - 1) / zb, g.nxh, nload * g.nd);
  size_t lds = sizeof(cplx<T>) * (size_t)(g.ny + zb * lds_stride<T>(g.ny));
  auto go = [&](auto kern) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, g, py, twy, zb, B, A, sstride, st);
  };
  if (ct_plan<96>(py, g.ny)) go(k_yinv<T, true, 96>);
  else if (ct_plan<48>(py, g.ny)) go(k_yinv<T, true, 48>);
  else if (P3K) go(k_yinv<T, true>);
  else if (ct_plan<128>(py, g.ny)) go(k_yinv<T, false, 128>);
  else if (ct_plan<64>(py, g.ny)) go(k_yinv<T, false, 64>);
  else if (ct_plan<256>(py, g.ny)) go(k_yinv<T, false, 256>);
  else if (ct_plan<32>(py, g.ny)) go(k_yinv<T, false, 32>);
  else if (ct_plan<16>(py, g.ny)) go(k_yinv<T, false, 16>);
  else go(k_yinv<T, false>);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xinv(const Grid& g, const AxisPlan& px, const cplx<double>* twx, int mode,
                       const cplx<T>* A, long long sstride, T* out, T* x, T* p,
                       long long fstride, int nload, const PcgState* st, hipStream_t s) {
  const bool P3K = px.n % 3 == 0;
  const int kRows = xpass_rows<T>(g, true);
  dim3 grid((g.ny + kRows - 1) / kRows, g.nz, nload * g.nd);
  size_t lds = sizeof(cplx<T>) * (size_t)(g.nx + (kRows / 2) * lds_stride<T>(g.nx) +
                                          kRows * (g.nxh + 1));
  auto go = [&](auto kern) {
    if (lds > 65536)
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, g, px, twx, mode, A, sstride, out, x,
                       p, fstride, st);
  };
  if (kRows == 32) {
    if (ct_plan<96>(px, g.nx)) go(k_xinv<T, true, 32, 96>);
    else if (ct_plan<48>(px, g.nx)) go(k_xinv<T, true, 32, 48>);
    else if (P3K) go(k_xinv<T, true, 32>);
    else if (ct_plan<128>(px, g.nx)) go(k_xinv<T, false, 32, 128>);
    else if (ct_plan<64>(px, g.nx)) go(k_xinv<T, false, 32, 64>);
    else if (ct_plan<32>(px, g.nx)) go(k_xinv<T, false, 32, 32>);
    else go(k_xinv<T, false, 32>);
  } else if (kRows == 8) {
    if (P3K) go(k_xinv<T, true, 8>);
    else if (ct_plan<256>(px, g.nx)) go(k_xinv<T, false, 8, 256>);
    else go(k_xinv<T, false, 8>);
  } else {
    if (ct_plan<96>(px, g.nx)) go(k_xinv<T, true, 16, 96>);
    else if (ct_plan<48>(px, g.nx)) go(k_xinv<T, true, 16, 48>);
    else if (P3K) go(k_xinv<T, true, 16>);
    else if (ct_plan<128>(px, g.nx)) go(k_xinv<T, false, 16, 128>);
    else if (ct_plan<256>(px, g.nx)) go(k_xinv<T, false, 16, 256>);
    else if (ct_plan<64>(px, g.nx)) go(k_xinv<T, false, 16, 64>);
    else if (ct_plan<32>(px, g.nx)) go(k_xinv<T, false, 16, 32>);
    else go(k_xinv<T, false, 16>);
  }
  return hipGetLastError();
}

hipError_t launch_symbol(const Grid& g, const cplx<double>* spec, long long sstride,
                         double* kplus, int* bad, hipStream_t s) {
  long long nfreq = (long long)g.nxh * g.ny * g.nz;
  int blocks = (int)((nfreq + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_symbol, dim3(blocks), dim3(256), 0, s, g, spec, sstride, kplus, bad);
  return hipGetLastError();
}

hipError_t launch_cast_symbol(long long count, const double* src, float* dst, hipStream_t s) {
  int blocks = (int)((count + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_cast_symbol, dim3(blocks), dim3(256), 0, s, count, src, dst);
  return hipGetLastError();
}

#define FH_INST(T)                                                                              \
  template hipError_t launch_xfwd<T>(const Grid&, const AxisPlan&, const cplx<double>*, int,  \
                                     T*, long long, const T*, long long, cplx<T>*, long long,  \
                                     int, const PcgState*, hipStream_t);                       \
  template hipError_t launch_yfwd<T>(const Grid&, const AxisPlan&, const cplx<double>*,       \
                                     const cplx<T>*, cplx<T>*, long long, int,                 \
                                     const PcgState*, hipStream_t);                            \
  template hipError_t launch_zpass<T>(const Grid&, const AxisPlan&, const cplx<double>*, int, \
                                      cplx<T>*, long long, const T*, int, const PcgState*,     \
                                      double*, int*, hipStream_t);                             \
  template hipError_t launch_yinv<T>(const Grid&, const AxisPlan&, const cplx<double>*,       \
                                     const cplx<T>*, cplx<T>*, long long, int,                 \
                                     const PcgState*, hipStream_t);                            \
  template hipError_t launch_xinv<T>(const Grid&, const AxisPlan&, const cplx<double>*, int,  \
                                     const cplx<T>*, long long, T*, T*, T*, long long, int,    \
                                     const PcgState*, hipStream_t);
FH_INST(double)
FH_INST(float)

}  // namespace fh
