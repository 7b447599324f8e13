// Learned warm start: a 3D convolutional encoder-decoder that maps the phase
// field of a two-phase microstructure to an initial fluctuation field for
// PCG (the initial guess u_(0) of Alg. 1, which the paper takes as zero).
// Training and inference run on the GPU with the kernels below:
//   * 3x3x3 periodic convolutions as implicit GEMMs on the CDNA4 matrix
//     cores (v_mfma_f32_16x16x32_bf16): BF16 operands, FP32 accumulation,
//     the periodic input halo staged through LDS; the same kernel computes
//     the input gradient with flipped, transposed weights;
//   * weight gradients as MFMA contractions over voxels, with channel-major,
//     x-shifted copies of the layer input so that every operand load is an
//     aligned 16-byte read;
//   * pooling, up-sampling, skip concatenation, the 1x1 head, the H^1 loss,
//     Adam and the weight packing as plain memory-bound kernels.
// Network (levels n, n/2, n/4, n/8 with 16/32/64/64 channels), loss and
// storage precision are defined by the FP64 reference the tests compare
// against; the activation is a leaky ReLU with slope 1/8.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fh.h"
#include "../../include/fh_net.h"
#include "fh_internal.h"

namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kSlope = 0.125f;
constexpr int kOut = 18;
constexpr int kHeadIn = 16;
constexpr int kLayers = 14;

struct LayerDef {
  int cin, cout, level;
};
constexpr LayerDef kL[kLayers] = {{3, 16, 0},   {16, 16, 0}, {16, 32, 1}, {32, 32, 1},
                                  {32, 64, 2},  {64, 64, 2}, {64, 64, 3}, {64, 64, 3},
                                  {128, 64, 2}, {64, 64, 2}, {96, 32, 1}, {32, 32, 1},
                                  {48, 16, 0},  {16, 16, 0}};
inline int cinp(int l) { return (kL[l].cin + 15) / 16 * 16; }

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float leaky_grad(float y) { return y > 0.0f ? 1.0f : kSlope; }
__device__ __forceinline__ int wrap(int i, int s) { return i < 0 ? i + s : (i >= s ? i - s : i); }

// ------------------------------------------------------------ convolution
// y[b][v][co] = epi( sum_t sum_ci W[t][co][ci] x[b][v + d_t][ci] ), channels
// last.  The reduction index k = (tap, ci) runs over 16-channel chunks of the
// input staged in LDS with a one-voxel periodic halo; an MFMA step covers two
// taps x 16 channels (k = 32), 14 steps per chunk (the last one pairs tap 26
// with a zero-weight dummy).  Weights come packed per step:
//   w[chunk][step][co][32], k = 8 g + e <-> tap 2 step + (g >> 1),
//   channel 16 chunk + 8 (g & 1) + e.
// MFMA roles: rows = 16 voxels of the tile, columns = 16 output channels.
// A wave owns RW row groups x NCT column tiles; a block (4 waves) covers
// a tx x ty x tz tile and NCT*16 output channels.
struct ConvArgs {
  const uint16_t* x;
  const uint16_t* w;
  const float* bias;     // forward: bias, else null
  const uint16_t* mask;  // input gradient: multiply by leaky'(mask) (stride cout), else null
  uint16_t* y;
  int cin, cout, s, tx, ty, tz, act, ngroups;
};

constexpr int kMaxHalo = 18 * 10 * 6;

template <int NCT, int RW>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  __shared__ uint4 lds[2 * kMaxHalo];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int s = a.s;
  const int ntx = s / a.tx, nty = s / a.ty, ntz = s / a.tz;
  int bid = blockIdx.x;
  const int tix = bid % ntx;
  bid /= ntx;
  const int tiy = bid % nty;
  bid /= nty;
  const int tiz = bid % ntz;
  bid /= ntz;
  const int grp = bid % a.ngroups;
  const int b = bid / a.ngroups;
  const int HX = a.tx + 2, HY = a.ty + 2, HZ = a.tz + 2, HV = HX * HY * HZ;
  const int x0 = tix * a.tx, y0 = tiy * a.ty, z0 = tiz * a.tz;
  const long long V = (long long)s * s * s;
  const uint16_t* xb = a.x + (long long)b * V * a.cin;
  int hbase[RW];
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int q = (wave * RW + rr) * 16 + i16;
    const int tx = q % a.tx, ty = (q / a.tx) % a.ty, tz = q / (a.tx * a.ty);
    hbase[rr] = ((tz + 1) * HY + (ty + 1)) * HX + (tx + 1);
  }
  f32x4 acc[RW][NCT];
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[rr][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int co0 = grp * NCT * 16;
  const int nchunk = a.cin >> 4;
  const int half = g & 1;
  for (int ch = 0; ch < nchunk; ++ch) {
    __syncthreads();
    for (int idx = tid; idx < 2 * HV; idx += 256) {
      const int hv = idx >> 1, h = idx & 1;
      const int hx = hv % HX, t = hv / HX, hy = t % HY, hz = t / HY;
      const int gx = wrap(x0 + hx - 1, s), gy = wrap(y0 + hy - 1, s), gz = wrap(z0 + hz - 1, s);
      lds[h * HV + hv] = *reinterpret_cast<const uint4*>(
          xb + (((long long)gz * s + gy) * s + gx) * a.cin + ch * 16 + h * 8);
    }
    __syncthreads();
    const uint16_t* wch = a.w + (long long)ch * 14 * a.cout * 32;
#pragma unroll
    for (int st = 0; st < 14; ++st) {
      int tap = 2 * st + (g >> 1);
      tap = tap > 26 ? 26 : tap;
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
      const int off = (dz * HY + dy) * HX + dx;
      bf16x8 bw[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        bw[ct] = *reinterpret_cast<const bf16x8*>(
            wch + ((long long)st * a.cout + co0 + ct * 16 + i16) * 32 + g * 8);
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(&lds[half * HV + hbase[rr] + off]);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[rr][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[ct], acc[rr][ct], 0, 0, 0);
      }
    }
  }
  // epilogue: lane holds rows 4 g + j (voxels) of column i16 (channel)
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int co = co0 + ct * 16 + i16;
      const float bv = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = (wave * RW + rr) * 16 + 4 * g + j;
        const int tx = q % a.tx, ty = (q / a.tx) % a.ty, tz = q / (a.tx * a.ty);
        const long long gv = ((long long)(z0 + tz) * s + (y0 + ty)) * s + (x0 + tx);
        const long long o = ((long long)b * V + gv) * a.cout + co;
        float v = acc[rr][ct][j] + bv;
        if (a.act) v = v > 0.0f ? v : kSlope * v;
        if (a.mask) v *= leaky_grad(bf2f(a.mask[o]));
        a.y[o] = f2bf(v);
      }
    }
}

// ------------------------------------------------------- weight gradient
// dW[t][o][c] = sum_v dZ[o][v] X[c][v + d_t].  MFMA roles: rows = 16 output
// channels (A = dZ, channel-major), columns = 16 input channels (B = X,
// channel-major), k = 32 consecutive voxels (four 8-voxel groups of one x
// row, one group per 16 lanes).  For every (dz, dy) row a lane loads its
// aligned 8 voxels once plus the single voxel on each side (periodic in x)
// and forms the dx = -1, 0, +1 operands with 16-bit funnel shifts, so each
// input row is read once for its three x taps.  A wave owns one (o, c) tile
// for all 27 taps and a contiguous range of k steps; partial sums go to
// part[split][t][o][c] and the per-channel sums of dZ (the bias gradient)
// to bpart[split][o].
struct WgradArgs {
  const uint16_t* xt;   // [B][cinp][V] channel-major layer input
  const uint16_t* dzt;  // [B][cout][V]
  float* part;
  float* bpart;
  int B, s, cinp, cout, nsplit, ntiles;
  long long ksteps;
};

__device__ __forceinline__ unsigned fshift16(unsigned lo, unsigned hi) {
  return (lo >> 16) | (hi << 16);
}

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
  const int lane = threadIdx.x & 63;
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= a.ntiles * a.nsplit) return;
  const int tile = wid % a.ntiles, split = wid / a.ntiles;
  const int nto = a.cout / 16;
  const int ot = tile % nto, it = tile / nto;
  const int i16 = lane & 15, g = lane >> 4;
  const int s = a.s;
  const long long V = (long long)s * s * s;
  const long long k0 = a.ksteps * split / a.nsplit, k1 = a.ksteps * (split + 1) / a.nsplit;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  for (long long ks = k0; ks < k1; ++ks) {
    const long long kv = ks * 32;
    const int b = (int)(kv / V);
    const long long v = kv - (long long)b * V + 8 * g;
    const int x = (int)(v % s), y = (int)((v / s) % s), z = (int)(v / ((long long)s * s));
    const int xl = x == 0 ? s - 1 : x - 1, xr = x + 8 == s ? 0 : x + 8;
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(
        a.dzt + ((long long)b * a.cout + ot * 16 + i16) * V + v);
#pragma unroll
    for (int e = 0; e < 8; ++e) bsum += bf2f((unsigned short)av[e]);
    const uint16_t* xc = a.xt + ((long long)b * a.cinp + it * 16 + i16) * V;
#pragma unroll
    for (int dzi = 0; dzi < 3; ++dzi) {
      const int zz = wrap(z + dzi - 1, s);
#pragma unroll
      for (int dyi = 0; dyi < 3; ++dyi) {
        const int yy = wrap(y + dyi - 1, s);
        const uint16_t* row = xc + ((long long)zz * s + yy) * s;
        const uint4 c = *reinterpret_cast<const uint4*>(row + x);
        const unsigned L = row[xl], R = row[xr];
        const unsigned s0 = fshift16(c.x, c.y), s1 = fshift16(c.y, c.z), s2 = fshift16(c.z, c.w);
        const uint4 lft = {L | (c.x << 16), s0, s1, s2};
        const uint4 rgt = {s0, s1, s2, fshift16(c.w, R)};
        const int t0 = dzi * 9 + dyi * 3;
        acc[t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&lft), acc[t0], 0, 0, 0);
        acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&c), acc[t0 + 1], 0, 0, 0);
        acc[t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&rgt), acc[t0 + 2], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      a.part[(((long long)split * 27 + t) * a.cout + ot * 16 + 4 * g + j) * a.cinp + it * 16 +
             i16] = acc[t][j];
  bsum += __shfl_xor(bsum, 16);
  bsum += __shfl_xor(bsum, 32);
  if (it == 0 && g == 0) a.bpart[(long long)split * a.cout + ot * 16 + i16] = bsum;
}

// The same products for grids with s >= 32 (a k step is 32 voxels of one x
// row): the k steps of a wave run along y within one (b, z, x-half) column,
// and the nine input rows of consecutive steps overlap in six, so a step
// loads only the three rows at y + 1 (one per dz) and shifts the other six
// along; a wave that starts a column, or starts mid-column, loads all nine.
// The next step's dZ tile and new rows are loaded while the current step's
// products run.  Two waves per SIMD (at most 256 registers): 112 TFLOP/s at
// 64^3 and batch 8, against 73 for the nine-row kernel; one wave per SIMD
// with the compiler's 336 registers, 103.
struct XRow {
  uint4 c;        // the lane's 8 aligned voxels
  unsigned l, r;  // its neighbours at x - 1 and x + 8 (periodic)
};

__global__ void __launch_bounds__(256, 2) k_wgrad_roll(WgradArgs a) {
  const int lane = threadIdx.x & 63;
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= a.ntiles * a.nsplit) return;
  const int tile = wid % a.ntiles, split = wid / a.ntiles;
  const int nto = a.cout / 16;
  const int ot = tile % nto, it = tile / nto;
  const int i16 = lane & 15, g = lane >> 4;
  const int s = a.s, nxh = s / 32;
  const long long V = (long long)s * s * s;
  const long long k0 = a.ksteps * split / a.nsplit, k1 = a.ksteps * (split + 1) / a.nsplit;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  // k step -> (sample, z, x half, y), y fastest
  struct Pos {
    int b, z, xh, y;
  };
  auto pos = [&](long long ks) {
    Pos q;
    q.y = (int)(ks % s);
    const long long r = ks / s;
    q.xh = (int)(r % nxh);
    const long long r2 = r / nxh;
    q.z = (int)(r2 % s);
    q.b = (int)(r2 / s);
    return q;
  };
  auto load_row = [&](const Pos& q, int zz, int yy) {
    const int x = q.xh * 32 + 8 * g;
    const int xl = x == 0 ? s - 1 : x - 1, xr = x + 8 == s ? 0 : x + 8;
    const uint16_t* row =
        a.xt + ((long long)q.b * a.cinp + it * 16 + i16) * V + ((long long)zz * s + yy) * s;
    XRow o;
    o.c = *reinterpret_cast<const uint4*>(row + x);
    o.l = row[xl];
    o.r = row[xr];
    return o;
  };
  auto load_dz = [&](const Pos& q) {
    const long long v = ((long long)q.z * s + q.y) * s + q.xh * 32 + 8 * g;
    return *reinterpret_cast<const bf16x8*>(
        a.dzt + ((long long)q.b * a.cout + ot * 16 + i16) * V + v);
  };
  auto load_all = [&](const Pos& q, XRow (&w)[3][3]) {
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
        w[dz][dy] = load_row(q, wrap(q.z + dz - 1, s), wrap(q.y + dy - 1, s));
  };
  if (k0 >= k1) return;
  // w[dz][dy]: input row (z + dz - 1, y + dy - 1) of the current step; the
  // next step's dZ tile and, when it continues the column, its three new
  // rows are loaded while the current step's products run
  XRow w[3][3], nw[3];
  Pos cur = pos(k0);
  load_all(cur, w);
  bf16x8 av = load_dz(cur);
  for (long long ks = k0; ks < k1; ++ks) {
    const bool more = ks + 1 < k1;
    Pos nxt = cur;
    bool cont = false;
    bf16x8 an = av;
    if (more) {
      nxt = pos(ks + 1);
      cont = nxt.b == cur.b && nxt.z == cur.z && nxt.xh == cur.xh && nxt.y == cur.y + 1;
      if (cont) {
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) nw[dz] = load_row(nxt, wrap(nxt.z + dz - 1, s), wrap(nxt.y + 1, s));
      }
      an = load_dz(nxt);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) bsum += bf2f((unsigned short)av[e]);
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const uint4 c = w[dz][dy].c;
        const unsigned s0 = fshift16(c.x, c.y), s1 = fshift16(c.y, c.z), s2 = fshift16(c.z, c.w);
        const uint4 lft = {w[dz][dy].l | (c.x << 16), s0, s1, s2};
        const uint4 rgt = {s0, s1, s2, fshift16(c.w, w[dz][dy].r)};
        const int t0 = dz * 9 + dy * 3;
        acc[t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&lft), acc[t0], 0, 0, 0);
        acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&c), acc[t0 + 1], 0, 0, 0);
        acc[t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(&rgt), acc[t0 + 2], 0, 0, 0);
      }
    if (!more) break;
    if (cont) {
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        w[dz][0] = w[dz][1];
        w[dz][1] = w[dz][2];
        w[dz][2] = nw[dz];
      }
    } else {
      load_all(nxt, w);
    }
    av = an;
    cur = nxt;
  }
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      a.part[(((long long)split * 27 + t) * a.cout + ot * 16 + 4 * g + j) * a.cinp + it * 16 +
             i16] = acc[t][j];
  bsum += __shfl_xor(bsum, 16);
  bsum += __shfl_xor(bsum, 32);
  if (it == 0 && g == 0) a.bpart[(long long)split * a.cout + ot * 16 + i16] = bsum;
}

// Column sums of part[nrow][ncol] in two fixed-order stages: block (x, r)
// sums rows r, r + R, r + 2R, ... of its 256 columns into p2[r][col]; then
// out[map(col)] = sum_r p2[r][col], where col = a * cinp + c maps to
// a * cin + c for c < cin (dropping padded channels) and is dropped else.
__global__ void k_colsum1(const float* part, long long nrow, long long ncol, int R, double* p2) {
  const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncol) return;
  double acc = 0.0;
  for (long long row = blockIdx.y; row < nrow; row += R) acc += part[row * ncol + col];
  p2[(long long)blockIdx.y * ncol + col] = acc;
}
__global__ void k_colsum2(const double* p2, int R, long long ncol, int cinp, int cin, float* out) {
  const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncol) return;
  double acc = 0.0;
  for (int r = 0; r < R; ++r) acc += p2[(long long)r * ncol + col];
  const int c = (int)(col % cinp);
  if (c < cin) out[(col / cinp) * cin + c] = (float)acc;
}

// channels-last [B][V][C] -> channel-major [ncopy][B][C][V]; with ncopy = 3,
// copy d holds the input shifted by d - 1 in x
__global__ void k_prep_shifted(const uint16_t* x, int C, int s, int B, int ncopy, uint16_t* out) {
  const long long V = (long long)s * s * s;
  const int ng = C / 8;
  const long long total = (long long)B * ng * V;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long v = i % V;
  const long long r = i / V;
  const int cg = (int)(r % ng), b = (int)(r / ng);
  const uint4 raw = *reinterpret_cast<const uint4*>(x + ((long long)b * V + v) * C + 8 * cg);
  const unsigned short* e = reinterpret_cast<const unsigned short*>(&raw);
  const int xx = (int)(v % s);
  const long long rowbase = v - xx;
  for (int d = 0; d < ncopy; ++d) {
    const int dx = ncopy == 3 ? d - 1 : 0;
    const int xd = wrap(xx - dx, s);
    uint16_t* o = out + (((long long)d * B + b) * C + 8 * cg) * V + rowbase + xd;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[(long long)k * V] = e[k];
  }
}

// ------------------------------------------------- elementwise and small
__global__ void k_features(const uint8_t* phase, const int* order, const float* gamma, int B,
                           long long V, uint16_t* I) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * V) return;
  const int b = (int)(i / V);
  const long long v = i - (long long)b * V;
  const int smp = order ? order[b] : b;
  const float gm = gamma[b];
  const bool chi = phase[(long long)smp * V + v] == 1;
  const unsigned short gb = f2bf(gm);
  uint4 lo, hi;
  lo.x = (chi ? 0x3f80u : 0u) | ((unsigned)(chi ? gb : 0) << 16);
  lo.y = gb;
  lo.z = lo.w = 0u;
  hi.x = hi.y = hi.z = hi.w = 0u;
  uint4* o = reinterpret_cast<uint4*>(I + i * 16);
  o[0] = lo;
  o[1] = hi;
}

// P[b][vc][c] = bf16(mean of the 8 children)
__global__ void k_pool(const uint16_t* x, int C, int s, int B, uint16_t* out) {
  const int h = s / 2;
  const long long Vc = (long long)h * h * h;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * Vc * C) return;
  const int c = (int)(i % C);
  const long long r = i / C;
  const long long vc = r % Vc;
  const int b = (int)(r / Vc);
  const int xc = (int)(vc % h), yc = (int)((vc / h) % h), zc = (int)(vc / ((long long)h * h));
  const long long V = (long long)s * s * s;
  float acc = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const long long v = ((long long)(2 * zc + (k >> 2)) * s + (2 * yc + ((k >> 1) & 1))) * s +
                        (2 * xc + (k & 1));
    acc += bf2f(x[((long long)b * V + v) * C + c]);
  }
  out[i] = f2bf(acc * 0.125f);
}

// C[b][v] = [coarse[b][parent(v)][0:Cu], skip[b][v][0:Cs]] in 8-channel groups
__global__ void k_concat(const uint16_t* coarse, int Cu, const uint16_t* skip, int Cs, int s,
                         int B, uint16_t* out) {
  const int Ct = Cu + Cs, ng = Ct / 8;
  const long long V = (long long)s * s * s;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * V * ng) return;
  const int cg = (int)(i % ng);
  const long long r = i / ng;
  const long long v = r % V;
  const int b = (int)(r / V);
  const int h = s / 2;
  uint4 val;
  if (cg * 8 < Cu) {
    const int x = (int)(v % s), y = (int)((v / s) % s), z = (int)(v / ((long long)s * s));
    const long long vc = ((long long)(z / 2) * h + y / 2) * h + x / 2;
    val = *reinterpret_cast<const uint4*>(coarse + ((long long)b * h * h * h + vc) * Cu + cg * 8);
  } else {
    val = *reinterpret_cast<const uint4*>(skip + ((long long)b * V + v) * Cs + (cg * 8 - Cu));
  }
  *reinterpret_cast<uint4*>(out + ((long long)b * V + v) * Ct + cg * 8) = val;
}

// coarse gradient of nearest up-sampling: sum of the 8 children of dC[.][0:Cu]
__global__ void k_upsum(const uint16_t* dc, int Ct, int Cu, int s, int B, uint16_t* out) {
  const int h = s / 2;
  const long long Vc = (long long)h * h * h, V = (long long)s * s * s;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * Vc * Cu) return;
  const int c = (int)(i % Cu);
  const long long r = i / Cu;
  const long long vc = r % Vc;
  const int b = (int)(r / Vc);
  const int xc = (int)(vc % h), yc = (int)((vc / h) % h), zc = (int)(vc / ((long long)h * h));
  float acc = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const long long v = ((long long)(2 * zc + (k >> 2)) * s + (2 * yc + ((k >> 1) & 1))) * s +
                        (2 * xc + (k & 1));
    acc += bf2f(dc[((long long)b * V + v) * Ct + c]);
  }
  out[i] = f2bf(acc);
}

// dE[b][v][c] = dC[b][v][Cu + c] + leaky'(E[b][v][c]) dP[b][parent(v)][c] / 8
__global__ void k_combine(const uint16_t* dc, int Ct, int Cu, const uint16_t* E, const uint16_t* dP,
                          int C, int s, int B, uint16_t* out) {
  const long long V = (long long)s * s * s;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * V * C) return;
  const int c = (int)(i % C);
  const long long r = i / C;
  const long long v = r % V;
  const int b = (int)(r / V);
  const int h = s / 2;
  const int x = (int)(v % s), y = (int)((v / s) % s), z = (int)(v / ((long long)s * s));
  const long long vc = ((long long)(z / 2) * h + y / 2) * h + x / 2;
  const float up = bf2f(dP[((long long)b * h * h * h + vc) * C + c]);
  const float val = bf2f(dc[((long long)b * V + v) * Ct + Cu + c]) + leaky_grad(bf2f(E[i])) * up * 0.125f;
  out[i] = f2bf(val);
}

// head: O[b][o][v] = sum_c Wh[o][c] D0[b][v][c] + bh[o]  (FP32 out)
__global__ void k_head(const uint16_t* d0, const float* wh, const float* bh, long long V, int B,
                       float* O) {
  __shared__ float w[kOut * kHeadIn + kOut];
  for (int k = threadIdx.x; k < kOut * kHeadIn + kOut; k += blockDim.x)
    w[k] = k < kOut * kHeadIn ? wh[k] : bh[k - kOut * kHeadIn];
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * V) return;
  const int b = (int)(i / V);
  const long long v = i - (long long)b * V;
  float d[kHeadIn];
  const uint4* src = reinterpret_cast<const uint4*>(d0 + i * kHeadIn);
  for (int q = 0; q < 2; ++q) {
    const uint4 raw = src[q];
    const unsigned short* e = reinterpret_cast<const unsigned short*>(&raw);
    for (int k = 0; k < 8; ++k) d[q * 8 + k] = bf2f(e[k]);
  }
  for (int o = 0; o < kOut; ++o) {
    float acc = w[kOut * kHeadIn + o];
    for (int c = 0; c < kHeadIn; ++c) acc += w[o * kHeadIn + c] * d[c];
    O[((long long)b * kOut + o) * V + v] = acc;
  }
}

// dD0[b][v][c] = leaky'(D0) sum_o Wh[o][c] dO[b][o][v]
__global__ void k_head_bwd(const float* dO, const uint16_t* d0, const float* wh, long long V,
                           int B, uint16_t* dd0) {
  __shared__ float w[kOut * kHeadIn];
  for (int k = threadIdx.x; k < kOut * kHeadIn; k += blockDim.x) w[k] = wh[k];
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * V) return;
  const int b = (int)(i / V);
  const long long v = i - (long long)b * V;
  float g[kOut];
  for (int o = 0; o < kOut; ++o) g[o] = dO[((long long)b * kOut + o) * V + v];
  uint4 out[2];
  unsigned short* oe = reinterpret_cast<unsigned short*>(out);
  const uint4* src = reinterpret_cast<const uint4*>(d0 + i * kHeadIn);
  uint4 raw[2] = {src[0], src[1]};
  const unsigned short* de = reinterpret_cast<const unsigned short*>(raw);
  for (int c = 0; c < kHeadIn; ++c) {
    float acc = 0.0f;
    for (int o = 0; o < kOut; ++o) acc += w[o * kHeadIn + c] * g[o];
    oe[c] = f2bf(leaky_grad(bf2f(de[c])) * acc);
  }
  uint4* dst = reinterpret_cast<uint4*>(dd0 + i * kHeadIn);
  dst[0] = out[0];
  dst[1] = out[1];
}

// head weight gradient: per block of 256 voxels (one sample), thread p < 288
// sums dO[o][v] D0[v][c] (o = p / 16, c = p % 16), thread 288 + o sums dO[o][v]
constexpr int kHeadChunk = 256;
constexpr int kHeadNP = kOut * kHeadIn + kOut;
__global__ void __launch_bounds__(320) k_head_wgrad(const float* dO, const uint16_t* d0,
                                                    long long V, float* part) {
  __shared__ float sg[kOut][kHeadChunk];
  __shared__ float sd[kHeadChunk][kHeadIn + 1];
  const long long chunks = V / kHeadChunk;
  const int b = (int)(blockIdx.x / chunks);
  const long long v0 = (blockIdx.x % chunks) * kHeadChunk;
  for (int k = threadIdx.x; k < kOut * kHeadChunk; k += blockDim.x) {
    const int o = k / kHeadChunk, vv = k % kHeadChunk;
    sg[o][vv] = dO[((long long)b * kOut + o) * V + v0 + vv];
  }
  for (int k = threadIdx.x; k < kHeadChunk * kHeadIn; k += blockDim.x) {
    const int vv = k / kHeadIn, c = k % kHeadIn;
    sd[vv][c] = bf2f(d0[((long long)b * V + v0 + vv) * kHeadIn + c]);
  }
  __syncthreads();
  const int p = threadIdx.x;
  if (p >= kHeadNP) return;
  float acc = 0.0f;
  if (p < kOut * kHeadIn) {
    const int o = p / kHeadIn, c = p % kHeadIn;
    for (int vv = 0; vv < kHeadChunk; ++vv) acc += sg[o][vv] * sd[vv][c];
  } else {
    const int o = p - kOut * kHeadIn;
    for (int vv = 0; vv < kHeadChunk; ++vv) acc += sg[o][vv];
  }
  part[(long long)blockIdx.x * kHeadNP + p] = acc;
}


// loss = mean_{b,o,v,d} (e[v + e_d] - e[v])^2, e = O - T; dO = dloss/dO.
constexpr int kLossBlocks = 2048;
__global__ void k_loss(const float* O, const uint16_t* T, const int* order, int s, int B,
                       double inv_m, float* dO, double* part) {
  __shared__ double sh[256];
  const long long V = (long long)s * s * s;
  const long long total = (long long)B * kOut * V;
  double contrib = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (long long)gridDim.x * 256) {
    const long long v = i % V;
    const long long bo = i / V;
    const int o = (int)(bo % kOut), b = (int)(bo / kOut);
    const int smp = order ? order[b] : b;
    const float* Ob = O + bo * V;
    const uint16_t* Tb = T + ((long long)smp * kOut + o) * V;
    const int x = (int)(v % s), y = (int)((v / s) % s), z = (int)(v / ((long long)s * s));
    auto e = [&](int zz, int yy, int xx) {
      const long long w = ((long long)zz * s + yy) * s + xx;
      return Ob[w] - bf2f(Tb[w]);
    };
    const float e0 = e(z, y, x);
    const float ex = e(z, y, wrap(x + 1, s)), exm = e(z, y, wrap(x - 1, s));
    const float ey = e(z, wrap(y + 1, s), x), eym = e(z, wrap(y - 1, s), x);
    const float ez = e(wrap(z + 1, s), y, x), ezm = e(wrap(z - 1, s), y, x);
    dO[i] = (float)(2.0 * inv_m) * (6.0f * e0 - ex - exm - ey - eym - ez - ezm);
    contrib += (double)(ex - e0) * (ex - e0) + (double)(ey - e0) * (ey - e0) +
               (double)(ez - e0) * (ez - e0);
  }
  sh[threadIdx.x] = contrib;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv_m;
}

__global__ void k_sum_double(const double* part, int n, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) acc += part[k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// global gradient norm -> clipping factor min(1, clip / |g|) (FP64 sums)
__global__ void k_sqnorm_part(const float* g, long long n, double* part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc += (double)g[i] * g[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_clip_factor(const double* part, int nb, double clip, float* factor) {
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int k = 0; k < nb; ++k) acc += part[k];
  const double nrm = sqrt(acc);
  *factor = (float)(nrm > clip ? clip / nrm : 1.0);
}

// omb1 = 1 - b1 and omb2 = 1 - b2 come from the host in FP64 (in FP32,
// 1 - 0.999f is 0.00100005, a 5e-5 relative error in the second moment)
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float omb1, float omb2, float eps, float c1, float c2,
                       const float* factor) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = factor ? g[i] * *factor : g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// master FP32 weights -> packed BF16 operands (forward and input gradient),
// BF16-rounded bias
__global__ void k_pack(const float* W, const float* bias, int cin, int cinp, int cout,
                       uint16_t* wf, uint16_t* wd, float* bout) {
  const long long nf = (long long)(cinp / 16) * 14 * cout * 32;
  const long long nd = wd ? (long long)(cout / 16) * 14 * cinp * 32 : 0;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) {
    const int k = (int)(i % 32);
    long long r = i / 32;
    const int co = (int)(r % cout);
    r /= cout;
    const int st = (int)(r % 14);
    const int ch = (int)(r / 14);
    const int g = k >> 3, e = k & 7;
    const int tap = 2 * st + (g >> 1), ci = ch * 16 + 8 * (g & 1) + e;
    float val = 0.0f;
    if (tap <= 26 && ci < cin) val = W[((long long)tap * cout + co) * cin + ci];
    wf[i] = f2bf(val);
  } else if (i < nf + nd) {
    const long long j = i - nf;
    const int k = (int)(j % 32);
    long long r = j / 32;
    const int ci = (int)(r % cinp);
    r /= cinp;
    const int st = (int)(r % 14);
    const int ch = (int)(r / 14);
    const int g = k >> 3, e = k & 7;
    const int tap = 2 * st + (g >> 1), co = ch * 16 + 8 * (g & 1) + e;
    float val = 0.0f;
    if (tap <= 26 && ci < cin) val = W[((long long)(26 - tap) * cout + co) * cin + ci];
    wd[j] = f2bf(val);
  } else if (i < nf + nd + cout) {
    const int o = (int)(i - nf - nd);
    bout[o] = bf2f(f2bf(bias[o]));
  }
}

__global__ void k_round(const float* src, float* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = bf2f(f2bf(src[i]));
}

__global__ void k_pack_target(const double* u, long long n, double scale, uint16_t* t) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = f2bf((float)(u[i] * scale));
}

// per-channel sums of O [18][V] (FP64 partials, then a fixed-order sum)
__global__ void k_chan_part(const float* O, long long V, int nb, double* part) {
  __shared__ double sh[256];
  const int ch = blockIdx.y;
  const long long per = (V + nb - 1) / nb;
  const long long v0 = blockIdx.x * per, v1 = min(V, v0 + per);
  double acc = 0.0;
  for (long long v = v0 + threadIdx.x; v < v1; v += 256) acc += O[(long long)ch * V + v];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)ch * nb + blockIdx.x] = sh[0];
}
__global__ void k_chan_mean(const double* part, int nb, long long V, double* mean) {
  const int ch = threadIdx.x;
  if (ch >= kOut) return;
  double acc = 0.0;
  for (int k = 0; k < nb; ++k) acc += part[(long long)ch * nb + k];
  mean[ch] = acc / (double)V;
}
// x[l][c][v] = scale sum_j E[l][j] (O[3 j + c][v] - mean[3 j + c])
__global__ void k_warm_x(const float* O, const double* mean, const double* E, int nload,
                         long long V, double scale, long long F, double* x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * V) return;
  const int c = (int)(i / V);
  const long long v = i - (long long)c * V;
  double o[6];
  for (int j = 0; j < 6; ++j) o[j] = (double)O[(long long)(3 * j + c) * V + v] - mean[3 * j + c];
  for (int l = 0; l < nload; ++l) {
    double acc = 0.0;
    for (int j = 0; j < 6; ++j) acc += E[l * 6 + j] * o[j];
    x[(long long)l * F + i] = scale * acc;
  }
}

inline unsigned nblk(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ================================================================= context
struct fh_net {
  int device = 0;
  hipStream_t stream = nullptr;
  int n = 0, maxb = 0;
  int s[4];
  long long V[4];
  std::string err;
  long long P = 0;
  long long offw[kLayers + 1], offb[kLayers + 1];
  char* mem = nullptr;
  float *p = nullptr, *gr = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wf[kLayers], *wd[kLayers];
  float* bias[kLayers];
  float *wh = nullptr, *bh = nullptr;
  uint16_t *I, *e0a, *e0, *p0, *e1a, *e1, *p1, *e2a, *e2, *p2, *b3a, *b3, *c2, *d2a, *d2, *c1,
      *d1a, *d1, *c0, *d0a, *d0;
  float *O, *dO;
  uint16_t *dc0, *dc1, *dc2, *ta, *tb, *xs, *dzt;
  float *wpart, *bpart, *hpart;
  double* csum;
  size_t wpart_n = 0, bpart_n = 0, csum_n = 0;
  double *lpart, *scal, *chpart, *chmean, *Edev;
  float* gamma_dev;
  float* clipf;
  int* order_dev = nullptr;
  long long order_n = 0;
  long long adam_t = 0;
  bool packed = false;
  // timing by class (FH_NET_K_*) with HIP events
  bool time_on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_cls;
  int ev_used = 0;
  double ms[FH_NET_K_NCLASS] = {0};
  long long launches[FH_NET_K_NCLASS] = {0};
  double flops[FH_NET_K_NCLASS] = {0};
};

namespace {

int nfail(fh_net* N, int code, const std::string& msg) {
  N->err = msg;
  return code;
}

#define NCHK(N, expr)                                                           \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) return nfail(N, FH_EDEVICE, std::string(#expr) + ": " + \
                                                          hipGetErrorString(e_)); \
  } while (0)

int tbegin(fh_net* N, int cls) {
  if (!N->time_on) return -1;
  if (N->ev_used + 2 > (int)N->ev.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      N->ev.push_back(e);
    }
    N->ev_cls.resize(N->ev.size() / 2 + 1);
  }
  const int slot = N->ev_used;
  N->ev_used += 2;
  N->ev_cls[slot / 2] = cls;
  hipEventRecord(N->ev[slot], N->stream);
  return slot;
}
void tend(fh_net* N, int slot) {
  if (slot >= 0) hipEventRecord(N->ev[slot + 1], N->stream);
}
void tcollect(fh_net* N) {
  if (!N->time_on || N->ev_used == 0) return;
  hipStreamSynchronize(N->stream);
  for (int k = 0; k < N->ev_used; k += 2) {
    float t = 0.0f;
    hipEventElapsedTime(&t, N->ev[k], N->ev[k + 1]);
    N->ms[N->ev_cls[k / 2]] += t;
    N->launches[N->ev_cls[k / 2]] += 1;
  }
  N->ev_used = 0;
}
struct TScope {
  fh_net* N;
  int slot;
  TScope(fh_net* n, int cls) : N(n), slot(tbegin(n, cls)) {}
  ~TScope() { tend(N, slot); }
};
// flush the event pool before it runs out of pre-created pairs
void tmaybe_flush(fh_net* N) {
  if (N->time_on && N->ev_used > 4096) tcollect(N);
}

template <int NCT, int RW>
hipError_t launch_conv_t(const ConvArgs& a, int B, hipStream_t st) {
  const int nblocks = B * a.ngroups * (a.s / a.tx) * (a.s / a.ty) * (a.s / a.tz);
  hipLaunchKernelGGL((k_conv<NCT, RW>), dim3(nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// y = conv(x) (forward, with bias and leaky ReLU) or the input gradient
// (w = flipped transposed weights, no bias, optional leaky' mask).
int conv(fh_net* N, const uint16_t* x, int cin, const uint16_t* w, const float* bias,
         const uint16_t* mask, uint16_t* y, int cout, int s, int B, bool act, int cls,
         double flops) {
  const int nct = cout / 16;
  int NCT = nct <= 4 ? nct : (nct == 6 ? 3 : 4);
  ConvArgs a{x, w, bias, mask, y, cin, cout, s, 0, 0, 0, act ? 1 : 0, nct / NCT};
  const int RW = NCT <= 2 ? 8 : 4;
  if (s >= 16) {
    a.tx = 16;
    a.ty = 8;
    a.tz = RW / 2;
  } else {
    a.tx = 8;
    a.ty = 8;
    a.tz = RW;
  }
  if (cin % 16 || cout % 16 || s % a.tx || s % a.ty || s % a.tz ||
      (a.tx + 2) * (a.ty + 2) * (a.tz + 2) > kMaxHalo)
    return nfail(N, FH_EINVAL, "conv shape not supported");
  TScope ts(N, cls);
  N->flops[cls] += flops;
  hipError_t e;
  switch (NCT) {
    case 1: e = launch_conv_t<1, 8>(a, B, N->stream); break;
    case 2: e = launch_conv_t<2, 8>(a, B, N->stream); break;
    case 3: e = launch_conv_t<3, 4>(a, B, N->stream); break;
    default: e = launch_conv_t<4, 4>(a, B, N->stream); break;
  }
  NCHK(N, e);
  return FH_OK;
}

// out <- column sums of part[nrow][ncol] (see k_colsum1/2)
int colsum(fh_net* N, const float* part, long long nrow, long long ncol, int cinp, int cin,
           float* out) {
  int R = (int)std::min<long long>(nrow, 64);
  R = (int)std::max<long long>(1, std::min<long long>(R, (long long)(N->csum_n / ncol)));
  hipLaunchKernelGGL(k_colsum1, dim3(nblk(ncol), R), dim3(256), 0, N->stream, part, nrow, ncol, R,
                     N->csum);
  hipLaunchKernelGGL(k_colsum2, dim3(nblk(ncol)), dim3(256), 0, N->stream, N->csum, R, ncol, cinp,
                     cin, out);
  NCHK(N, hipGetLastError());
  return FH_OK;
}

// weight and bias gradient of layer l from its input x (channels last,
// cinp channels) and the output gradient dz (cout channels)
int wgrad(fh_net* N, int l, const uint16_t* x, const uint16_t* dz, int B) {
  const int ci = cinp(l), cin = kL[l].cin, co = kL[l].cout, s = N->s[kL[l].level];
  const long long V = N->V[kL[l].level];
  TScope ts(N, FH_NET_K_WGRAD);
  N->flops[FH_NET_K_WGRAD] += 2.0 * B * V * 27.0 * cin * co;
  hipLaunchKernelGGL(k_prep_shifted, dim3(nblk((long long)B * (ci / 8) * V)), dim3(256), 0,
                     N->stream, x, ci, s, B, 1, N->xs);
  NCHK(N, hipGetLastError());
  hipLaunchKernelGGL(k_prep_shifted, dim3(nblk((long long)B * (co / 8) * V)), dim3(256), 0,
                     N->stream, dz, co, s, B, 1, N->dzt);
  NCHK(N, hipGetLastError());
  const int ntiles = (co / 16) * (ci / 16);
  const long long ksteps = (long long)B * V / 32;
  long long nsplit = std::max<long long>(1, (4096 + ntiles - 1) / ntiles);
  nsplit = std::min(nsplit, std::max<long long>(1, ksteps / 16));
  nsplit = std::min<long long>(nsplit, 1024);
  nsplit = std::min<long long>(nsplit, (long long)(N->wpart_n / (27LL * co * ci)));
  nsplit = std::min<long long>(nsplit, (long long)(N->bpart_n / co));
  WgradArgs a{N->xs, N->dzt, N->wpart, N->bpart, B, s, ci, co, (int)nsplit, ntiles, ksteps};
  if (s >= 32)
    hipLaunchKernelGGL(k_wgrad_roll, dim3(nblk((long long)ntiles * nsplit, 4)), dim3(256), 0,
                       N->stream, a);
  else
    hipLaunchKernelGGL(k_wgrad, dim3(nblk((long long)ntiles * nsplit, 4)), dim3(256), 0,
                       N->stream, a);
  NCHK(N, hipGetLastError());
  int rc = colsum(N, N->wpart, nsplit, 27LL * co * ci, ci, cin, N->gr + N->offw[l]);
  if (!rc) rc = colsum(N, N->bpart, nsplit, co, co, co, N->gr + N->offb[l]);
  return rc;
}

int pack_all(fh_net* N) {
  for (int l = 0; l < kLayers; ++l) {
    const int ci = cinp(l), co = kL[l].cout;
    const long long nf = (long long)(ci / 16) * 14 * co * 32;
    const long long nd = N->wd[l] ? (long long)(co / 16) * 14 * ci * 32 : 0;
    hipLaunchKernelGGL(k_pack, dim3(nblk(nf + nd + co)), dim3(256), 0, N->stream,
                       N->p + N->offw[l], N->p + N->offb[l], kL[l].cin, ci, co, N->wf[l],
                       N->wd[l], N->bias[l]);
    NCHK(N, hipGetLastError());
  }
  hipLaunchKernelGGL(k_round, dim3(nblk(kOut * kHeadIn)), dim3(256), 0, N->stream,
                     N->p + N->offw[kLayers], N->wh, kOut * kHeadIn);
  hipLaunchKernelGGL(k_round, dim3(1), dim3(64), 0, N->stream, N->p + N->offb[kLayers], N->bh,
                     kOut);
  NCHK(N, hipGetLastError());
  N->packed = true;
  return FH_OK;
}

double conv_flops(const fh_net* N, int l, int B) {
  return 2.0 * B * N->V[kL[l].level] * 27.0 * kL[l].cin * kL[l].cout;
}

// forward pass for B samples: phase + order (null = identity), gamma on device
int forward(fh_net* N, int B, const uint8_t* phase, const int* order, const float* gamma) {
  if (!N->packed) {
    int rc = pack_all(N);
    if (rc) return rc;
  }
  const int s0 = N->s[0], s1 = N->s[1], s2 = N->s[2], s3 = N->s[3];
  {
    TScope ts(N, FH_NET_K_OTHER);
    hipLaunchKernelGGL(k_features, dim3(nblk((long long)B * N->V[0])), dim3(256), 0, N->stream,
                       phase, order, gamma, B, N->V[0], N->I);
    NCHK(N, hipGetLastError());
  }
  int rc;
  auto F = [&](int l, const uint16_t* x, uint16_t* y) {
    return conv(N, x, cinp(l), N->wf[l], N->bias[l], nullptr, y, kL[l].cout, N->s[kL[l].level],
                B, true, FH_NET_K_CONV, conv_flops(N, l, B));
  };
  auto pool = [&](const uint16_t* x, int C, int s, uint16_t* y) {
    TScope ts(N, FH_NET_K_OTHER);
    hipLaunchKernelGGL(k_pool, dim3(nblk((long long)B * (s / 2) * (s / 2) * (s / 2) * C)),
                       dim3(256), 0, N->stream, x, C, s, B, y);
    return hipGetLastError() == hipSuccess ? FH_OK : nfail(N, FH_EDEVICE, "pool launch");
  };
  auto cat = [&](const uint16_t* coarse, int Cu, const uint16_t* skip, int Cs, int s,
                 uint16_t* y) {
    TScope ts(N, FH_NET_K_OTHER);
    hipLaunchKernelGGL(k_concat, dim3(nblk((long long)B * s * s * s * ((Cu + Cs) / 8))),
                       dim3(256), 0, N->stream, coarse, Cu, skip, Cs, s, B, y);
    return hipGetLastError() == hipSuccess ? FH_OK : nfail(N, FH_EDEVICE, "concat launch");
  };
  if ((rc = F(0, N->I, N->e0a)) || (rc = F(1, N->e0a, N->e0)) || (rc = pool(N->e0, 16, s0, N->p0)) ||
      (rc = F(2, N->p0, N->e1a)) || (rc = F(3, N->e1a, N->e1)) || (rc = pool(N->e1, 32, s1, N->p1)) ||
      (rc = F(4, N->p1, N->e2a)) || (rc = F(5, N->e2a, N->e2)) || (rc = pool(N->e2, 64, s2, N->p2)) ||
      (rc = F(6, N->p2, N->b3a)) || (rc = F(7, N->b3a, N->b3)) ||
      (rc = cat(N->b3, 64, N->e2, 64, s2, N->c2)) || (rc = F(8, N->c2, N->d2a)) ||
      (rc = F(9, N->d2a, N->d2)) || (rc = cat(N->d2, 64, N->e1, 32, s1, N->c1)) ||
      (rc = F(10, N->c1, N->d1a)) || (rc = F(11, N->d1a, N->d1)) ||
      (rc = cat(N->d1, 32, N->e0, 16, s0, N->c0)) || (rc = F(12, N->c0, N->d0a)) ||
      (rc = F(13, N->d0a, N->d0)))
    return rc;
  (void)s3;
  TScope ts(N, FH_NET_K_OTHER);
  hipLaunchKernelGGL(k_head, dim3(nblk((long long)B * N->V[0])), dim3(256), 0, N->stream, N->d0,
                     N->wh, N->bh, N->V[0], B, N->O);
  NCHK(N, hipGetLastError());
  return FH_OK;
}

// loss and gradient for B samples (after forward); targets gathered by order
int backward(fh_net* N, int B, const uint16_t* target, const int* order, double* loss_dev) {
  const int s0 = N->s[0], s1 = N->s[1], s2 = N->s[2];
  const long long V0 = N->V[0];
  {
    TScope ts(N, FH_NET_K_OTHER);
    const long long tot = (long long)B * kOut * V0;
    hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, N->stream, N->O, target, order,
                       s0, B, 1.0 / (3.0 * (double)tot), N->dO, N->lpart);
    hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, N->stream, N->lpart, kLossBlocks,
                       loss_dev);
    // head
    const unsigned nhb = (unsigned)(B * (V0 / kHeadChunk));
    hipLaunchKernelGGL(k_head_wgrad, dim3(nhb), dim3(320), 0, N->stream, N->dO, N->d0, V0,
                       N->hpart);
    NCHK(N, hipGetLastError());
    int rc0 = colsum(N, N->hpart, nhb, kHeadNP, kHeadNP, kHeadNP, N->gr + N->offw[kLayers]);
    if (rc0) return rc0;
    hipLaunchKernelGGL(k_head_bwd, dim3(nblk((long long)B * V0)), dim3(256), 0, N->stream, N->dO,
                       N->d0, N->wh, V0, B, N->ta);
    NCHK(N, hipGetLastError());
  }
  int rc;
  // input gradient of layer l: dz (cout ch) -> y (cinp ch), masked by the
  // layer input when that input is an activation output
  auto D = [&](int l, const uint16_t* dz, const uint16_t* mask, uint16_t* y) {
    return conv(N, dz, kL[l].cout, N->wd[l], nullptr, mask, y, cinp(l), N->s[kL[l].level], B,
                false, FH_NET_K_DGRAD, conv_flops(N, l, B));
  };
  auto W = [&](int l, const uint16_t* x, const uint16_t* dz) { return wgrad(N, l, x, dz, B); };
  auto upsum = [&](const uint16_t* dc, int Ct, int Cu, int s, uint16_t* y) {
    TScope ts(N, FH_NET_K_OTHER);
    hipLaunchKernelGGL(k_upsum, dim3(nblk((long long)B * (s / 2) * (s / 2) * (s / 2) * Cu)),
                       dim3(256), 0, N->stream, dc, Ct, Cu, s, B, y);
    return hipGetLastError() == hipSuccess ? FH_OK : nfail(N, FH_EDEVICE, "upsum launch");
  };
  auto combine = [&](const uint16_t* dc, int Ct, int Cu, const uint16_t* E, const uint16_t* dP,
                     int C, int s, uint16_t* y) {
    TScope ts(N, FH_NET_K_OTHER);
    hipLaunchKernelGGL(k_combine, dim3(nblk((long long)B * s * s * s * C)), dim3(256), 0,
                       N->stream, dc, Ct, Cu, E, dP, C, s, B, y);
    return hipGetLastError() == hipSuccess ? FH_OK : nfail(N, FH_EDEVICE, "combine launch");
  };
  uint16_t *ta = N->ta, *tb = N->tb;
  if ((rc = W(13, N->d0a, ta)) || (rc = D(13, ta, N->d0a, tb)) ||
      (rc = W(12, N->c0, tb)) || (rc = D(12, tb, N->c0, N->dc0)) ||
      (rc = upsum(N->dc0, 48, 32, s0, ta)) ||
      (rc = W(11, N->d1a, ta)) || (rc = D(11, ta, N->d1a, tb)) ||
      (rc = W(10, N->c1, tb)) || (rc = D(10, tb, N->c1, N->dc1)) ||
      (rc = upsum(N->dc1, 96, 64, s1, ta)) ||
      (rc = W(9, N->d2a, ta)) || (rc = D(9, ta, N->d2a, tb)) ||
      (rc = W(8, N->c2, tb)) || (rc = D(8, tb, N->c2, N->dc2)) ||
      (rc = upsum(N->dc2, 128, 64, s2, ta)) ||
      (rc = W(7, N->b3a, ta)) || (rc = D(7, ta, N->b3a, tb)) ||
      (rc = W(6, N->p2, tb)) || (rc = D(6, tb, nullptr, ta)) ||
      (rc = combine(N->dc2, 128, 64, N->e2, ta, 64, s2, tb)) ||
      (rc = W(5, N->e2a, tb)) || (rc = D(5, tb, N->e2a, ta)) ||
      (rc = W(4, N->p1, ta)) || (rc = D(4, ta, nullptr, tb)) ||
      (rc = combine(N->dc1, 96, 64, N->e1, tb, 32, s1, ta)) ||
      (rc = W(3, N->e1a, ta)) || (rc = D(3, ta, N->e1a, tb)) ||
      (rc = W(2, N->p0, tb)) || (rc = D(2, tb, nullptr, ta)) ||
      (rc = combine(N->dc0, 48, 32, N->e0, ta, 16, s0, tb)) ||
      (rc = W(1, N->e0a, tb)) || (rc = D(1, tb, N->e0a, ta)) ||
      (rc = W(0, N->I, ta)))
    return rc;
  return FH_OK;
}

int adam_step(fh_net* N, const fh_adam& o) {
  N->adam_t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(o.beta1, (double)N->adam_t));
  const double c2 = 1.0 / (1.0 - std::pow(o.beta2, (double)N->adam_t));
  TScope ts(N, FH_NET_K_OTHER);
  const float* factor = nullptr;
  if (o.clip > 0.0) {
    const int nb = 256;
    hipLaunchKernelGGL(k_sqnorm_part, dim3(nb), dim3(256), 0, N->stream, N->gr, N->P,
                       N->lpart);
    hipLaunchKernelGGL(k_clip_factor, dim3(1), dim3(64), 0, N->stream, N->lpart, nb, o.clip,
                       N->clipf);
    factor = N->clipf;
  }
  hipLaunchKernelGGL(k_adam, dim3(nblk(N->P)), dim3(256), 0, N->stream, N->p, N->gr, N->m, N->v,
                     N->P, (float)o.lr, (float)o.beta1, (float)o.beta2, (float)(1.0 - o.beta1),
                     (float)(1.0 - o.beta2), (float)o.eps, (float)c1, (float)c2, factor);
  NCHK(N, hipGetLastError());
  N->packed = false;
  return pack_all(N);
}

int upload_gamma(fh_net* N, const float* gamma_host, int B) {
  NCHK(N, hipMemcpyAsync(N->gamma_dev, gamma_host, sizeof(float) * B, hipMemcpyHostToDevice,
                         N->stream));
  return FH_OK;
}

int check_batch(fh_net* N, int B) {
  if (B < 1 || B > N->maxb) return nfail(N, FH_EINVAL, "batch outside 1..max_batch");
  return FH_OK;
}

}  // namespace

// ================================================================ C-ABI
extern "C" {

long long fh_net_param_count(void) {
  long long n = 0;
  for (int l = 0; l < kLayers; ++l) n += 27LL * kL[l].cin * kL[l].cout + kL[l].cout;
  return n + kOut * kHeadIn + kOut;
}

int fh_net_create(fh_net** out, int device, int n, int max_batch) {
  if (!out) return FH_EINVAL;
  *out = nullptr;
  if (n < 64 || n > 256 || n % 64 || max_batch < 1 || max_batch > 64) return FH_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return FH_EDEVICE;
  fh_net* N = new fh_net();
  N->device = device;
  N->n = n;
  N->maxb = max_batch;
  for (int k = 0; k < 4; ++k) {
    N->s[k] = n >> k;
    N->V[k] = (long long)N->s[k] * N->s[k] * N->s[k];
  }
  long long off = 0;
  for (int l = 0; l < kLayers; ++l) {
    N->offw[l] = off;
    off += 27LL * kL[l].cin * kL[l].cout;
    N->offb[l] = off;
    off += kL[l].cout;
  }
  N->offw[kLayers] = off;
  off += kOut * kHeadIn;
  N->offb[kLayers] = off;
  off += kOut;
  N->P = off;
  // one allocation, carved into 256-byte aligned pieces
  const long long B = max_batch;
  std::vector<std::pair<void**, size_t>> parts;
  auto add = [&](void** p, size_t bytes) { parts.push_back({p, bytes}); };
  for (float** f : {&N->p, &N->gr, &N->m, &N->v}) add((void**)f, sizeof(float) * N->P);
  for (int l = 0; l < kLayers; ++l) {
    const int ci = cinp(l), co = kL[l].cout;
    add((void**)&N->wf[l], 2ULL * (ci / 16) * 14 * co * 32);
    N->wd[l] = nullptr;
    if (l > 0) add((void**)&N->wd[l], 2ULL * (co / 16) * 14 * ci * 32);
    add((void**)&N->bias[l], sizeof(float) * co);
  }
  add((void**)&N->wh, sizeof(float) * kOut * kHeadIn);
  add((void**)&N->bh, sizeof(float) * kOut);
  const long long *V = N->V;
  auto act = [&](uint16_t** p, int C, int lev) { add((void**)p, 2ULL * B * V[lev] * C); };
  act(&N->I, 16, 0); act(&N->e0a, 16, 0); act(&N->e0, 16, 0); act(&N->p0, 16, 1);
  act(&N->e1a, 32, 1); act(&N->e1, 32, 1); act(&N->p1, 32, 2);
  act(&N->e2a, 64, 2); act(&N->e2, 64, 2); act(&N->p2, 64, 3);
  act(&N->b3a, 64, 3); act(&N->b3, 64, 3); act(&N->c2, 128, 2);
  act(&N->d2a, 64, 2); act(&N->d2, 64, 2); act(&N->c1, 96, 1);
  act(&N->d1a, 32, 1); act(&N->d1, 32, 1); act(&N->c0, 48, 0);
  act(&N->d0a, 16, 0); act(&N->d0, 16, 0);
  add((void**)&N->O, sizeof(float) * B * kOut * V[0]);
  add((void**)&N->dO, sizeof(float) * B * kOut * V[0]);
  act(&N->dc0, 48, 0); act(&N->dc1, 96, 1); act(&N->dc2, 128, 2);
  act(&N->ta, 16, 0); act(&N->tb, 16, 0);
  add((void**)&N->xs, 2ULL * 3 * B * V[0] * 48);
  act(&N->dzt, 16, 0);
  N->wpart_n = 16ULL << 20;  // floats
  N->bpart_n = 1ULL << 16;
  add((void**)&N->wpart, sizeof(float) * N->wpart_n);
  add((void**)&N->bpart, sizeof(float) * N->bpart_n);
  add((void**)&N->hpart, sizeof(float) * (size_t)(B * (V[0] / kHeadChunk)) * kHeadNP);
  add((void**)&N->lpart, sizeof(double) * kLossBlocks);
  N->csum_n = 4ULL << 20;  // doubles
  add((void**)&N->csum, sizeof(double) * N->csum_n);
  add((void**)&N->scal, sizeof(double) * 8);
  add((void**)&N->chpart, sizeof(double) * kOut * 256);
  add((void**)&N->chmean, sizeof(double) * kOut);
  add((void**)&N->Edev, sizeof(double) * 6 * FH_MAX_LOADS);
  add((void**)&N->gamma_dev, sizeof(float) * 64);
  add((void**)&N->clipf, sizeof(float) * 4);
  size_t total = 0;
  for (auto& pr : parts) total += (pr.second + 255) & ~(size_t)255;
  if (hipMalloc((void**)&N->mem, total) != hipSuccess) {
    delete N;
    return FH_ENOMEM;
  }
  size_t pos = 0;
  for (auto& pr : parts) {
    *pr.first = N->mem + pos;
    pos += (pr.second + 255) & ~(size_t)255;
  }
  hipMemset(N->m, 0, sizeof(float) * N->P);
  hipMemset(N->v, 0, sizeof(float) * N->P);
  hipMemset(N->p, 0, sizeof(float) * N->P);
  hipDeviceSynchronize();
  *out = N;
  return FH_OK;
}

void fh_net_destroy(fh_net* N) {
  if (!N) return;
  hipSetDevice(N->device);
  if (N->stream) hipStreamSynchronize(N->stream);
  else hipDeviceSynchronize();
  for (hipEvent_t e : N->ev) hipEventDestroy(e);
  if (N->order_dev) hipFree(N->order_dev);
  hipFree(N->mem);
  delete N;
}

const char* fh_net_last_error(const fh_net* N) { return N ? N->err.c_str() : "null network"; }

int fh_net_set_stream(fh_net* N, void* stream) {
  if (!N) return FH_EINVAL;
  N->stream = (hipStream_t)stream;
  return FH_OK;
}

int fh_net_set_params(fh_net* N, const float* params) {
  if (!N || !params) return FH_EINVAL;
  hipSetDevice(N->device);
  NCHK(N, hipMemcpyAsync(N->p, params, sizeof(float) * N->P, hipMemcpyHostToDevice, N->stream));
  NCHK(N, hipMemsetAsync(N->m, 0, sizeof(float) * N->P, N->stream));
  NCHK(N, hipMemsetAsync(N->v, 0, sizeof(float) * N->P, N->stream));
  N->adam_t = 0;
  int rc = pack_all(N);
  if (rc) return rc;
  NCHK(N, hipStreamSynchronize(N->stream));
  return FH_OK;
}

int fh_net_get_params(fh_net* N, float* params) {
  if (!N || !params) return FH_EINVAL;
  hipSetDevice(N->device);
  NCHK(N, hipMemcpyAsync(params, N->p, sizeof(float) * N->P, hipMemcpyDeviceToHost, N->stream));
  NCHK(N, hipStreamSynchronize(N->stream));
  return FH_OK;
}

int fh_net_forward(fh_net* N, int batch, const uint8_t* phase_dev, const float* gamma,
                   float* out_dev) {
  if (!N || !phase_dev || !gamma || !out_dev) return FH_EINVAL;
  hipSetDevice(N->device);
  int rc = check_batch(N, batch);
  if (rc || (rc = upload_gamma(N, gamma, batch))) return rc;
  if ((rc = forward(N, batch, phase_dev, nullptr, N->gamma_dev))) return rc;
  NCHK(N, hipMemcpyAsync(out_dev, N->O, sizeof(float) * batch * kOut * N->V[0],
                         hipMemcpyDeviceToDevice, N->stream));
  NCHK(N, hipStreamSynchronize(N->stream));
  tcollect(N);
  return FH_OK;
}

int fh_net_gradient(fh_net* N, int batch, const uint8_t* phase_dev, const float* gamma,
                    const uint16_t* target_dev, double* loss, float* grad) {
  if (!N || !phase_dev || !gamma || !target_dev) return FH_EINVAL;
  hipSetDevice(N->device);
  int rc = check_batch(N, batch);
  if (rc || (rc = upload_gamma(N, gamma, batch))) return rc;
  if ((rc = forward(N, batch, phase_dev, nullptr, N->gamma_dev))) return rc;
  if ((rc = backward(N, batch, target_dev, nullptr, N->scal))) return rc;
  if (loss)
    NCHK(N, hipMemcpyAsync(loss, N->scal, sizeof(double), hipMemcpyDeviceToHost, N->stream));
  if (grad)
    NCHK(N, hipMemcpyAsync(grad, N->gr, sizeof(float) * N->P, hipMemcpyDeviceToHost, N->stream));
  NCHK(N, hipStreamSynchronize(N->stream));
  tcollect(N);
  return FH_OK;
}

int fh_net_adam(fh_net* N, const float* grad, const fh_adam* opt) {
  if (!N || !opt) return FH_EINVAL;
  hipSetDevice(N->device);
  if (grad)
    NCHK(N, hipMemcpyAsync(N->gr, grad, sizeof(float) * N->P, hipMemcpyHostToDevice, N->stream));
  int rc = adam_step(N, *opt);
  if (rc) return rc;
  NCHK(N, hipStreamSynchronize(N->stream));
  tcollect(N);
  return FH_OK;
}

int fh_net_train(fh_net* N, int nsamples, const uint8_t* phase_dev, const float* gamma,
                 const uint16_t* target_dev, int batch, int steps, const int* order,
                 const fh_adam* opt, double* loss) {
  if (!N || nsamples < 1 || !phase_dev || !gamma || !target_dev || steps < 0 || !order || !opt)
    return FH_EINVAL;
  hipSetDevice(N->device);
  int rc = check_batch(N, batch);
  if (rc) return rc;
  const long long norder = (long long)steps * batch;
  for (long long k = 0; k < norder; ++k)
    if (order[k] < 0 || order[k] >= nsamples) return nfail(N, FH_EINVAL, "order index out of range");
  if (norder > N->order_n) {
    if (N->order_dev) hipFree(N->order_dev);
    N->order_dev = nullptr;
    N->order_n = 0;
    NCHK(N, hipMalloc((void**)&N->order_dev, sizeof(int) * norder));
    N->order_n = norder;
  }
  float* gdev = nullptr;
  NCHK(N, hipMalloc((void**)&gdev, sizeof(float) * norder + sizeof(double) * (steps + 1)));
  double* ldev = reinterpret_cast<double*>(
      reinterpret_cast<char*>(gdev) + ((sizeof(float) * norder + 7) & ~(size_t)7));
  std::vector<float> gs(norder);
  for (long long k = 0; k < norder; ++k) gs[k] = gamma[order[k]];
  hipError_t e1 = hipMemcpyAsync(N->order_dev, order, sizeof(int) * norder, hipMemcpyHostToDevice,
                                 N->stream);
  hipError_t e2 = hipMemcpyAsync(gdev, gs.data(), sizeof(float) * norder, hipMemcpyHostToDevice,
                                 N->stream);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    hipFree(gdev);
    return nfail(N, FH_EDEVICE, "upload of the sample order failed");
  }
  for (int st = 0; st < steps && rc == FH_OK; ++st) {
    const int* ord = N->order_dev + (long long)st * batch;
    rc = forward(N, batch, phase_dev, ord, gdev + (long long)st * batch);
    if (!rc) rc = backward(N, batch, target_dev, ord, ldev + st);
    if (!rc) rc = adam_step(N, *opt);
    tmaybe_flush(N);
  }
  hipError_t es = hipStreamSynchronize(N->stream);
  if (!rc && es == hipSuccess && loss && steps > 0)
    es = hipMemcpy(loss, ldev, sizeof(double) * steps, hipMemcpyDeviceToHost);
  hipFree(gdev);
  if (rc) return rc;
  if (es != hipSuccess) return nfail(N, FH_EDEVICE, hipGetErrorString(es));
  tcollect(N);
  return FH_OK;
}

int fh_net_pack_target(fh_net* N, const double* u_dev, double scale, uint16_t* target_dev) {
  if (!N || !u_dev || !target_dev) return FH_EINVAL;
  hipSetDevice(N->device);
  const long long n = (long long)kOut * N->V[0];
  hipLaunchKernelGGL(k_pack_target, dim3(nblk(n)), dim3(256), 0, N->stream, u_dev, n, scale,
                     target_dev);
  NCHK(N, hipGetLastError());
  NCHK(N, hipStreamSynchronize(N->stream));
  return FH_OK;
}

int fh_net_layer(fh_net* N, int layer, int op, int batch, const uint16_t* x_dev,
                 const uint16_t* dz_dev, const uint16_t* mask_dev, void* out_dev) {
  if (!N || !out_dev) return FH_EINVAL;
  hipSetDevice(N->device);
  if (layer < 0 || layer >= kLayers) return nfail(N, FH_EINVAL, "layer index out of range");
  int rc = check_batch(N, batch);
  if (rc) return rc;
  if (!N->packed && (rc = pack_all(N))) return rc;
  const int l = layer, s = N->s[kL[l].level];
  if (op == FH_NET_OP_FORWARD) {
    if (!x_dev) return nfail(N, FH_EINVAL, "forward needs x");
    rc = conv(N, x_dev, cinp(l), N->wf[l], N->bias[l], nullptr, (uint16_t*)out_dev, kL[l].cout,
              s, batch, true, FH_NET_K_CONV, conv_flops(N, l, batch));
  } else if (op == FH_NET_OP_DGRAD) {
    if (!dz_dev) return nfail(N, FH_EINVAL, "input gradient needs dz");
    if (!N->wd[l]) return nfail(N, FH_EINVAL, "the first layer has no input gradient");
    rc = conv(N, dz_dev, kL[l].cout, N->wd[l], nullptr, mask_dev, (uint16_t*)out_dev, cinp(l), s,
              batch, false, FH_NET_K_DGRAD, conv_flops(N, l, batch));
  } else if (op == FH_NET_OP_WGRAD) {
    if (!x_dev || !dz_dev) return nfail(N, FH_EINVAL, "weight gradient needs x and dz");
    rc = wgrad(N, l, x_dev, dz_dev, batch);
    if (!rc) {
      const long long nw = 27LL * kL[l].cin * kL[l].cout;
      float* o = (float*)out_dev;
      NCHK(N, hipMemcpyAsync(o, N->gr + N->offw[l], nw * sizeof(float), hipMemcpyDeviceToDevice,
                             N->stream));
      NCHK(N, hipMemcpyAsync(o + nw, N->gr + N->offb[l], kL[l].cout * sizeof(float),
                             hipMemcpyDeviceToDevice, N->stream));
    }
  } else {
    return nfail(N, FH_EINVAL, "unknown layer operation");
  }
  if (rc) return rc;
  NCHK(N, hipStreamSynchronize(N->stream));
  return FH_OK;
}

int fh_net_set_timing(fh_net* N, int on) {
  if (!N) return FH_EINVAL;
  N->time_on = on != 0;
  for (int k = 0; k < FH_NET_K_NCLASS; ++k) {
    N->ms[k] = 0.0;
    N->launches[k] = 0;
    N->flops[k] = 0.0;
  }
  N->ev_used = 0;
  return FH_OK;
}

int fh_net_get_stats(fh_net* N, fh_net_stats* st) {
  if (!N || !st) return FH_EINVAL;
  tcollect(N);
  for (int k = 0; k < FH_NET_K_NCLASS; ++k) {
    st->kernel_ms[k] = N->ms[k];
    st->kernel_launches[k] = N->launches[k];
    st->flops[k] = N->flops[k];
  }
  st->adam_steps = N->adam_t;
  return FH_OK;
}

}  // extern "C"

// ----------------------------------------------- warm start for the solver
namespace fh {

// Initial fluctuation of the nload loads E (host, Mandel 6-vectors) for one
// microstructure: x[l] = scale sum_j E[l][j] (O_j - mean O_j), O = network
// output of the phase field with material descriptor gamma.
int net_warm_guess(fh_net* N, hipStream_t stream, const uint8_t* phase_dev, float gamma,
                   int nload, const double* E, double scale, double* x, long long F,
                   std::string* err) {
  if (nload < 1 || nload > FH_MAX_LOADS) {
    *err = "warm start: bad load count";
    return FH_EINVAL;
  }
  hipStream_t saved = N->stream;
  N->stream = stream;
  struct Restore {
    fh_net* N;
    hipStream_t s;
    ~Restore() { N->stream = s; }
  } restore{N, saved};
  int rc = upload_gamma(N, &gamma, 1);
  if (!rc) rc = forward(N, 1, phase_dev, nullptr, N->gamma_dev);
  if (rc) {
    *err = N->err;
    return rc;
  }
  const long long V = N->V[0];
  const int nb = 64;
  hipLaunchKernelGGL(k_chan_part, dim3(nb, kOut), dim3(256), 0, stream, N->O, V, nb, N->chpart);
  hipLaunchKernelGGL(k_chan_mean, dim3(1), dim3(64), 0, stream, N->chpart, nb, V, N->chmean);
  hipError_t e = hipMemcpyAsync(N->Edev, E, sizeof(double) * 6 * nload, hipMemcpyHostToDevice,
                                stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_warm_x, dim3(nblk(3 * V)), dim3(256), 0, stream, N->O, N->chmean,
                       N->Edev, nload, V, scale, F, x);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // E is a pageable host copy
  if (e != hipSuccess) {
    *err = std::string("warm start: ") + hipGetErrorString(e);
    return FH_EDEVICE;
  }
  tcollect(N);
  return FH_OK;
}

int net_grid(const fh_net* N) { return N->n; }

}  // namespace fh

extern "C" int fh_net_guess(fh_net* N, const uint8_t* phase_dev, float gamma, int nload,
                            const double* E, double length, double* x_dev) {
  if (!N || !phase_dev || !E || !x_dev || !(length > 0.0)) return FH_EINVAL;
  hipSetDevice(N->device);
  std::string err;
  const int rc = fh::net_warm_guess(N, N->stream, phase_dev, gamma, nload, E, length / N->n,
                                    x_dev, 3 * N->V[0], &err);
  if (rc) return nfail(N, rc, err);
  return FH_OK;
}
