// Matrix-free stiffness operator q = K u = D^T W C D u and the right-hand
// side b = -D^T W C e.
//
// Paper Sec. 3 (eqs. Du_mat, grad_componets, W_mat, lin_system) and Sec. 5.1:
// the gradient D is applied as a short stencil per pixel/voxel and the
// quadrature weights are fused into the transpose ("weighted divergence").
//
// Elastic hex8 kernel (3D trilinear hexahedra, 2x2x2 Gauss points,
// element-wise constant Mandel stiffness):
//   Per voxel the 8 corner values of each displacement component are mapped
//   to tensor-product modes (per axis: mean and difference).  In that basis
//   the gradient at the Gauss points is a sum over products of (xi - 1/2)
//   factors, and the 2-point Gauss rule is orthogonal on {1, xi - 1/2} with
//   weights 1 and 1/12.  The element energy therefore splits into seven
//   independent terms (mode sets M of size 0, 1, 2), each a 6 x 6 Mandel
//   contraction on at most six strain coefficients.  This is exactly the
//   2x2x2 quadrature of D^T W C D (no approximation) with about a third of
//   the arithmetic of the per-point form.
//   Work split: a block owns a TX x TY tile of output nodes and a chunk of z
//   planes, computes the (TX+1) x (TY+1) voxels that touch the tile, marches
//   in z keeping two node planes in LDS, carries the upper-face forces of the
//   previous voxel slab in registers, and sums the four in-plane voxel
//   contributions of every node through LDS in a fixed order (deterministic).
//   The energy u.Ku = sum_e u_e.K_e u_e is accumulated per owned voxel, which
//   gives the PCG inner product p.q without a second pass.
#include "fh_internal.h"

namespace fh {

__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ double block_sum_k(double v, double* sh) {
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

// One term of the modal energy for mode set M (bit 1 = x, 2 = y, 4 = z).
// w[c][m]: mode m of displacement component c; fh: modal forces.
template <typename T, int M>
__device__ __forceinline__ void modal_term(const T (&w)[3][8], T (&fh)[3][8], const T* __restrict__ C,
                                           const T ihx, const T ihy, const T ihz, double& energy) {
  constexpr bool X = !(M & 1), Y = !(M & 2), Z = !(M & 4);
  constexpr int nbits = ((M & 1) ? 1 : 0) + ((M & 2) ? 1 : 0) + ((M & 4) ? 1 : 0);
  const T cM = nbits == 0 ? T(1) : (nbits == 1 ? T(1.0 / 12.0) : T(1.0 / 144.0));
  const T s = T(0.70710678118654752440084436210485);
  constexpr bool nz[6] = {X, Y, Z, Y || Z, X || Z, X || Y};
  T E[6];
  E[0] = X ? w[0][M | 1] * ihx : T(0);
  E[1] = Y ? w[1][M | 2] * ihy : T(0);
  E[2] = Z ? w[2][M | 4] * ihz : T(0);
  E[3] = s * ((Z ? w[1][M | 4] * ihz : T(0)) + (Y ? w[2][M | 2] * ihy : T(0)));
  E[4] = s * ((Z ? w[0][M | 4] * ihz : T(0)) + (X ? w[2][M | 1] * ihx : T(0)));
  E[5] = s * ((Y ? w[0][M | 2] * ihy : T(0)) + (X ? w[1][M | 1] * ihx : T(0)));
  T S[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T acc = T(0);
    if (nz[i]) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (nz[k]) acc += C[i * 6 + k] * E[k];
    }
    S[i] = cM * acc;
  }
  double e = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
    if (nz[i]) e += (double)E[i] * (double)S[i];
  energy += e;
  if (X) fh[0][M | 1] += S[0] * ihx;
  if (Y) fh[1][M | 2] += S[1] * ihy;
  if (Z) fh[2][M | 4] += S[2] * ihz;
  if (Z) fh[1][M | 4] += s * S[3] * ihz;
  if (Y) fh[2][M | 2] += s * S[3] * ihy;
  if (Z) fh[0][M | 4] += s * S[4] * ihz;
  if (X) fh[2][M | 1] += s * S[4] * ihx;
  if (Y) fh[0][M | 2] += s * S[5] * ihy;
  if (X) fh[1][M | 1] += s * S[5] * ihx;
}

template <typename T, int TX, int TY>
struct HexCfg {
  static constexpr int EX = TX + 1, EY = TY + 1, PX = TX + 2, PY = TY + 2;
  static constexpr int NE = EX * EY, NP = PX * PY;
  // element slots laid out with the node-plane pitch PX (one unused slot per
  // row), so that the lanes of a wave touch consecutive LDS words
  static constexpr int NEL = (EY - 1) * PX + EX;
  static constexpr int NT = ((NEL + 63) / 64) * 64;
};

template <typename T, int TX, int TY>
__global__ void __launch_bounds__((HexCfg<T, TX, TY>::NT))
    k_kop_hex8_elastic(Grid g, int kz, const T* __restrict__ u, T* __restrict__ q,
                       const uint8_t* __restrict__ phase, const T* __restrict__ mat,
                       long long ustride, long long qstride, const PcgState* st, double* pq_part) {
  using Cfg = HexCfg<T, TX, TY>;
  constexpr int EX = Cfg::EX, PX = Cfg::PX, NE = Cfg::NE, NP = Cfg::NP;
  __shared__ T plane[2][3][NP];
  __shared__ T force[12][NE];
  __shared__ double red[32];
  const int ld = blockIdx.z;
  if (st && st[ld].status != ST_ACTIVE) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  const int ntx = (nx + TX - 1) / TX;
  const int x0 = (blockIdx.x % ntx) * TX, y0 = (blockIdx.x / ntx) * TY;
  const int z0 = blockIdx.y * kz;
  const int z1 = min(z0 + kz, nz);
  const T* __restrict__ ub = u + (long long)ld * ustride;
  T* __restrict__ qb = q + (long long)ld * qstride;
  const int tid = threadIdx.x;
  const bool is_elem = tid < NE;
  const int ei = tid % EX, ej = tid / EX;
  const int ex = wrapi(x0 - 1 + ei, nx), ey = wrapi(y0 - 1 + ej, ny);
  const bool own_xy = is_elem && ei >= 1 && ej >= 1 && (x0 + ei - 1 < nx) && (y0 + ej - 1 < ny);
  const T ihx = T(1.0 / g.h[0]), ihy = T(1.0 / g.h[1]), ihz = T(1.0 / g.h[2]);

  auto load_plane = [&](int zp, int buf) {
    const long long zoff = (long long)wrapi(zp, nz) * ny;
    for (int idx = tid; idx < NP; idx += blockDim.x) {
      const int a = idx % PX, b = idx / PX;
      const int gx = wrapi(x0 - 1 + a, nx), gy = wrapi(y0 - 1 + b, ny);
      const long long o = (zoff + gy) * nx + gx;
      plane[buf][0][idx] = ub[o];
      plane[buf][1][idx] = ub[N + o];
      plane[buf][2][idx] = ub[2 * N + o];
    }
  };

  T carry[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) carry[k] = T(0);
  double energy = 0.0;
  load_plane(z0 - 1, 0);
  const int nsteps = z1 - z0 + 1;
  for (int s = 0; s < nsteps; ++s) {
    const int zs = z0 - 1 + s;
    const int lo = s & 1, hi = lo ^ 1;
    load_plane(zs + 1, hi);
    __syncthreads();
    if (is_elem) {
      T w[3][8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int idx = (ej + ((a >> 1) & 1)) * PX + (ei + (a & 1));
        const int buf = (a >> 2) ? hi : lo;
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c][a] = plane[buf][c][idx];
      }
      // forward modal transform along x, y, z: (u0, u1) -> ((u0+u1)/2, u1-u0)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            if (a & bit) continue;
            const T u0 = w[c][a], u1 = w[c][a | bit];
            w[c][a] = T(0.5) * (u0 + u1);
            w[c][a | bit] = u1 - u0;
          }
        }
      }
      const uint8_t ph = phase[((long long)wrapi(zs, nz) * ny + ey) * nx + ex];
      const T* __restrict__ C = mat + (int)ph * 36;
      T fh[3][8];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 8; ++a) fh[c][a] = T(0);
      double e = 0.0;
      modal_term<T, 0>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 1>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 2>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 4>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 3>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 5>(w, fh, C, ihx, ihy, ihz, e);
      modal_term<T, 6>(w, fh, C, ihx, ihy, ihz, e);
      // transpose transform: (fm, fd) -> (fm/2 - fd, fm/2 + fd)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            if (a & bit) continue;
            const T fm = fh[c][a], fd = fh[c][a | bit];
            fh[c][a] = T(0.5) * fm - fd;
            fh[c][a | bit] = T(0.5) * fm + fd;
          }
        }
      }
      if (s > 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) force[c * 4 + k][tid] = fh[c][k] + carry[c * 4 + k];
        if (own_xy) energy += e;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) carry[c * 4 + k] = fh[c][k + 4];
    }
    __syncthreads();
    if (s > 0 && tid < TX * TY) {
      const int ox = tid % TX, oy = tid / TX;
      const int x = x0 + ox, y = y0 + oy;
      if (x < nx && y < ny) {
        const int e00 = oy * EX + ox;
        const long long o = ((long long)zs * ny + y) * nx + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T v = force[c * 4 + 3][e00] + force[c * 4 + 2][e00 + 1] +
                      force[c * 4 + 1][e00 + EX] + force[c * 4 + 0][e00 + EX + 1];
          qb[c * N + o] = v;
        }
      }
    }
  }
  if (pq_part) {
    const double tot = block_sum_k(energy, red);
    if (tid == 0) {
      const long long nb = (long long)gridDim.x * gridDim.y;
      pq_part[(long long)ld * nb + (long long)blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
  }
}

// ------------------------------------------------ isotropic hex8 kernel
// Same operator for isotropic phases, C = lambda 1(x)1 + 2 mu I (Mandel).
// Both modal transforms are pure sum/difference butterflies: the factors
// 1/2 of the mean modes are folded into per-term constants a_beta(M) =
// 2^-(2-|M|) / h_beta, which scale the gradient coefficients on the way in
// and the modal forces on the way out.  The PCG product p.q is taken at the
// output nodes (p is still in the LDS plane), so no per-voxel energy is
// formed.  The next node plane is prefetched into registers while the
// current slab is computed; the modal forces of a slab's upper face stay in
// registers until the next slab adds its own, and (FP64, cubic voxels) so do
// the in-plane modes of its node values, which are the next slab's lower
// face.  Three node planes rotate in
// LDS and the lower-face forces are double-buffered, so a slab needs one
// barrier: every buffer a step overwrites was last read before the previous
// step's barrier.
template <typename T, int M>
__device__ __forceinline__ void iso_term(const T (&w)[3][8], T (&f)[3][8], const T lam,
                                         const T mu2, const T ax, const T ay, const T az) {
  constexpr bool X = !(M & 1), Y = !(M & 2), Z = !(M & 4);
  const T s = T(0.70710678118654752440084436210485);
  const T sax = s * ax, say = s * ay, saz = s * az;
  // absent strain coefficients are -0, so sums with them fold away exactly
  const T z = T(-0.0);
  const T E0 = X ? w[0][M | 1] * ax : z;
  const T E1 = Y ? w[1][M | 2] * ay : z;
  const T E2 = Z ? w[2][M | 4] * az : z;
  const T E3 = (Z ? w[1][M | 4] * saz : z) + (Y ? w[2][M | 2] * say : z);
  const T E4 = (Z ? w[0][M | 4] * saz : z) + (X ? w[2][M | 1] * sax : z);
  const T E5 = (Y ? w[0][M | 2] * say : z) + (X ? w[1][M | 1] * sax : z);
  const T lt = lam * (E0 + E1 + E2);
  if (X) f[0][M | 1] += (lt + mu2 * E0) * ax;
  if (Y) f[1][M | 2] += (lt + mu2 * E1) * ay;
  if (Z) f[2][M | 4] += (lt + mu2 * E2) * az;
  const T S3 = mu2 * E3, S4 = mu2 * E4, S5 = mu2 * E5;
  if (Z) f[1][M | 4] += S3 * saz;
  if (Y) f[2][M | 2] += S3 * say;
  if (Z) f[0][M | 4] += S4 * saz;
  if (X) f[2][M | 1] += S4 * sax;
  if (Y) f[0][M | 2] += S5 * say;
  if (X) f[1][M | 1] += S5 * sax;
}

// The same term for cubic voxels (h_x = h_y = h_z).  With one a for every
// axis the two factors a of a term fold into its constants: l = V lambda c_M
// a^2, m = 2 V mu c_M a^2 and mh = m / 2 (the two 1/sqrt2 of a shear pair);
// lpm = l + m serves the terms with a single normal strain.  Each shear
// coefficient is then the plain sum of the cross derivatives present, and
// its stress goes back unscaled to both of them.
template <typename T, int M>
__device__ __forceinline__ void iso_term_cube(const T (&w)[3][8], T (&f)[3][8], const T l,
                                              const T m, const T mh, const T lpm) {
  constexpr bool X = !(M & 1), Y = !(M & 2), Z = !(M & 4);
  if constexpr (X + Y + Z == 1) {
    if constexpr (X) f[0][M | 1] += lpm * w[0][M | 1];
    if constexpr (Y) f[1][M | 2] += lpm * w[1][M | 2];
    if constexpr (Z) f[2][M | 4] += lpm * w[2][M | 4];
  } else {
    T sd;  // sum of the normal strain coefficients present
    if constexpr (X && Y && Z) sd = w[0][M | 1] + w[1][M | 2] + w[2][M | 4];
    else if constexpr (X && Y) sd = w[0][M | 1] + w[1][M | 2];
    else if constexpr (X && Z) sd = w[0][M | 1] + w[2][M | 4];
    else sd = w[1][M | 2] + w[2][M | 4];
    const T lt = l * sd;
    if constexpr (X) f[0][M | 1] += lt + m * w[0][M | 1];
    if constexpr (Y) f[1][M | 2] += lt + m * w[1][M | 2];
    if constexpr (Z) f[2][M | 4] += lt + m * w[2][M | 4];
  }
  if constexpr (Y && Z) {  // yz
    const T g = mh * (w[1][M | 4] + w[2][M | 2]);
    f[1][M | 4] += g;
    f[2][M | 2] += g;
  } else if constexpr (Z) {
    f[1][M | 4] += mh * w[1][M | 4];
  } else if constexpr (Y) {
    f[2][M | 2] += mh * w[2][M | 2];
  }
  if constexpr (X && Z) {  // xz
    const T g = mh * (w[0][M | 4] + w[2][M | 1]);
    f[0][M | 4] += g;
    f[2][M | 1] += g;
  } else if constexpr (Z) {
    f[0][M | 4] += mh * w[0][M | 4];
  } else if constexpr (X) {
    f[2][M | 1] += mh * w[2][M | 1];
  }
  if constexpr (X && Y) {  // xy
    const T g = mh * (w[0][M | 2] + w[1][M | 1]);
    f[0][M | 2] += g;
    f[1][M | 1] += g;
  } else if constexpr (Y) {
    f[0][M | 2] += mh * w[0][M | 2];
  } else if constexpr (X) {
    f[1][M | 1] += mh * w[1][M | 1];
  }
}

template <typename T, int TX, int TY, bool CUBE>
__global__ void __launch_bounds__((HexCfg<T, TX, TY>::NT), 3)
    k_kop_hex8_iso(Grid g, int kz, const T* __restrict__ u, T* __restrict__ q,
                   const uint8_t* __restrict__ phase, const T* __restrict__ lm,
                   long long ustride, long long qstride, const PcgState* st, double* pq_part) {
  using Cfg = HexCfg<T, TX, TY>;
  constexpr int EX = Cfg::EX, PX = Cfg::PX, NEL = Cfg::NEL, NP = Cfg::NP, NT = Cfg::NT;
  constexpr int NPF = (NP + NT - 1) / NT;  // plane nodes per thread
  // three rotating node planes: the next one is stored while the current
  // slab reads the other two, so one barrier per slab suffices
  __shared__ T plane[3][3][NP];
  __shared__ uint8_t phl[3][NP];  // voxel phases of the slab above each plane
  // lower-face corners 0..2 of the current slab, double-buffered across
  // slabs; corner 3 of a thread's element lands on its own output node and
  // stays in registers
  __shared__ T force[2][9][NEL];
  __shared__ double red[32];
  // per-phase {V lambda, 2 V mu}, sized by the launch (2 nphase_max)
  extern __shared__ __align__(16) unsigned char kop_dyn[];
  T* lmt = reinterpret_cast<T*>(kop_dyn);
  // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
  // that each XCD receives a contiguous range of tiles, whose halos then
  // meet in the same L2.
  int bt = blockIdx.x, bz = blockIdx.y, ld = blockIdx.z;
  {
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    if ((nb & 7) == 0) {
      const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      const int l = (b & 7) * (nb >> 3) + (b >> 3);
      bt = l % gridDim.x;
      bz = (l / gridDim.x) % gridDim.y;
      ld = l / (gridDim.x * gridDim.y);
    }
  }
  if (st && st[ld].status != ST_ACTIVE) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  const int ntx = (nx + TX - 1) / TX;
  const int x0 = (bt % ntx) * TX, y0 = (bt / ntx) * TY;
  const int z0 = bz * kz;
  const int z1 = min(z0 + kz, nz);
  const T* __restrict__ ub = u + (long long)ld * ustride;
  T* __restrict__ qb = q + (long long)ld * qstride;
  const int ms = ld / g.G;
  phase += ms * g.phase_stride;
  lm += ms * g.lm_stride;
  const int tid = threadIdx.x;
  // element (ei, ej) and output node (ox, oy) of this thread, both with pitch PX
  const int ei = tid % PX, ej = tid / PX;
  const bool is_elem = tid < NEL && ei < EX;
  const T ihx = T(1.0 / g.h[0]), ihy = T(1.0 / g.h[1]), ihz = T(1.0 / g.h[2]);
  const double ih2 = 1.0 / (g.h[0] * g.h[0]);
  const T k0 = T(ih2 / 16.0), k1 = T(ih2 / 48.0), k2 = T(ih2 / 144.0);
  const T k0h = T(ih2 / 32.0), k1h = T(ih2 / 96.0), k2h = T(ih2 / 288.0);

  int poff[NPF];
#pragma unroll
  for (int k = 0; k < NPF; ++k) {
    const int idx = tid + k * NT;
    const int a = idx % PX, b = idx / PX;
    poff[k] = idx < NP ? wrapi(y0 - 1 + b, ny) * nx + wrapi(x0 - 1 + a, nx) : -1;
  }
  // A plane fetch also brings the phases of the voxels whose lowest corner
  // is in that plane, so that one wait covers every global read of a step.
  T pf[NPF][3];
  uint8_t pph[NPF];
  auto fetch = [&](int zp) {
    const long long zb = (long long)wrapi(zp, nz) * ny * nx;
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if (poff[k] >= 0) {
        pf[k][0] = ub[zb + poff[k]];
        pf[k][1] = ub[N + zb + poff[k]];
        pf[k][2] = ub[2 * N + zb + poff[k]];
        pph[k] = phase[zb + poff[k]];
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if (poff[k] >= 0) {
        const int idx = tid + k * NT;
        plane[buf][0][idx] = pf[k][0];
        plane[buf][1][idx] = pf[k][1];
        plane[buf][2][idx] = pf[k][2];
        phl[buf][idx] = pph[k];
      }
  };

  for (int i = tid; i < 2 * g.nphase_max; i += NT) lmt[i] = lm[i];
  T carry[12];  // upper-face modes of the previous slab
#pragma unroll
  for (int r = 0; r < 12; ++r) carry[r] = T(0);
  double dot = 0.0;
  // in-plane modes (sum and difference along x, then y) of the four nodes
  // of an element's face, into w[c][base + 0..3]
  auto face_modes = [&](const T (&pl)[3][NP], int e0, T (&w)[3][8], int base) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = e0 + (k >> 1) * PX + (k & 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c][base + k] = pl[c][idx];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bit = 1; bit < 4; bit <<= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k & bit) continue;
          const T u0 = w[c][base + k], u1 = w[c][base + (k | bit)];
          w[c][base + k] = u0 + u1;
          w[c][base + (k | bit)] = u1 - u0;
        }
  };
  fetch(z0 - 1);
  store(0);
  fetch(z0);
  store(1);
  if (z0 + 1 <= z1) fetch(z0 + 1);
  __syncthreads();
  const int nsteps = z1 - z0 + 1;
  int blo = 0, bhi = 1, bnx = 2;
  // In-plane modes of the first slab's lower face; each later slab's lower
  // face is the previous slab's upper face, so its in-plane transform is
  // carried instead of redone.  Taken for FP64 on cubic voxels only: in
  // FP32 the register copies of the carry cost more than the adds they
  // save, and the general-voxel kernel would spill.
  constexpr bool FC = CUBE && sizeof(T) == 8;
  T fwd[12];
  if (FC && is_elem) {
    T w[3][8];
    face_modes(plane[0], ej * PX + ei, w, 0);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) fwd[c * 4 + k] = w[c][k];
  }
  for (int s = 0; s < nsteps; ++s) {
    const int zs = z0 - 1 + s;
    const int fb = s & 1;
    const int ox = ei, oy = ej;
    const bool out_ok = s > 0 && ox < TX && oy < TY && x0 + ox < nx && y0 + oy < ny;
    const long long o = ((long long)zs * ny + (y0 + oy)) * nx + (x0 + ox);
    T own[3] = {T(0), T(0), T(0)};
    if (is_elem) {
      // in-plane modes of the upper face's four nodes (x, then y), kept for
      // the next slab, whose lower face it is; then the z butterfly with the
      // lower face's
      T w[3][8];
      if constexpr (FC) {
        face_modes(plane[bhi], ej * PX + ei, w, 4);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const T lo = fwd[c * 4 + k], hi = w[c][k | 4];
            fwd[c * 4 + k] = hi;
            w[c][k] = lo + hi;
            w[c][k | 4] = hi - lo;
          }
      } else {  // both faces, then z
        face_modes(plane[blo], ej * PX + ei, w, 0);
        face_modes(plane[bhi], ej * PX + ei, w, 4);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const T lo = w[c][k], hi = w[c][k | 4];
            w[c][k] = lo + hi;
            w[c][k | 4] = hi - lo;
          }
      }
      const int ph = phl[blo][ej * PX + ei];
      const T lam = lmt[2 * ph], mu2 = lmt[2 * ph + 1];
      // -0 is the identity of addition, so the first sum into a mode and the
      // inverse butterflies of the never-written mode 0 fold away exactly
      T f[3][8];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 8; ++a) f[c][a] = T(-0.0);
      if constexpr (CUBE) {
        // c_M a^2 = h^-2 / 16, / 48, / 144 for |M| = 0, 1, 2
        const T l0 = lam * k0, m0 = mu2 * k0, h0 = mu2 * k0h;
        iso_term_cube<T, 0>(w, f, l0, m0, h0, T(0));
        const T l1 = lam * k1, m1 = mu2 * k1, h1 = mu2 * k1h;
        iso_term_cube<T, 1>(w, f, l1, m1, h1, T(0));
        iso_term_cube<T, 2>(w, f, l1, m1, h1, T(0));
        iso_term_cube<T, 4>(w, f, l1, m1, h1, T(0));
        const T p2 = (lam + mu2) * k2, h2 = mu2 * k2h;
        iso_term_cube<T, 3>(w, f, T(0), T(0), h2, p2);
        iso_term_cube<T, 5>(w, f, T(0), T(0), h2, p2);
        iso_term_cube<T, 6>(w, f, T(0), T(0), h2, p2);
      } else {
        {  // |M| = 0: c_M = 1, a = h^-1 / 4
          const T qx = T(0.25) * ihx, qy = T(0.25) * ihy, qz = T(0.25) * ihz;
          iso_term<T, 0>(w, f, lam, mu2, qx, qy, qz);
        }
        {  // |M| = 1: c_M = 1/12, a = h^-1 / 2
          const T l1 = lam * T(1.0 / 12.0), m1 = mu2 * T(1.0 / 12.0);
          const T hx = T(0.5) * ihx, hy = T(0.5) * ihy, hz = T(0.5) * ihz;
          iso_term<T, 1>(w, f, l1, m1, hx, hy, hz);
          iso_term<T, 2>(w, f, l1, m1, hx, hy, hz);
          iso_term<T, 4>(w, f, l1, m1, hx, hy, hz);
        }
        {  // |M| = 2: c_M = 1/144, a = h^-1
          const T l2 = lam * T(1.0 / 144.0), m2 = mu2 * T(1.0 / 144.0);
          iso_term<T, 3>(w, f, l2, m2, ihx, ihy, ihz);
          iso_term<T, 5>(w, f, l2, m2, ihx, ihy, ihz);
          iso_term<T, 6>(w, f, l2, m2, ihx, ihy, ihz);
        }
      }
      // Transpose transform, z first: (fm, fd) -> (fm - fd, fm + fd) gives
      // the modes of the lower and upper faces.  The upper face of this slab
      // is the lower face of the next, so its modes are carried and added to
      // the next slab's before the in-plane transform, which thus runs once
      // per face.
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T fl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int r = c * 4 + k;
          const T fm = f[c][k], fd = f[c][k | 4];
          fl[k] = fm - fd;
          if (s > 0) fl[k] += carry[r];
          carry[r] = fm + fd;
        }
        if (s > 0) {
#pragma unroll
          for (int bit = 1; bit < 4; bit <<= 1)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if (k & bit) continue;
              const T fm = fl[k], fd = fl[k | bit];
              fl[k] = fm - fd;
              fl[k | bit] = fm + fd;
            }
#pragma unroll
          for (int k = 0; k < 3; ++k) force[fb][c * 3 + k][tid] = fl[k];
          own[c] = fl[3];
        }
      }
    }
    // p at this step's output node (plane zs, still in LDS) for p.q
    T pd0 = T(0), pd1 = T(0), pd2 = T(0);
    if (out_ok) {
      const int pidx = (oy + 1) * PX + (ox + 1);
      pd0 = plane[blo][0][pidx];
      pd1 = plane[blo][1][pidx];
      pd2 = plane[blo][2][pidx];
    }
    // plane zs+2 goes into the buffer of plane zs-1, which no thread reads
    // any more (every thread passed the previous barrier after its last
    // read); then prefetch zs+3
    if (zs + 2 <= z1) {
      store(bnx);
      if (zs + 3 <= z1) fetch(zs + 3);
    }
    __syncthreads();
    if (out_ok) {
      const int e00 = oy * PX + ox;
      const T pd[3] = {pd0, pd1, pd2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T v = own[c] + force[fb][c * 3 + 2][e00 + 1] + force[fb][c * 3 + 1][e00 + PX] +
                    force[fb][c * 3 + 0][e00 + PX + 1];
        qb[c * N + o] = v;
        dot += (double)pd[c] * (double)v;
      }
    }
    const int t = blo;
    blo = bhi;
    bhi = bnx;
    bnx = t;
  }
  if (pq_part) {
    const double tot = block_sum_k(dot, red);
    if (tid == 0) {
      const long long nb = (long long)gridDim.x * gridDim.y;
      pq_part[(long long)ld * nb + (long long)bz * gridDim.x + bt] = tot;
    }
  }
}

// ------------------------------------------------- scalar hex8 kernel
// q = K u for heat conduction with an isotropic conductivity k per voxel
// (a per-voxel field, or a per-phase table): Sec. 3 with A = k I (App. A).
// In the modal (mean/difference) basis of a voxel's 8 corner values the
// 2x2x2 Gauss energy is diagonal: mode m with bit beta set carries the
// gradient along beta, and the element force of mode m is the mode times
// V k sum_beta c_M(m, beta) a_beta^2, with c_M = (1/12)^|M| and a_beta =
// 2^-(2-|M|) / h_beta as in the isotropic elastic kernel (M = the other
// difference bits of m).  Same z march as that kernel: node planes in LDS,
// lower-face forces exchanged, upper-face modes carried to the next slab.
// A block applies the operator to NL load cases at once (the z index of the
// grid counts groups of NL): the voxel coefficients are read once for all of
// them, each barrier serves all of them, and their independent arithmetic
// interleaves.  Cases past nload, or no longer active, are skipped.
template <typename T, int TX, int TY, int NL>
__global__ void __launch_bounds__((HexCfg<T, TX, TY>::NT), 4)
    k_kop_hex8_scalar(Grid g, int kz, int nload, const T* __restrict__ u, T* __restrict__ q,
                      const uint8_t* __restrict__ phase, const T* __restrict__ kfield,
                      const T* __restrict__ sk, long long ustride, long long qstride,
                      const PcgState* st, double* pq_part) {
  using Cfg = HexCfg<T, TX, TY>;
  constexpr int EX = Cfg::EX, PX = Cfg::PX, NEL = Cfg::NEL, NP = Cfg::NP, NT = Cfg::NT;
  constexpr int NPF = (NP + NT - 1) / NT;
  __shared__ T plane[2][NL][NP];
  __shared__ T cpl[2][NP];  // coefficients of the slab above each plane
  __shared__ T force[4][NL][NEL];
  __shared__ double red[4 * NL];
  extern __shared__ __align__(16) unsigned char kop_dyn[];
  T* skt = reinterpret_cast<T*>(kop_dyn);  // V k per phase (field: V)
  int bt = blockIdx.x, bz = blockIdx.y, lg = blockIdx.z;
  {
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    if ((nb & 7) == 0) {
      const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      const int l = (b & 7) * (nb >> 3) + (b >> 3);
      bt = l % gridDim.x;
      bz = (l / gridDim.x) % gridDim.y;
      lg = l / (gridDim.x * gridDim.y);
    }
  }
  const int ld0 = lg * NL;
  bool act[NL];
  bool any = false;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const int ld = ld0 + l;
    act[l] = ld < nload && (!st || st[ld].status == ST_ACTIVE);
    any = any || act[l];
  }
  if (!any) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ntx = (nx + TX - 1) / TX;
  const int x0 = (bt % ntx) * TX, y0 = (bt / ntx) * TY;
  const int z0 = bz * kz;
  const int z1 = min(z0 + kz, nz);
  const T* __restrict__ ub = u + (long long)ld0 * ustride;
  T* __restrict__ qb = q + (long long)ld0 * qstride;
  const int tid = threadIdx.x;
  // element (ei, ej) and output node (ox, oy) of this thread, both with pitch PX
  const int ei = tid % PX, ej = tid / PX;
  const bool is_elem = tid < NEL && ei < EX;
  // modal factors: d[m] = sum over the difference bits beta of m of
  // c_M(m, beta) a_beta^2 (mode 0, the mean, carries no gradient)
  T d[8];
  {
    const T ih[3] = {T(1.0 / g.h[0]), T(1.0 / g.h[1]), T(1.0 / g.h[2])};
    d[0] = T(0);
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      const int nbits = (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1);
      const int mo = nbits - 1;  // |M| for every beta of m
      const T cm = mo == 0 ? T(1) : (mo == 1 ? T(1.0 / 12.0) : T(1.0 / 144.0));
      const T sc = mo == 0 ? T(0.25) : (mo == 1 ? T(0.5) : T(1));
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (m & (1 << b)) acc += cm * (sc * ih[b]) * (sc * ih[b]);
      d[m] = acc;
    }
  }
  int poff[NPF];
#pragma unroll
  for (int k = 0; k < NPF; ++k) {
    const int idx = tid + k * NT;
    const int a = idx % PX, b = idx / PX;
    poff[k] = idx < NP ? wrapi(y0 - 1 + b, ny) * nx + wrapi(x0 - 1 + a, nx) : -1;
  }
  // A plane fetch also brings the coefficients (field value or phase) of the
  // voxels whose lowest corner is in that plane: one wait per step.
  T pf[NPF][NL], pc[NPF];
#pragma unroll
  for (int k = 0; k < NPF; ++k)
#pragma unroll
    for (int l = 0; l < NL; ++l) pf[k][l] = T(0);
  auto fetch = [&](int zp) {
    const long long zb = (long long)wrapi(zp, nz) * ny * nx;
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if (poff[k] >= 0) {
#pragma unroll
        for (int l = 0; l < NL; ++l)
          if (act[l]) pf[k][l] = ub[l * ustride + zb + poff[k]];
        pc[k] = kfield ? kfield[zb + poff[k]] : T(phase[zb + poff[k]]);
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if (poff[k] >= 0) {
#pragma unroll
        for (int l = 0; l < NL; ++l) plane[buf][l][tid + k * NT] = pf[k][l];
        cpl[buf][tid + k * NT] = pc[k];
      }
  };
  for (int i = tid; i < g.nphase_max; i += NT) skt[i] = sk[i];
  T carry[NL][4];  // upper-face modes of the previous slab
  double dot[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    dot[l] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) carry[l][k] = T(0);
  }
  fetch(z0 - 1);
  store(0);
  fetch(z0);
  store(1);
  if (z0 + 1 <= z1) fetch(z0 + 1);
  const int nsteps = z1 - z0 + 1;
  for (int s = 0; s < nsteps; ++s) {
    const int zs = z0 - 1 + s;
    const int blo = s & 1, bhi = blo ^ 1;
    const int ox = ei, oy = ej;
    const bool out_ok = s > 0 && ox < TX && oy < TY && x0 + ox < nx && y0 + oy < ny;
    const long long o = ((long long)zs * ny + (y0 + oy)) * nx + (x0 + ox);
    __syncthreads();
    if (is_elem) {
      const T csrc = cpl[blo][ej * PX + ei];
      const T kk = kfield ? skt[0] * csrc : skt[(int)csrc];
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        if (!act[l]) continue;
        T w[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int idx = (ej + ((a >> 1) & 1)) * PX + (ei + (a & 1));
          w[a] = plane[(a >> 2) ? bhi : blo][l][idx];
        }
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            if (a & bit) continue;
            const T u0 = w[a], u1 = w[a | bit];
            w[a] = u0 + u1;
            w[a | bit] = u1 - u0;
          }
        // mode 0 (the mean) carries no gradient; -0 keeps its butterflies
        // exact and lets them fold away
        T f[8];
        f[0] = T(-0.0);
#pragma unroll
        for (int a = 1; a < 8; ++a) f[a] = kk * d[a] * w[a];
        // transpose transform, z first; the upper face's modes are carried
        // to the next slab and added before the in-plane transform
        T fl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T fm = f[k], fd = f[k | 4];
          fl[k] = fm - fd;
          if (s > 0) fl[k] += carry[l][k];
          carry[l][k] = fm + fd;
        }
        if (s > 0) {
#pragma unroll
          for (int bit = 1; bit < 4; bit <<= 1)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if (k & bit) continue;
              const T fm = fl[k], fd = fl[k | bit];
              fl[k] = fm - fd;
              fl[k | bit] = fm + fd;
            }
#pragma unroll
          for (int k = 0; k < 4; ++k) force[k][l][tid] = fl[k];
        }
      }
    }
    T pd[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) pd[l] = out_ok ? plane[blo][l][(oy + 1) * PX + (ox + 1)] : T(0);
    __syncthreads();
    if (zs + 2 <= z1) {
      store(blo);
      if (zs + 3 <= z1) fetch(zs + 3);
    }
    if (out_ok) {
      const int e00 = oy * PX + ox;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        if (!act[l]) continue;
        const T v = force[3][l][e00] + force[2][l][e00 + 1] + force[1][l][e00 + PX] +
                    force[0][l][e00 + PX + 1];
        qb[l * qstride + o] = v;
        dot[l] += (double)pd[l] * (double)v;
      }
    }
  }
  if (pq_part) {
    const long long nb = (long long)gridDim.x * gridDim.y;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const double tot = block_sum_k(dot[l], red + 4 * l);
      if (tid == 0 && act[l]) pq_part[(long long)(ld0 + l) * nb + (long long)bz * gridDim.x + bt] = tot;
    }
  }
}

// 16 x 8 output nodes per block (17 x 9 elements, 3 waves; about 25 KB of
// LDS in FP64 for elasticity, and four blocks per CU at 162 VGPRs).  Tile
// sweep at 128^3, 6 loads, FP64, with an earlier form of the kernel that
// kept the carry in LDS: 32x8 480 us, 32x4 353 us, 16x4 363 us, 16x8 317 us
// per launch.
constexpr int kHexTX = 16, kHexTY = 8;

// z chunk per block (16 x 8 tiles, 128^3, FP64: kz 16 / 32 / 64 -> 317 /
// 320 / 338 us).
static int hex_kz(const Grid& g, int tbytes) {
  (void)tbytes;
  if (g.kz > 0) return g.kz;
  return g.nz >= 64 ? 16 : 8;
}

int kop_nblocks(const Grid& g, bool hex_elastic, int tbytes) {
  if (hex_elastic) {
    const int kz = hex_kz(g, tbytes);
    const int ntiles = ((g.nx + kHexTX - 1) / kHexTX) * ((g.ny + kHexTY - 1) / kHexTY);
    return ntiles * ((g.nz + kz - 1) / kz);
  }
  long long blocks = (g.N + 255) / 256;
  return (int)(blocks > 2048 ? 2048 : blocks);
}

template <typename T>
hipError_t launch_kop_hex8_elastic(const Grid& g, const T* u, T* q, const uint8_t* phase,
                                   const T* mat, int nload, long long ustride, long long qstride,
                                   const PcgState* st, double* pq_part, int* nblocks_out,
                                   hipStream_t s) {
  constexpr int TX = kHexTX, TY = kHexTY;
  using Cfg = HexCfg<T, TX, TY>;
  const int kz = hex_kz(g, (int)sizeof(T));
  const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  dim3 grid(ntiles, (g.nz + kz - 1) / kz, nload);
  if (nblocks_out) *nblocks_out = grid.x * grid.y;
  hipLaunchKernelGGL((k_kop_hex8_elastic<T, TX, TY>), grid, dim3(Cfg::NT), 0, s, g, kz, u, q,
                     phase, mat, ustride, qstride, st, pq_part);
  return hipGetLastError();
}

// ------------------------------------------------ node-centric operator
// Used for 2D stencils (quad4, tri2) and the 3D scalar hex8: per node, sum
// over the pixels e = I - c_a that contain it of the element-matrix rows.
// ke holds per-phase element matrices (NC*ND)^2, row index a*ND + alpha,
// already integrated on the host; kfield (if set) scales a unit matrix.
template <typename T, int DIM, int ND>
__global__ void __launch_bounds__(256)
    k_kop_generic(Grid g, const T* __restrict__ u, T* __restrict__ q,
                  const uint8_t* __restrict__ phase, const T* __restrict__ kfield,
                  const T* __restrict__ ke, long long ustride, long long qstride,
                  const PcgState* st, double* pq_part) {
  constexpr int NC = 1 << DIM, NK = NC * ND;
  __shared__ double red[8];
  const int ld = blockIdx.y;
  if (st && st[ld].status != ST_ACTIVE) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long N = g.N;
  const T* __restrict__ ub = u + (long long)ld * ustride;
  T* __restrict__ qb = q + (long long)ld * qstride;
  double dot = 0.0;
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx);
    const int y = (int)((I / nx) % ny);
    const int z = (int)(I / ((long long)nx * ny));
    T acc[ND];
#pragma unroll
    for (int al = 0; al < ND; ++al) acc[al] = T(0);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const int exx = wrapi(x - ax, nx), eyy = wrapi(y - ay, ny), ezz = wrapi(z - az, nz);
      const long long e = ((long long)ezz * ny + eyy) * nx + exx;
      const T* Ke = phase ? ke + (size_t)phase[e] * NK * NK : ke;
      const T sc = kfield ? kfield[e] : T(1);
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const long long J = ((long long)wrapi(ezz + bz, nz) * ny + wrapi(eyy + by, ny)) * nx +
                            wrapi(exx + bx, nx);
#pragma unroll
        for (int be = 0; be < ND; ++be) {
          const T uj = sc * ub[be * N + J];
#pragma unroll
          for (int al = 0; al < ND; ++al) acc[al] += Ke[(a * ND + al) * NK + b * ND + be] * uj;
        }
      }
    }
#pragma unroll
    for (int al = 0; al < ND; ++al) {
      qb[al * N + I] = acc[al];
      dot += (double)ub[al * N + I] * (double)acc[al];
    }
  }
  if (pq_part) {
    const double tot = block_sum_k(dot, red);
    if (threadIdx.x == 0) pq_part[(long long)ld * gridDim.x + blockIdx.x] = tot;
  }
}

template <typename T>
hipError_t launch_kop_generic(const Grid& g, int elem, const T* u, T* q, const uint8_t* phase,
                              const T* kfield, const T* ke, int nload, long long ustride,
                              long long qstride, const PcgState* st, double* pq_part,
                              int* nblocks_out, hipStream_t s) {
  (void)elem;
  const int blocks = kop_nblocks(g, false);
  dim3 grid((unsigned)blocks, nload);
  if (nblocks_out) *nblocks_out = (int)blocks;
  if (g.dim == 3 && g.nd == 1)
    hipLaunchKernelGGL((k_kop_generic<T, 3, 1>), grid, dim3(256), 0, s, g, u, q, phase, kfield,
                       ke, ustride, qstride, st, pq_part);
  else if (g.dim == 2 && g.nd == 1)
    hipLaunchKernelGGL((k_kop_generic<T, 2, 1>), grid, dim3(256), 0, s, g, u, q, phase, kfield,
                       ke, ustride, qstride, st, pq_part);
  else if (g.dim == 2 && g.nd == 2)
    hipLaunchKernelGGL((k_kop_generic<T, 2, 2>), grid, dim3(256), 0, s, g, u, q, phase, kfield,
                       ke, ustride, qstride, st, pq_part);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// -------------------------------------------------------------- RHS
// b[alpha][I] = -sum_a fe[t(e)][load][a*nd + alpha] (* k(e)), e = I - c_a.
// Corner contributions are added in antipodal pairs (a, NC-1-a): in a
// homogeneous medium each pair cancels exactly, so b = 0 exactly there.
// The phases (or conductivities) of the nc pixels around node I are read
// once and serve every load case and component.
__global__ void k_rhs(Grid g, int nc, const uint8_t* __restrict__ phase,
                      const double* __restrict__ kfield, const double* __restrict__ fe,
                      int nload, double* __restrict__ b, long long bstride) {
  const int nx = g.nx, ny = g.ny, nz = g.nz, nd = g.nd;
  const long long N = g.N;
  const int nk = nc * nd;
  for (long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x; I < N;
       I += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(I % nx);
    const int y = (int)((I / nx) % ny);
    const int z = (int)(I / ((long long)nx * ny));
    int t[8];
    double sc[8];
#pragma unroll
    for (int aa = 0; aa < 8; ++aa) {
      if (aa >= nc) break;
      const int ax = aa & 1, ay = (aa >> 1) & 1, az = (aa >> 2) & 1;
      const long long e = ((long long)wrapi(z - az, nz) * ny + wrapi(y - ay, ny)) * nx +
                          wrapi(x - ax, nx);
      t[aa] = phase ? phase[e] : 0;
      sc[aa] = kfield ? kfield[e] : 1.0;
    }
    for (int ld = 0; ld < nload; ++ld) {
      for (int al = 0; al < nd; ++al) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a >= nc / 2) break;
          const int a2 = nc - 1 - a;
          const double pair = sc[a] * fe[((size_t)t[a] * nload + ld) * nk + a * nd + al] +
                              sc[a2] * fe[((size_t)t[a2] * nload + ld) * nk + a2 * nd + al];
          acc += pair;
        }
        b[(long long)ld * bstride + al * N + I] = -acc;
      }
    }
  }
}

hipError_t launch_rhs(const Grid& g, int elem, const uint8_t* phase, const double* kfield,
                      const double* fe, int nphase_tables, int nload, double* b,
                      long long bstride, hipStream_t s) {
  (void)nphase_tables;
  (void)elem;
  if (g.tn) return launch_rhs_tn(g, phase, kfield, fe, nload, b, bstride, s);
  const int nc = g.dim == 3 ? 8 : 4;
  long long blocks = (g.N + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)blocks), dim3(256), 0, s, g, nc, phase, kfield, fe,
                     nload, b, bstride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_kop_hex8_iso(const Grid& g, const T* u, T* q, const uint8_t* phase,
                               const T* lm, int nload, long long ustride, long long qstride,
                               const PcgState* st, double* pq_part, int* nblocks_out,
                               hipStream_t s) {
  constexpr int TX = kHexTX, TY = kHexTY;
  using Cfg = HexCfg<T, TX, TY>;
  const int kz = hex_kz(g, (int)sizeof(T));
  const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  dim3 grid(ntiles, (g.nz + kz - 1) / kz, nload);
  if (nblocks_out) *nblocks_out = grid.x * grid.y;
  const size_t lds = sizeof(T) * 2 * (size_t)(g.nphase_max > 0 ? g.nphase_max : 1);
  if (g.h[0] == g.h[1] && g.h[0] == g.h[2])
    hipLaunchKernelGGL((k_kop_hex8_iso<T, TX, TY, true>), grid, dim3(Cfg::NT), lds, s, g, kz, u, q,
                       phase, lm, ustride, qstride, st, pq_part);
  else
    hipLaunchKernelGGL((k_kop_hex8_iso<T, TX, TY, false>), grid, dim3(Cfg::NT), lds, s, g, kz, u,
                       q, phase, lm, ustride, qstride, st, pq_part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_kop_hex8_scalar(const Grid& g, const T* u, T* q, const uint8_t* phase,
                                  const T* kfield, const T* sk, int nload, long long ustride,
                                  long long qstride, const PcgState* st, double* pq_part,
                                  int* nblocks_out, hipStream_t s) {
  constexpr int TX = kHexTX, TY = kHexTY;
  const int kz = hex_kz(g, (int)sizeof(T));
  const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
  // load cases per block (FP32): three where that leaves no block with one
  // case alone (3, 6, ... and 5 = 3 + 2 fit best), else pairs.  FP64 keeps
  // one: its three-case kernel needs 118 VGPRs against 74, and with 15
  // instead of 24 waves per CU it was slower (256^3, 3 loads: 425 against
  // 367 us per launch; FP32 198 against 236 us).
  const int NL = sizeof(T) == 8 || nload == 1 ? 1 : ((nload == 2 || nload == 4) ? 2 : 3);
  dim3 grid(ntiles, (g.nz + kz - 1) / kz, (nload + NL - 1) / NL);
  if (nblocks_out) *nblocks_out = grid.x * grid.y;
  const size_t lds = sizeof(T) * (size_t)(g.nphase_max > 0 ? g.nphase_max : 1);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(HexCfg<T, TX, TY>::NT), lds, s, g, kz, nload, u, q,
                       phase, kfield, sk, ustride, qstride, st, pq_part);
  };
  if (NL == 1) go(k_kop_hex8_scalar<T, TX, TY, 1>);
  else if (NL == 2) go(k_kop_hex8_scalar<T, TX, TY, 2>);
  else go(k_kop_hex8_scalar<T, TX, TY, 3>);
  return hipGetLastError();
}
template hipError_t launch_kop_hex8_scalar<double>(const Grid&, const double*, double*,
                                                   const uint8_t*, const double*, const double*,
                                                   int, long long, long long, const PcgState*,
                                                   double*, int*, hipStream_t);
template hipError_t launch_kop_hex8_scalar<float>(const Grid&, const float*, float*,
                                                  const uint8_t*, const float*, const float*, int,
                                                  long long, long long, const PcgState*, double*,
                                                  int*, hipStream_t);

template hipError_t launch_kop_hex8_iso<double>(const Grid&, const double*, double*,
                                                const uint8_t*, const double*, int, long long,
                                                long long, const PcgState*, double*, int*,
                                                hipStream_t);
template hipError_t launch_kop_hex8_iso<float>(const Grid&, const float*, float*, const uint8_t*,
                                               const float*, int, long long, long long,
                                               const PcgState*, double*, int*, hipStream_t);

template hipError_t launch_kop_hex8_elastic<double>(const Grid&, const double*, double*,
                                                    const uint8_t*, const double*, int,
                                                    long long, long long, const PcgState*,
                                                    double*, int*, hipStream_t);
template hipError_t launch_kop_hex8_elastic<float>(const Grid&, const float*, float*,
                                                   const uint8_t*, const float*, int, long long,
                                                   long long, const PcgState*, double*, int*,
                                                   hipStream_t);
template hipError_t launch_kop_generic<double>(const Grid&, int, const double*, double*,
                                               const uint8_t*, const double*, const double*,
                                               int, long long, long long, const PcgState*,
                                               double*, int*, hipStream_t);
template hipError_t launch_kop_generic<float>(const Grid&, int, const float*, float*,
                                              const uint8_t*, const float*, const float*, int,
                                              long long, long long, const PcgState*, double*,
                                              int*, hipStream_t);

}  // namespace fh
