// Internal declarations shared by the HIP translation units of libfh.
// Device code targets gfx950 (CDNA4): 64-wide wavefronts, 160 KB LDS per
// workgroup, FP64 vector ALU.  Nothing here is part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace fh {

// ---------------------------------------------------------------- PCG state
// Per load case, device resident.  Kernels read alpha/beta/status from here so
// that no host round trip is needed inside an iteration.
enum : int {
  ST_ACTIVE = 0,
  ST_CONVERGED = 1,
  ST_MAXIT = 2,
  ST_BREAKDOWN = 3,
  ST_CONVERGED_PENDING = 4,  // converged this iteration, x update still due
  ST_MAXIT_PENDING = 5,
};

struct PcgState {
  double rho, rho0, alpha, beta, eta2, last;
  int iter, status, itmax, pad;
};

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }

// -------------------------------------------------------------- geometry
struct Grid {
  int nx, ny, nz;      // nz = 1 in 2D
  int dim;             // 2 or 3
  int nd;              // dofs per node (d or 1)
  int nxh;             // nx/2 + 1
  long long N;         // nx*ny*nz
  double h[3];         // grid spacing
  int nphase_max;      // number of material tables the operator may index
  // Batched solves: load index ld belongs to microstructure ld / G, whose
  // phase grid, material table and K^+ sit at these strides (G large and
  // strides 0 for a single microstructure).
  int G;
  long long phase_stride, kplus_stride;
  int lm_stride;
  // launch shapes (0 = default): operator z-chunk, y-pass lines per block,
  // z-pass ky lines per block, FP32 x-pass rows per block (16 or 32) -- set
  // by the autotuner for batched solves
  int kz, zb, kyb, xrows;
  // two-node stencil (N_n = 2): the nd = 2 fields are the corner and centre
  // node sets, K^+ is a Hermitian block stored as {k00, k11, Re k01, Im k01}
  int tn;
};

// FFT plan for one axis length: radix of stage i (applied first to last) in
// bits 4i..4i+3 of `code` (a packed word keeps the plan in scalar registers).
struct AxisPlan {
  int n;
  int nstage;
  unsigned code;
};

// ------------------------------------------------------ kernel launchers
// All launchers enqueue on `s` and return hipError_t of the launch.

// Operator q = K u (eq. lin_system), element-wise constant materials.
//   elastic hex8: mat = nphase x 36 (Mandel, pre-multiplied by the voxel
//   volume); partial energies u.Ku per block go to pq_part (may be null).
template <typename T>
hipError_t launch_kop_hex8_elastic(const Grid& g, const T* u, T* q, const uint8_t* phase,
                                   const T* mat, int nload, long long ustride, long long qstride,
                                   const PcgState* st, double* pq_part, int* nblocks_out,
                                   hipStream_t s);
// isotropic phases: lm = nphase x {V lambda, 2 V mu}.
template <typename T>
hipError_t launch_kop_hex8_iso(const Grid& g, const T* u, T* q, const uint8_t* phase,
                               const T* lm, int nload, long long ustride, long long qstride,
                               const PcgState* st, double* pq_part, int* nblocks_out,
                               hipStream_t s);
// scalar hex8 conduction, isotropic k per voxel: kk = sk[0] * kfield[e]
// (field) or sk[phase[e]] (sk = V k per phase); g.nphase_max table entries.
template <typename T>
hipError_t launch_kop_hex8_scalar(const Grid& g, const T* u, T* q, const uint8_t* phase,
                                  const T* kfield, const T* sk, int nload, long long ustride,
                                  long long qstride, const PcgState* st, double* pq_part,
                                  int* nblocks_out, hipStream_t s);
// node-centric generic operator with per-phase element matrices (2D
// elements, 3D scalar hex8): ke = nphase x (nc*nd)^2, or a unit element
// matrix scaled by a per-voxel field kfield.
template <typename T>
hipError_t launch_kop_generic(const Grid& g, int elem, const T* u, T* q, const uint8_t* phase,
                              const T* kfield, const T* ke, int nload, long long ustride,
                              long long qstride, const PcgState* st, double* pq_part,
                              int* nblocks_out, hipStream_t s);
// b = -D^T W C e: fe = nphase x nload x (nc*nd) element forces of the
// uniform strain, or unit forces scaled by kfield.
hipError_t launch_rhs(const Grid& g, int elem, const uint8_t* phase, const double* kfield,
                      const double* fe, int nphase_tables, int nload, double* b,
                      long long bstride, hipStream_t s);

// FFT passes (layouts in fft.hip).  modes below.
enum XfwdMode { XF_PLAIN = 0, XF_UPDATE_R = 1 };
enum XinvMode { XI_PLAIN = 0, XI_INIT_P = 1, XI_PCG = 2 };
enum ZMode { Z_FORWARD_ONLY = 0, Z_SOLVE = 1 };

template <typename T>
hipError_t launch_xfwd(const Grid& g, const AxisPlan& px, const cplx<double>* twx, int mode,
                       T* r, long long rstride, const T* q, long long qstride, cplx<T>* A,
                       long long sstride, int nload, const PcgState* st, hipStream_t s);
template <typename T>
hipError_t launch_yfwd(const Grid& g, const AxisPlan& py, const cplx<double>* twy,
                       const cplx<T>* A, cplx<T>* B, long long sstride, int nload,
                       const PcgState* st, hipStream_t s);
template <typename T>
hipError_t launch_zpass(const Grid& g, const AxisPlan& pz, const cplx<double>* twz, int mode,
                        cplx<T>* B, long long sstride, const T* kplus, int nload,
                        const PcgState* st, double* rz_part, int* nblocks_out, hipStream_t s);
template <typename T>
hipError_t launch_yinv(const Grid& g, const AxisPlan& py, const cplx<double>* twy,
                       const cplx<T>* B, cplx<T>* A, long long sstride, int nload,
                       const PcgState* st, hipStream_t s);
template <typename T>
hipError_t launch_xinv(const Grid& g, const AxisPlan& px, const cplx<double>* twx, int mode,
                       const cplx<T>* A, long long sstride, T* out, T* x, T* p,
                       long long fstride, int nload, const PcgState* st, hipStream_t s);

// Symbol K^+ (Alg. 2 + eq. block_inversion) from the forward spectra of the
// impulse responses: spec[beta] = spectrum of Kref i^beta (B layout).
hipError_t launch_symbol(const Grid& g, const cplx<double>* spec, long long sstride,
                         double* kplus, int* bad_flag, hipStream_t s);
hipError_t launch_cast_symbol(long long count, const double* src, float* dst, hipStream_t s);

// Guaranteed eigenvalue bounds (Sec. 4.3): per node the min / max of the
// per-voxel generalized eigenvalue pairs over the 2^dim voxels sharing the
// node (tab: lo/hi per phase table, or the unit-conductivity pair scaled by
// kfield).  lo/hi (N values each) may be null; range[0..1] = global min/max.
// part holds 2 doubles per block (node_bounds_partials blocks).
int node_bounds_partials(const Grid& g);
hipError_t launch_node_bounds(const Grid& g, const uint8_t* phase, const double* kfield,
                              const double* tab, double* lo, double* hi, double* part,
                              double* range, hipStream_t s);

// Elasto-plastic material stage (plastic.hip).  mode 0 = residual: stress
// at e + D u from the committed state, tangent per point, element forces;
// mode 1 = tangent operator on u (= p); mode 2 = commit the internal
// variables at e + D u.  part (may be null): plastic_parts() doubles per
// block (macro stress 6, sum fe^2, sum K, sum a, sum v v^T (21), plastic
// points).  Launch with plastic_blocks(g, max) blocks.
int plastic_parts();
int plastic_blocks(const Grid& g, int max_blocks);
hipError_t launch_plastic_stage(int mode, const Grid& g, const uint8_t* phase,
                                const double* params, const double* E, const double* u,
                                double* fe, double* eps_p, double* alpha, double* ta, double* tv,
                                double* part, int nblocks, hipStream_t s);
// out[c][I] = sign * sum of the 8 element forces at node I; part (may be
// null): one partial per block of sum (dot ? dot : out) * out.
hipError_t launch_gather_nodes(const Grid& g, const double* fe, double sign, double* out,
                               const double* dot, double* part, int nblocks, hipStream_t s);

// Two-node stencil (tn.hip), 2D scalar: operator from per-phase 5 x 5
// element matrices (or a unit matrix scaled by kfield); right-hand side from
// per-phase x load element forces (5 each); Hermitian K^+ / N from the
// impulse-response spectra (part: 1024 doubles of scratch).
template <typename T>
hipError_t launch_kop_tn(const Grid& g, const T* u, T* q, const uint8_t* phase, const T* kfield,
                         const T* ke, int nload, long long ustride, long long qstride,
                         const PcgState* st, double* pq_part, int* nblocks_out, hipStream_t s);
hipError_t launch_rhs_tn(const Grid& g, const uint8_t* phase, const double* kfield,
                         const double* fe, int nload, double* b, long long bstride,
                         hipStream_t s);
hipError_t launch_symbol_tn(const Grid& g, const cplx<double>* spec, long long sstride,
                            double* kplus, int* bad_flag, double* part, hipStream_t s);

// Strain-based scheme (sb.hip), 3D hex8, quadrature-point fields [6][8][N].
// A 6x6 matrix (m, row-major) and a 6-vector (v) passed by value.
struct Mat6 {
  double m[36];
  double v[6];
};
// fe = element forces of tau = C_phase (x + E) (x may be null; E 6 values or
// null); C = nphase x 36 Mandel tables.
hipError_t launch_sb_cdiv(const Grid& g, const uint8_t* phase, const double* C, const double* x,
                          const double* E, double* fe, hipStream_t s);
// out = D z at the Gauss points
hipError_t launch_sb_grad(const Grid& g, const double* z, double* out, hipStream_t s);
// part[sb_dot_partials(g)] = per-block sums of w (a + Ea)^T M (b + Eb),
// M = Mc (36 values) or the voxel's C when C is not null
int sb_dot_partials(const Grid& g);
hipError_t launch_sb_dot(const Grid& g, const uint8_t* phase, const double* C, const double* Mc,
                         const double* a, const double* Ea, const double* b, const double* Eb,
                         double* part, hipStream_t s);
// p = r + beta p
hipError_t launch_sb_xpby(double* p, const double* r, double beta, long long n, hipStream_t s);

// Number of per-load partial sums the operator and z-pass launches write.
// (tbytes = sizeof of the field type: the default z chunk depends on it)
int kop_nblocks(const Grid& g, bool hex_elastic, int tbytes = 8);
template <typename T>
int zpass_nblocks(const Grid& g);

// Reductions and PCG scalar updates.
hipError_t launch_finalize_init(PcgState* st, const double* part, int nb, int nload,
                                hipStream_t s);
hipError_t launch_finalize_alpha(PcgState* st, const double* part, int nb, int nload,
                                 hipStream_t s);
hipError_t launch_finalize_beta(PcgState* st, const double* part, int nb, int nload,
                                double* hist, int hist_len, hipStream_t s);
hipError_t launch_dot_partials(const double* a, const double* b, long long n, double* part,
                               int nb, hipStream_t s);
hipError_t launch_sum_partials(const double* part, int nb, double* out, hipStream_t s);
hipError_t launch_pair_dots(const double* A, const double* B, long long F, int G, int nms,
                            int nchunk, double* part, double* out, hipStream_t s);
hipError_t launch_phase_count(const uint8_t* phase, long long n, int nphase,
                              unsigned long long* counts, int* bad, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, T v, long long n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s);
hipError_t launch_axpy(double* y, double a, const double* x, long long n, hipStream_t s);
// y = x - mean(x) per component: not needed on the hot path.
hipError_t launch_cast_d2f(const double* src, float* dst, long long n, hipStream_t s);
hipError_t launch_add_f2d(double* dst, const float* src, long long n, hipStream_t s);
hipError_t launch_residual(double* r, const double* b, const double* Kx, long long n,
                           hipStream_t s);
// per load case (blockIdx.y): dst = (float) src where the load is active;
// dst += src where mask[load] != 0
hipError_t launch_cast_masked(const double* src, float* dst, long long F, int nload,
                              const PcgState* st, hipStream_t s);
hipError_t launch_add_masked(double* dst, const float* src, long long F, int nload,
                             const int* mask, hipStream_t s);
hipError_t launch_impulse(double* f, long long n, long long pos, hipStream_t s);
hipError_t launch_field_sum(const double* x, long long n, double* out_part, int nb,
                            hipStream_t s);
// *flag |= 1 if some x[i] is not a positive finite number (flag not cleared)
hipError_t launch_flag_nonpositive(const double* x, long long n, int* flag, hipStream_t s);
// x[seg][.] -= its mean for nseg segments of n values (part: nseg x nchunk)
hipError_t launch_remove_mean(double* x, int nseg, long long n, double* part, int nchunk,
                              hipStream_t s);

}  // namespace fh

// learned warm start (net.hip)
struct fh_net;
#include <string>
namespace fh {
int net_warm_guess(fh_net* net, hipStream_t stream, const uint8_t* phase_dev, float gamma,
                   int nload, const double* E, double scale, double* x, long long F,
                   std::string* err);
int net_grid(const fh_net* net);
}  // namespace fh
