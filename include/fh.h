/*
 * fh.h -- C-ABI of the MI355X FFT-preconditioned finite-element
 * homogenization solver (Ladecky et al., "Optimal FFT-accelerated Finite
 * Element Solver for Homogenization").
 *
 * What the library computes
 *   For a periodic cell discretised on a regular grid with a one-node
 *   stencil (Sec. 3, Fig. tiling) and an element-wise constant linear
 *   material, it solves for every macroscopic load e_j the linear system
 *   K u_j = b_j with K = D^T W C D and b_j = -D^T W C e_j (eq. lin_system with
 *   u_(0) = 0) by PCG (Sec. 4.1, Alg. 1) preconditioned with the pseudo-inverse
 *   of the reference stiffness Kref = D^T W Cref D (eq. Kref), applied as
 *   F^H K^+ F (eq. M_inverse) with K^ assembled by Alg. 2.  PCG stops when the
 *   Kref^-1-norm of the residual has dropped by eta (Sec. 6, termination
 *   criteria).  The homogenized tensor is returned in energy form
 *   C_hom[i][j] = (1/|Y|) sum_Q w_Q (e_i + D u_i)^T C (e_j + D u_j).
 *
 * Conventions
 *   Grid n = (nx, ny, nz) (nz = 1 in 2D), cell lengths l (h = l/n).  Every
 *   grid array is x-fastest: element (x, y, z) at x + nx*(y + ny*z).  A voxel
 *   (pixel) belongs to its lowest corner node.  Nodal fields are
 *   component-major: u[c][z][y][x], c < nd (nd = d for elasticity, 1 for
 *   scalar problems).  Strains and materials use Mandel notation
 *   (Sec. 2, eq. mandel_grad): 3D order 11, 22, 33, 23, 13, 12 with sqrt(2)
 *   on shear; 2D order 11, 22, 12.  A scalar material is the d x d
 *   conductivity (App. A).
 *
 * Memory
 *   Pointers whose name ends in _dev are device pointers (HBM of the device
 *   given to fh_create); all other array pointers are host pointers.  The
 *   caller owns every array it passes; the library copies host inputs and
 *   reads device inputs during the call (a device phase/conductivity field
 *   must stay alive until the next fh_set_* call or fh_destroy).  Device work
 *   runs on the stream set by fh_set_stream (default: the null stream); calls
 *   that return results to the host synchronise that stream.  Device scratch
 *   comes from a caller-bound workspace (fh_bind_workspace) or, if none is
 *   bound, from hipMalloc inside the library.
 *
 * Errors
 *   0 = success; > 0 warning with a valid result (FH_NOT_CONVERGED);
 *   < 0 error, no result.  fh_last_error() returns a message for the last
 *   failing call on the context.  A context is not thread-safe.
 */
#ifndef FH_H
#define FH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FH_OK 0
#define FH_NOT_CONVERGED 1
#define FH_EINVAL (-1)
#define FH_ENOMEM (-2)
#define FH_EDEVICE (-3)
#define FH_ENOTSPD (-4)
#define FH_ESTATE (-5)

#define FH_SCALAR 0  /* thermal conduction (App. A)            */
#define FH_ELASTIC 1 /* small-strain elasticity (Sec. 2)       */

#define FH_HEX8 0  /* 3D trilinear hexahedron, 2x2x2 Gauss points, w = V_p/8 */
#define FH_QUAD4 1 /* 2D bilinear quadrilateral, 2x2 Gauss points, w = V_p/4 (Fig. tiling a.2) */
#define FH_TRI2 2  /* 2D two linear triangles per pixel, split along (0,0)-(1,1),
                      one centroid point each, w = V_p/2 (Fig. tiling b.2) */
#define FH_TRI4 3  /* 2D two-node stencil (N_n = 2, Fig. tiling c.2): every pixel
                      carries its lowest corner node and its centre node and
                      is cut into four linear triangles (centre + one pixel
                      edge), one centroid point each, w = V_p/4.  Scalar
                      problems only.  A nodal field holds two node sets,
                      u[0][y][x] at the corners and u[1][y][x] at the centres
                      (2 N doubles), and the symbol is a Hermitian 2 x 2
                      block per frequency whose zero-frequency block has rank
                      1 (fh_get_symbol: {k00, k11, Re k01, Im k01} of K^+ / N
                      per frequency, each as a separate [kx][ky] plane).      */

#define FH_FP64 0          /* every kernel in FP64                                 */
#define FH_FP32_REFINED 1  /* FP32 operator/FFT/solve inside FP64 refinement       */

#define FH_MAX_LOADS 32

/* fh_opts.flags: record a HIP event pair on the solve stream around every
 * kernel launch of the PCG loop and report per-class totals in fh_stats.   */
#define FH_FLAG_TIME_KERNELS 1
/* fh_opts.flags: rebuild the reference material, the Alg. 2 symbol and the
 * right-hand sides even if the inputs have not changed since the last solve */
#define FH_FLAG_REBUILD 2
/* fh_opts.flags: start every load case from the learned warm start of the
 * network attached with fh_set_warm_start instead of from zero (see there) */
#define FH_FLAG_WARM_START 4
/* fh_opts.flags, with FH_FLAG_TIME_KERNELS: record the event pairs only in
 * every 8th PCG iteration (loop iterations 4, 12, 20, ...).  Each timed launch leaves the GPU idle for a few
 * microseconds around its events, so timing every launch slows the loop;
 * the per-class totals then cover the sampled iterations only.             */
#define FH_FLAG_TIME_SAMPLED 8
/* fh_opts.flags for fh_solve_batch: solve the grid-size groups one after
 * another instead of concurrently (each group on its own stream)           */
#define FH_FLAG_BATCH_SERIAL 16
/* fh_opts.flags: capture one PCG iteration in a hipGraph on a private
 * stream of the context (forked from and joined back to the stream of
 * fh_set_stream with events) and replay it, instead of launching every
 * kernel from the host; the iterations that FH_FLAG_TIME_KERNELS samples
 * are launched from the host either way.  Both paths run the same kernels
 * in the same order and give the same bits.  (At 128^3 the host launches
 * already queue back to back: replay measured 0.5 % slower.)              */
#define FH_FLAG_GRAPH 32

/* kernel classes of fh_stats.kernel_ms / kernel_launches                  */
#define FH_K_OPERATOR 0   /* q = K p (+ p.q partials)                       */
#define FH_K_XFWD 1       /* r -= alpha q, forward real FFT along x          */
#define FH_K_YFWD 2       /* forward FFT along y                             */
#define FH_K_ZSOLVE 3     /* FFT along z, K^+ block solve, r.z, inverse z    */
#define FH_K_YINV 4       /* inverse FFT along y                             */
#define FH_K_XINV 5       /* inverse real FFT along x, x += alpha p, p update */
#define FH_K_SCALAR 6     /* single-block scalar updates (alpha, beta, stop) */
#define FH_K_NCLASS 8

typedef struct fh_ctx fh_ctx;
#ifndef FH_NET_TYPEDEF
#define FH_NET_TYPEDEF
typedef struct fh_net fh_net; /* learned warm start, fh_net.h */
#endif

typedef struct fh_opts {
  double eta;       /* relative Kref^-1-norm tolerance (Sec. 6); e.g. 1e-10       */
  int itmax;        /* PCG iteration cap per load case (Alg. 1 it_max^CG)         */
  int precision;    /* FH_FP64 or FH_FP32_REFINED                                 */
  int poll;         /* iterations between host convergence polls (0 = default)   */
  int flags;        /* FH_FLAG_* bits                                             */
  double eta_inner; /* FH_FP32_REFINED: sweep k of the refinement brings the
                       residual to max(eta_inner^(k+1), eta/2) times that of b
                       (0 = sqrt(eta) when eta >= 1e-6, else 1e-4)                */
  const double *guess_dev; /* initial fluctuation u_(0) of Alg. 1 for every load
                       case (device, nload x nd x N; NULL = zero).  It is shifted
                       to zero mean per component and screened: a load case keeps
                       it only if r0.M r0 < b.M b (r0 = b - K u_(0)), else it
                       starts from zero.  The stopping test stays relative to
                       b.M b, so results are comparable with zero starts.       */
} fh_opts;

typedef struct fh_stats {
  int nload;
  int iterations[FH_MAX_LOADS]; /* PCG iterations per load case (inner, summed)  */
  int status[FH_MAX_LOADS];     /* 0 converged, 1 not converged, < 0 error       */
  double rel_res[FH_MAX_LOADS]; /* final sqrt(r.z / r0.z0)                        */
  int outer[FH_MAX_LOADS];      /* refinement sweeps (FH_FP32_REFINED)            */
  double setup_ms;              /* Cref, Alg. 2 symbol, right-hand sides          */
  double solve_ms;              /* PCG loops of all load cases                    */
  double chom_ms;               /* homogenized-tensor reduction                   */
  long long dof;                /* nd * N                                         */
  double kernel_ms[FH_K_NCLASS];      /* summed event-timed durations       */
  long long kernel_launches[FH_K_NCLASS];
  int guess_used[FH_MAX_LOADS];   /* 1 if the initial guess was kept          */
  double guess_res[FH_MAX_LOADS]; /* sqrt(r0.M r0 / b.M b) of the guess       */
  double guess_ms;                /* warm-start inference + screen             */
  long long kernel_issued[FH_K_NCLASS]; /* launches per class, timed or not
                                           (kernel_launches counts the timed
                                           ones, FH_FLAG_TIME_SAMPLED)       */
  double kernel_units[FH_K_NCLASS]; /* load cases processed by the timed
                                       launches of each class (a launch skips
                                       load cases that have stopped), so bytes
                                       per timed launch = bytes per load case
                                       x kernel_units / kernel_launches     */
} fh_stats;

/* Context on HIP device `device`.  Returns FH_EDEVICE if it cannot be used. */
int fh_create(fh_ctx **out, int device);
void fh_destroy(fh_ctx *ctx);
const char *fh_last_error(const fh_ctx *ctx);

/* HIP stream (hipStream_t) all device work is issued on; NULL = null stream. */
int fh_set_stream(fh_ctx *ctx, void *hip_stream);

/* Grid and discretisation (Sec. 3).  dim = 2 or 3; n[2] ignored (taken as 1)
 * in 2D; l = cell edge lengths (NULL = all 1).  problem = FH_SCALAR or
 * FH_ELASTIC; element = FH_HEX8 (dim 3) or FH_QUAD4 / FH_TRI2 (dim 2).
 * nx and ny must be even; every n must be a product of 2 and 3 and at
 * most 256.  Invalidates phases, loads and results.                          */
int fh_set_grid(fh_ctx *ctx, int dim, const int n[3], const double l[3], int problem,
                int element);

/* Element-wise constant material (Sec. 4.3): phase_dev = uint8 per voxel
 * (device, N bytes), mat = nphase tables (host), each m x m row-major with
 * m = d_m (elastic, Mandel) or d (scalar conductivity).  Tables must be
 * symmetric; nphase in 1..256.  Phase ids >= nphase make fh_solve fail.   */
int fh_set_phases(fh_ctx *ctx, const uint8_t *phase_dev, int nphase, const double *mat);

/* Per-voxel scalar conductivity A = k I (scalar problems, FH_HEX8):
 * k_dev = N doubles on the device, all > 0.                                 */
int fh_set_conductivity_field(fh_ctx *ctx, const double *k_dev);

/* Reference material Cref (eq. Kref), m x m host, symmetric positive
 * definite; NULL = quadrature-weighted mean of the material (Sec. 6.2).    */
int fh_set_reference(fh_ctx *ctx, const double *Cref);

/* Macroscopic strains / gradients e_j (Sec. 2, App. A): nload x m host
 * (Mandel for elasticity), nload in 1..FH_MAX_LOADS.                        */
int fh_set_load(fh_ctx *ctx, int nload, const double *E);

/* Device bytes the next fh_solve needs for the current grid and loads, and
 * binding of a caller-owned device buffer of at least that size (256-byte
 * aligned).  Binding NULL returns to library-owned memory.                 */
int fh_workspace_size(fh_ctx *ctx, size_t *bytes);
int fh_bind_workspace(fh_ctx *ctx, void *dev, size_t bytes);

/* Setup (Alg. 2 and right-hand sides) followed by one PCG solve per load
 * case, then the homogenized tensor.  opt may be NULL (eta 1e-10, itmax
 * 10000, FP64).  Returns FH_NOT_CONVERGED if any load case hit itmax,
 * FH_ENOTSPD on PCG breakdown (p.q <= 0) or a non-SPD Cref block.         */
int fh_solve(fh_ctx *ctx, const fh_opts *opt, fh_stats *st);

/* Learned warm start (fh_net.h): with FH_FLAG_WARM_START, fh_solve runs the
 * network on the phase field and takes u_(0) = (l/n) sum_j E_j O_j, shifted
 * to zero mean, as initial guess of every load case (screened as guess_dev).
 * Needs 3D elasticity with FH_HEX8 on a cubic n^3 grid equal to the
 * network's, cubic cell, two isotropic phases (0 = matrix, 1 = inclusion);
 * gamma = log10(C1[0][0] / C0[0][0]) / 3.  The network must outlive its use;
 * NULL detaches.                                                            */
int fh_set_warm_start(fh_ctx *ctx, fh_net *net);

/* Results of the last fh_solve: fluctuation u_j (device, nd*N doubles,
 * zero-mean representative) and the homogenized tensor (host, nload x nload,
 * the full m x m tensor when the loads are the m unit vectors).            */
int fh_get_fluctuation(fh_ctx *ctx, int load, double *u_dev);
int fh_get_homogenized(fh_ctx *ctx, double *Chom);
/* Reference material actually used (host, m x m) and the convergence
 * history sqrt(r_k.z_k / r0.z0), k = 1..iterations (host, up to max).     */
int fh_get_reference(fh_ctx *ctx, double *Cref);
int fh_get_history(fh_ctx *ctx, int load, double *hist, int max, int *count);

/* Step-level entry points (same kernels as fh_solve, for parity checks).
 * All need fh_set_grid and a material; the symbol is (re)built if needed.
 *   q_dev = K u_dev                     (eq. lin_system, matrix-free)
 *   z_dev = M^+ r_dev = F^H K^+ F r     (eq. M_inverse)
 *   b_dev = -D^T W C e                  for the macroscopic strain E (host)
 *   kplus_dev = K^+(xi)/N, [s][kx][ky][kz], kx < nx/2+1, s over the
 *     nd(nd+1)/2 symmetric entries ordered as the Mandel pairs
 *     (00, 11, 22, 12, 02, 01) in 3D, (00, 11, 01) in 2D, (00) scalar.
 *   fh_solve_rhs: PCG for K u = b_dev (b_dev zero-mean), result in u_dev. */
int fh_apply_operator(fh_ctx *ctx, const double *u_dev, double *q_dev);
int fh_apply_preconditioner(fh_ctx *ctx, const double *r_dev, double *z_dev);
int fh_compute_rhs(fh_ctx *ctx, const double *E, double *b_dev);
int fh_get_symbol(fh_ctx *ctx, double *kplus_dev);
int fh_solve_rhs(fh_ctx *ctx, const double *b_dev, double *u_dev, const fh_opts *opt,
                 fh_stats *st);

/* Same result as fh_compute_rhs, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the element-force tables are staged in a static device
 * array of 6144 doubles (48 KiB) that the library holds on every device it
 * runs on until the process ends; no hipMalloc, hipFree or allocating
 * routine is called.  Needs the same set-up as fh_compute_rhs (grid and
 * material).  FH_EINVAL if the tables (material tables x corners x
 * components) would exceed the array -- impossible within fh_set_phases'
 * limits.  All contexts on one device share the array: calls that overlap in
 * time on one device (other threads, other streams) race and must be
 * serialised by the caller.  The call synchronises the context's stream.  */
int fh_compute_rhs_noalloc(fh_ctx *ctx, const double *E, double *b_dev);

/* ----------------------------------------- eigenvalue bounds (Sec. 4.3)
 * Guaranteed two-sided bounds on the eigenvalues of the preconditioned
 * operator Kref^+ K.  For every node I, lambda_I^L (lambda_I^U) is the
 * smallest (largest) generalized eigenvalue of the pair (C, Cref) over the
 * quadrature points in the support of the node's basis function; with
 * materials constant per pixel/voxel that is the min (max) over the 2^dim
 * pixels/voxels that have I as a corner.  Counting every nodal bound nd
 * times and sorting the two lists gives bounds on all eigenvalues of
 * Kref^+ K; kappa = lambda_max / lambda_min bounds its condition number
 * (Sec. 4.3), and ceil(sqrt(kappa)/2 ln(2/eta)) bounds the PCG iterations
 * to reduce the energy-norm error by eta (classical CG estimate).         */
typedef struct fh_bounds {
  double lambda_min;        /* min over nodes of lambda_I^L                  */
  double lambda_max;        /* max over nodes of lambda_I^U                  */
  double kappa;             /* lambda_max / lambda_min                       */
  int predicted_iterations; /* ceil(sqrt(kappa)/2 ln(2/eta)) (0 if eta bad)  */
  int pad;
} fh_bounds;

/* Cref: d_m x d_m (or d x d) reference, or NULL for the context's reference
 * (the one given to fh_set_reference, else the quadrature-weighted mean of
 * Sec. 6.2).  lo_dev / hi_dev: device arrays of N doubles (node order of the
 * grid) that receive lambda_I^L and lambda_I^U, or NULL.  Needs a grid and
 * a material.  FH_ENOTSPD if Cref is not SPD.                              */
int fh_eigen_bounds(fh_ctx *ctx, const double *Cref, double eta, double *lo_dev,
                    double *hi_dev, fh_bounds *out);

/* Reference material choice by the bound on the condition number (Sec. 4.3,
 * Sec. 6.2): FH_REF_MEAN = quadrature-weighted mean, FH_REF_IDENTITY = I_s
 * (the identity in Mandel / scalar notation), FH_REF_BEST = the candidate
 * with the smallest kappa among the mean, I_s and, for 3D elasticity with
 * isotropic phases, the isotropic reference whose bulk-to-shear ratio
 * minimises kappa (its shear modulus is the mean's).  The choice becomes
 * the context's reference (as fh_set_reference); Cref_out (d_m x d_m, may
 * be NULL) receives it, out (may be NULL) its bounds
 * (predicted_iterations = 0).                                              */
#define FH_REF_MEAN 0
#define FH_REF_IDENTITY 1
#define FH_REF_BEST 2
int fh_choose_reference(fh_ctx *ctx, int strategy, double *Cref_out, fh_bounds *out);

/* ------------------------------- elasto-plastic Newton loop (Alg. 1)
 * Nonlinear equilibrium D^T W sigma(e + D u) = 0 (Sec. 3, eq.
 * non_lin_system) for 3D hex8 elasticity with small-strain von Mises
 * plasticity and linear isotropic hardening per phase (the small-strain
 * counterpart of the Sec. 6.3 material): bulk modulus K, shear modulus G,
 * initial yield stress sy0, hardening modulus H (yield stress sy0 + H alpha,
 * alpha the equivalent plastic strain).  The stress update is the radial
 * return with its consistent tangent (Simo & Hughes, Sec. 3.3); internal
 * variables (plastic strain, alpha) live at the 8 Gauss points of every
 * voxel and are committed at the end of each load increment.
 *
 * Newton step i (Alg. 1, eq. lin_system): b = -D^T W sigma(e + D u_(i)),
 * K_(i) = D^T W C_(i) D with the per-point tangent C_(i); the preconditioner
 * is re-assembled (Alg. 2) every step from the quadrature-weighted mean of
 * C_(i) (FH_NEWTON_REF_TANGENT) or once from the mean elastic stiffness
 * (FH_NEWTON_REF_ELASTIC); PCG to eta_cg (Sec. 6 relative Kref^-1-norm);
 * u_(i+1) = u_(i) + du; stop when ||du|| <= eta_newton ||u_(i+1)||.  A
 * residual whose 2-norm is at most 1e-12 of the 2-norm of the element forces
 * it sums is rounding noise (a uniform stress) and ends the loop without a
 * step.  Increment k applies e = (k / nincrement) E_final and starts from
 * the previous increment's u.                                             */
#define FH_MAX_INCREMENTS 64
#define FH_MAX_NEWTON 64
#define FH_NEWTON_REF_TANGENT 0
#define FH_NEWTON_REF_ELASTIC 1

typedef struct fh_newton_opts {
  double eta_newton; /* Newton tolerance on ||du|| / ||u||                 */
  double eta_cg;     /* PCG tolerance per Newton step                      */
  int itmax_newton;  /* Newton steps per increment (<= FH_MAX_NEWTON)      */
  int itmax_cg;      /* PCG iterations per Newton step                     */
  int nincrement;    /* load increments (<= FH_MAX_INCREMENTS)              */
  int ref_mode;      /* FH_NEWTON_REF_TANGENT or FH_NEWTON_REF_ELASTIC      */
} fh_newton_opts;

typedef struct fh_newton_stats {
  int nincrement;
  int newton_steps[FH_MAX_INCREMENTS];   /* steps taken per increment          */
  int converged[FH_MAX_INCREMENTS];      /* 1 if the Newton test was met        */
  int pcg_iterations[FH_MAX_INCREMENTS][FH_MAX_NEWTON];
  double du_ratio[FH_MAX_INCREMENTS][FH_MAX_NEWTON]; /* ||du|| / ||u_(i+1)|| */
  double macro_stress[FH_MAX_INCREMENTS][6]; /* (1/|Y|) sum_Q w_Q sigma_Q,
                                                Mandel, at the converged u */
  double plastic_fraction[FH_MAX_INCREMENTS]; /* share of yielding points   */
  int total_pcg;                         /* PCG iterations of all steps        */
  double solve_ms;
} fh_newton_stats;

/* phase_dev: uint8 N_p grid (device, [z][y][x]), read by every later call;
 * params: nphase x {K, G, sy0, H} (host, copied), K, G, H > 0, sy0 >= 0.
 * Sets the phases' elastic stiffnesses as fh_set_phases does (so the linear
 * entry points keep working) and allocates the per-point state: about
 * 1.1 kB per voxel, library-owned, freed by fh_set_grid, fh_set_phases,
 * fh_set_conductivity_field or fh_destroy.  Needs a 3D FH_HEX8 FH_ELASTIC
 * grid.                                                                    */
int fh_set_plastic_phases(fh_ctx *ctx, const uint8_t *phase_dev, int nphase,
                          const double *params);
/* E_final: 6 Mandel components (host).  opt NULL = {1e-8, 1e-10, 50, 10000,
 * 1, FH_NEWTON_REF_TANGENT}.  Starts from u = 0 and a virgin state.
 * Returns FH_OK, FH_NOT_CONVERGED (an increment hit itmax_newton or a step
 * hit itmax_cg; the state is still committed and the loop continues),
 * FH_ENOTSPD (PCG breakdown), FH_EINVAL / FH_ESTATE.  The caller's
 * fh_set_reference choice is restored afterwards.                         */
int fh_newton_solve(fh_ctx *ctx, const double *E_final, const fh_newton_opts *opt,
                    fh_newton_stats *st);
/* Device copies (any may be NULL): u_dev 3 x N ([comp][z][y][x]), eps_p_dev
 * 6 x 8 x N ([Mandel comp][Gauss point][voxel]), alpha_dev 8 x N; Gauss
 * point q = qx + 2 qy + 4 qz at reference coordinates 1/2 -+ 1/(2 sqrt 3).  */
int fh_get_plastic_state(fh_ctx *ctx, double *u_dev, double *eps_p_dev, double *alpha_dev);

/* ---------------- strain-based scheme with the FE projection (Sec. 7.1)
 * The same linear problem as fh_solve, solved with the strain field at the
 * Gauss points as the unknown (eq. projection_chceme): CG on
 * Gamma0 C eps = -Gamma0 C e, Gamma0 = D (D^T W Cref D)^+ D^T W, with the
 * pseudo-inverse applied by the displacement scheme's FFT preconditioner
 * (same Cref, symbol and zero-frequency rule).  CG runs in the inner
 * product <a, b> = sum_Q w_Q a_Q^T Cref b_Q and stops when
 * sqrt(<r, r> / <r0, r0>) <= eta; since r = D z for the displacement
 * scheme's preconditioned residual z, this is the Sec. 6 stopping test and
 * the iterates are eps_k = D u_k (the paper's equivalence).  3D hex8
 * elasticity with a phase field; every load case of fh_set_load, one after
 * another, FP64 (opt->precision must be FH_FP64; flags and guess are
 * ignored).  Afterwards fh_get_homogenized returns the energy-form C_hom of
 * the strain fields, fh_get_history the residual history of each load, and
 * fh_stats the iterations.  Library-owned device memory: (nload + 3) x 48 N
 * + 24 N doubles, kept until the grid changes or the context is destroyed. */
int fh_solve_strain_based(fh_ctx *ctx, const fh_opts *opt, fh_stats *st);
/* eps_dev: 6 x 8 x N doubles (device): strain fluctuation D u of load
 * `load` at the Gauss points, [Mandel comp][Gauss point q = qx + 2 qy +
 * 4 qz][voxel].  FH_ESTATE before fh_solve_strain_based (or after a later
 * fh_solve).                                                               */
int fh_get_strain(fh_ctx *ctx, int load, double *eps_dev);

/* ------------------------------------------------------------ batches
 * Many independent microstructures (possibly of different grid sizes), each
 * solved for the same nload macroscopic strains.  Systems are grouped by grid
 * size; within a group every stage of an iteration is one launch over all
 * microstructures x load cases, one PCG iteration is captured in a hipGraph
 * and replayed, and the launch shapes (operator z-chunk, FFT lines per block)
 * are chosen per grid size by timing candidates on the group's own data.
 * Every microstructure gets its own mean reference material and Alg. 2
 * symbol.  Phases must be isotropic (C = lambda 1(x)1 + 2 mu I, Mandel).  */
typedef struct fh_system {
  const uint8_t *phase_dev; /* n0*n1*n2 bytes on the device                  */
  int n[3];                 /* 3D grid, sizes as for fh_set_grid             */
  int nphase;               /* 1..16                                         */
  const double *mat;        /* nphase x 6 x 6 Mandel stiffness tables (host)  */
  double *u_dev;            /* optional output (device, nload x 3 x N doubles):
                               the fluctuation fields of this system           */
} fh_system;

#define FH_MAX_GROUPS 16
typedef struct fh_batch_report {
  int ngroups;
  int n[FH_MAX_GROUPS][3];
  int nsys[FH_MAX_GROUPS];
  int kz[FH_MAX_GROUPS], zb[FH_MAX_GROUPS], kyb[FH_MAX_GROUPS]; /* tuned shapes */
  double tune_ms[FH_MAX_GROUPS], setup_ms[FH_MAX_GROUPS], solve_ms[FH_MAX_GROUPS];
  int xrows[FH_MAX_GROUPS]; /* tuned rows per block of the FP32 x passes     */
} fh_batch_report;

/* Solve nsys systems (elasticity, FH_HEX8) for the nload strains E (host,
 * nload x 6 Mandel, nload <= 8).  chom (host, nsys x nload x nload) receives
 * each system's homogenized tensor in energy form; st (may be NULL) one
 * fh_stats per system; rep (may be NULL) the per-group tuning and timings.
 * opt as for fh_solve (FH_FP32_REFINED recommended).  At most FH_MAX_GROUPS
 * distinct grid sizes.  With a workspace bound to ctx (fh_bind_workspace) of
 * at least fh_batch_workspace_size bytes, the groups take their fields,
 * spectra and K^+ from it (disjoint regions, overwritten by the call);
 * otherwise they allocate them.  A bound workspace that is too small is
 * FH_ENOMEM.  Small per-group tables (packed phases, twiddles, material
 * tables) are allocated inside the call either way.                       */
int fh_solve_batch(fh_ctx *ctx, int nsys, const fh_system *sys, int nload, const double *E,
                   const fh_opts *opt, double *chom, fh_stats *st, fh_batch_report *rep);

/* Device bytes fh_solve_batch takes from a bound workspace for these
 * systems and nload load cases (arguments as for fh_solve_batch).          */
int fh_batch_workspace_size(fh_ctx *ctx, int nsys, const fh_system *sys, int nload,
                            size_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* FH_H */
