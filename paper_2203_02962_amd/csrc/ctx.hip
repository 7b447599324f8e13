// Host side of the C-ABI: context, setup (reference material, Alg. 2 symbol,
// right-hand sides), the PCG driver and the homogenized tensor.
//
// Setup follows the paper: Cref defaults to the quadrature-weighted mean of
// the material (Sec. 6.2); K^ comes from Alg. 2 -- the operator kernel is
// applied to the nd unit impulses with the uniform reference material and the
// responses are transformed with the forward FFT passes -- and every block is
// inverted (zero block at zero frequency, eq. block_inversion).  The PCG loop
// (Sec. 4.1, Alg. 1 with a linear material) runs entirely on the device; the
// host only enqueues iterations and polls the per-load status every `poll`
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <condition_variable>
#include <mutex>
#include <thread>

#include "../../include/fh.h"
#include "fh_internal.h"

using fh::cplx;

// Staging for fh_compute_rhs_noalloc: the element forces of the uniform
// strain, one table per material table (at most 256 tables x 8 corners x 3
// components).  Every device holds its own copy for the life of the process.
// In host code the array's name is not a device address: the address of the
// current device's copy comes from hipGetSymbolAddress (scratch_ptr below).
constexpr int kRhsScratchDoubles = 256 * 8 * 3;
static __device__ __align__(256) double scratch[kRhsScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.  Returns null if the lookup fails.
double* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_dev[device] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[device];
}
}  // namespace

// chunks of the load-pair dot products behind C_hom, and of the one-dot-per-
// system reductions (refinement norms, warm-start screen)
constexpr int kPairChunks = 1024;
constexpr int kSysChunks = 512;

struct fh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  bool has_grid = false;
  fh::Grid g{};
  int problem = FH_SCALAR, element = FH_HEX8;
  double l[3] = {1, 1, 1};
  fh::AxisPlan px{}, py{}, pz{};
  cplx<double>* twx = nullptr;
  cplx<double>* twy = nullptr;
  cplx<double>* twz = nullptr;

  int mat_kind = 0;  // 0 none, 1 phases, 2 conductivity field
  bool phases_checked = false;
  const uint8_t* phase_dev = nullptr;
  const double* kfield_dev = nullptr;
  int nphase = 0;
  std::vector<double> mat;  // nphase * m * m

  bool cref_user = false;
  std::vector<double> cref_in, cref;  // m * m

  int nload = 0;
  std::vector<double> loads;  // nload * m

  void* ws_user = nullptr;
  size_t ws_user_bytes = 0;
  void* ws_own = nullptr;
  size_t ws_own_bytes = 0;

  // small device tables (library-owned)
  double* mat_dev = nullptr;   // K operator tables (double)
  float* mat_dev_f = nullptr;  // float copy
  double* ref_dev = nullptr;   // Kref operator tables
  double* fe_dev = nullptr;    // RHS element forces
  size_t mat_dev_n = 0, ref_dev_n = 0, fe_dev_n = 0;
  // isotropic hex8 elasticity: {V lambda, 2 V mu} per phase (and for Cref)
  bool iso = false, ref_iso = false;
  // scalar hex8 with isotropic conductivity: V k per phase (a field: {V})
  bool sc = false, ref_sc = false;
  double* sk_dev = nullptr;
  float* sk_dev_f = nullptr;
  double* ref_sk_dev = nullptr;
  size_t sk_dev_n = 0, ref_sk_dev_n = 0;
  double* lm_dev = nullptr;
  double* bound_tab_dev = nullptr;  // eigenvalue pairs per material table (Sec. 4.3)
  size_t bound_tab_n = 0;
  // elasto-plastic Newton loop (fh_set_plastic_phases, fh_newton_solve):
  // per-phase {K, G, sy0, H}; per-point committed state and tangent; the
  // element forces of the material stage; the displacement of the loop
  bool plastic = false;
  bool qp_tangent = false;  // apply_K uses the per-point tangent
  std::vector<double> pl_params;
  double* pl_params_dev = nullptr;
  double *pl_eps_p = nullptr, *pl_alpha = nullptr, *pl_ta = nullptr, *pl_tv = nullptr;
  double *pl_fe = nullptr, *pl_u = nullptr, *pl_part = nullptr;
  // strain-based scheme (fh_solve_strain_based): strain fields of every load
  // case, CG vectors, element forces, raw Mandel tables; library-owned
  double *sb_eps = nullptr, *sb_r = nullptr, *sb_p = nullptr, *sb_q = nullptr;
  double *sb_fe = nullptr, *sb_C = nullptr;
  int sb_nload = 0;
  bool sb_solved = false;
  int pl_nb = 0;   // blocks of the material-stage launches
  int pl_nbg = 0;  // blocks of the node gather (p.q partials)
  float* lm_dev_f = nullptr;
  double* ref_lm_dev = nullptr;
  size_t lm_dev_n = 0, ref_lm_dev_n = 0;
  unsigned long long* counts_dev = nullptr;
  int* flag_dev = nullptr;
  double* host_pinned = nullptr;  // pinned staging
  size_t host_pinned_n = 0;

  // workspace carve (set by bind_layout)
  struct Layout {
    size_t bytes = 0;
    double *x, *r, *p, *q, *b;
    cplx<double> *A, *B, *spec;
    double* kplus;
    float* kplus_f;
    float *x32, *r32, *p32, *q32;
    float* kf32;  // float copy of a per-voxel conductivity
    cplx<float> *A32, *B32;
    double *d64;  // refinement: correction accumulator
    fh::PcgState* st;
    double *pq_part, *rz_part, *hist, *dot_part, *scal;
    double *sysdot, *sysdot_part;  // one dot per system (refinement norms)
    double* pair_part;             // load-pair dot partials + results (C_hom)
    int* mask;                     // per-system flags
    uint8_t* phase0;
    int nb_kop, nb_z, nb_z32, hist_len;
  } L{};
  bool layout_ok = false;
  int layout_nload = -1;

  // live kernel timing (FH_FLAG_TIME_KERNELS): event pairs recorded on the
  // solve stream around each launch, read back at every poll
  struct KTimer {
    bool on = false;
    int period = 1;      // time every period-th PCG iteration
    bool sample = true;  // the current iteration is timed
    std::vector<hipEvent_t> ev;  // 2 per slot
    std::vector<int> cls;
    size_t used = 0;
    double ms[FH_K_NCLASS] = {};
    long long n[FH_K_NCLASS] = {};       // timed launches
    long long issued[FH_K_NCLASS] = {};  // all launches while on
    // load-case units of the timed launches: the PCG loop index of every
    // timed launch of the current pcg_run, resolved to the number of load
    // cases still iterating once their final counts are known
    int cur_iter = 0;
    std::vector<std::pair<int, int>> timed_iters;  // (class, loop index)
    double units[FH_K_NCLASS] = {};
  } kt;

  // batched solves: nms microstructures of this grid, G = loads each
  int nms = 1;
  bool use_graph = false;
  bool own_stream = false;
  // single solves: one PCG iteration replayed from a hipGraph on a private
  // stream (the caller's stream may be the null stream, which cannot be
  // captured), forked from and joined back to `stream` with the two events
  bool graph = false;  // FH_FLAG_GRAPH of the current solve
  hipStream_t gstream = nullptr;
  hipEvent_t gfork = nullptr, gjoin = nullptr;
  uint8_t* phase_pack = nullptr;
  std::vector<std::vector<double>> cmean_ms;
  std::vector<unsigned long long> phase_counts;  // voxels per phase (compute_mean)

  bool symbol_ok = false;
  bool rhs_ok = false;
  bool solved = false;
  std::vector<double> chom;
  std::vector<double> cmean;
  std::vector<std::vector<double>> history;
  fh_stats last{};
  fh_net* net = nullptr;  // learned warm start (fh_set_warm_start)
};

namespace {

int fail(fh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                           \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess)                                                           \
      return fail(ctx, FH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// stored K^+ entries per frequency: the unique entries of a real symmetric
// block, or 4 reals of the Hermitian two-node block
int nsym_of(const fh::Grid& g) { return g.tn ? 4 : g.nd * (g.nd + 1) / 2; }

int mdim(const fh_ctx* c) {
  const int d = c->g.dim;
  return c->problem == FH_ELASTIC ? d * (d + 1) / 2 : d;
}

bool factor_ok(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

fh::AxisPlan make_plan(int n) {
  fh::AxisPlan p{};
  p.n = n;
  int m = n;
  auto push = [&](unsigned r) { p.code |= r << (4 * p.nstage); ++p.nstage; };
  while (m % 8 == 0) { push(8); m /= 8; }
  while (m % 4 == 0) { push(4); m /= 4; }
  while (m % 2 == 0) { push(2); m /= 2; }
  while (m % 3 == 0) { push(3); m /= 3; }
  return p;
}

// exp(-2 pi i k / n) with the angle reduced to [0, pi/4] by symmetry and
// evaluated in long double.
std::vector<cplx<double>> twiddle_table(int n) {
  std::vector<cplx<double>> t(n);
  for (int k = 0; k < n; ++k) {
    // angle = 2 pi k / n, use exact integer reduction modulo n
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k /
                          (long double)n;
    t[k].re = (double)cosl(a);
    t[k].im = (double)(-sinl(a));
    // exact values at multiples of quarter turns
    if ((4LL * k) % n == 0) {
      const int q = (int)((4LL * k) / n) % 4;
      const double cs[4] = {1, 0, -1, 0}, sn[4] = {0, 1, 0, -1};
      t[k].re = cs[q];
      t[k].im = -sn[q];
    }
  }
  return t;
}

// ---------------------------------------------------- element definitions
// Reference stencils of the paper's Fig. tiling (one-node, N_n = 1):
//   hex8 / quad4: corners a with bit k = offset along axis k, Gauss points
//   1/2 -+ 1/(2 sqrt 3) per axis, weights V_p/2^d;
//   tri2: pixel split along (0,0)-(1,1), centroid points, weights V_p/2.
struct ElemDef {
  int dim, nc, nq;
  std::vector<double> grad;  // [q][a][k] reference gradients
  std::vector<double> wfrac;
};

ElemDef make_element(int element) {
  ElemDef e{};
  if (element == FH_TRI4) {
    // corners 0..3 (bit 0 = x, bit 1 = y offset), centre 4; triangles on the
    // bottom, right, top and left pixel edges, each with the centre
    e.dim = 2; e.nc = 5; e.nq = 4;
    e.grad.assign(4 * 5 * 2, 0.0);
    auto G = [&](int q, int a, double gx, double gy) {
      e.grad[(q * 5 + a) * 2 + 0] = gx;
      e.grad[(q * 5 + a) * 2 + 1] = gy;
    };
    G(0, 0, -1, -1); G(0, 1, 1, -1); G(0, 4, 0, 2);   // bottom: 1-x-y, x-y, 2y
    G(1, 1, 1, -1);  G(1, 3, 1, 1);  G(1, 4, -2, 0);  // right: x-y, x+y-1, 2-2x
    G(2, 3, 1, 1);   G(2, 2, -1, 1); G(2, 4, 0, -2);  // top: x+y-1, y-x, 2-2y
    G(3, 2, -1, 1);  G(3, 0, -1, -1); G(3, 4, 2, 0);  // left: y-x, 1-x-y, 2x
    e.wfrac = {0.25, 0.25, 0.25, 0.25};
    return e;
  }
  if (element == FH_TRI2) {
    e.dim = 2; e.nc = 4; e.nq = 2;
    e.grad.assign(2 * 4 * 2, 0.0);
    auto G = [&](int q, int a, double gx, double gy) {
      e.grad[(q * 4 + a) * 2 + 0] = gx;
      e.grad[(q * 4 + a) * 2 + 1] = gy;
    };
    // lower triangle (0,0),(1,0),(1,1): lambda = 1-x, x-y, y
    G(0, 0, -1, 0); G(0, 1, 1, -1); G(0, 3, 0, 1);
    // upper triangle (0,0),(1,1),(0,1): lambda = 1-y, x, y-x
    G(1, 0, 0, -1); G(1, 3, 1, 0); G(1, 2, -1, 1);
    e.wfrac = {0.5, 0.5};
    return e;
  }
  const int dim = element == FH_HEX8 ? 3 : 2;
  e.dim = dim; e.nc = 1 << dim; e.nq = 1 << dim;
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  e.grad.assign((size_t)e.nq * e.nc * dim, 0.0);
  for (int q = 0; q < e.nq; ++q) {
    double xi[3];
    for (int k = 0; k < dim; ++k) xi[k] = gp[(q >> k) & 1];
    for (int a = 0; a < e.nc; ++a)
      for (int k = 0; k < dim; ++k) {
        double v = ((a >> k) & 1) ? 1.0 : -1.0;
        for (int j = 0; j < dim; ++j)
          if (j != k) v *= ((a >> j) & 1) ? xi[j] : 1.0 - xi[j];
        e.grad[((size_t)q * e.nc + a) * dim + k] = v;
      }
  }
  e.wfrac.assign(e.nq, 1.0 / e.nq);
  return e;
}

// strain row m receives coef * d u_alpha / d x_beta (Mandel, eq. mandel_grad)
struct GradRow { int m, alpha, beta; double coef; };
std::vector<GradRow> grad_rows(int problem, int dim) {
  const double s = std::sqrt(0.5);
  if (problem == FH_SCALAR) {
    std::vector<GradRow> r;
    for (int b = 0; b < dim; ++b) r.push_back({b, 0, b, 1.0});
    return r;
  }
  if (dim == 2) return {{0, 0, 0, 1}, {1, 1, 1, 1}, {2, 0, 1, s}, {2, 1, 0, s}};
  return {{0, 0, 0, 1}, {1, 1, 1, 1}, {2, 2, 2, 1}, {3, 1, 2, s}, {3, 2, 1, s},
          {4, 0, 2, s}, {4, 2, 0, s}, {5, 0, 1, s}, {5, 1, 0, s}};
}

// degrees of freedom per node (the two-node stencil's fields are node sets)
int pnd(const fh_ctx* c) { return c->problem == FH_ELASTIC ? c->g.dim : 1; }

// B_q (m x nc*nd) in physical coordinates
std::vector<double> bmat(const fh_ctx* c, const ElemDef& e, int q) {
  const int m = mdim(c), nd = pnd(c), nk = e.nc * nd;
  std::vector<double> B((size_t)m * nk, 0.0);
  for (const GradRow& r : grad_rows(c->problem, e.dim))
    for (int a = 0; a < e.nc; ++a)
      B[(size_t)r.m * nk + a * nd + r.alpha] +=
          r.coef * e.grad[((size_t)q * e.nc + a) * e.dim + r.beta] / c->g.h[r.beta];
  return B;
}

double voxel_volume(const fh_ctx* c) {
  double v = 1.0;
  for (int k = 0; k < c->g.dim; ++k) v *= c->g.h[k];
  return v;
}

// K_e = sum_q w_q B_q^T C B_q
std::vector<double> element_matrix(const fh_ctx* c, const double* C) {
  const ElemDef e = make_element(c->element);
  const int m = mdim(c), nk = e.nc * pnd(c);
  const double Vp = voxel_volume(c);
  std::vector<double> K((size_t)nk * nk, 0.0);
  for (int q = 0; q < e.nq; ++q) {
    const std::vector<double> B = bmat(c, e, q);
    const double w = e.wfrac[q] * Vp;
    std::vector<double> CB((size_t)m * nk, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < nk; ++j) {
        double s = 0;
        for (int k = 0; k < m; ++k) s += C[i * m + k] * B[(size_t)k * nk + j];
        CB[(size_t)i * nk + j] = s;
      }
    for (int i = 0; i < nk; ++i)
      for (int j = 0; j < nk; ++j) {
        double s = 0;
        for (int k = 0; k < m; ++k) s += B[(size_t)k * nk + i] * CB[(size_t)k * nk + j];
        K[(size_t)i * nk + j] += w * s;
      }
  }
  return K;
}

// Element force of a uniform strain: f = (int_e B dx)^T (C E); the integral
// of every shape-function derivative over a pixel is +-V_p / (2^(d-1) h_beta)
// for all three stencils (divergence theorem), so antipodal corners get
// exactly opposite forces.
std::vector<double> uniform_strain_force(const fh_ctx* c, const double* C, const double* E) {
  if (c->element == FH_TRI4) {
    // f = sum_q w_q B_q^T (C E)
    const ElemDef el = make_element(FH_TRI4);
    const int m = mdim(c), nk = el.nc * pnd(c);
    std::vector<double> sig(m, 0.0), f(nk, 0.0);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) sig[i] += C[i * m + k] * E[k];
    for (int q = 0; q < el.nq; ++q) {
      const std::vector<double> B = bmat(c, el, q);
      const double w = el.wfrac[q] * voxel_volume(c);
      for (int j = 0; j < nk; ++j)
        for (int i = 0; i < m; ++i) f[j] += w * B[(size_t)i * nk + j] * sig[i];
    }
    return f;
  }
  const int m = mdim(c), nd = c->g.nd, dim = c->g.dim, nc = 1 << dim;
  const double Vp = voxel_volume(c);
  std::vector<double> sig(m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) sig[i] += C[i * m + k] * E[k];
  std::vector<double> f((size_t)nc * nd, 0.0);
  const double scale = Vp / (double)(1 << (dim - 1));
  for (int a = 0; a < nc; ++a) {
    for (const GradRow& r : grad_rows(c->problem, dim)) {
      const double g = (((a >> r.beta) & 1) ? 1.0 : -1.0) * scale / c->g.h[r.beta];
      f[(size_t)a * nd + r.alpha] += r.coef * g * sig[r.m];
    }
  }
  return f;
}

bool cholesky_ok(const std::vector<double>& A, int m) {
  std::vector<double> L(A);
  for (int j = 0; j < m; ++j) {
    double d = L[j * m + j];
    for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = L[i * m + j];
      for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = s / d;
    }
  }
  return true;
}

bool hex_elastic(const fh_ctx* c) { return c->element == FH_HEX8 && c->problem == FH_ELASTIC; }
bool hex_scalar(const fh_ctx* c) {
  return c->element == FH_HEX8 && c->problem == FH_SCALAR && c->g.dim == 3;
}
// the material operator runs the tiled z-march kernels (elastic, or scalar
// with isotropic conductivity): their partial-sum count differs
bool hex_tiled(const fh_ctx* c) { return hex_elastic(c) || (hex_scalar(c) && c->sc); }
// A = k I (d x d): returns k, or -1
double isotropic_k(const double* A, int d) {
  double mx = 0.0;
  for (int i = 0; i < d * d; ++i) mx = std::max(mx, std::fabs(A[i]));
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double v = A[i * d + j];
      if (i != j && std::fabs(v) > 1e-14 * mx) return -1.0;
      if (i == j && std::fabs(v - A[0]) > 1e-14 * mx) return -1.0;
    }
  return A[0] > 0.0 ? A[0] : -1.0;
}

void free_plastic(fh_ctx* c) {
  for (double** p : {&c->pl_params_dev, &c->pl_eps_p, &c->pl_alpha, &c->pl_ta, &c->pl_tv,
                     &c->pl_fe, &c->pl_u, &c->pl_part}) {
    hipFree(*p);
    *p = nullptr;
  }
  c->plastic = false;
  c->qp_tangent = false;
  c->pl_params.clear();
}

void free_sb(fh_ctx* c) {
  for (double** p : {&c->sb_eps, &c->sb_r, &c->sb_p, &c->sb_q, &c->sb_fe, &c->sb_C}) {
    hipFree(*p);
    *p = nullptr;
  }
  c->sb_nload = 0;
  c->sb_solved = false;
}

void free_tables(fh_ctx* c) {
  hipFree(c->lm_dev); c->lm_dev = nullptr;
  hipFree(c->lm_dev_f); c->lm_dev_f = nullptr;
  hipFree(c->ref_lm_dev); c->ref_lm_dev = nullptr;
  hipFree(c->sk_dev); c->sk_dev = nullptr;
  hipFree(c->sk_dev_f); c->sk_dev_f = nullptr;
  hipFree(c->ref_sk_dev); c->ref_sk_dev = nullptr;
  c->sk_dev_n = c->ref_sk_dev_n = 0;
  c->sc = c->ref_sc = false;
  c->lm_dev_n = c->ref_lm_dev_n = 0;
  c->iso = c->ref_iso = false;
  hipFree(c->mat_dev); c->mat_dev = nullptr;
  hipFree(c->mat_dev_f); c->mat_dev_f = nullptr;
  hipFree(c->ref_dev); c->ref_dev = nullptr;
  hipFree(c->fe_dev); c->fe_dev = nullptr;
  c->mat_dev_n = c->ref_dev_n = c->fe_dev_n = 0;
}

// Operator tables: hex8 elastic -> V_p * C per phase (36); otherwise the
// element matrices per phase (or the unit-conductivity matrix for a field).
std::vector<double> operator_tables(const fh_ctx* c, const double* mats, int count) {
  const int m = mdim(c);
  std::vector<double> out;
  if (hex_elastic(c)) {
    const double Vp = voxel_volume(c);
    for (int p = 0; p < count; ++p)
      for (int i = 0; i < 36; ++i) out.push_back(Vp * mats[(size_t)p * m * m + i]);
    return out;
  }
  for (int p = 0; p < count; ++p) {
    std::vector<double> K = element_matrix(c, mats + (size_t)p * m * m);
    out.insert(out.end(), K.begin(), K.end());
  }
  return out;
}

// Isotropic Mandel stiffness C = lambda 1(x)1 + 2 mu I?  Returns
// {V lambda, 2 V mu} in lm when it is (to 1e-13 of the largest entry).
bool isotropic_lm(const double* C, double Vp, double lm[2]) {
  double mx = 0;
  for (int i = 0; i < 36; ++i) mx = std::max(mx, std::fabs(C[i]));
  const double lam = C[0 * 6 + 1], mu2 = C[3 * 6 + 3];
  const double tol = 1e-13 * mx;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double want = 0.0;
      if (i < 3 && j < 3) want = lam + (i == j ? mu2 : 0.0);
      else if (i == j) want = mu2;
      if (std::fabs(C[i * 6 + j] - want) > tol) return false;
    }
  lm[0] = Vp * lam;
  lm[1] = Vp * mu2;
  return true;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Compute the workspace layout (offsets relative to base; base may be null
// for sizing).
size_t layout(fh_ctx* c, char* base, fh_ctx::Layout* Lout) {
  fh_ctx::Layout L{};
  const fh::Grid& g = c->g;
  const int nl = std::max(1, c->nload);
  const long long F = (long long)g.nd * g.N;
  const long long S = (long long)g.nd * g.nxh * g.ny * g.nz;
  const long long nfreq = (long long)g.nxh * g.ny * g.nz;
  const int nsym = nsym_of(g);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  L.x = (double*)take(sizeof(double) * F * nl);
  L.r = (double*)take(sizeof(double) * F * nl);
  L.p = (double*)take(sizeof(double) * F * nl);
  L.q = (double*)take(sizeof(double) * F * nl);
  L.b = (double*)take(sizeof(double) * F * nl);
  L.A = (cplx<double>*)take(sizeof(cplx<double>) * S * nl);
  L.B = (cplx<double>*)take(sizeof(cplx<double>) * S * nl);
  L.spec = (cplx<double>*)take(sizeof(cplx<double>) * S * g.nd);
  L.kplus = (double*)take(sizeof(double) * nfreq * nsym * c->nms);
  L.kplus_f = (float*)take(sizeof(float) * nfreq * nsym * c->nms);
  L.x32 = (float*)take(sizeof(float) * F * nl);
  L.r32 = (float*)take(sizeof(float) * F * nl);
  L.p32 = (float*)take(sizeof(float) * F * nl);
  L.q32 = (float*)take(sizeof(float) * F * nl);
  L.A32 = (cplx<float>*)take(sizeof(cplx<float>) * S * nl);
  L.B32 = (cplx<float>*)take(sizeof(cplx<float>) * S * nl);
  L.d64 = (double*)take(sizeof(double) * F * nl);
  L.kf32 = (float*)take(sizeof(float) * (size_t)g.N);
  L.st = (fh::PcgState*)take(sizeof(fh::PcgState) * nl);
  {
    // partial sums sized for the smallest launch shapes the tuner may pick
    fh::Grid gw = g;
    gw.kz = 4;
    gw.kyb = 1;
    L.nb_kop = std::max(fh::kop_nblocks(gw, true), fh::kop_nblocks(gw, false));
    L.nb_z = fh::zpass_nblocks<double>(gw);
    L.nb_z32 = fh::zpass_nblocks<float>(gw);
  }
  const int nbz = std::max(L.nb_z, L.nb_z32);
  L.pq_part = (double*)take(sizeof(double) * (size_t)L.nb_kop * nl);
  L.rz_part = (double*)take(sizeof(double) * (size_t)nbz * nl);
  L.hist_len = 20000;
  L.hist = (double*)take(sizeof(double) * (size_t)L.hist_len * nl);
  L.dot_part = (double*)take(sizeof(double) * 1024);
  L.scal = (double*)take(sizeof(double) * 64);
  L.sysdot = (double*)take(sizeof(double) * nl);
  L.sysdot_part = (double*)take(sizeof(double) * nl * kSysChunks);
  // load-pair dot partials and results: one solve (kPairChunks chunks) or a
  // batch group (64 chunks per microstructure), up to 8 x 8 pairs each
  L.pair_part = (double*)take(sizeof(double) *
                              std::max<size_t>(kPairChunks * 64 + 128,
                                               (size_t)c->nms * (64 * 64 + 2 * 64)));
  L.mask = (int*)take(sizeof(int) * nl);
  L.phase0 = (uint8_t*)take((size_t)g.N);
  L.bytes = off;
  if (Lout) *Lout = L;
  return off;
}

int ensure_layout(fh_ctx* c) {
  if (c->layout_ok && c->layout_nload == c->nload) return FH_OK;
  size_t need = layout(c, nullptr, nullptr);
  char* base = nullptr;
  if (c->ws_user) {
    if (c->ws_user_bytes < need)
      return fail(c, FH_ENOMEM, "bound workspace too small: need " + std::to_string(need) +
                                    " bytes");
    base = (char*)c->ws_user;
  } else {
    if (c->ws_own_bytes < need) {
      hipFree(c->ws_own);
      c->ws_own = nullptr;
      c->ws_own_bytes = 0;
      if (hipMalloc(&c->ws_own, need) != hipSuccess)
        return fail(c, FH_ENOMEM, "hipMalloc of workspace failed (" + std::to_string(need) +
                                      " bytes)");
      c->ws_own_bytes = need;
    }
    base = (char*)c->ws_own;
  }
  layout(c, base, &c->L);
  c->layout_ok = true;
  c->layout_nload = c->nload;
  c->symbol_ok = false;
  c->rhs_ok = false;
  HIPCHK(c, hipMemsetAsync(c->L.phase0, 0, (size_t)c->g.N, c->stream));
  return FH_OK;
}

int ensure_pinned(fh_ctx* c, size_t n) {
  if (c->host_pinned_n >= n) return FH_OK;
  if (c->host_pinned) hipHostFree(c->host_pinned);
  c->host_pinned = nullptr;
  c->host_pinned_n = 0;
  HIPCHK(c, hipHostMalloc((void**)&c->host_pinned, n * sizeof(double), hipHostMallocDefault));
  c->host_pinned_n = n;
  return FH_OK;
}

int upload_f(fh_ctx* c, float** dst, const std::vector<double>& v) {
  hipFree(*dst);
  *dst = nullptr;
  std::vector<float> f(v.begin(), v.end());
  HIPCHK(c, hipMalloc((void**)dst, f.size() * sizeof(float)));
  HIPCHK(c, hipMemcpy(*dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  return FH_OK;
}

int upload(fh_ctx* c, double** dst, size_t* dst_n, const std::vector<double>& v) {
  if (*dst_n < v.size()) {
    hipFree(*dst);
    *dst = nullptr;
    HIPCHK(c, hipMalloc((void**)dst, v.size() * sizeof(double)));
    *dst_n = v.size();
  }
  HIPCHK(c, hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  // the host vector is a temporary of the caller: wait until it is copied
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

// Apply K (or Kref when `ref`) to nload fields (double).
int apply_K(fh_ctx* c, bool ref, const double* u, double* q, int nload, long long stride,
            const fh::PcgState* st, double* pq) {
  fh::Grid g = c->g;
  g.nphase_max = (!ref && c->mat_kind == 1) ? c->nphase : 1;
  const uint8_t* ph = ref ? c->L.phase0 : (c->mat_kind == 1 ? c->phase_dev : nullptr);
  const double* kf = ref ? nullptr : (c->mat_kind == 2 ? c->kfield_dev : nullptr);
  const double* tab = ref ? c->ref_dev : c->mat_dev;
  int nb = 0;
  if (!ref && c->qp_tangent) {
    // per-point tangent of the Newton step (one load case)
    if (nload != 1) return fail(c, FH_EINVAL, "the tangent operator takes one field");
    HIPCHK(c, fh::launch_plastic_stage(1, g, c->phase_dev, c->pl_params_dev, nullptr, u,
                                       c->pl_fe, nullptr, nullptr, c->pl_ta, c->pl_tv, nullptr,
                                       c->pl_nb, c->stream));
    HIPCHK(c, fh::launch_gather_nodes(g, c->pl_fe, 1.0, q, pq ? u : nullptr, pq, c->pl_nbg,
                                      c->stream));
  } else if (c->element == FH_TRI4) {
    if (!ph && !kf) ph = c->L.phase0;
    HIPCHK(c, fh::launch_kop_tn<double>(g, u, q, ph, kf, tab, nload, stride, stride, st, pq, &nb,
                                        c->stream));
  } else if (hex_scalar(c) && (ref ? c->ref_sc : c->sc)) {
    HIPCHK(c, fh::launch_kop_hex8_scalar<double>(g, u, q, kf ? nullptr : (ph ? ph : c->L.phase0),
                                                 kf, ref ? c->ref_sk_dev : c->sk_dev, nload,
                                                 stride, stride, st, pq, &nb, c->stream));
  } else if (hex_elastic(c) && (ref ? c->ref_iso : c->iso)) {
    const double* lm = ref ? c->ref_lm_dev : c->lm_dev;
    HIPCHK(c, fh::launch_kop_hex8_iso<double>(g, u, q, ph, lm, nload, stride, stride, st, pq,
                                              &nb, c->stream));
  } else if (hex_elastic(c)) {
    HIPCHK(c, fh::launch_kop_hex8_elastic<double>(g, u, q, ph, tab, nload, stride, stride, st,
                                                  pq, &nb, c->stream));
  } else {
    if (!ph && !kf) ph = c->L.phase0;
    HIPCHK(c, fh::launch_kop_generic<double>(g, c->element, u, q, ph, kf, tab, nload, stride,
                                             stride, st, pq, &nb, c->stream));
  }
  return FH_OK;
}

int apply_K32(fh_ctx* c, const float* u, float* q, int nload, long long stride,
              const fh::PcgState* st, double* pq) {
  fh::Grid g = c->g;
  g.nphase_max = c->mat_kind == 1 ? c->nphase : 1;
  const uint8_t* ph = c->mat_kind == 1 ? c->phase_dev : nullptr;
  int nb = 0;
  if (c->element == FH_TRI4) {
    const float* kf = c->mat_kind == 2 ? c->L.kf32 : nullptr;
    HIPCHK(c, fh::launch_kop_tn<float>(g, u, q, kf ? nullptr : ph, kf, c->mat_dev_f, nload,
                                       stride, stride, st, pq, &nb, c->stream));
  } else if (hex_scalar(c) && c->sc) {
    const float* kf = c->mat_kind == 2 ? c->L.kf32 : nullptr;
    HIPCHK(c, fh::launch_kop_hex8_scalar<float>(g, u, q, kf ? nullptr : ph, kf, c->sk_dev_f,
                                                nload, stride, stride, st, pq, &nb, c->stream));
  } else if (hex_elastic(c) && c->iso) {
    HIPCHK(c, fh::launch_kop_hex8_iso<float>(g, u, q, ph, c->lm_dev_f, nload, stride, stride,
                                             st, pq, &nb, c->stream));
  } else if (hex_elastic(c)) {
    HIPCHK(c, fh::launch_kop_hex8_elastic<float>(g, u, q, ph, c->mat_dev_f, nload, stride,
                                                 stride, st, pq, &nb, c->stream));
  } else {
    const float* kf = c->mat_kind == 2 ? c->L.kf32 : nullptr;
    HIPCHK(c, fh::launch_kop_generic<float>(g, c->element, u, q, ph, kf, c->mat_dev_f, nload,
                                            stride, stride, st, pq, &nb, c->stream));
  }
  return FH_OK;
}

// M^+ on nload fields (double): r -> z in `out` (plain mode) using A/B.
int precond_fields(fh_ctx* c, double* r, double* out, int nload, long long fstride) {
  const fh::Grid& g = c->g;
  const long long S = (long long)g.nd * g.nxh * g.ny * g.nz;
  HIPCHK(c, fh::launch_xfwd<double>(g, c->px, c->twx, fh::XF_PLAIN, r, fstride, nullptr, 0,
                                    c->L.A, S, nload, nullptr, c->stream));
  HIPCHK(c, fh::launch_yfwd<double>(g, c->py, c->twy, c->L.A, c->L.B, S, nload, nullptr,
                                    c->stream));
  int nb = 0;
  HIPCHK(c, fh::launch_zpass<double>(g, c->pz, c->twz, fh::Z_SOLVE, c->L.B, S, c->L.kplus,
                                     nload, nullptr, nullptr, &nb, c->stream));
  HIPCHK(c, fh::launch_yinv<double>(g, c->py, c->twy, c->L.B, c->L.A, S, nload, nullptr,
                                    c->stream));
  HIPCHK(c, fh::launch_xinv<double>(g, c->px, c->twx, fh::XI_PLAIN, c->L.A, S, out, nullptr,
                                    nullptr, fstride, nload, nullptr, c->stream));
  return FH_OK;
}

int check_material(fh_ctx* c) {
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  if (c->mat_kind == 0) return fail(c, FH_ESTATE, "no material set");
  if (c->mat_kind == 1 && !c->phases_checked) {
    // every phase id must index a table before any kernel reads the tables
    HIPCHK(c, hipMemsetAsync(c->flag_dev, 0, sizeof(int), c->stream));
    HIPCHK(c, hipMemsetAsync(c->counts_dev, 0, 256 * sizeof(unsigned long long), c->stream));
    HIPCHK(c, fh::launch_phase_count(c->phase_dev, c->g.N, c->nphase, c->counts_dev, c->flag_dev,
                                     c->stream));
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, FH_EINVAL, "phase id >= nphase in phase field");
    c->phases_checked = true;
  }
  return FH_OK;
}

// Quadrature-weighted mean of the material (Sec. 6.2) into c->cmean; for a
// phase field also the voxel count of every phase into c->phase_counts.
int compute_mean(fh_ctx* c) {
  const fh::Grid& g = c->g;
  const int m = mdim(c);
  c->cmean.assign((size_t)m * m, 0.0);
  HIPCHK(c, hipMemsetAsync(c->flag_dev, 0, sizeof(int), c->stream));
  if (c->mat_kind == 1) {
    HIPCHK(c, hipMemsetAsync(c->counts_dev, 0, 256 * sizeof(unsigned long long), c->stream));
    HIPCHK(c, fh::launch_phase_count(c->phase_dev, g.N, c->nphase, c->counts_dev, c->flag_dev,
                                     c->stream));
    unsigned long long counts[256];
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(counts, c->counts_dev, sizeof(counts), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(&bad, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, FH_EINVAL, "phase id >= nphase in phase field");
    c->phase_counts.assign(counts, counts + c->nphase);
    for (int p = 0; p < c->nphase; ++p)
      for (int i = 0; i < m * m; ++i)
        c->cmean[i] += (double)counts[p] * c->mat[(size_t)p * m * m + i];
    for (double& v : c->cmean) v /= (double)g.N;
  } else {
    const int nb = 1024;
    HIPCHK(c, fh::launch_flag_nonpositive(c->kfield_dev, g.N, c->flag_dev, c->stream));
    HIPCHK(c, fh::launch_field_sum(c->kfield_dev, g.N, c->L.dot_part, nb, c->stream));
    HIPCHK(c, fh::launch_sum_partials(c->L.dot_part, nb, c->L.scal, c->stream));
    double ks = 0;
    int badk = 0;
    HIPCHK(c, hipMemcpyAsync(&ks, c->L.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&badk, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (badk || !(ks > 0.0))
      return fail(c, FH_EINVAL, "conductivity field must be positive and finite in every voxel");
    for (int i = 0; i < m; ++i) c->cmean[i * m + i] = ks / (double)g.N;
  }
  return FH_OK;
}

// Reference material, symbol (Alg. 2) and Kref tables.
int build_symbol(fh_ctx* c) {
  int rc = check_material(c);
  if (rc) return rc;
  rc = ensure_layout(c);
  if (rc) return rc;
  if (c->symbol_ok) return FH_OK;
  const fh::Grid& g = c->g;
  const int m = mdim(c);
  rc = compute_mean(c);
  if (rc) return rc;
  c->cref = c->cref_user ? c->cref_in : c->cmean;
  if (!cholesky_ok(c->cref, m)) return fail(c, FH_ENOTSPD, "reference material is not SPD");
  rc = upload(c, &c->ref_dev, &c->ref_dev_n, operator_tables(c, c->cref.data(), 1));
  if (rc) return rc;
  c->ref_iso = false;
  if (hex_elastic(c)) {
    std::vector<double> lm(2);
    if (isotropic_lm(c->cref.data(), voxel_volume(c), lm.data())) {
      rc = upload(c, &c->ref_lm_dev, &c->ref_lm_dev_n, lm);
      if (rc) return rc;
      c->ref_iso = true;
    }
  }
  c->ref_sc = false;
  if (hex_scalar(c)) {
    const double kr = isotropic_k(c->cref.data(), 3);
    if (kr > 0.0) {
      rc = upload(c, &c->ref_sk_dev, &c->ref_sk_dev_n,
                  std::vector<double>{voxel_volume(c) * kr});
      if (rc) return rc;
      c->ref_sc = true;
    }
  }
  // Alg. 2: impulse responses of Kref, forward FFT, per-frequency inverse
  const long long F = (long long)g.nd * g.N;
  const long long S = (long long)g.nd * g.nxh * g.ny * g.nz;
  for (int be = 0; be < g.nd; ++be) {
    HIPCHK(c, fh::launch_impulse(c->L.x, F, (long long)be * g.N, c->stream));
    rc = apply_K(c, true, c->L.x, c->L.q, 1, F, nullptr, nullptr);
    if (rc) return rc;
    HIPCHK(c, fh::launch_xfwd<double>(g, c->px, c->twx, fh::XF_PLAIN, c->L.q, F, nullptr, 0,
                                      c->L.A, S, 1, nullptr, c->stream));
    HIPCHK(c, fh::launch_yfwd<double>(g, c->py, c->twy, c->L.A, c->L.spec + be * S, S, 1,
                                      nullptr, c->stream));
    int nb = 0;
    HIPCHK(c, fh::launch_zpass<double>(g, c->pz, c->twz, fh::Z_FORWARD_ONLY, c->L.spec + be * S,
                                       S, nullptr, 1, nullptr, nullptr, &nb, c->stream));
  }
  HIPCHK(c, hipMemsetAsync(c->flag_dev, 0, sizeof(int), c->stream));
  if (g.tn)
    HIPCHK(c, fh::launch_symbol_tn(g, c->L.spec, S, c->L.kplus, c->flag_dev, c->L.dot_part,
                                   c->stream));
  else
    HIPCHK(c, fh::launch_symbol(g, c->L.spec, S, c->L.kplus, c->flag_dev, c->stream));
  const long long nsym_n = (long long)g.nxh * g.ny * g.nz * nsym_of(g);
  HIPCHK(c, fh::launch_cast_symbol(nsym_n, c->L.kplus, c->L.kplus_f, c->stream));
  if (c->mat_kind == 2) HIPCHK(c, fh::launch_cast_d2f(c->kfield_dev, c->L.kf32, g.N, c->stream));
  int bad = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) return fail(c, FH_ENOTSPD, "reference symbol has a non-SPD block");
  c->symbol_ok = true;
  return FH_OK;
}

int build_rhs(fh_ctx* c) {
  if (c->rhs_ok) return FH_OK;
  if (c->nload < 1) return fail(c, FH_ESTATE, "fh_set_load not called");
  const fh::Grid& g = c->g;
  const int m = mdim(c);
  const int ntab = c->mat_kind == 1 ? c->nphase : 1;
  std::vector<double> fe;
  const std::vector<double> unit = [&] {
    std::vector<double> I((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) I[i * m + i] = 1.0;
    return I;
  }();
  for (int t = 0; t < ntab; ++t) {
    const double* C = c->mat_kind == 1 ? c->mat.data() + (size_t)t * m * m : unit.data();
    for (int j = 0; j < c->nload; ++j) {
      std::vector<double> f = uniform_strain_force(c, C, c->loads.data() + (size_t)j * m);
      fe.insert(fe.end(), f.begin(), f.end());
    }
  }
  int rc = upload(c, &c->fe_dev, &c->fe_dev_n, fe);
  if (rc) return rc;
  const long long F = (long long)g.nd * g.N;
  HIPCHK(c, fh::launch_rhs(g, c->element, c->mat_kind == 1 ? c->phase_dev : nullptr,
                           c->mat_kind == 2 ? c->kfield_dev : nullptr, c->fe_dev, ntab,
                           c->nload, c->L.b, F, c->stream));
  c->rhs_ok = true;
  return FH_OK;
}

int kt_begin(fh_ctx* c, int cls);
void kt_end(fh_ctx* c, int slot);
void kt_collect(fh_ctx* c);
#define KT(cls, stmt)                    \
  do {                                   \
    const int _slot = kt_begin(c, cls);  \
    stmt;                                \
    kt_end(c, _slot);                    \
  } while (0)

// Launch counts of one replayed iteration, per kernel class (the replay
// records no events, so kt_begin does not see its launches).
void kt_count_iteration(fh_ctx* c) {
  for (int cls : {FH_K_OPERATOR, FH_K_XFWD, FH_K_YFWD, FH_K_ZSOLVE, FH_K_YINV, FH_K_XINV})
    c->kt.issued[cls] += 1;
  c->kt.issued[FH_K_SCALAR] += 2;
}

// Moves a context's work to its private stream for the PCG loop of a single
// solve and back: an event on the caller's stream orders the loop after the
// set-up, an event on the private stream orders the caller's later work
// after the loop.  The private stream and events are created on first use
// and kept until fh_destroy.
struct GraphStream {
  fh_ctx* c;
  hipStream_t saved = nullptr;
  bool on = false;
  explicit GraphStream(fh_ctx* cc) : c(cc) {}
  int fork() {
    if (!c->gstream) {
      // all three or none: a failure leaves nothing half-made behind
      hipStream_t st = nullptr;
      hipEvent_t ef = nullptr, ej = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&ef, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&ej, hipEventDisableTiming) != hipSuccess) {
        if (ej) hipEventDestroy(ej);
        if (ef) hipEventDestroy(ef);
        if (st) hipStreamDestroy(st);
        return fail(c, FH_EDEVICE, "stream or event creation for graph replay failed");
      }
      c->gstream = st;
      c->gfork = ef;
      c->gjoin = ej;
    }
    HIPCHK(c, hipEventRecord(c->gfork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->gfork, 0));
    saved = c->stream;
    c->stream = c->gstream;
    on = true;
    return FH_OK;
  }
  ~GraphStream() {
    if (!on) return;
    hipEventRecord(c->gjoin, c->gstream);
    hipStreamWaitEvent(saved, c->gjoin, 0);
    c->stream = saved;
  }
};

// ------------------------------------------------------------------ PCG
// One PCG solve per load case on buffers of type T (double, or float for the
// inner solves of the refinement).  The right-hand side must already be in
// `r`; x is zeroed here.  Load cases whose initial state is not ACTIVE are
// skipped by every kernel.  Scalars, reductions and the stopping test are
// FP64 in both cases.  The host only polls the per-load status every `poll`
// iterations.
template <typename T>
struct PcgBufs {
  T *x, *r, *p, *q;
  cplx<T> *A, *B;
  const T* kplus;
};

int apply_KT(fh_ctx* c, const double* u, double* q, int nload, long long F,
             const fh::PcgState* st, double* pq) {
  return apply_K(c, false, u, q, nload, F, st, pq);
}
int apply_KT(fh_ctx* c, const float* u, float* q, int nload, long long F,
             const fh::PcgState* st, double* pq) {
  return apply_K32(c, u, q, nload, F, st, pq);
}

// With zero_x false, x keeps its content (an initial guess whose residual is
// already in r) and the PCG updates add to it.  eta2v (optional) gives each
// load case its own squared tolerance relative to its initial r.z.
template <typename T>
int pcg_run(fh_ctx* c, int nload, const PcgBufs<T>& bf, double eta, int itmax, int poll,
            const std::vector<int>& active, std::vector<fh::PcgState>& out,
            bool zero_x = true, const std::vector<double>* eta2v = nullptr,
            const std::vector<int>* itmaxv = nullptr) {
  const fh::Grid& g = c->g;
  const long long F = (long long)g.nd * g.N;
  const long long S = (long long)g.nd * g.nxh * g.ny * g.nz;
  fh_ctx::Layout& L = c->L;
  std::vector<fh::PcgState> hs(nload);
  for (int j = 0; j < nload; ++j) {
    hs[j] = fh::PcgState{};
    hs[j].status = active[j] ? fh::ST_ACTIVE : fh::ST_CONVERGED;
    hs[j].eta2 = eta2v ? (*eta2v)[j] : eta * eta;
    hs[j].itmax = itmaxv ? std::max(1, (*itmaxv)[j]) : itmax;
  }
  const bool single_graph = !c->use_graph && c->graph;
  GraphStream gs(c);
  if (single_graph) {
    const int rc = gs.fork();
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpyAsync(L.st, hs.data(), sizeof(fh::PcgState) * nload, hipMemcpyHostToDevice,
                           c->stream));
  if (zero_x) HIPCHK(c, fh::launch_fill<T>(bf.x, T(0), F * nload, c->stream));
  // z0 = M r0, p0 = z0, rho0 = r0.z0
  int nbz = 0;
  HIPCHK(c, fh::launch_xfwd<T>(g, c->px, c->twx, fh::XF_PLAIN, bf.r, F, nullptr, 0, bf.A, S,
                               nload, L.st, c->stream));
  HIPCHK(c, fh::launch_yfwd<T>(g, c->py, c->twy, bf.A, bf.B, S, nload, L.st, c->stream));
  HIPCHK(c, fh::launch_zpass<T>(g, c->pz, c->twz, fh::Z_SOLVE, bf.B, S, bf.kplus, nload, L.st,
                                L.rz_part, &nbz, c->stream));
  HIPCHK(c, fh::launch_yinv<T>(g, c->py, c->twy, bf.B, bf.A, S, nload, L.st, c->stream));
  HIPCHK(c, fh::launch_xinv<T>(g, c->px, c->twx, fh::XI_INIT_P, bf.A, S, nullptr, nullptr, bf.p,
                               F, nload, L.st, c->stream));
  HIPCHK(c, fh::launch_finalize_init(L.st, L.rz_part, nbz, nload, c->stream));
  const int nbk = c->qp_tangent ? c->pl_nbg : fh::kop_nblocks(g, hex_tiled(c), (int)sizeof(T));
  auto one_iteration = [&]() -> int {
      int rc = 0;
      KT(FH_K_OPERATOR, rc = apply_KT(c, bf.p, bf.q, nload, F, L.st, L.pq_part));
      if (rc) return rc;
      KT(FH_K_SCALAR, HIPCHK(c, fh::launch_finalize_alpha(L.st, L.pq_part, nbk, nload,
                                                          c->stream)));
      KT(FH_K_XFWD, HIPCHK(c, fh::launch_xfwd<T>(g, c->px, c->twx, fh::XF_UPDATE_R, bf.r, F,
                                                 bf.q, F, bf.A, S, nload, L.st, c->stream)));
      KT(FH_K_YFWD, HIPCHK(c, fh::launch_yfwd<T>(g, c->py, c->twy, bf.A, bf.B, S, nload, L.st,
                                                 c->stream)));
      KT(FH_K_ZSOLVE, HIPCHK(c, fh::launch_zpass<T>(g, c->pz, c->twz, fh::Z_SOLVE, bf.B, S,
                                                    bf.kplus, nload, L.st, L.rz_part, &nbz,
                                                    c->stream)));
      KT(FH_K_SCALAR, HIPCHK(c, fh::launch_finalize_beta(L.st, L.rz_part, nbz, nload, L.hist,
                                                         L.hist_len, c->stream)));
      KT(FH_K_YINV, HIPCHK(c, fh::launch_yinv<T>(g, c->py, c->twy, bf.B, bf.A, S, nload, L.st,
                                                 c->stream)));
      KT(FH_K_XINV, HIPCHK(c, fh::launch_xinv<T>(g, c->px, c->twx, fh::XI_PCG, bf.A, S, nullptr,
                                                 bf.x, bf.p, F, nload, L.st, c->stream)));
      return FH_OK;
  };
  // One iteration (all kernels, all load cases, all systems of a batch) is
  // captured in a hipGraph and replayed; kernels read everything that
  // changes from the device-resident PCG state, so the same graph serves
  // every iteration.  Batched solves capture on their group's own stream;
  // single solves with FH_FLAG_GRAPH move to the context's private stream
  // for the loop.
  hipGraphExec_t exec = nullptr;
  if (c->use_graph || single_graph) {
    hipGraph_t graph = nullptr;
    const bool kt_was = c->kt.on;
    c->kt.on = false;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int rc = one_iteration();
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->kt.on = kt_was;
    if (rc) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    HIPCHK(c, e);
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    HIPCHK(c, ei);
  }
  struct ExecGuard {
    hipGraphExec_t e;
    ~ExecGuard() { if (e) hipGraphExecDestroy(e); }
  } guard{exec};
  int done_iters = 0;
  const int cap = itmax + 2;
  // Iterations until the next status poll.  After the first window the
  // count follows the observed contraction of sqrt(r.z / r0.z0) since the
  // previous poll, so that the loop stops close to the last load's
  // convergence instead of running up to poll - 1 iterations in which every
  // load case has stopped (those launches only test the status and exit).
  int window = poll;
  std::vector<double> prev_last(nload, 1.0);
  std::vector<int> prev_iter(nload, 0);
  while (true) {
    for (int k = 0; k < window && done_iters < cap; ++k, ++done_iters) {
      // sampled iterations sit mid-way between the 16-iteration status
      // polls: the iteration right after a poll starts on an idle GPU, and
      // its first event pair would include the host's launch latency
      const bool sampled = done_iters % c->kt.period == c->kt.period / 2;
      if (exec && !(c->kt.on && sampled)) {
        HIPCHK(c, hipGraphLaunch(exec, c->stream));
        if (c->kt.on) kt_count_iteration(c);
      } else {
        c->kt.sample = sampled;
        c->kt.cur_iter = done_iters;
        const int rc = one_iteration();
        c->kt.sample = true;
        if (rc) return rc;
      }
    }
    HIPCHK(c, hipMemcpyAsync(hs.data(), L.st, sizeof(fh::PcgState) * nload,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    kt_collect(c);
    bool any = false;
    for (auto& st : hs) any |= (st.status == fh::ST_ACTIVE);
    if (!any || done_iters >= cap) break;
    window = poll;
    for (int j = 0; j < nload; ++j) {
      const fh::PcgState& sj = hs[j];
      if (sj.status != fh::ST_ACTIVE) continue;
      const int di = sj.iter - prev_iter[j];
      if (di > 0 && sj.last > 0.0 && prev_last[j] > 0.0 && sj.last < prev_last[j]) {
        const double rate = std::pow(sj.last / prev_last[j], 1.0 / di);
        const double need = std::log(std::sqrt(sj.eta2) / sj.last) / std::log(rate);
        if (std::isfinite(need)) window = std::min(window, std::max(1, (int)std::ceil(need)));
      }
      prev_last[j] = sj.last;
      prev_iter[j] = sj.iter;
    }
  }
  // A load case takes part in loop iteration k (0-based) of this run if it
  // started active and its final count exceeds k: its last iteration still
  // runs every pass (the x update of a converged load is due then).
  for (const auto& ti : c->kt.timed_iters) {
    int act = 0;
    for (int j = 0; j < nload; ++j) act += (active[j] && ti.second < hs[j].iter) ? 1 : 0;
    c->kt.units[ti.first] += act;
  }
  c->kt.timed_iters.clear();
  out = hs;
  return FH_OK;
}

// Plain FP64 solve of K x = b for the right-hand sides in L.b.
int pcg64(fh_ctx* c, int nload, double eta, int itmax, int poll, std::vector<fh::PcgState>& out) {
  const long long F = (long long)c->g.nd * c->g.N;
  fh_ctx::Layout& L = c->L;
  HIPCHK(c, fh::launch_copy(L.r, L.b, F * nload, c->stream));
  PcgBufs<double> bf{L.x, L.r, L.p, L.q, L.A, L.B, L.kplus};
  return pcg_run<double>(c, nload, bf, eta, itmax, poll, std::vector<int>(nload, 1), out);
}

// Plain FP64 solve from the screened initial guess in L.x, whose residual is in
// L.r: rr[j] = r0.M r0 of the starting point, rb[j] = b.M b.  The stopping
// test stays relative to b.M b (rho <= eta^2 rb); load cases that already
// meet it do no iteration.  Reported residuals are relative to b.
int pcg64_warm(fh_ctx* c, int nload, double eta, int itmax, int poll,
               const std::vector<double>& rb, const std::vector<double>& rr,
               std::vector<fh::PcgState>& out) {
  fh_ctx::Layout& L = c->L;
  std::vector<int> active(nload, 1);
  std::vector<double> eta2(nload, eta * eta);
  for (int j = 0; j < nload; ++j) {
    if (!(rb[j] > 0.0) || rr[j] <= eta * eta * rb[j]) active[j] = 0;
    else if (rr[j] != rb[j]) eta2[j] = eta * eta * rb[j] / rr[j];
  }
  PcgBufs<double> bf{L.x, L.r, L.p, L.q, L.A, L.B, L.kplus};
  int rc = pcg_run<double>(c, nload, bf, eta, itmax, poll, active, out, false, &eta2);
  if (rc) return rc;
  for (int j = 0; j < nload; ++j) {
    const double f = rb[j] > 0.0 ? std::sqrt(std::max(rr[j], 0.0) / rb[j]) : 0.0;
    if (!active[j]) {
      out[j] = fh::PcgState{};
      out[j].status = fh::ST_CONVERGED;
      out[j].last = f;
    } else {
      out[j].last *= f;
    }
  }
  return FH_OK;
}

// Inner FP32 tolerance when the caller gives none.  FP32 PCG stagnates near
// 1e-6 relative, so each sweep asks for at most 1e-3..1e-4: sqrt(eta) for
// loose outer targets (two sweeps), 1e-4 for tight ones.
double default_eta_inner(const fh_opts& o) {
  if (o.eta_inner > 0.0) return o.eta_inner;
  return o.eta >= 1e-6 ? std::sqrt(o.eta) : 1e-4;
}

// FP32-in-FP64 iterative refinement (FH_FP32_REFINED).  Outer loop in FP64:
// residual r = b - K x with the FP64 operator, its Kref^-1-norm sqrt(r.M r)
// with the FP64 preconditioner (the same stopping rule as the plain solve,
// relative to the norm of b), then an inner PCG in FP32 for K d = r to the
// relative tolerance eta_inner and x += d in FP64.  out[j].iter holds the
// summed inner iterations, outer[j] the number of sweeps.
// With rho_ref set, the caller has put an initial guess in L.x and its
// residual in L.r, and the stopping test is relative to rho_ref (b.M b).
int pcg_refined(fh_ctx* c, int nload, double eta, double eta_in, int itmax, int poll,
                std::vector<fh::PcgState>& out, std::vector<int>& outer,
                const std::vector<double>* rho_ref = nullptr) {
  const fh::Grid& g = c->g;
  const long long F = (long long)g.nd * g.N;
  fh_ctx::Layout& L = c->L;
  std::vector<double> rho0(nload, 0.0), rho(nload, 0.0);
  std::vector<int> active(nload, 1), total(nload, 0), status(nload, fh::ST_ACTIVE);
  std::vector<double> last(nload, 1.0);
  outer.assign(nload, 0);
  int* mask_dev = L.mask;
  if (!rho_ref) {
    HIPCHK(c, fh::launch_fill<double>(L.x, 0.0, F * nload, c->stream));
    HIPCHK(c, fh::launch_copy(L.r, L.b, F * nload, c->stream));
  }
  const int max_outer = 64;
  for (int sweep = 0; sweep <= max_outer; ++sweep) {
    // Kref^-1-norm of the FP64 residual
    int rc = precond_fields(c, L.r, L.q, nload, F);
    if (rc) return rc;
    // r_j . z_j for every system in one launch (fixed-order sums)
    HIPCHK(c, fh::launch_pair_dots(L.r, L.q, F, 1, nload, kSysChunks, L.sysdot_part, L.sysdot,
                                   c->stream));
    std::vector<double> dots(nload, 0.0);
    HIPCHK(c, hipMemcpyAsync(dots.data(), L.sysdot, sizeof(double) * nload,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool any = false;
    for (int j = 0; j < nload; ++j) {
      if (!active[j]) continue;
      rho[j] = dots[j];
      if (sweep == 0) rho0[j] = rho_ref ? (*rho_ref)[j] : rho[j];
      if (!(rho0[j] > 0.0)) {
        active[j] = 0;
        status[j] = rho0[j] == 0.0 ? fh::ST_CONVERGED : fh::ST_BREAKDOWN;
        last[j] = 0.0;
        continue;
      }
      last[j] = rho[j] > 0.0 ? std::sqrt(rho[j] / rho0[j]) : 0.0;
      if (rho[j] <= eta * eta * rho0[j]) {
        active[j] = 0;
        status[j] = fh::ST_CONVERGED;
      } else if (sweep == max_outer || total[j] >= itmax) {
        active[j] = 0;
        status[j] = fh::ST_MAXIT;
      }
      any |= active[j] != 0;
    }
    if (!any) break;
    // inner FP32 solve K d = r (cast per active load), d in x32
    std::vector<fh::PcgState> ist(nload);
    for (int j = 0; j < nload; ++j) {
      ist[j] = fh::PcgState{};
      ist[j].status = active[j] ? fh::ST_ACTIVE : fh::ST_CONVERGED;
    }
    HIPCHK(c, hipMemcpyAsync(L.st, ist.data(), sizeof(fh::PcgState) * nload,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, fh::launch_cast_masked(L.r, L.r32, F, nload, L.st, c->stream));
    PcgBufs<float> bf{L.x32, L.r32, L.p32, L.q32, L.A32, L.B32, L.kplus_f};
    // sweep k aims at |r| <= tau_k |b| (M-norms), tau_k = max(eta_in^(k+1),
    // eta/2): the inner tolerance relative to the current residual is
    // tau_k sqrt(rho0 / rho), kept within [1e-5, 0.5] (FP32 PCG stalls
    // below about 1e-6).  A warm start that already removed part of b, or a
    // last sweep that only needs a little more, asks the inner solve for less.
    std::vector<double> eta2(nload, eta_in * eta_in);
    const double tau = std::max(std::pow(eta_in, sweep + 1), 0.5 * eta);
    for (int j = 0; j < nload; ++j)
      if (active[j] && rho[j] > 0.0) {
        const double rel = std::min(0.5, std::max(1e-5, tau * std::sqrt(rho0[j] / rho[j])));
        eta2[j] = rel * rel;
      }
    // the inner sweeps share the caller's iteration cap (Alg. 1 it_max^CG):
    // each may run only what the earlier sweeps of its load case left
    std::vector<int> left(nload, 1);
    for (int j = 0; j < nload; ++j) left[j] = std::max(1, itmax - total[j]);
    std::vector<fh::PcgState> hs;
    rc = pcg_run<float>(c, nload, bf, eta_in, std::max(1, itmax), poll, active, hs, true, &eta2,
                        &left);
    if (rc) return rc;
    for (int j = 0; j < nload; ++j)
      if (active[j]) {
        total[j] += hs[j].iter;
        outer[j] += 1;
        if (hs[j].status == fh::ST_BREAKDOWN) {
          active[j] = 0;
          status[j] = fh::ST_BREAKDOWN;
        }
      }
    HIPCHK(c, hipMemcpyAsync(mask_dev, active.data(), sizeof(int) * nload, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, fh::launch_add_masked(L.x, L.x32, F, nload, mask_dev, c->stream));
    // r = b - K x in FP64
    rc = apply_K(c, false, L.x, L.q, nload, F, nullptr, nullptr);
    if (rc) return rc;
    HIPCHK(c, fh::launch_residual(L.r, L.b, L.q, F * nload, c->stream));
  }
  out.assign(nload, fh::PcgState{});
  for (int j = 0; j < nload; ++j) {
    out[j].iter = total[j];
    out[j].status = status[j] == fh::ST_ACTIVE ? fh::ST_MAXIT : status[j];
    out[j].last = last[j];
  }
  return FH_OK;
}

void record_history(fh_ctx* c, const std::vector<fh::PcgState>& hs, int nload,
                    const std::vector<double>* scale = nullptr) {
  c->history.assign(nload, {});
  std::vector<double> h((size_t)c->L.hist_len * nload);
  hipMemcpyAsync(h.data(), c->L.hist, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                 c->stream);
  hipStreamSynchronize(c->stream);
  for (int j = 0; j < nload; ++j) {
    const int n = std::min(hs[j].iter, c->L.hist_len);
    c->history[j].assign(h.begin() + (size_t)j * c->L.hist_len,
                         h.begin() + (size_t)j * c->L.hist_len + n);
    if (scale)
      for (double& v : c->history[j]) v *= (*scale)[j];
  }
}

// Initial guess for fh_solve (opts.guess_dev or the learned warm start) into
// L.x, shifted to zero mean per component, and the screen: rb = b.M b, rr =
// r0.M r0 of the kept starting point (a load case whose guess is not better
// than zero restarts from zero, rr = rb).  L.r holds the starting residual.
int prepare_guess(fh_ctx* c, const fh_opts& o, std::vector<double>& rb,
                  std::vector<double>& rr, std::vector<double>& gres, std::vector<int>& used) {
  const fh::Grid& g = c->g;
  const int nl = c->nload;
  const long long F = (long long)g.nd * g.N;
  fh_ctx::Layout& L = c->L;
  if (o.flags & FH_FLAG_WARM_START) {
    if (!c->net) return fail(c, FH_ESTATE, "warm start requested but no network attached");
    const int n = g.nx;
    if (!hex_elastic(c) || g.dim != 3 || g.ny != n || g.nz != n || fh::net_grid(c->net) != n ||
        c->l[1] != c->l[0] || c->l[2] != c->l[0])
      return fail(c, FH_EINVAL, "warm start needs 3D hex8 elasticity on the network's cubic grid");
    if (c->mat_kind != 1 || c->nphase != 2 || !c->iso)
      return fail(c, FH_EINVAL, "warm start needs two isotropic phases");
    const double r = c->mat[36] / c->mat[0];
    if (!(r > 0.0)) return fail(c, FH_EINVAL, "warm start: bad phase stiffness ratio");
    const float gamma = (float)(std::log10(r) / 3.0);
    std::string err;
    const int rc = fh::net_warm_guess(c->net, c->stream, c->phase_dev, gamma, nl,
                                      c->loads.data(), c->l[0] / n, L.x, F, &err);
    if (rc) return fail(c, rc, err);
  } else {
    HIPCHK(c, hipMemcpyAsync(L.x, o.guess_dev, sizeof(double) * F * nl, hipMemcpyDeviceToDevice,
                             c->stream));
  }
  HIPCHK(c, fh::launch_remove_mean(L.x, nl * g.nd, g.N, L.sysdot_part, 16, c->stream));
  auto dots = [&](const double* a, const double* b, std::vector<double>& out) -> int {
    HIPCHK(c, fh::launch_pair_dots(a, b, F, 1, nl, kSysChunks, L.sysdot_part, L.sysdot,
                                   c->stream));
    out.assign(nl, 0.0);
    HIPCHK(c, hipMemcpyAsync(out.data(), L.sysdot, sizeof(double) * nl, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FH_OK;
  };
  int rc = precond_fields(c, L.b, L.q, nl, F);
  if (rc || (rc = dots(L.b, L.q, rb))) return rc;
  if ((rc = apply_K(c, false, L.x, L.q, nl, F, nullptr, nullptr))) return rc;
  HIPCHK(c, fh::launch_residual(L.r, L.b, L.q, F * nl, c->stream));
  if ((rc = precond_fields(c, L.r, L.q, nl, F)) || (rc = dots(L.r, L.q, rr))) return rc;
  used.assign(nl, 0);
  gres.assign(nl, 0.0);
  for (int j = 0; j < nl; ++j) {
    gres[j] = rb[j] > 0.0 ? std::sqrt(std::max(rr[j], 0.0) / rb[j]) : 0.0;
    used[j] = rr[j] < rb[j] ? 1 : 0;
    if (!used[j]) {
      HIPCHK(c, fh::launch_fill<double>(L.x + j * F, 0.0, F, c->stream));
      HIPCHK(c, fh::launch_copy(L.r + j * F, L.b + j * F, F, c->stream));
      rr[j] = rb[j];
    }
  }
  return FH_OK;
}

int status_code(int st) {
  switch (st) {
    case fh::ST_CONVERGED:
    case fh::ST_CONVERGED_PENDING: return 0;
    case fh::ST_MAXIT:
    case fh::ST_MAXIT_PENDING: return 1;
    default: return FH_ENOTSPD;
  }
}

int fill_stats(fh_ctx* c, const std::vector<fh::PcgState>& hs, int nload, fh_stats* st) {
  fh_stats s{};
  s.nload = nload;
  s.dof = (long long)c->g.nd * c->g.N;
  int rc = FH_OK;
  for (int j = 0; j < nload && j < FH_MAX_LOADS; ++j) {
    s.iterations[j] = hs[j].iter;
    s.status[j] = status_code(hs[j].status);
    s.rel_res[j] = hs[j].last;
    s.outer[j] = 0;
    if (s.status[j] < 0) rc = FH_ENOTSPD;
    else if (s.status[j] > 0 && rc == FH_OK) rc = FH_NOT_CONVERGED;
  }
  c->last = s;
  if (st) *st = s;
  if (rc == FH_ENOTSPD) fail(c, rc, "PCG breakdown (p.q <= 0 or r.z < 0)");
  return rc;
}

int kt_begin(fh_ctx* c, int cls) {
  fh_ctx::KTimer& t = c->kt;
  if (!t.on) return -1;
  t.issued[cls] += 1;
  if (!t.sample) return -1;
  if (t.used * 2 + 2 > t.ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      hipEventDestroy(a);
      return -1;
    }
    t.ev.push_back(a);
    t.ev.push_back(b);
    t.cls.push_back(0);
  }
  const int slot = (int)t.used++;
  t.cls[slot] = cls;
  t.timed_iters.emplace_back(cls, t.cur_iter);
  hipEventRecord(t.ev[2 * slot], c->stream);
  return slot;
}

void kt_end(fh_ctx* c, int slot) {
  if (slot >= 0) hipEventRecord(c->kt.ev[2 * slot + 1], c->stream);
}

// after a stream synchronisation: fold the recorded pairs into the totals
void kt_collect(fh_ctx* c) {
  fh_ctx::KTimer& t = c->kt;
  for (size_t i = 0; i < t.used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) == hipSuccess) {
      t.ms[t.cls[i]] += ms;
      t.n[t.cls[i]] += 1;
    }
  }
  t.used = 0;
}

struct KScope {
  fh_ctx* c;
  int slot;
  KScope(fh_ctx* cc, int cls) : c(cc), slot(kt_begin(cc, cls)) {}
  ~KScope() { kt_end(c, slot); }
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace


// ================================================================ batches
namespace {

double time_launches(fh_ctx* c, const std::function<int()>& launch, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30;
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return 1e30;
  }
  double ms = 1e30;
  if (launch() == FH_OK) {  // warm-up
    hipEventRecord(a, c->stream);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = launch() == FH_OK;
    hipEventRecord(b, c->stream);
    float t = 0.f;
    if (ok && hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&t, a, b) == hipSuccess)
      ms = t / reps;
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

// Choose the operator z-chunk and the FFT lines per block for this grid by
// timing the FP32 kernels (the refinement's inner loop) on the group's own
// buffers.  The candidates are timed on at most 24 load cases: enough blocks
// to fill the GPU at these grid sizes, at a fraction of the cost.
int autotune(fh_ctx* c, int nload_all, double* tune_ms) {
  auto t0 = std::chrono::steady_clock::now();
  const int nload_total = std::min(nload_all, 24);
  fh::Grid& g = c->g;
  const long long F = (long long)g.nd * g.N;
  const long long S = (long long)g.nd * g.nxh * g.ny * g.nz;
  fh_ctx::Layout& L = c->L;
  HIPCHK(c, fh::launch_fill<float>(L.p32, 0.f, F * nload_total, c->stream));
  HIPCHK(c, fh::launch_fill<float>(L.q32, 0.f, F * nload_total, c->stream));
  HIPCHK(c, fh::launch_fill<float>(L.r32, 0.f, F * nload_total, c->stream));
  const int reps = 3;
  int best = g.kz;
  double bt = 1e30;
  for (int kz : {4, 8, 16, 32}) {
    if (kz > g.nz) continue;
    g.kz = kz;
    const double t = time_launches(c, [&] {
      return apply_K32(c, L.p32, L.q32, nload_total, F, nullptr, nullptr);
    }, reps);
    if (t < bt) { bt = t; best = kz; }
  }
  g.kz = best;
  best = 0;
  bt = 1e30;
  for (int zb : {2, 4, 8, 16}) {
    if (zb * g.ny > 2048 || zb > g.nz) continue;
    g.zb = zb;
    const double t = time_launches(c, [&] {
      return fh::launch_yfwd<float>(g, c->py, c->twy, L.A32, L.B32, S, nload_total, nullptr,
                                    c->stream) == hipSuccess ? FH_OK : FH_EDEVICE;
    }, reps);
    if (t < bt) { bt = t; best = zb; }
  }
  g.zb = best;
  best = 0;
  bt = 1e30;
  for (int kyb : {1, 2, 4, 8, 16}) {
    if (kyb * g.nd * g.nz > 2048 || kyb > g.ny) continue;
    g.kyb = kyb;
    int nb = 0;
    const double t = time_launches(c, [&] {
      return fh::launch_zpass<float>(g, c->pz, c->twz, fh::Z_FORWARD_ONLY, L.B32, S, nullptr,
                                     nload_total, nullptr, nullptr, &nb,
                                     c->stream) == hipSuccess ? FH_OK : FH_EDEVICE;
    }, reps);
    if (t < bt) { bt = t; best = kyb; }
  }
  g.kyb = best;
  // rows per block of the FP32 x passes (forward and inverse timed together)
  best = 16;
  bt = 1e30;
  for (int xr : {16, 32}) {
    if (xr == 32 && g.nx > 128) continue;
    g.xrows = xr;
    const double t = time_launches(c, [&] {
      if (fh::launch_xfwd<float>(g, c->px, c->twx, fh::XF_PLAIN, L.r32, F, nullptr, 0, L.A32, S,
                                 nload_total, nullptr, c->stream) != hipSuccess)
        return FH_EDEVICE;
      return fh::launch_xinv<float>(g, c->px, c->twx, fh::XI_PLAIN, L.A32, S, L.q32, nullptr,
                                    nullptr, F, nload_total, nullptr,
                                    c->stream) == hipSuccess ? FH_OK : FH_EDEVICE;
    }, reps);
    if (t < bt) { bt = t; best = xr; }
  }
  g.xrows = best;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *tune_ms = ms_since(t0);
  return FH_OK;
}

// Start line for the solves of concurrently running groups: every group
// finishes its set-up and launch-shape tuning (timed on an otherwise idle
// GPU, one group at a time under `tune_mu`) before any group starts solving.
struct BatchGate {
  std::mutex tune_mu, mu;
  std::condition_variable cv;
  int waiting = 0, total = 1;
  void arrive() {
    std::unique_lock<std::mutex> lk(mu);
    if (++waiting >= total) cv.notify_all();
    else cv.wait(lk, [&] { return waiting >= total; });
  }
};

int batch_group(fh_ctx* parent, const std::vector<int>& idx, const fh_system* sys, int nload,
                const double* E, const fh_opts& o, double* chom, fh_stats* st,
                fh_batch_report* rep, int gi, BatchGate* gate, char* region,
                size_t region_bytes) {
  // the gate is passed exactly once, whatever path leaves this function
  struct Arrive {
    BatchGate* g;
    bool done = false;
    void now() { if (g && !done) { done = true; g->arrive(); } }
    ~Arrive() { now(); }
  } arrive{gate};
  std::unique_lock<std::mutex> tune_lock;
  if (gate) tune_lock = std::unique_lock<std::mutex>(gate->tune_mu);
  fh_ctx* c = nullptr;
  if (fh_create(&c, parent->device) != FH_OK) return fail(parent, FH_EDEVICE, "fh_create");
  struct Owner {
    fh_ctx* c;
    ~Owner() { fh_destroy(c); }
  } owner{c};
  auto pfail = [&](int rc) { return fail(parent, rc, c->err); };
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(parent, FH_EDEVICE, "stream creation failed");
  c->own_stream = true;
  const fh_system& s0 = sys[idx[0]];
  int rc = fh_set_grid(c, 3, s0.n, nullptr, FH_ELASTIC, FH_HEX8);
  if (rc) return pfail(rc);
  auto t0 = std::chrono::steady_clock::now();
  const fh::Grid g0 = c->g;
  const int nms = (int)idx.size();
  const long long N = g0.N, F = 3 * N;
  const long long nfreq = (long long)g0.nxh * g0.ny * g0.nz;
  const long long S = 3 * nfreq;
  const double Vp = voxel_volume(c);
  int np = 1;
  for (int i : idx) np = std::max(np, sys[i].nphase);
  // packed phases and per-microstructure {V lambda, 2 V mu} tables
  if (hipMalloc((void**)&c->phase_pack, (size_t)nms * N) != hipSuccess)
    return fail(parent, FH_ENOMEM, "phase pack allocation failed");
  std::vector<double> lm((size_t)nms * 2 * np, 0.0);
  for (int ms = 0; ms < nms; ++ms) {
    const fh_system& sy = sys[idx[ms]];
    HIPCHK(parent, hipMemcpyAsync(c->phase_pack + (size_t)ms * N, sy.phase_dev, (size_t)N,
                                  hipMemcpyDeviceToDevice, c->stream));
    for (int p = 0; p < sy.nphase; ++p)
      if (!isotropic_lm(sy.mat + (size_t)p * 36, Vp, lm.data() + ((size_t)ms * np + p) * 2))
        return fail(parent, FH_EINVAL, "batched solves need isotropic phases");
  }
  if ((rc = upload(c, &c->lm_dev, &c->lm_dev_n, lm)) || (rc = upload_f(c, &c->lm_dev_f, lm)))
    return pfail(rc);
  c->iso = true;
  c->mat_kind = 1;
  c->phase_dev = c->phase_pack;
  c->nphase = np;
  c->g.nphase_max = np;
  c->phases_checked = true;
  c->nms = nms;
  c->nload = nms * nload;
  c->loads.clear();
  for (int ms = 0; ms < nms; ++ms) c->loads.insert(c->loads.end(), E, E + (size_t)nload * 6);
  if (region) {  // a region of the caller's bound workspace
    c->ws_user = region;
    c->ws_user_bytes = region_bytes;
  }
  if ((rc = ensure_layout(c))) return pfail(rc);
  fh_ctx::Layout& L = c->L;
  // per microstructure: Cref = mean (Sec. 6.2), Alg. 2 symbol, right-hand sides
  c->cmean_ms.assign(nms, std::vector<double>(36, 0.0));
  for (int ms = 0; ms < nms; ++ms) {
    const fh_system& sy = sys[idx[ms]];
    HIPCHK(parent, hipMemsetAsync(c->flag_dev, 0, sizeof(int), c->stream));
    HIPCHK(parent, hipMemsetAsync(c->counts_dev, 0, 256 * sizeof(unsigned long long), c->stream));
    HIPCHK(parent, fh::launch_phase_count(c->phase_pack + (size_t)ms * N, N, sy.nphase,
                                          c->counts_dev, c->flag_dev, c->stream));
    unsigned long long counts[256];
    int bad = 0;
    HIPCHK(parent, hipMemcpyAsync(counts, c->counts_dev, sizeof(counts), hipMemcpyDeviceToHost,
                                  c->stream));
    HIPCHK(parent, hipMemcpyAsync(&bad, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost,
                                  c->stream));
    HIPCHK(parent, hipStreamSynchronize(c->stream));
    if (bad) return fail(parent, FH_EINVAL, "phase id >= nphase in a batched system");
    std::vector<double>& cm = c->cmean_ms[ms];
    for (int p = 0; p < sy.nphase; ++p)
      for (int i = 0; i < 36; ++i) cm[i] += (double)counts[p] * sy.mat[(size_t)p * 36 + i];
    for (double& v : cm) v /= (double)N;
    std::vector<double> rlm(2);
    if (!cholesky_ok(cm, 6) || !isotropic_lm(cm.data(), Vp, rlm.data()))
      return fail(parent, FH_ENOTSPD, "mean reference material not SPD/isotropic");
    if ((rc = upload(c, &c->ref_lm_dev, &c->ref_lm_dev_n, rlm))) return pfail(rc);
    c->ref_iso = true;
    c->cref = cm;
    for (int be = 0; be < 3; ++be) {
      HIPCHK(parent, fh::launch_impulse(L.x, F, (long long)be * N, c->stream));
      if ((rc = apply_K(c, true, L.x, L.q, 1, F, nullptr, nullptr))) return pfail(rc);
      HIPCHK(parent, fh::launch_xfwd<double>(c->g, c->px, c->twx, fh::XF_PLAIN, L.q, F, nullptr,
                                             0, L.A, S, 1, nullptr, c->stream));
      HIPCHK(parent, fh::launch_yfwd<double>(c->g, c->py, c->twy, L.A, L.spec + be * S, S, 1,
                                             nullptr, c->stream));
      int nb = 0;
      HIPCHK(parent, fh::launch_zpass<double>(c->g, c->pz, c->twz, fh::Z_FORWARD_ONLY,
                                              L.spec + be * S, S, nullptr, 1, nullptr, nullptr,
                                              &nb, c->stream));
    }
    HIPCHK(parent, hipMemsetAsync(c->flag_dev, 0, sizeof(int), c->stream));
    HIPCHK(parent, fh::launch_symbol(c->g, L.spec, S, L.kplus + (size_t)ms * 6 * nfreq,
                                     c->flag_dev, c->stream));
    std::vector<double> fe;
    for (int p = 0; p < np; ++p)
      for (int j = 0; j < nload; ++j) {
        std::vector<double> f(24, 0.0);
        if (p < sy.nphase) f = uniform_strain_force(c, sy.mat + (size_t)p * 36, E + (size_t)j * 6);
        fe.insert(fe.end(), f.begin(), f.end());
      }
    if ((rc = upload(c, &c->fe_dev, &c->fe_dev_n, fe))) return pfail(rc);
    HIPCHK(parent, fh::launch_rhs(c->g, c->element, c->phase_pack + (size_t)ms * N, nullptr,
                                  c->fe_dev, np, nload, L.b + (size_t)ms * nload * F, F,
                                  c->stream));
    HIPCHK(parent, hipMemcpyAsync(&bad, c->flag_dev, sizeof(int), hipMemcpyDeviceToHost,
                                  c->stream));
    HIPCHK(parent, hipStreamSynchronize(c->stream));
    if (bad) return fail(parent, FH_ENOTSPD, "reference symbol has a non-SPD block");
  }
  HIPCHK(parent, fh::launch_cast_symbol((long long)nms * 6 * nfreq, L.kplus, L.kplus_f,
                                        c->stream));
  c->symbol_ok = c->rhs_ok = true;
  // batched addressing: system ld -> microstructure ld / nload
  c->g.G = nload;
  c->g.phase_stride = N;
  c->g.kplus_stride = 6 * nfreq;
  c->g.lm_stride = 2 * np;
  HIPCHK(parent, hipStreamSynchronize(c->stream));
  const double setup_ms = ms_since(t0);
  double tune_ms = 0.0;
  if ((rc = autotune(c, c->nload, &tune_ms))) return pfail(rc);
  if (gate) tune_lock.unlock();
  arrive.now();
  // solve all microstructures x loads together
  auto t1 = std::chrono::steady_clock::now();
  c->use_graph = true;
  std::vector<fh::PcgState> hs;
  std::vector<int> outer;
  if (o.precision == FH_FP32_REFINED)
    rc = pcg_refined(c, c->nload, o.eta, default_eta_inner(o), o.itmax,
                     o.poll > 0 ? o.poll : 8, hs, outer);
  else
    rc = pcg64(c, c->nload, o.eta, o.itmax, o.poll > 0 ? o.poll : 16, hs);
  if (rc) return pfail(rc);
  // homogenized tensors (energy form, as fh_solve)
  if ((rc = apply_K(c, false, L.x, L.q, c->nload, F, nullptr, nullptr))) return pfail(rc);
  const int nchunk = 64;
  // fh_solve_batch admits nload <= 8, the size the buffer is laid out for
  double* part = L.pair_part;                                // nms x nchunk x nload^2
  double* dots = part + (size_t)nms * nchunk * nload * nload;  // 2 x nms x nload^2
  hipError_t e1 = fh::launch_pair_dots(L.b, L.x, F, nload, nms, nchunk, part, dots, c->stream);
  hipError_t e2 = fh::launch_pair_dots(L.x, L.q, F, nload, nms, nchunk, part,
                                       dots + (size_t)nms * nload * nload, c->stream);
  std::vector<double> hd((size_t)2 * nms * nload * nload);
  hipError_t e3 = hipMemcpyAsync(hd.data(), dots, hd.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream);
  hipError_t e4 = hipStreamSynchronize(c->stream);
  if (e1 || e2 || e3 || e4) return fail(parent, FH_EDEVICE, "batched C_hom reduction failed");
  const double solve_ms = ms_since(t1);
  for (int ms = 0; ms < nms; ++ms)
    if (sys[idx[ms]].u_dev)
      HIPCHK(parent, hipMemcpyAsync(sys[idx[ms]].u_dev, L.x + (size_t)ms * nload * F,
                                    sizeof(double) * nload * F, hipMemcpyDeviceToDevice,
                                    c->stream));
  HIPCHK(parent, hipStreamSynchronize(c->stream));
  const double vol = c->l[0] * c->l[1] * c->l[2];
  for (int ms = 0; ms < nms; ++ms) {
    const int sid = idx[ms];
    const double* bu = hd.data() + (size_t)ms * nload * nload;
    const double* uk = hd.data() + ((size_t)nms + ms) * nload * nload;
    double* H = chom + (size_t)sid * nload * nload;
    for (int i = 0; i < nload; ++i)
      for (int j = 0; j < nload; ++j) {
        double e = 0;
        for (int a = 0; a < 6; ++a)
          for (int b = 0; b < 6; ++b)
            e += E[(size_t)i * 6 + a] * c->cmean_ms[ms][a * 6 + b] * E[(size_t)j * 6 + b];
        H[i * nload + j] = e + (-bu[i * nload + j] - bu[j * nload + i] + uk[i * nload + j]) / vol;
      }
    if (st) {
      fh_stats s{};
      s.nload = nload;
      s.dof = F;
      for (int j = 0; j < nload; ++j) {
        const fh::PcgState& p = hs[(size_t)ms * nload + j];
        s.iterations[j] = p.iter;
        s.status[j] = status_code(p.status);
        s.rel_res[j] = p.last;
        s.outer[j] = outer.empty() ? 0 : outer[(size_t)ms * nload + j];
      }
      s.setup_ms = setup_ms;
      s.solve_ms = solve_ms;
      st[sid] = s;
    }
  }
  if (rep && gi < FH_MAX_GROUPS) {
    for (int k = 0; k < 3; ++k) rep->n[gi][k] = (&g0.nx)[k];
    rep->nsys[gi] = nms;
    rep->kz[gi] = c->g.kz;
    rep->zb[gi] = c->g.zb;
    rep->kyb[gi] = c->g.kyb;
    rep->xrows[gi] = c->g.xrows;
    rep->tune_ms[gi] = tune_ms;
    rep->setup_ms[gi] = setup_ms;
    rep->solve_ms[gi] = solve_ms;
  }
  for (const fh::PcgState& p : hs)
    if (status_code(p.status) < 0) return fail(parent, FH_ENOTSPD, "PCG breakdown in a batch");
  for (const fh::PcgState& p : hs)
    if (status_code(p.status) > 0) return FH_NOT_CONVERGED;
  return FH_OK;
}

}  // namespace

// Systems grouped by grid size, in order of first appearance.
int batch_groups(fh_ctx* c, int nsys, const fh_system* sys,
                 std::vector<std::vector<int>>& groups) {
  std::vector<std::array<int, 3>> sizes;
  groups.clear();
  for (int i = 0; i < nsys; ++i) {
    const fh_system& s = sys[i];
    if (!s.phase_dev || !s.mat || s.nphase < 1 || s.nphase > 16)
      return fail(c, FH_EINVAL, "bad system " + std::to_string(i));
    for (int k = 0; k < 3; ++k)
      if (s.n[k] < 2 || s.n[k] > 256 || !factor_ok(s.n[k]) || (k < 2 && s.n[k] % 2))
        return fail(c, FH_EINVAL, "bad grid size in system " + std::to_string(i));
    std::array<int, 3> key{s.n[0], s.n[1], s.n[2]};
    auto it = std::find(sizes.begin(), sizes.end(), key);
    if (it == sizes.end()) {
      sizes.push_back(key);
      groups.push_back({i});
    } else {
      groups[it - sizes.begin()].push_back(i);
    }
  }
  if ((int)groups.size() > FH_MAX_GROUPS) return fail(c, FH_EINVAL, "too many grid sizes");
  return FH_OK;
}

// Device bytes of one group's layout (fields, spectra, K^+, partial sums):
// the same computation as ensure_layout on a host-only context that carries
// the group's grid and load count.
size_t batch_group_bytes(const int n[3], int nms, int nload) {
  fh_ctx t;
  t.g.nx = n[0];
  t.g.ny = n[1];
  t.g.nz = n[2];
  t.g.dim = 3;
  t.g.nd = 3;
  t.g.nxh = n[0] / 2 + 1;
  t.g.N = (long long)n[0] * n[1] * n[2];
  t.g.nphase_max = 1;
  t.g.G = nload;
  t.nms = nms;
  t.nload = nms * nload;
  return align_up(layout(&t, nullptr, nullptr));
}

extern "C" int fh_batch_workspace_size(fh_ctx* c, int nsys, const fh_system* sys, int nload,
                                       size_t* bytes) {
  if (!c || nsys < 1 || !sys || nload < 1 || nload > 8 || !bytes) return FH_EINVAL;
  std::vector<std::vector<int>> groups;
  const int rc = batch_groups(c, nsys, sys, groups);
  if (rc) return rc;
  size_t total = 0;
  for (const auto& gr : groups) total += batch_group_bytes(sys[gr[0]].n, (int)gr.size(), nload);
  *bytes = total;
  return FH_OK;
}

extern "C" int fh_solve_batch(fh_ctx* c, int nsys, const fh_system* sys, int nload,
                              const double* E, const fh_opts* opt, double* chom, fh_stats* st,
                              fh_batch_report* rep) {
  if (!c || nsys < 1 || !sys || nload < 1 || nload > 8 || !E || !chom) return FH_EINVAL;
  hipSetDevice(c->device);
  fh_opts o{1e-10, 10000, FH_FP64, 0, 0, 0.0};
  if (opt) o = *opt;
  if (!(o.eta > 0.0) || o.itmax < 1) return fail(c, FH_EINVAL, "bad eta/itmax");
  std::vector<std::vector<int>> groups;
  int grc = batch_groups(c, nsys, sys, groups);
  if (grc) return grc;
  // with a workspace bound to the context, every group takes its layout
  // from it (disjoint regions in group order) instead of allocating one
  std::vector<char*> region(groups.size(), nullptr);
  std::vector<size_t> region_bytes(groups.size(), 0);
  if (c->ws_user) {
    size_t off = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      region_bytes[gi] = batch_group_bytes(sys[groups[gi][0]].n, (int)groups[gi].size(), nload);
      region[gi] = (char*)c->ws_user + off;
      off += region_bytes[gi];
    }
    if (off > c->ws_user_bytes)
      return fail(c, FH_ENOMEM, "bound workspace too small for the batch: need " +
                                    std::to_string(off) + " bytes");
  }
  if (rep) *rep = fh_batch_report{};
  if (rep) rep->ngroups = (int)groups.size();
  if (c->stream) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipDeviceSynchronize());
  }
  int worst = FH_OK;
  const int ng = (int)groups.size();
  if ((o.flags & FH_FLAG_BATCH_SERIAL) || ng == 1) {
    for (int gi = 0; gi < ng; ++gi) {
      const int rc = batch_group(c, groups[gi], sys, nload, E, o, chom, st, rep, gi, nullptr,
                                 region[gi], region_bytes[gi]);
      if (rc < 0) return rc;
      if (rc > 0) worst = rc;
    }
    return worst;
  }
  // groups of different grid sizes run concurrently, one host thread and one
  // stream each; every thread reports into its own error holder
  BatchGate gate;
  gate.total = ng;
  std::vector<fh_ctx> holders(ng);
  std::vector<int> rcs(ng, FH_OK);
  std::vector<std::thread> threads;
  int started = 0;
  for (int gi = 0; gi < ng; ++gi) holders[gi].device = c->device;
  try {
    for (int gi = 0; gi < ng; ++gi) {
      threads.emplace_back([&, gi] {
        hipSetDevice(c->device);
        try {
          rcs[gi] = batch_group(&holders[gi], groups[gi], sys, nload, E, o, chom, st, rep, gi,
                                &gate, region[gi], region_bytes[gi]);
        } catch (...) {  // host allocation failure inside the group
          rcs[gi] = FH_ENOMEM;
          holders[gi].err = "host exception in batch group " + std::to_string(gi);
        }
      });
      ++started;
    }
  } catch (...) {
    // a thread could not be started: the running groups stop waiting for
    // it at the start line, and the rest run here one after another
    {
      std::lock_guard<std::mutex> lk(gate.mu);
      gate.total = started;
      if (gate.waiting >= gate.total) gate.cv.notify_all();
    }
  }
  for (std::thread& t : threads) t.join();
  for (int gi = started; gi < ng; ++gi)
    rcs[gi] = batch_group(&holders[gi], groups[gi], sys, nload, E, o, chom, st, rep, gi, nullptr,
                          region[gi], region_bytes[gi]);
  for (int gi = 0; gi < ng; ++gi) {
    if (rcs[gi] < 0) return fail(c, rcs[gi], holders[gi].err);
    if (rcs[gi] > 0) worst = rcs[gi];
  }
  return worst;
}

// ================================================================ C-ABI
extern "C" {

int fh_create(fh_ctx** out, int device) {
  if (!out) return FH_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FH_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return FH_EDEVICE;
  if (!scratch_ptr(device)) return FH_EDEVICE;
  fh_ctx* c = new fh_ctx();
  c->device = device;
  if (hipMalloc((void**)&c->counts_dev, 256 * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc((void**)&c->flag_dev, sizeof(int)) != hipSuccess) {
    delete c;
    return FH_EDEVICE;
  }
  *out = c;
  return FH_OK;
}

void fh_destroy(fh_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  hipFree(c->ws_own);
  free_tables(c);
  free_plastic(c);
  free_sb(c);
  hipFree(c->bound_tab_dev);
  hipFree(c->counts_dev);
  hipFree(c->flag_dev);
  hipFree(c->twx);
  hipFree(c->twy);
  hipFree(c->twz);
  if (c->host_pinned) hipHostFree(c->host_pinned);
  for (hipEvent_t e : c->kt.ev) hipEventDestroy(e);
  hipFree(c->phase_pack);
  if (c->gstream) {
    hipStreamSynchronize(c->gstream);
    hipStreamDestroy(c->gstream);
  }
  if (c->gfork) hipEventDestroy(c->gfork);
  if (c->gjoin) hipEventDestroy(c->gjoin);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
}

const char* fh_last_error(const fh_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fh_set_stream(fh_ctx* c, void* s) {
  if (!c) return FH_EINVAL;
  c->stream = (hipStream_t)s;
  return FH_OK;
}

int fh_set_grid(fh_ctx* c, int dim, const int n[3], const double l[3], int problem,
                int element) {
  if (!c || !n) return FH_EINVAL;
  hipSetDevice(c->device);
  if (dim != 2 && dim != 3) return fail(c, FH_EINVAL, "dim must be 2 or 3");
  if (problem != FH_SCALAR && problem != FH_ELASTIC) return fail(c, FH_EINVAL, "bad problem");
  if ((dim == 3) != (element == FH_HEX8) ||
      (element != FH_HEX8 && element != FH_QUAD4 && element != FH_TRI2 && element != FH_TRI4))
    return fail(c, FH_EINVAL, "element does not match dim");
  if (element == FH_TRI4 && problem != FH_SCALAR)
    return fail(c, FH_EINVAL, "the two-node stencil is built for scalar problems");
  int nn[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  for (int k = 0; k < 3; ++k)
    if (nn[k] < 1 || nn[k] > 256 || !factor_ok(nn[k]))
      return fail(c, FH_EINVAL, "grid sizes must be products of 2 and 3 and at most 256");
  if (nn[0] % 2 || nn[1] % 2) return fail(c, FH_EINVAL, "nx and ny must be even");
  if (dim == 3 && nn[2] < 2) return fail(c, FH_EINVAL, "nz must be >= 2 in 3D");
  for (int k = 0; k < dim; ++k)
    if (l && !(l[k] > 0.0)) return fail(c, FH_EINVAL, "cell lengths must be positive");
  c->g = fh::Grid{};
  c->g.nx = nn[0];
  c->g.ny = nn[1];
  c->g.nz = nn[2];
  c->g.dim = dim;
  c->g.nd = (problem == FH_ELASTIC ? dim : 1) * (element == FH_TRI4 ? 2 : 1);
  c->g.tn = element == FH_TRI4 ? 1 : 0;
  c->g.nxh = nn[0] / 2 + 1;
  c->g.N = (long long)nn[0] * nn[1] * nn[2];
  c->g.nphase_max = 1;
  c->g.G = 1 << 30;
  for (int k = 0; k < 3; ++k) {
    c->l[k] = (l && k < dim) ? l[k] : 1.0;
    c->g.h[k] = c->l[k] / nn[k];
  }
  c->problem = problem;
  c->element = element;
  c->px = make_plan(nn[0]);
  c->py = make_plan(nn[1]);
  c->pz = make_plan(nn[2]);
  auto up = [&](cplx<double>** dst, int len) -> int {
    hipFree(*dst);
    *dst = nullptr;
    std::vector<cplx<double>> t = twiddle_table(len);
    HIPCHK(c, hipMalloc((void**)dst, sizeof(cplx<double>) * len));
    HIPCHK(c, hipMemcpy(*dst, t.data(), sizeof(cplx<double>) * len, hipMemcpyHostToDevice));
    return FH_OK;
  };
  int rc;
  if ((rc = up(&c->twx, nn[0])) || (rc = up(&c->twy, nn[1])) || (rc = up(&c->twz, nn[2])))
    return rc;
  c->has_grid = true;
  c->mat_kind = 0;
  c->nload = 0;
  // a reference set for the previous grid has the previous problem's size
  c->cref_user = false;
  c->cref_in.clear();
  c->cref.clear();
  c->layout_ok = false;
  c->symbol_ok = c->rhs_ok = c->solved = false;
  free_tables(c);
  free_plastic(c);
  free_sb(c);
  return FH_OK;
}

int fh_set_phases(fh_ctx* c, const uint8_t* phase_dev, int nphase, const double* mat) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  if (!phase_dev || !mat || nphase < 1 || nphase > 256)
    return fail(c, FH_EINVAL, "bad phase arguments");
  const int m = mdim(c);
  for (int p = 0; p < nphase; ++p)
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const double a = mat[(size_t)p * m * m + i * m + j], b = mat[(size_t)p * m * m + j * m + i];
        if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 * (std::fabs(a) + std::fabs(b)))
          return fail(c, FH_EINVAL, "material tables must be finite and symmetric");
      }
  if (c->plastic) free_plastic(c);
  c->phase_dev = phase_dev;
  c->nphase = nphase;
  c->g.nphase_max = nphase;
  c->phases_checked = false;
  c->mat.assign(mat, mat + (size_t)nphase * m * m);
  c->kfield_dev = nullptr;
  c->mat_kind = 1;
  std::vector<double> tab = operator_tables(c, c->mat.data(), nphase);
  int rc = upload(c, &c->mat_dev, &c->mat_dev_n, tab);
  if (rc) return rc;
  c->iso = false;
  if (hex_elastic(c)) {
    std::vector<double> lm(2 * (size_t)nphase);
    bool all = true;
    for (int p = 0; p < nphase && all; ++p)
      all = isotropic_lm(c->mat.data() + (size_t)p * 36, voxel_volume(c), lm.data() + 2 * p);
    if (all) {
      rc = upload(c, &c->lm_dev, &c->lm_dev_n, lm);
      if (rc) return rc;
      rc = upload_f(c, &c->lm_dev_f, lm);
      if (rc) return rc;
      c->iso = true;
    }
  }
  rc = upload_f(c, &c->mat_dev_f, tab);
  if (rc) return rc;
  c->sc = false;
  if (hex_scalar(c)) {
    std::vector<double> sk((size_t)nphase);
    bool all = true;
    for (int p = 0; p < nphase && all; ++p) {
      const double k = isotropic_k(c->mat.data() + (size_t)p * 9, 3);
      all = k > 0.0;
      sk[p] = voxel_volume(c) * k;
    }
    if (all) {
      if ((rc = upload(c, &c->sk_dev, &c->sk_dev_n, sk)) || (rc = upload_f(c, &c->sk_dev_f, sk)))
        return rc;
      c->sc = true;
    }
  }
  c->symbol_ok = c->rhs_ok = c->solved = false;
  return FH_OK;
}

int fh_set_conductivity_field(fh_ctx* c, const double* k_dev) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  if (c->problem != FH_SCALAR) return fail(c, FH_EINVAL, "conductivity field needs FH_SCALAR");
  if (!k_dev) return fail(c, FH_EINVAL, "null field");
  if (c->plastic) free_plastic(c);
  c->kfield_dev = k_dev;
  c->phase_dev = nullptr;
  c->mat_kind = 2;
  c->nphase = 0;
  std::vector<double> I((size_t)c->g.dim * c->g.dim, 0.0);
  for (int i = 0; i < c->g.dim; ++i) I[i * c->g.dim + i] = 1.0;
  c->mat = I;
  std::vector<double> tab = operator_tables(c, I.data(), 1);
  int rc = upload(c, &c->mat_dev, &c->mat_dev_n, tab);
  if (rc) return rc;
  rc = upload_f(c, &c->mat_dev_f, tab);
  if (rc) return rc;
  c->sc = false;
  if (hex_scalar(c)) {
    const std::vector<double> sk{voxel_volume(c)};
    if ((rc = upload(c, &c->sk_dev, &c->sk_dev_n, sk)) || (rc = upload_f(c, &c->sk_dev_f, sk)))
      return rc;
    c->sc = true;
  }
  c->symbol_ok = c->rhs_ok = c->solved = false;
  return FH_OK;
}

int fh_set_reference(fh_ctx* c, const double* Cref) {
  if (!c) return FH_EINVAL;
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  const int m = mdim(c);
  if (!Cref) {
    c->cref_user = false;
  } else {
    std::vector<double> v(Cref, Cref + (size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        if (std::fabs(v[i * m + j] - v[j * m + i]) > 1e-12 * (std::fabs(v[i * m + j]) + 1e-300))
          return fail(c, FH_EINVAL, "Cref must be symmetric");
    if (!cholesky_ok(v, m)) return fail(c, FH_ENOTSPD, "Cref is not positive definite");
    c->cref_in = v;
    c->cref_user = true;
  }
  c->symbol_ok = false;
  c->solved = false;
  return FH_OK;
}

int fh_set_load(fh_ctx* c, int nload, const double* E) {
  if (!c) return FH_EINVAL;
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  if (nload < 1 || nload > FH_MAX_LOADS || !E) return fail(c, FH_EINVAL, "bad loads");
  const int m = mdim(c);
  for (int i = 0; i < nload * m; ++i)
    if (!std::isfinite(E[i])) return fail(c, FH_EINVAL, "loads must be finite");
  c->nload = nload;
  c->loads.assign(E, E + (size_t)nload * m);
  c->rhs_ok = false;
  c->solved = false;
  return FH_OK;
}

int fh_workspace_size(fh_ctx* c, size_t* bytes) {
  if (!c || !bytes) return FH_EINVAL;
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  *bytes = layout(c, nullptr, nullptr);
  return FH_OK;
}

int fh_bind_workspace(fh_ctx* c, void* dev, size_t bytes) {
  if (!c) return FH_EINVAL;
  if (dev && ((uintptr_t)dev % 256)) return fail(c, FH_EINVAL, "workspace must be 256-byte aligned");
  c->ws_user = dev;
  c->ws_user_bytes = dev ? bytes : 0;
  c->layout_ok = false;
  c->symbol_ok = c->rhs_ok = c->solved = false;
  return FH_OK;
}

int fh_solve(fh_ctx* c, const fh_opts* opt, fh_stats* st) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  fh_opts o{1e-10, 10000, FH_FP64, 0, 0, 0.0};
  if (opt) o = *opt;
  if (!(o.eta > 0.0) || o.itmax < 1) return fail(c, FH_EINVAL, "bad eta/itmax");
  if (o.precision != FH_FP64 && o.precision != FH_FP32_REFINED)
    return fail(c, FH_EINVAL, "bad precision");

  if (c->nload < 1) return fail(c, FH_ESTATE, "fh_set_load not called");
  const int poll = o.poll > 0 ? o.poll : 16;
  auto t0 = std::chrono::steady_clock::now();
  c->solved = false;
  c->sb_solved = false;
  c->kt.on = (o.flags & FH_FLAG_TIME_KERNELS) != 0;
  c->kt.period = (o.flags & FH_FLAG_TIME_SAMPLED) ? 8 : 1;
  c->kt.sample = true;
  c->graph = (o.flags & FH_FLAG_GRAPH) != 0;
  if (o.flags & FH_FLAG_REBUILD) c->symbol_ok = c->rhs_ok = false;
  c->kt.used = 0;
  c->kt.timed_iters.clear();
  for (int k = 0; k < FH_K_NCLASS; ++k) {
    c->kt.ms[k] = 0.0;
    c->kt.n[k] = 0;
    c->kt.issued[k] = 0;
    c->kt.units[k] = 0.0;
  }
  int rc = build_symbol(c);
  if (rc) return rc;
  rc = build_rhs(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double setup_ms = ms_since(t0);
  auto t1 = std::chrono::steady_clock::now();
  std::vector<fh::PcgState> hs;
  std::vector<int> outer;
  const bool warm = (o.flags & FH_FLAG_WARM_START) || o.guess_dev;
  std::vector<double> rb, rr, gres;
  std::vector<int> used;
  double guess_ms = 0.0;
  if (warm) {
    if ((rc = ensure_layout(c))) return rc;
    rc = prepare_guess(c, o, rb, rr, gres, used);
    if (rc) return rc;
    guess_ms = ms_since(t1);
  }
  if (o.precision == FH_FP32_REFINED) {
    rc = pcg_refined(c, c->nload, o.eta, default_eta_inner(o), o.itmax, o.poll > 0 ? o.poll : 8,
                     hs, outer, warm ? &rb : nullptr);
  } else if (warm) {
    rc = pcg64_warm(c, c->nload, o.eta, o.itmax, poll, rb, rr, hs);
  } else {
    rc = pcg64(c, c->nload, o.eta, o.itmax, poll, hs);
  }
  if (rc) return rc;
  const double solve_ms = ms_since(t1);
  auto t2 = std::chrono::steady_clock::now();
  // homogenized tensor, energy form:
  // C[i][j] = e_i.Cmean e_j + (-b_i.u_j - b_j.u_i + u_i.K u_j) / |Y|
  const fh::Grid& g = c->g;
  const long long F = (long long)g.nd * g.N;
  const int nl = c->nload, m = mdim(c);
  rc = apply_K(c, false, c->L.x, c->L.q, nl, F, nullptr, nullptr);
  if (rc) return rc;
  std::vector<double> bu((size_t)nl * nl), uKu((size_t)nl * nl);
  if (nl <= 8) {
    // all load pairs in one pass over the fields (fixed-order chunk sums)
    const int nchunk = kPairChunks;
    double* part = c->L.pair_part;            // nchunk x nl^2
    double* out = part + (size_t)nchunk * 64;  // 2 x 64
    HIPCHK(c, fh::launch_pair_dots(c->L.b, c->L.x, F, nl, 1, nchunk, part, out, c->stream));
    HIPCHK(c, fh::launch_pair_dots(c->L.x, c->L.q, F, nl, 1, nchunk, part, out + 64,
                                   c->stream));
    HIPCHK(c, hipMemcpyAsync(bu.data(), out, sizeof(double) * nl * nl, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(uKu.data(), out + 64, sizeof(double) * nl * nl,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    double* scal = c->L.scal;
    const int nb = 1024;
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        HIPCHK(c, fh::launch_dot_partials(c->L.b + i * F, c->L.x + j * F, F, c->L.dot_part, nb,
                                          c->stream));
        HIPCHK(c, fh::launch_sum_partials(c->L.dot_part, nb, scal, c->stream));
        double v = 0;
        HIPCHK(c, hipMemcpyAsync(&v, scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, fh::launch_dot_partials(c->L.x + i * F, c->L.q + j * F, F, c->L.dot_part, nb,
                                          c->stream));
        HIPCHK(c, fh::launch_sum_partials(c->L.dot_part, nb, scal + 1, c->stream));
        double w = 0;
        HIPCHK(c, hipMemcpyAsync(&w, scal + 1, sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bu[(size_t)i * nl + j] = v;
        uKu[(size_t)i * nl + j] = w;
      }
  }
  double vol = 1.0;
  for (int k = 0; k < g.dim; ++k) vol *= c->l[k];
  c->chom.assign((size_t)nl * nl, 0.0);
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < nl; ++j) {
      double e = 0;
      const double* Ei = c->loads.data() + (size_t)i * m;
      const double* Ej = c->loads.data() + (size_t)j * m;
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) e += Ei[a] * c->cmean[a * m + b] * Ej[b];
      c->chom[(size_t)i * nl + j] =
          e + (-bu[(size_t)i * nl + j] - bu[(size_t)j * nl + i] + uKu[(size_t)i * nl + j]) / vol;
    }
  const double chom_ms = ms_since(t2);
  std::vector<double> hscale;
  if (warm && o.precision != FH_FP32_REFINED) {
    hscale.resize(nl);
    for (int j = 0; j < nl; ++j) hscale[j] = rb[j] > 0.0 ? std::sqrt(rr[j] / rb[j]) : 0.0;
  }
  if (o.precision == FH_FP32_REFINED) c->history.assign(nl, {});
  else record_history(c, hs, nl, warm ? &hscale : nullptr);
  c->solved = true;
  rc = fill_stats(c, hs, nl, st);
  for (int j = 0; j < nl && j < FH_MAX_LOADS && warm; ++j) {
    c->last.guess_used[j] = used[j];
    c->last.guess_res[j] = gres[j];
  }
  c->last.guess_ms = guess_ms;
  for (int j = 0; j < nl && j < FH_MAX_LOADS && j < (int)outer.size(); ++j)
    c->last.outer[j] = outer[j];
  c->last.setup_ms = setup_ms;
  c->last.solve_ms = solve_ms;
  c->last.chom_ms = chom_ms;
  for (int k = 0; k < FH_K_NCLASS; ++k) {
    c->last.kernel_ms[k] = c->kt.ms[k];
    c->last.kernel_launches[k] = c->kt.n[k];
    c->last.kernel_issued[k] = c->kt.issued[k];
    c->last.kernel_units[k] = c->kt.units[k];
  }
  c->kt.on = false;
  if (st) *st = c->last;
  return rc;
}

int fh_set_warm_start(fh_ctx* c, fh_net* net) {
  if (!c) return FH_EINVAL;
  c->net = net;
  return FH_OK;
}

int fh_get_fluctuation(fh_ctx* c, int load, double* u_dev) {
  if (!c || !u_dev) return FH_EINVAL;
  if (!c->solved) return fail(c, FH_ESTATE, "no solution available");
  if (load < 0 || load >= c->nload) return fail(c, FH_EINVAL, "bad load index");
  const long long F = (long long)c->g.nd * c->g.N;
  HIPCHK(c, hipMemcpyAsync(u_dev, c->L.x + load * F, F * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

int fh_get_homogenized(fh_ctx* c, double* Chom) {
  if (!c || !Chom) return FH_EINVAL;
  if (!c->solved && !c->sb_solved) return fail(c, FH_ESTATE, "no solution available");
  std::memcpy(Chom, c->chom.data(), c->chom.size() * sizeof(double));
  return FH_OK;
}

int fh_get_reference(fh_ctx* c, double* Cref) {
  if (!c || !Cref) return FH_EINVAL;
  if (!c->symbol_ok) return fail(c, FH_ESTATE, "reference not built yet");
  const size_t mm = (size_t)mdim(c) * mdim(c);
  if (c->cref.size() != mm) return fail(c, FH_ESTATE, "reference does not match the grid");
  std::memcpy(Cref, c->cref.data(), mm * sizeof(double));
  return FH_OK;
}

int fh_get_history(fh_ctx* c, int load, double* hist, int max, int* count) {
  if (!c || !count) return FH_EINVAL;
  if (load < 0 || load >= (int)c->history.size()) return fail(c, FH_EINVAL, "bad load index");
  const std::vector<double>& h = c->history[load];
  const int n = std::min((int)h.size(), max);
  if (hist && n > 0) std::memcpy(hist, h.data(), n * sizeof(double));
  *count = (int)h.size();
  return FH_OK;
}

int fh_apply_operator(fh_ctx* c, const double* u_dev, double* q_dev) {
  if (!c || !u_dev || !q_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  int rc = check_material(c);
  if (rc) return rc;
  const long long F = (long long)c->g.nd * c->g.N;
  rc = apply_K(c, false, u_dev, q_dev, 1, F, nullptr, nullptr);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

int fh_apply_preconditioner(fh_ctx* c, const double* r_dev, double* z_dev) {
  if (!c || !r_dev || !z_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  int rc = build_symbol(c);
  if (rc) return rc;
  const long long F = (long long)c->g.nd * c->g.N;
  HIPCHK(c, fh::launch_copy(c->L.r, r_dev, F, c->stream));
  rc = precond_fields(c, c->L.r, z_dev, 1, F);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

}  // extern "C"

namespace {
// Element forces of the uniform strain E for every material table (one unit
// table for a conductivity field), as k_rhs reads them.
int rhs_force_tables(fh_ctx* c, const double* E, std::vector<double>& fe) {
  int rc = check_material(c);
  if (rc) return rc;
  const int m = mdim(c);
  for (int i = 0; i < m; ++i)
    if (!std::isfinite(E[i])) return fail(c, FH_EINVAL, "loads must be finite");
  const int ntab = c->mat_kind == 1 ? c->nphase : 1;
  std::vector<double> unit((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) unit[i * m + i] = 1.0;
  fe.clear();
  for (int t = 0; t < ntab; ++t) {
    const double* C = c->mat_kind == 1 ? c->mat.data() + (size_t)t * m * m : unit.data();
    std::vector<double> f = uniform_strain_force(c, C, E);
    fe.insert(fe.end(), f.begin(), f.end());
  }
  return FH_OK;
}
}  // namespace

extern "C" {

int fh_compute_rhs_noalloc(fh_ctx* c, const double* E, double* b_dev) {
  if (!c || !E || !b_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  std::vector<double> fe;
  int rc = rhs_force_tables(c, E, fe);
  if (rc) return rc;
  if (fe.size() > (size_t)kRhsScratchDoubles)
    return fail(c, FH_EINVAL, "element force tables need " + std::to_string(fe.size()) +
                                  " doubles, the static staging holds " +
                                  std::to_string(kRhsScratchDoubles));
  double* stage = scratch_ptr(c->device);
  if (!stage) return fail(c, FH_EDEVICE, "hipGetSymbolAddress of the staging array failed");
  const int ntab = c->mat_kind == 1 ? c->nphase : 1;
  // every entry k_rhs reads is written here, so nothing of an earlier call
  // (a larger table) is ever read
  HIPCHK(c, hipMemcpyAsync(stage, fe.data(), fe.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, fh::launch_rhs(c->g, c->element, c->mat_kind == 1 ? c->phase_dev : nullptr,
                           c->mat_kind == 2 ? c->kfield_dev : nullptr, stage, ntab, 1, b_dev, 0,
                           c->stream));
  // the host table must outlive the copy, and the staging the kernel
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

int fh_compute_rhs(fh_ctx* c, const double* E, double* b_dev) {
  if (!c || !E || !b_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  std::vector<double> fe;
  int rc = rhs_force_tables(c, E, fe);
  if (rc) return rc;
  const int ntab = c->mat_kind == 1 ? c->nphase : 1;
  double* tmp = nullptr;
  HIPCHK(c, hipMalloc((void**)&tmp, fe.size() * sizeof(double)));
  hipError_t e1 = hipMemcpyAsync(tmp, fe.data(), fe.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream);
  hipError_t e2 = fh::launch_rhs(c->g, c->element, c->mat_kind == 1 ? c->phase_dev : nullptr,
                                 c->mat_kind == 2 ? c->kfield_dev : nullptr, tmp, ntab, 1, b_dev,
                                 0, c->stream);
  hipError_t e3 = hipStreamSynchronize(c->stream);
  hipFree(tmp);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
    return fail(c, FH_EDEVICE, "rhs kernel failed");
  return FH_OK;
}

int fh_get_symbol(fh_ctx* c, double* kplus_dev) {
  if (!c || !kplus_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  int rc = build_symbol(c);
  if (rc) return rc;
  const fh::Grid& g = c->g;
  const long long n = (long long)g.nxh * g.ny * g.nz * nsym_of(g);
  HIPCHK(c, hipMemcpyAsync(kplus_dev, c->L.kplus, n * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

int fh_solve_rhs(fh_ctx* c, const double* b_dev, double* u_dev, const fh_opts* opt,
                 fh_stats* st) {
  if (!c || !b_dev || !u_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  fh_opts o{1e-10, 10000, FH_FP64, 0, 0, 0.0};
  if (opt) o = *opt;
  if (!(o.eta > 0.0) || o.itmax < 1) return fail(c, FH_EINVAL, "bad eta/itmax");
  if (c->nload < 1) {
    // a single slot is enough
    c->nload = 1;
    c->loads.assign(mdim(c), 0.0);
    c->rhs_ok = false;
  }
  c->kt.on = false;
  int rc = build_symbol(c);
  if (rc) return rc;
  const long long F = (long long)c->g.nd * c->g.N;
  HIPCHK(c, fh::launch_copy(c->L.b, b_dev, F, c->stream));
  c->rhs_ok = false;  // slot 0 of b now holds the caller's vector
  c->solved = false;
  std::vector<fh::PcgState> hs;
  rc = pcg64(c, 1, o.eta, o.itmax, o.poll > 0 ? o.poll : 16, hs);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(u_dev, c->L.x, F * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  record_history(c, hs, 1);
  return fill_stats(c, hs, 1, st);
}

}  // extern "C"

// ============================================ eigenvalue bounds (Sec. 4.3)
namespace {

// Eigenvalues of a symmetric m x m matrix (cyclic Jacobi rotations).
std::vector<double> sym_eigvals(std::vector<double> A, int m) {
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i * m + j] * A[i * m + j];
        if (i != j) off += A[i * m + j] * A[i * m + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {  // columns p, q
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = cs * akp - sn * akq;
          A[k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {  // rows p, q
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = cs * apk - sn * aqk;
          A[q * m + k] = sn * apk + cs * aqk;
        }
      }
  }
  std::vector<double> ev(m);
  for (int i = 0; i < m; ++i) ev[i] = A[i * m + i];
  return ev;
}

// Smallest and largest generalized eigenvalue of (C, R), R SPD: the
// eigenvalues of L^-1 C L^-T with R = L L^T.
bool gen_eig_range(const double* C, const std::vector<double>& R, int m, double* lo, double* hi) {
  std::vector<double> L(R);
  for (int j = 0; j < m; ++j) {
    double d = L[j * m + j];
    for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double sm = L[i * m + j];
      for (int k = 0; k < j; ++k) sm -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = sm / d;
    }
    for (int k = j + 1; k < m; ++k) L[j * m + k] = 0.0;
  }
  // Y = L^-1 C (forward substitution per column), then A = L^-1 Y^T
  std::vector<double> Y((size_t)m * m), A((size_t)m * m);
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      double sm = C[i * m + col];
      for (int k = 0; k < i; ++k) sm -= L[i * m + k] * Y[k * m + col];
      Y[i * m + col] = sm / L[i * m + i];
    }
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      double sm = Y[col * m + i];  // (Y^T)[i][col]
      for (int k = 0; k < i; ++k) sm -= L[i * m + k] * A[k * m + col];
      A[i * m + col] = sm / L[i * m + i];
    }
  for (int i = 0; i < m; ++i)  // symmetrise the rounding
    for (int j = i + 1; j < m; ++j) A[i * m + j] = A[j * m + i] = 0.5 * (A[i * m + j] + A[j * m + i]);
  const std::vector<double> ev = sym_eigvals(A, m);
  *lo = *std::min_element(ev.begin(), ev.end());
  *hi = *std::max_element(ev.begin(), ev.end());
  return true;
}

// Per material table, the (lo, hi) generalized eigenvalue pair of
// (C_table, R); for a conductivity field, the pair of the unit conductivity.
int bound_tables(fh_ctx* c, const std::vector<double>& R, std::vector<double>& tab) {
  const int m = mdim(c);
  tab.clear();
  if (c->mat_kind == 1) {
    for (int p = 0; p < c->nphase; ++p) {
      double lo, hi;
      if (!gen_eig_range(c->mat.data() + (size_t)p * m * m, R, m, &lo, &hi))
        return fail(c, FH_ENOTSPD, "reference material is not SPD");
      tab.push_back(lo);
      tab.push_back(hi);
    }
  } else {
    std::vector<double> I((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) I[i * m + i] = 1.0;
    double lo, hi;
    if (!gen_eig_range(I.data(), R, m, &lo, &hi))
      return fail(c, FH_ENOTSPD, "reference material is not SPD");
    tab = {lo, hi};
  }
  return FH_OK;
}

// Classical CG estimate: the energy-norm error falls by eta within
// ceil(sqrt(kappa)/2 ln(2/eta)) iterations.
int cg_iteration_bound(double kappa, double eta) {
  if (!(kappa >= 1.0) || !(eta > 0.0) || eta >= 2.0) return 0;
  const double v = std::ceil(0.5 * std::sqrt(kappa) * std::log(2.0 / eta));
  return v > 2e9 ? 2000000000 : (int)v;
}

// Range of the nodal bounds for reference R over the whole grid: from the
// phases present (every voxel's pair is some node's extreme), or from the
// kernel's reduction for a conductivity field.
int bounds_range(fh_ctx* c, const std::vector<double>& R, double* lo, double* hi,
                 double* lo_dev, double* hi_dev) {
  std::vector<double> tab;
  int rc = bound_tables(c, R, tab);
  if (rc) return rc;
  if (c->mat_kind == 1 && !lo_dev && !hi_dev) {
    double a = HUGE_VAL, b = -HUGE_VAL;
    for (int p = 0; p < c->nphase; ++p)
      if (c->phase_counts[p] > 0) {
        a = std::min(a, tab[2 * p]);
        b = std::max(b, tab[2 * p + 1]);
      }
    *lo = a;
    *hi = b;
    return FH_OK;
  }
  rc = upload(c, &c->bound_tab_dev, &c->bound_tab_n, tab);
  if (rc) return rc;
  const fh::Grid& g = c->g;
  double* part = c->L.dot_part;  // 1024 doubles: 2 per block
  if (fh::node_bounds_partials(g) * 2 > 1024) return fail(c, FH_EINVAL, "bounds partials");
  HIPCHK(c, fh::launch_node_bounds(g, c->mat_kind == 1 ? c->phase_dev : nullptr,
                                   c->mat_kind == 2 ? c->kfield_dev : nullptr, c->bound_tab_dev,
                                   lo_dev, hi_dev, part, c->L.scal, c->stream));
  double r[2];
  HIPCHK(c, hipMemcpyAsync(r, c->L.scal, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *lo = r[0];
  *hi = r[1];
  return FH_OK;
}

// Isotropic Mandel stiffness with bulk modulus K and shear modulus G.
std::vector<double> iso_mandel(double K, double G) {
  std::vector<double> C(36, 0.0);
  const double lam = K - 2.0 * G / 3.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 6 + j] = lam + (i == j ? 2.0 * G : 0.0);
  for (int i = 3; i < 6; ++i) C[i * 6 + i] = 2.0 * G;
  return C;
}

}  // namespace

extern "C" {

int fh_eigen_bounds(fh_ctx* c, const double* Cref, double eta, double* lo_dev, double* hi_dev,
                    fh_bounds* out) {
  if (!c || !out) return FH_EINVAL;
  hipSetDevice(c->device);
  int rc = check_material(c);
  if (rc) return rc;
  if (c->element == FH_TRI4)
    return fail(c, FH_EINVAL, "eigenvalue bounds are built for one-node stencils");
  if ((rc = ensure_layout(c))) return rc;
  if ((rc = compute_mean(c))) return rc;
  const int m = mdim(c);
  std::vector<double> R = Cref ? std::vector<double>(Cref, Cref + (size_t)m * m)
                               : (c->cref_user ? c->cref_in : c->cmean);
  double lo = 0, hi = 0;
  if ((rc = bounds_range(c, R, &lo, &hi, lo_dev, hi_dev))) return rc;
  fh_bounds b{};
  b.lambda_min = lo;
  b.lambda_max = hi;
  b.kappa = hi / lo;
  b.predicted_iterations = cg_iteration_bound(b.kappa, eta);
  *out = b;
  return FH_OK;
}

int fh_choose_reference(fh_ctx* c, int strategy, double* Cref_out, fh_bounds* out) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  if (strategy < FH_REF_MEAN || strategy > FH_REF_BEST)
    return fail(c, FH_EINVAL, "unknown reference strategy");
  int rc = check_material(c);
  if (rc) return rc;
  if (c->element == FH_TRI4)
    return fail(c, FH_EINVAL, "eigenvalue bounds are built for one-node stencils");
  if ((rc = ensure_layout(c))) return rc;
  if ((rc = compute_mean(c))) return rc;
  const int m = mdim(c);
  std::vector<double> ident((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) ident[i * m + i] = 1.0;
  auto kappa_of = [&](const std::vector<double>& R, double* kap) -> int {
    double lo = 0, hi = 0;
    const int r = bounds_range(c, R, &lo, &hi, nullptr, nullptr);
    if (r) return r;
    *kap = hi / lo;
    return FH_OK;
  };
  std::vector<std::vector<double>> cand;
  if (strategy == FH_REF_MEAN || strategy == FH_REF_BEST) cand.push_back(c->cmean);
  if (strategy == FH_REF_IDENTITY || strategy == FH_REF_BEST) cand.push_back(ident);
  if (strategy == FH_REF_BEST && c->mat_kind == 1 && m == 6) {
    // isotropic phases: the isotropic reference with the smallest bound.  The
    // generalized eigenvalues of two isotropic stiffnesses are the ratios of
    // their bulk and shear moduli, so the bound depends only on K_r / G_r;
    // golden-section search in log(K_r / G_r), with G_r fixed by the mean.
    bool all_iso = true;
    for (int p = 0; p < c->nphase && all_iso; ++p) {
      double lm[2];
      all_iso = isotropic_lm(c->mat.data() + (size_t)p * 36, 1.0, lm);
    }
    double lmm[2];
    if (all_iso && isotropic_lm(c->cmean.data(), 1.0, lmm)) {
      const double Gm = 0.5 * lmm[1], Km = lmm[0] + lmm[1] / 3.0;
      auto f = [&](double s, double* kap) {  // s = log(K_r/G_r) - log(K_m/G_m)
        return kappa_of(iso_mandel(Km * std::exp(s), Gm), kap);
      };
      double a = -12.0, b = 12.0;
      const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
      double x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1, f2;
      if ((rc = f(x1, &f1)) || (rc = f(x2, &f2))) return rc;
      for (int it = 0; it < 80; ++it) {
        if (f1 <= f2) {
          b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a);
          if ((rc = f(x1, &f1))) return rc;
        } else {
          a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a);
          if ((rc = f(x2, &f2))) return rc;
        }
      }
      cand.push_back(iso_mandel(Km * std::exp(f1 <= f2 ? x1 : x2), Gm));
    }
  }
  int best = -1;
  double kbest = HUGE_VAL;
  for (size_t i = 0; i < cand.size(); ++i) {
    double k = 0;
    if ((rc = kappa_of(cand[i], &k))) return rc;
    if (k < kbest) {  // first of equal bounds wins: mean, then I_s
      kbest = k;
      best = (int)i;
    }
  }
  if ((rc = fh_set_reference(c, cand[best].data()))) return rc;
  if (Cref_out) std::copy(cand[best].begin(), cand[best].end(), Cref_out);
  if (out) {
    double lo = 0, hi = 0;
    if ((rc = bounds_range(c, cand[best], &lo, &hi, nullptr, nullptr))) return rc;
    out->lambda_min = lo;
    out->lambda_max = hi;
    out->kappa = hi / lo;
    out->predicted_iterations = 0;
  }
  return FH_OK;
}

}  // extern "C"

// ==================================== elasto-plastic Newton loop (Alg. 1)
namespace {

// Host sums (fixed order) of the material stage's per-block partials.
int plastic_sums(fh_ctx* c, std::vector<double>& out) {
  const int np = fh::plastic_parts();
  std::vector<double> part((size_t)c->pl_nb * np);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->pl_part, part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out.assign(np, 0.0);
  for (int b = 0; b < c->pl_nb; ++b)
    for (int k = 0; k < np; ++k) out[k] += part[(size_t)b * np + k];
  return FH_OK;
}

// sum of squares of a nodal field (device partials, fixed-order sum)
int field_dot(fh_ctx* c, const double* a, const double* b, long long n, double* out) {
  const int nb = 1024;
  HIPCHK(c, fh::launch_dot_partials(a, b, n, c->L.dot_part, nb, c->stream));
  HIPCHK(c, fh::launch_sum_partials(c->L.dot_part, nb, c->L.scal, c->stream));
  HIPCHK(c, hipMemcpyAsync(out, c->L.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

}  // namespace

extern "C" {

int fh_set_plastic_phases(fh_ctx* c, const uint8_t* phase_dev, int nphase, const double* params) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->has_grid) return fail(c, FH_ESTATE, "fh_set_grid not called");
  if (!hex_elastic(c) || c->g.dim != 3)
    return fail(c, FH_EINVAL, "plastic phases need 3D hex8 elasticity");
  if (!phase_dev || !params || nphase < 1 || nphase > 256)
    return fail(c, FH_EINVAL, "bad phase arguments");
  for (int p = 0; p < nphase; ++p) {
    const double K = params[4 * p], G = params[4 * p + 1], sy = params[4 * p + 2],
                 H = params[4 * p + 3];
    if (!(K > 0.0) || !(G > 0.0) || !(sy >= 0.0) || !(H > 0.0) || !std::isfinite(K) ||
        !std::isfinite(G) || !std::isfinite(sy) || !std::isfinite(H))
      return fail(c, FH_EINVAL, "plastic phase needs K > 0, G > 0, sy0 >= 0, H > 0 (finite)");
  }
  // the elastic stiffness of every phase: the material of the linear problem
  std::vector<double> mats((size_t)nphase * 36, 0.0);
  for (int p = 0; p < nphase; ++p) {
    const double K = params[4 * p], G = params[4 * p + 1];
    double* C = mats.data() + (size_t)p * 36;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) C[i * 6 + j] = K - 2.0 * G / 3.0 + (i == j ? 2.0 * G : 0.0);
    for (int i = 3; i < 6; ++i) C[i * 6 + i] = 2.0 * G;
  }
  int rc = fh_set_phases(c, phase_dev, nphase, mats.data());
  if (rc) return rc;
  const long long N = c->g.N;
  c->pl_params.assign(params, params + 4 * (size_t)nphase);
  c->pl_nb = fh::plastic_blocks(c->g, 2048);
  struct Buf { double** p; size_t n; };
  const Buf bufs[] = {{&c->pl_params_dev, 4 * (size_t)nphase}, {&c->pl_eps_p, 48 * (size_t)N},
                      {&c->pl_alpha, 8 * (size_t)N}, {&c->pl_ta, 8 * (size_t)N},
                      {&c->pl_tv, 48 * (size_t)N}, {&c->pl_fe, 24 * (size_t)N},
                      {&c->pl_u, 3 * (size_t)N},
                      {&c->pl_part, (size_t)c->pl_nb * fh::plastic_parts()}};
  for (const Buf& b : bufs) {
    if (hipMalloc((void**)b.p, b.n * sizeof(double)) != hipSuccess) {
      free_plastic(c);
      return fail(c, FH_ENOMEM, "hipMalloc of the plastic state failed");
    }
  }
  HIPCHK(c, hipMemcpy(c->pl_params_dev, params, 4 * (size_t)nphase * sizeof(double),
                      hipMemcpyHostToDevice));
  c->plastic = true;
  return FH_OK;
}

int fh_newton_solve(fh_ctx* c, const double* E_final, const fh_newton_opts* opt,
                    fh_newton_stats* st) {
  if (!c || !E_final) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->plastic) return fail(c, FH_ESTATE, "fh_set_plastic_phases not called");
  fh_newton_opts o{1e-8, 1e-10, 50, 10000, 1, FH_NEWTON_REF_TANGENT};
  if (opt) o = *opt;
  if (!(o.eta_newton > 0.0) || !(o.eta_cg > 0.0) || o.itmax_newton < 1 || o.itmax_cg < 1 ||
      o.nincrement < 1 || o.nincrement > FH_MAX_INCREMENTS ||
      o.itmax_newton > FH_MAX_NEWTON ||
      (o.ref_mode != FH_NEWTON_REF_TANGENT && o.ref_mode != FH_NEWTON_REF_ELASTIC))
    return fail(c, FH_EINVAL, "bad Newton options");
  for (int m = 0; m < 6; ++m)
    if (!std::isfinite(E_final[m])) return fail(c, FH_EINVAL, "loads must be finite");
  int rc = check_material(c);
  if (rc) return rc;
  if ((rc = ensure_layout(c))) return rc;
  c->pl_nbg = fh::plastic_blocks(c->g, c->L.nb_kop);
  auto t0 = std::chrono::steady_clock::now();
  const fh::Grid& g = c->g;
  const long long N = g.N, F = 3 * N;
  fh_ctx::Layout& L = c->L;
  fh_newton_stats s{};
  s.nincrement = o.nincrement;
  // the caller's reference is restored at the end
  const bool user_was = c->cref_user;
  const std::vector<double> user_in = c->cref_in;
  struct Restore {
    fh_ctx* c;
    bool user;
    const std::vector<double>& in;
    ~Restore() {
      c->qp_tangent = false;
      c->cref_user = user;
      c->cref_in = in;
      c->symbol_ok = false;
      c->solved = false;
    }
  } restore{c, user_was, user_in};
  HIPCHK(c, fh::launch_fill<double>(c->pl_eps_p, 0.0, 48 * N, c->stream));
  HIPCHK(c, fh::launch_fill<double>(c->pl_alpha, 0.0, 8 * N, c->stream));
  HIPCHK(c, fh::launch_fill<double>(c->pl_u, 0.0, F, c->stream));
  const double vol = c->l[0] * c->l[1] * c->l[2];
  std::vector<double> sums;
  bool elastic_ref_done = false;
  int result = FH_OK;
  for (int k = 1; k <= o.nincrement; ++k) {
    double E[6];
    for (int m = 0; m < 6; ++m) E[m] = E_final[m] * ((double)k / o.nincrement);
    bool conv = false;
    int steps = 0;
    for (int i = 0; i < o.itmax_newton; ++i) {
      // material stage at u_(i): stress, tangent, element forces; b = -D^T W sigma
      c->qp_tangent = false;
      HIPCHK(c, fh::launch_plastic_stage(0, g, c->phase_dev, c->pl_params_dev, E, c->pl_u,
                                         c->pl_fe, c->pl_eps_p, c->pl_alpha, c->pl_ta, c->pl_tv,
                                         c->pl_part, c->pl_nb, c->stream));
      HIPCHK(c, fh::launch_gather_nodes(g, c->pl_fe, -1.0, L.b, nullptr, nullptr, c->pl_nbg,
                                        c->stream));
      if ((rc = plastic_sums(c, sums))) return rc;
      double bb = 0.0;
      if ((rc = field_dot(c, L.b, L.b, F, &bb))) return rc;
      steps = i + 1;
      if (std::sqrt(bb) <= 1e-12 * std::sqrt(sums[6])) {
        // equilibrium to rounding (e.g. a uniform stress): no step
        s.pcg_iterations[k - 1][i] = 0;
        s.du_ratio[k - 1][i] = 0.0;
        conv = true;
        break;
      }
      // reference material: mean of the current tangent (Alg. 1 assembles
      // the preconditioner every step), or the mean elastic stiffness once
      if (o.ref_mode == FH_NEWTON_REF_TANGENT || !elastic_ref_done) {
        std::vector<double> Cr(36, 0.0);
        if (o.ref_mode == FH_NEWTON_REF_TANGENT) {
          const double Ks = sums[7] / vol, As = sums[8] / vol;
          for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
              const double one = (a < 3 && b < 3) ? 1.0 : 0.0;
              Cr[a * 6 + b] = Ks * one + As * ((a == b ? 1.0 : 0.0) - one / 3.0);
            }
          int t = 9;
          for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b, ++t) {
              Cr[a * 6 + b] -= sums[t] / vol;
              if (b != a) Cr[b * 6 + a] -= sums[t] / vol;
            }
          c->cref_in = Cr;
          c->cref_user = true;
        } else {
          c->cref_user = false;  // the mean elastic stiffness (Sec. 6.2)
          elastic_ref_done = true;
        }
        c->symbol_ok = false;
        if ((rc = build_symbol(c))) return rc;
      }
      // PCG for K_(i) du = b with the per-point tangent
      c->qp_tangent = true;
      HIPCHK(c, fh::launch_copy(L.r, L.b, F, c->stream));
      PcgBufs<double> bf{L.x, L.r, L.p, L.q, L.A, L.B, L.kplus};
      std::vector<fh::PcgState> hs;
      c->kt.on = false;
      rc = pcg_run<double>(c, 1, bf, o.eta_cg, o.itmax_cg, 16, std::vector<int>(1, 1), hs);
      c->qp_tangent = false;
      if (rc) return rc;
      s.pcg_iterations[k - 1][i] = hs[0].iter;
      s.total_pcg += hs[0].iter;
      const int pst = status_code(hs[0].status);
      if (pst < 0) return fail(c, FH_ENOTSPD, "PCG breakdown in a Newton step");
      if (pst > 0) result = FH_NOT_CONVERGED;
      HIPCHK(c, fh::launch_axpy(c->pl_u, 1.0, L.x, F, c->stream));
      double dd = 0.0, uu = 0.0;
      if ((rc = field_dot(c, L.x, L.x, F, &dd)) || (rc = field_dot(c, c->pl_u, c->pl_u, F, &uu)))
        return rc;
      const double ndu = std::sqrt(dd), nu = std::sqrt(uu);
      s.du_ratio[k - 1][i] = nu > 0.0 ? ndu / nu : 0.0;
      if (ndu <= o.eta_newton * nu) {
        conv = true;
        break;
      }
    }
    s.newton_steps[k - 1] = steps;
    s.converged[k - 1] = conv ? 1 : 0;
    if (!conv) result = FH_NOT_CONVERGED;
    // commit the internal variables at the converged displacement
    HIPCHK(c, fh::launch_plastic_stage(2, g, c->phase_dev, c->pl_params_dev, E, c->pl_u, nullptr,
                                       c->pl_eps_p, c->pl_alpha, nullptr, nullptr, c->pl_part,
                                       c->pl_nb, c->stream));
    if ((rc = plastic_sums(c, sums))) return rc;
    for (int m = 0; m < 6; ++m) s.macro_stress[k - 1][m] = sums[m] / vol;
    s.plastic_fraction[k - 1] = sums[30] / (8.0 * (double)N);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  s.solve_ms = ms_since(t0);
  if (st) *st = s;
  return result;
}

int fh_get_plastic_state(fh_ctx* c, double* u_dev, double* eps_p_dev, double* alpha_dev) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->plastic) return fail(c, FH_ESTATE, "fh_set_plastic_phases not called");
  const long long N = c->g.N;
  if (u_dev)
    HIPCHK(c, hipMemcpyAsync(u_dev, c->pl_u, 3 * N * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  if (eps_p_dev)
    HIPCHK(c, hipMemcpyAsync(eps_p_dev, c->pl_eps_p, 48 * N * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  if (alpha_dev)
    HIPCHK(c, hipMemcpyAsync(alpha_dev, c->pl_alpha, 8 * N * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

}  // extern "C"

// ============================ strain-based scheme with FE projection (Sec. 7.1)
namespace {

// Gamma0 tau = D Kref^+ D^T W tau with tau = C (x + E) (x may be null):
// element forces, nodal sum (sign), FFT pseudo-inverse, gradient.
int sb_green(fh_ctx* c, const double* x, const double* E, double sign, double* out) {
  const fh::Grid& g = c->g;
  const long long F = 3 * g.N;
  HIPCHK(c, fh::launch_sb_cdiv(g, c->phase_dev, c->sb_C, x, E, c->sb_fe, c->stream));
  HIPCHK(c, fh::launch_gather_nodes(g, c->sb_fe, sign, c->L.r, nullptr, nullptr,
                                    fh::plastic_blocks(g, 2048), c->stream));
  int rc = precond_fields(c, c->L.r, c->L.q, 1, F);
  if (rc) return rc;
  HIPCHK(c, fh::launch_sb_grad(g, c->L.q, out, c->stream));
  return FH_OK;
}

int sb_dot(fh_ctx* c, const double* C, const double* Mc, const double* a, const double* Ea,
           const double* b, const double* Eb, double* out) {
  const fh::Grid& g = c->g;
  const int nb = fh::sb_dot_partials(g);
  HIPCHK(c, fh::launch_sb_dot(g, c->phase_dev, C, Mc, a, Ea, b, Eb, c->L.dot_part, c->stream));
  HIPCHK(c, fh::launch_sum_partials(c->L.dot_part, nb, c->L.scal, c->stream));
  HIPCHK(c, hipMemcpyAsync(out, c->L.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

}  // namespace

extern "C" {

int fh_solve_strain_based(fh_ctx* c, const fh_opts* opt, fh_stats* st) {
  if (!c) return FH_EINVAL;
  hipSetDevice(c->device);
  fh_opts o{1e-10, 10000, FH_FP64, 0, 0, 0.0};
  if (opt) o = *opt;
  if (!(o.eta > 0.0) || o.itmax < 1) return fail(c, FH_EINVAL, "bad eta/itmax");
  if (o.precision != FH_FP64) return fail(c, FH_EINVAL, "the strain-based scheme runs in FP64");
  if (!c->has_grid || !hex_elastic(c) || c->g.dim != 3)
    return fail(c, FH_EINVAL, "the strain-based scheme needs 3D hex8 elasticity");
  if (c->mat_kind != 1) return fail(c, FH_ESTATE, "fh_set_phases not called");
  if (c->nload < 1) return fail(c, FH_ESTATE, "fh_set_load not called");
  c->kt.on = false;
  auto t0 = std::chrono::steady_clock::now();
  int rc = build_symbol(c);
  if (rc) return rc;
  const double t_setup = ms_since(t0);
  const fh::Grid& g = c->g;
  const long long N = g.N, Q = 48 * N;
  const int nl = c->nload;
  if (c->sb_nload != nl) {
    free_sb(c);
    struct Buf { double** p; size_t n; };
    const Buf bufs[] = {{&c->sb_eps, (size_t)nl * Q}, {&c->sb_r, (size_t)Q}, {&c->sb_p, (size_t)Q},
                        {&c->sb_q, (size_t)Q}, {&c->sb_fe, 24 * (size_t)N},
                        {&c->sb_C, 36 * (size_t)c->nphase}};
    for (const Buf& b : bufs)
      if (hipMalloc((void**)b.p, b.n * sizeof(double)) != hipSuccess) {
        free_sb(c);
        return fail(c, FH_ENOMEM, "hipMalloc of the strain-based fields failed");
      }
    c->sb_nload = nl;
  }
  HIPCHK(c, hipMemcpy(c->sb_C, c->mat.data(), 36 * (size_t)c->nphase * sizeof(double),
                      hipMemcpyHostToDevice));
  c->sb_solved = false;
  c->solved = false;
  const double* Cref = c->cref.data();
  std::vector<fh::PcgState> hs(nl);
  c->history.assign(nl, {});
  t0 = std::chrono::steady_clock::now();
  for (int j = 0; j < nl; ++j) {
    const double* E = c->loads.data() + 6 * (size_t)j;
    double* x = c->sb_eps + (size_t)j * Q;
    fh::PcgState& s = hs[j];
    s = fh::PcgState{};
    HIPCHK(c, fh::launch_fill<double>(x, 0.0, Q, c->stream));
    // r0 = -Gamma0 C e, p0 = r0
    if ((rc = sb_green(c, nullptr, E, -1.0, c->sb_r))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->sb_p, c->sb_r, Q * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    double rho = 0.0;
    if ((rc = sb_dot(c, nullptr, Cref, c->sb_r, nullptr, c->sb_r, nullptr, &rho))) return rc;
    s.rho0 = rho;
    s.status = fh::ST_CONVERGED;
    if (!(rho > 0.0)) continue;
    s.status = fh::ST_MAXIT;
    for (int k = 1; k <= o.itmax; ++k) {
      if ((rc = sb_green(c, c->sb_p, nullptr, 1.0, c->sb_q))) return rc;
      double pq = 0.0;
      if ((rc = sb_dot(c, nullptr, Cref, c->sb_p, nullptr, c->sb_q, nullptr, &pq))) return rc;
      if (!(pq > 0.0)) {
        s.status = fh::ST_BREAKDOWN;
        break;
      }
      const double alpha = rho / pq;
      HIPCHK(c, fh::launch_axpy(x, alpha, c->sb_p, Q, c->stream));
      HIPCHK(c, fh::launch_axpy(c->sb_r, -alpha, c->sb_q, Q, c->stream));
      double rho_new = 0.0;
      if ((rc = sb_dot(c, nullptr, Cref, c->sb_r, nullptr, c->sb_r, nullptr, &rho_new)))
        return rc;
      s.iter = k;
      s.last = rho_new > 0.0 ? std::sqrt(rho_new / s.rho0) : 0.0;
      c->history[j].push_back(s.last);
      if (!(rho_new >= 0.0)) {
        s.status = fh::ST_BREAKDOWN;
        break;
      }
      if (rho_new <= o.eta * o.eta * s.rho0) {
        s.status = fh::ST_CONVERGED;
        break;
      }
      HIPCHK(c, fh::launch_sb_xpby(c->sb_p, c->sb_r, rho_new / rho, Q, c->stream));
      rho = rho_new;
    }
  }
  const double t_solve = ms_since(t0);
  // C_hom[i][j] = (1/|Y|) sum_Q w (e_i + eps_i)^T C (e_j + eps_j)
  t0 = std::chrono::steady_clock::now();
  const double vol = c->l[0] * c->l[1] * c->l[2];
  c->chom.assign((size_t)nl * nl, 0.0);
  for (int i = 0; i < nl; ++i)
    for (int j = i; j < nl; ++j) {
      double v = 0.0;
      if ((rc = sb_dot(c, c->sb_C, nullptr, c->sb_eps + (size_t)i * Q, c->loads.data() + 6 * i,
                       c->sb_eps + (size_t)j * Q, c->loads.data() + 6 * j, &v)))
        return rc;
      c->chom[(size_t)i * nl + j] = c->chom[(size_t)j * nl + i] = v / vol;
    }
  c->sb_solved = true;
  rc = fill_stats(c, hs, nl, nullptr);
  c->last.setup_ms = t_setup;
  c->last.solve_ms = t_solve;
  c->last.chom_ms = ms_since(t0);
  if (st) *st = c->last;
  return rc;
}

int fh_get_strain(fh_ctx* c, int load, double* eps_dev) {
  if (!c || !eps_dev) return FH_EINVAL;
  hipSetDevice(c->device);
  if (!c->sb_solved) return fail(c, FH_ESTATE, "fh_solve_strain_based not called");
  if (load < 0 || load >= c->sb_nload) return fail(c, FH_EINVAL, "load index out of range");
  const long long Q = 48 * c->g.N;
  HIPCHK(c, hipMemcpyAsync(eps_dev, c->sb_eps + (size_t)load * Q, Q * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FH_OK;
}

}  // extern "C"
