// Solver orchestration on the host: batched (F)GMRES, the multigrid cycle,
// the adaptive setup and the outer FP64 solve.
//
// Paper section 4: FGMRES at the top level (goal residual 1e-10), a
// (non-block) FGMRES on the middle level to r_m ~ 7e-2 preconditioned by the
// next level, GMRES on the bottom level to r_b ~ 1e-1; orthogonalisation by
// classical Gram-Schmidt without re-orthogonalisation.  Section 2: the
// preconditioner combines the coarse-grid correction with SAP smoothing.
//
// Every column (one rhs x one twisted mass) runs its own Arnoldi process; all
// columns advance together through batched kernels, and each column's
// solution uses exactly the iterations up to the one at which it met its own
// tolerance.  The small Hessenberg least-squares problems are solved on the
// host after one device->host copy per iteration.
#include <algorithm>
#include <chrono>
#include <complex>
#include <functional>
#include <map>
#include <tuple>

#include "common.h"
#include "hess_eig.h"
#include "device.h"

namespace ddamg {

void build_geometry(ddamg_ctx* c, int level, const int* dims, const int* grp, int dof, bool fine);
void random_fill(ddamg_ctx* c, int level, const MV& X, int ncol, uint64_t seed);

using cd = std::complex<double>;
using Precond = std::function<void(const MV& v, const MV& z, const double* d_mu)>;
constexpr int KMAX = 64;

// ------------------------------------------------------------ kernels ---
// x_col /= sqrt(n2_col): one lane per 16-byte chunk (column t = unit mod T)
template <typename C>
__global__ void k_normalize(C* __restrict__ x, const double* __restrict__ n2, size_t nunits, int T,
                            size_t tile_units) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const size_t col = (u / tile_units) * T + u % T;
    const double v = n2[col];
    C a = x[u];
    if constexpr (sizeof(a.x) == 8) {
      const double sc = v > 0 ? 1.0 / sqrt(v) : 0.0;
      a.x *= sc; a.y *= sc;
    } else {
      const float sc = (float)(v > 0 ? 1.0 / sqrt(v) : 0.0);
      a.x *= sc; a.y *= sc; a.z *= sc; a.w *= sc;
    }
    x[u] = a;
  }
}

void mv_normalize(ddamg_ctx* c, const MV& x, const double* d_n2) {
  DD_CHECK(x.prec == P64 || x.prec == P32, DDAMG_EINVAL, "mv_normalize: FP64 or FP32");
  const size_t tile_units = (size_t)x.nchunk * x.nsites * x.T, nunits = tile_units * x.ntiles;
  size_t g = (nunits + 255) / 256;
  if (g > 65536) g = 65536;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_normalize<double2>, dim3((unsigned)g), dim3(256), 0, c->stream, (double2*)x.p, d_n2, nunits,
                       x.T, tile_units);
  else
    hipLaunchKernelGGL(k_normalize<float4>, dim3((unsigned)g), dim3(256), 0, c->stream, (float4*)x.p, d_n2, nunits,
                       x.T, tile_units);
  DD_HIP(hipGetLastError());
}

// One-reduction Arnoldi step.  dots: [j+2][ncol] complex, <V_q, w> for q <= j
// and <w, w> last.  osc[col] = 1 / ||w - V h|| predicted as
// sqrt(<w, w> - sum_q |h_q|^2) (Pythagoras: the orthogonalised vector and the
// projection are orthogonal); when that difference is not safely positive
// (cancellation) the scale falls back to 1 / ||w||, and the norm measured in
// the update pass corrects it.  A zero w gets osc = 0.
__global__ void k_lowsync_scale(int j, int ncol, const double* __restrict__ dots, double* __restrict__ osc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncol) return;
  const double om = dots[((size_t)(j + 1) * ncol + i) * 2];
  double s = om;
  for (int q = 0; q <= j; ++q) {
    const double re = dots[((size_t)q * ncol + i) * 2], im = dots[((size_t)q * ncol + i) * 2 + 1];
    s -= re * re + im * im;
  }
  osc[i] = om > 0 ? 1.0 / sqrt(s > 1e-6 * om ? s : om) : 0.0;
}

// The correcting rescale of the one-reduction step: columns whose stored
// vector's squared norm n2 is off 1 by more than tau are divided by sqrt(n2);
// the others are left untouched (and not read).
template <typename C>
__global__ void k_renorm(C* __restrict__ x, const double* __restrict__ n2, size_t nunits, int T, size_t tile_units,
                         double tau) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const size_t col = (u / tile_units) * T + u % T;
    const double v = n2[col];
    if (!(v > 0) || fabs(v - 1.0) <= tau) continue;
    C a = x[u];
    if constexpr (sizeof(a.x) == 8) {
      const double sc = 1.0 / sqrt(v);
      a.x *= sc; a.y *= sc;
    } else {
      const float sc = (float)(1.0 / sqrt(v));
      a.x *= sc; a.y *= sc; a.z *= sc; a.w *= sc;
    }
    x[u] = a;
  }
}

// Tolerance on |n2 - 1| below which the predicted normalisation stands: far
// above the prediction's rounding error (FP64 dots) and the stored vector's
// own rounding, so that only a prediction that cancelled is corrected.
static double renorm_tau(const ddamg_ctx* c, int prec) {
  if (c->gram_lowsync == 2) return -1.0;
  return prec == P64 ? 1e-12 : 1e-6;
}

static void mv_renorm(ddamg_ctx* c, const MV& x, const double* d_n2, double tau) {
  const size_t tile_units = (size_t)x.nchunk * x.nsites * x.T, nunits = tile_units * x.ntiles;
  size_t g = (nunits + 255) / 256;
  if (g > 65536) g = 65536;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_renorm<double2>, dim3((unsigned)g), dim3(256), 0, c->stream, (double2*)x.p, d_n2, nunits,
                       x.T, tile_units, tau);
  else
    hipLaunchKernelGGL(k_renorm<float4>, dim3((unsigned)g), dim3(256), 0, c->stream, (float4*)x.p, d_n2, nunits,
                       x.T, tile_units, tau);
  DD_HIP(hipGetLastError());
}

// Doublets: the two columns of a pair form one vector, so their dots and
// squared norms are summed and the sum given to both.  h: [nq][ncol] complex.
__global__ void k_pair_sum_c(double* __restrict__ h, int nq, int ncol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = ncol / 2;
  if (i >= nq * np) return;
  const int q = i / np, pr = i % np;
  double* a = h + ((size_t)q * ncol + 2 * pr) * 2;
  const double re = a[0] + a[2], im = a[1] + a[3];
  a[0] = a[2] = re;
  a[1] = a[3] = im;
}

__global__ void k_pair_sum_r(double* __restrict__ n2, int ncol) {
  const int pr = blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= ncol / 2) return;
  const double v = n2[2 * pr] + n2[2 * pr + 1];
  n2[2 * pr] = n2[2 * pr + 1] = v;
}

static void pair_sum_c(ddamg_ctx* c, double* h, int nq, int ncol) {
  const int n = nq * (ncol / 2);
  hipLaunchKernelGGL(k_pair_sum_c, dim3((n + 255) / 256), dim3(256), 0, c->stream, h, nq, ncol);
  DD_HIP(hipGetLastError());
}

static void pair_sum_r(ddamg_ctx* c, double* n2, int ncol) {
  hipLaunchKernelGGL(k_pair_sum_r, dim3((ncol / 2 + 255) / 256), dim3(256), 0, c->stream, n2, ncol);
  DD_HIP(hipGetLastError());
}

// While alive, the fine operator is the doublet operator with epsbar per
// column at `eps` (or the flavour-diagonal one with eps = nullptr).
struct NDScope {
  ddamg_ctx* c;
  const double* saved;
  NDScope(ddamg_ctx* c_, const double* eps) : c(c_), saved(c_->nd_eps) { c->nd_eps = eps; }
  ~NDScope() { c->nd_eps = saved; }
};

// dst (FP16 basis, same layout) = src (FP32) / sqrt(n2_col) * hscale: the
// normalisation and the store of a new basis vector in one pass
__global__ void k_normalize_f16(const float* __restrict__ src, _Float16* __restrict__ dst,
                                const double* __restrict__ n2, size_t nunits, int T, size_t tile_units,
                                double hscale) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(u / tile_units) * T + (int)(u % T);
    const double v = n2[col];
    const float sc = (float)(v > 0 ? hscale / sqrt(v) : 0.0);
    const float4 a = reinterpret_cast<const float4*>(src)[u];
    _Float16* d = dst + u * 4;
    d[0] = (_Float16)(a.x * sc);
    d[1] = (_Float16)(a.y * sc);
    d[2] = (_Float16)(a.z * sc);
    d[3] = (_Float16)(a.w * sc);
  }
}

static void mv_normalize_into_f16(ddamg_ctx* c, const MV& src, const double* d_n2, const MV& dst) {
  DD_CHECK(src.prec == P32 && dst.prec == P16 && src.reals() == dst.reals(), DDAMG_EINVAL, "normalize into FP16");
  const size_t tile_units = (size_t)src.nchunk * src.nsites * src.T, nunits = tile_units * src.ntiles;
  size_t g = (nunits + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_normalize_f16, dim3((unsigned)g), dim3(256), 0, c->stream, src.as<float>(),
                     dst.as<_Float16>(), d_n2, nunits, src.T, tile_units, dst.hscale);
  DD_HIP(hipGetLastError());
}

// alpha = <q, r> / <q, q> per column (MR step), 0 where <q,q> = 0
__global__ void k_mr_alpha(const double* __restrict__ qr, const double* __restrict__ qq, double* __restrict__ a,
                           int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = qq[i];
  a[2 * i] = d > 0 ? qr[2 * i] / d : 0.0;
  a[2 * i + 1] = d > 0 ? qr[2 * i + 1] / d : 0.0;
}

// -------------------------------------------------------- workspaces ---
struct LW {
  int cap = 0;                   // tiles
  int prec = 0;
  std::vector<MV> V, Z;
  MV zt, rc, ec, res, s, q, rho;
  MV cb, cx, cb2, cx2;           // outer solve: active right-hand sides / solutions (ping-pong)
  int vprec = -1;                // storage precision of the Arnoldi basis V (P16 or the working precision)
  MV wt, vi;                     // FP16 basis: working-precision new vector and preconditioner input
  double* d_h = nullptr;         // [KMAX][ncol] complex dots + [ncol] norm
  double* d_aux = nullptr;       // [ncol] complex scratch for MR / coefficients
  double* d_vsc = nullptr;       // FP16 basis: [KMAX+1][ncol] 1/c_j^2 of the stored vectors + [ncol] store scale
  double* d_osc = nullptr;       // [ncol] output scales of the one-reduction Arnoldi step
  int* d_map = nullptr;          // [3][ncol] column maps of the outer solve's scheduler
  double* d_muc = nullptr;       // [ncol] shifts of the active columns
  double* d_epsc = nullptr;      // [ncol] doublet coupling epsbar of the active columns
  struct GraphState* gs = nullptr;   // captured GMRES steps (unpreconditioned solves)
};

// Captured Arnoldi steps of an unpreconditioned GMRES(m) on one workspace:
// one executable graph per step j, valid for one tile count, restart length
// and set of tile-shape knobs; every buffer a graph touches is owned here or
// by the workspace, so the recorded pointers stay valid until the workspace
// is reallocated (which destroys the graphs).
struct GraphState {
  int nt = -1, m = 0, ncol = 0, g5 = 0;
  int knobs[7] = {0, 0, 0, 0, 0, 0, 0};
  double *d_H = nullptr, *d_cs = nullptr, *d_sn = nullptr, *d_g = nullptr, *d_tol = nullptr, *d_est = nullptr;
  double *d_n2 = nullptr, *d_cbuf = nullptr, *d_part = nullptr, *d_mu = nullptr, *d_coef = nullptr;
  double *d_osc = nullptr, *d_apart = nullptr;   // one-reduction step: output scales, update partials
  int *d_kc = nullptr, *d_done = nullptr;
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> exec;
};

static void destroy_graphs(ddamg_ctx* c, GraphState* g) {
  if (!g) return;
  for (auto e : g->exec)
    if (e) hipGraphExecDestroy(e);
  for (auto q : g->graph)
    if (q) hipGraphDestroy(q);
  double* dbl[] = {g->d_H, g->d_cs, g->d_sn, g->d_g, g->d_tol, g->d_est, g->d_n2, g->d_cbuf, g->d_part, g->d_mu,
                   g->d_coef, g->d_osc, g->d_apart};
  for (double* p : dbl)
    if (p) c->pool.release(p);
  if (g->d_kc) c->pool.release(g->d_kc);
  if (g->d_done) c->pool.release(g->d_done);
  delete g;
}

struct Work {
  std::map<std::tuple<int, int, int>, LW> lw;   // (level, precision, role)
};

static Work& work(ddamg_ctx* c) {
  if (!c->work) c->work = new Work();
  return *static_cast<Work*>(c->work);
}

void free_work(ddamg_ctx* c) {
  if (!c->work) return;
  for (auto& kv : static_cast<Work*>(c->work)->lw) destroy_graphs(c, kv.second.gs);
  delete static_cast<Work*>(c->work);
  c->work = nullptr;
}

// Workspace of one Krylov solver: role 0 for the solver of a level, role 1
// for the inner FGMRES of the outer solve (same level, its own basis).
static LW& lw(ddamg_ctx* c, int level, int prec, int ntiles, int role = 0) {
  LW& w = work(c).lw[{level, prec, role}];
  // the inner FGMRES of the outer solve, and (coarse_fp16) the solves of the
  // coarse levels, may keep their bases in FP16
  if (w.vprec < 0)
    w.vprec = (prec == P32 && ((role == 1 && c->p.inner_fp16) || (role == 0 && level > 0 && c->p.coarse_fp16)))
                  ? P16 : prec;
  if (ntiles > w.cap) {
    for (auto& m : w.V) mv_free(c, m);
    for (auto& m : w.Z) mv_free(c, m);
    MV* all[] = {&w.zt, &w.rc, &w.ec, &w.res, &w.s, &w.q, &w.rho, &w.cb, &w.cx, &w.cb2, &w.cx2, &w.wt, &w.vi};
    for (MV* m : all) mv_free(c, *m);
    w.V.clear();
    w.Z.clear();
    if (w.d_h) c->pool.release(w.d_h);
    if (w.d_aux) c->pool.release(w.d_aux);
    if (w.d_vsc) c->pool.release(w.d_vsc);
    if (w.d_osc) c->pool.release(w.d_osc);
    if (w.d_map) c->pool.release(w.d_map);
    if (w.d_muc) c->pool.release(w.d_muc);
    if (w.d_epsc) c->pool.release(w.d_epsc);
    w.d_map = nullptr;
    w.d_muc = nullptr;
    w.d_epsc = nullptr;
    destroy_graphs(c, w.gs);
    w.gs = nullptr;
    w.cap = ntiles;
    w.prec = prec;
    const int ncol = ntiles * c->T;
    w.d_h = (double*)c->pool.alloc(((size_t)KMAX * ncol * 2 + ncol) * sizeof(double));
    w.d_aux = (double*)c->pool.alloc((size_t)KMAX * ncol * 2 * sizeof(double));
    w.d_vsc = (double*)c->pool.alloc((size_t)(KMAX + 2) * ncol * sizeof(double));
    w.d_osc = (double*)c->pool.alloc((size_t)ncol * sizeof(double));
  }
  return w;
}

static MV get(ddamg_ctx* c, MV& slot, int level, int prec, int cap, int nt) {
  if (!slot.p) slot = mv_alloc(c, level, prec, cap * c->T);
  return slot.tiles(0, nt);
}

static MV basis(ddamg_ctx* c, std::vector<MV>& vec, int j, int level, int prec, int cap, int nt) {
  while ((int)vec.size() <= j) vec.push_back(MV{});
  return get(c, vec[j], level, prec, cap, nt);
}

// ------------------------------------------------------------ Krylov ---
struct KrylovOut {
  std::vector<int> iters;
  std::vector<double> relres;   // Arnoldi estimate / ||b|| at exit
  int total = 0;
};

static double host_norm_guard(double v) { return v > 0 ? std::sqrt(v) : 0.0; }

// Host-side state of one restarted (F)GMRES cycle over ncol lockstep columns:
// Hessenberg matrices, Givens rotations and right-hand sides per column.
struct Cycle {
  int m = 0;
  std::vector<cd> H, g, sn;
  std::vector<double> cs, hbuf, coef;
  std::vector<int> kc;          // Arnoldi steps used per column (-1: all of the cycle)
  // FP16 basis stored unnormalised: entry scale c_j of each stored vector,
  // 1/c_j^2 and the store scale of the next vector (uploaded each step)
  std::vector<double> cj, vsc, nstore, osc_exact;
  std::vector<double> osc;      // one-reduction step: output scales of the last step (host copy)
  bool pairs = false;           // doublets: columns 2i, 2i+1 form one Krylov vector
  Cycle(int ncol, int m_) : m(m_), H((size_t)ncol * (m_ + 1) * m_), g((size_t)ncol * (m_ + 1)), sn((size_t)ncol * m_),
                            cs((size_t)ncol * m_), hbuf((size_t)KMAX * ncol * 2 + ncol), kc(ncol),
                            cj((size_t)(m_ + 1) * ncol, 1.0), vsc((size_t)(KMAX + 2) * ncol, 1.0), nstore(ncol, 1.0),
                            osc_exact(ncol, 1.0), osc(ncol, 1.0) {}
};

// One (F)GMRES cycle on the first nt tiles of the level's workspace: V[0]
// holds the residual r with per-column norms beta (host; d_n2 holds their
// squares).  Up to min(m, budget) Arnoldi steps with classical Gram-Schmidt
// (one fused multi-dot and multi-axpy per step, section 4), per-column Givens
// least squares on the host, then x += Z y (or V y).  Columns flagged done take
// no step; a column whose estimate meets tol_abs stops at that step.  Returns
// the number of steps; cy.kc[i] the steps that entered column i's update.
static int gmres_cycle(ddamg_ctx* c, int level, LW& w, int nt, const MV& x, const double* d_mu, const Precond* pc,
                       int zprec, int budget, bool fixed, const std::vector<double>& beta, std::vector<char>& done,
                       const std::vector<double>& tol_abs, std::vector<double>& est, const std::vector<double>& bn,
                       Cycle& cy, double* d_n2, int& total, bool pc_f16 = false) {
  const int prec = x.prec, ncol = nt * c->T, cap = w.cap, m = cy.m, vprec = w.vprec;
  const bool half = vprec != prec;   // FP16 basis: new vectors are formed in the working precision
  MV r = half ? get(c, w.wt, level, prec, cap, nt) : basis(c, w.V, 0, level, vprec, cap, nt);
  if (half) mv_normalize_into_f16(c, r, d_n2, basis(c, w.V, 0, level, vprec, cap, nt));
  else mv_normalize(c, r, d_n2);
  // FP16 basis: later vectors are stored unnormalised, as w' / nstore (nstore:
  // a prediction of |w'| made before it is known), and carry the entry scale
  // c_j = |w'| / nstore; the first one is normalised (c_0 = 1).  The stored
  // vectors are used as they are (preconditioner and operator inputs, Z):
  // the Arnoldi relation then holds with H_qj = <v_q, A z_j>, v_q = V_q / c_q
  const double hscale = half ? basis(c, w.V, 0, level, vprec, cap, nt).hscale : 1.0;
  double* d_cinv2 = w.d_vsc;
  double* d_osc = w.d_vsc + (size_t)(KMAX + 1) * ncol;
  if (half) {
    for (int i = 0; i < ncol; ++i) {
      cy.cj[i] = 1.0;
      cy.nstore[i] = 1.0;
      cy.vsc[i] = 1.0;
      cy.vsc[(size_t)(KMAX + 1) * ncol + i] = hscale;
    }
    DD_HIP(hipMemcpyAsync(d_cinv2, cy.vsc.data(), ncol * sizeof(double), hipMemcpyHostToDevice, c->stream));
    DD_HIP(hipMemcpyAsync(d_osc, cy.vsc.data() + (size_t)(KMAX + 1) * ncol, ncol * sizeof(double), hipMemcpyHostToDevice,
                          c->stream));
  }
  for (int i = 0; i < ncol; ++i) {
    cy.kc[i] = done[i] ? 0 : -1;
    for (int j = 0; j <= m; ++j) cy.g[(size_t)i * (m + 1) + j] = 0;
    cy.g[(size_t)i * (m + 1)] = beta[i];
  }
  int jj = 0;
  for (int j = 0; j < m && j < budget; ++j) {
    MV vj = basis(c, w.V, j, level, vprec, cap, nt);
    // the one-tile MFMA coarse stencil reads the FP16 basis vector itself
    const bool op_f16 = half && !pc && level > 0 && coarse_takes_f16(c, level, nt);
    if (half && !pc_f16 && !op_f16) {
      MV v32 = get(c, w.vi, level, prec, cap, nt);
      mv_copy(c, vj, v32);
      vj = v32;
    }
    MV z = vj;
    if (pc) {
      z = basis(c, w.Z, j, level, zprec, cap, nt);
      (*pc)(vj, z, d_mu);
    }
    MV vn = half ? get(c, w.wt, level, prec, cap, nt) : basis(c, w.V, j + 1, level, vprec, cap, nt);
    if (z.prec != prec && !op_f16) {
      MV zt = get(c, w.zt, level, prec, cap, nt);
      mv_copy(c, z, zt);
      operator_apply(c, level, zt, vn, d_mu);
    } else {
      operator_apply(c, level, z, vn, d_mu);
    }
    const bool one_red = !half && c->gram_lowsync != 0 && (vprec == P32 || vprec == P64);
    std::vector<MV> Vs(j + 2);
    for (int i = 0; i <= j; ++i) Vs[i] = basis(c, w.V, i, level, vprec, cap, nt);
    if (one_red) {
      // one reduction per step: the dots with the basis and |w|^2 together,
      // then w - V h stored already scaled by the predicted 1 / h_{j+1,j},
      // its norm measured in the same pass (DDAMG_KNOB_GRAM_ONE_REDUCTION)
      Vs[j + 1] = vn;
      mv_multidot(c, Vs.data(), j + 2, vn, w.d_h);
      if (cy.pairs) pair_sum_c(c, w.d_h, j + 2, ncol);
      hipLaunchKernelGGL(k_lowsync_scale, dim3((ncol + 63) / 64), dim3(64), 0, c->stream, j, ncol, w.d_h, w.d_osc);
      DD_HIP(hipGetLastError());
      mv_multiaxpy_scale_norm2(c, Vs.data(), j + 1, w.d_h, vn, -1, w.d_osc, d_n2, nullptr);
      if (cy.pairs) pair_sum_r(c, d_n2, ncol);
      mv_renorm(c, vn, d_n2, renorm_tau(c, vprec));
      copy_to_host(c, w.d_osc, cy.osc.data(), ncol * sizeof(double));
    } else {
    mv_multidot(c, Vs.data(), j + 1, vn, w.d_h);
    if (cy.pairs) pair_sum_c(c, w.d_h, j + 1, ncol);
    if (half)   // w' straight into the next FP16 basis vector, unnormalised
      mv_multiaxpy_norm2_into_f16(c, Vs.data(), j + 1, w.d_h, d_cinv2, vn, basis(c, w.V, j + 1, level, vprec, cap, nt),
                                  d_osc, d_n2);
    else
      mv_multiaxpy_norm2(c, Vs.data(), j + 1, w.d_h, vn, -1, d_n2);
    if (cy.pairs) pair_sum_r(c, d_n2, ncol);
    }
    // one copy of the dots and the norm
    const size_t nh = (size_t)(j + 1) * ncol * 2;
    copy_to_host(c, w.d_h, cy.hbuf.data(), nh * sizeof(double));
    copy_to_host(c, d_n2, cy.hbuf.data() + (size_t)KMAX * ncol * 2, ncol * sizeof(double));
    if (!half && !one_red) mv_normalize(c, vn, d_n2);
    ++total;
    jj = j + 1;
    bool alld = true;
    if (half) {   // entry scale of the vector just stored, and the store scale of the next
      // an entry scale far from 1 (a norm far from its prediction) would
      // leave the stored FP16 entries near the subnormal range or waste
      // their range: the pass is then run again (w and the dots are still
      // intact) with each column stored at its exact norm (c = 1)
      const double bound = c->fp16_rescale;
      bool redo = false;
      for (int i = 0; i < ncol; ++i) {
        const double hn = host_norm_guard(cy.hbuf[(size_t)KMAX * ncol * 2 + i]);
        const double cn = hn / cy.nstore[i];
        if (hn > 0 && (cn * bound < 1.0 || cn > bound)) redo = true;
      }
      if (redo) {
        for (int i = 0; i < ncol; ++i) {
          const double hn = host_norm_guard(cy.hbuf[(size_t)KMAX * ncol * 2 + i]);
          cy.osc_exact[i] = hscale / (hn > 0 ? hn : cy.nstore[i]);
        }
        DD_HIP(hipMemcpyAsync(d_osc, cy.osc_exact.data(), ncol * sizeof(double), hipMemcpyHostToDevice, c->stream));
        mv_multiaxpy_norm2_into_f16(c, Vs.data(), j + 1, w.d_h, d_cinv2, vn,
                                    basis(c, w.V, j + 1, level, vprec, cap, nt), d_osc, d_n2);
        c->st.fp16_restores++;
      }
      for (int i = 0; i < ncol; ++i) {
        const double hn = host_norm_guard(cy.hbuf[(size_t)KMAX * ncol * 2 + i]);
        const double cn = hn > 0 && !redo ? hn / cy.nstore[i] : 1.0;
        // the next norm is predicted as c_{j+1} times this step's norm for a
        // unit input (hn / c_j), which keeps the entry scales near 1
        if (hn > 0) cy.nstore[i] = cn * hn / cy.cj[(size_t)j * ncol + i];
        cy.cj[(size_t)(j + 1) * ncol + i] = cn;
        cy.vsc[(size_t)(j + 1) * ncol + i] = 1.0 / (cn * cn);
        cy.vsc[(size_t)(KMAX + 1) * ncol + i] = hscale / cy.nstore[i];
      }
      DD_HIP(hipMemcpyAsync(d_cinv2 + (size_t)(j + 1) * ncol, cy.vsc.data() + (size_t)(j + 1) * ncol,
                            ncol * sizeof(double), hipMemcpyHostToDevice, c->stream));
      DD_HIP(hipMemcpyAsync(d_osc, cy.vsc.data() + (size_t)(KMAX + 1) * ncol, ncol * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
    }
    for (int i = 0; i < ncol; ++i) {
      cd* Hc = &cy.H[(size_t)i * (m + 1) * m];
      for (int q = 0; q <= j; ++q) {   // dots with the stored vectors, over their entry scale
        const double cq = half ? cy.cj[(size_t)q * ncol + i] : 1.0;
        Hc[(size_t)q * m + j] =
            cd(cy.hbuf[((size_t)q * ncol + i) * 2], cy.hbuf[((size_t)q * ncol + i) * 2 + 1]) / cq;
      }
      double hn = host_norm_guard(cy.hbuf[(size_t)KMAX * ncol * 2 + i]);
      if (one_red) hn = cy.osc[i] > 0 ? hn / cy.osc[i] : 0.0;   // |w - V h| = sqrt(n2) / osc
      Hc[(size_t)(j + 1) * m + j] = hn;
      if (done[i] && cy.kc[i] >= 0) continue;
      // apply the previous rotations to column j
      for (int q = 0; q < j; ++q) {
        const cd a = Hc[(size_t)q * m + j], bb = Hc[(size_t)(q + 1) * m + j];
        const double cq = cy.cs[(size_t)i * m + q];
        const cd sq = cy.sn[(size_t)i * m + q];
        Hc[(size_t)q * m + j] = cq * a + sq * bb;
        Hc[(size_t)(q + 1) * m + j] = -std::conj(sq) * a + cq * bb;
      }
      const cd a = Hc[(size_t)j * m + j], bb = Hc[(size_t)(j + 1) * m + j];
      double cc;
      cd ss, rr;
      if (std::abs(bb) == 0) { cc = 1; ss = 0; rr = a; }
      else if (std::abs(a) == 0) { cc = 0; ss = std::conj(bb) / std::abs(bb); rr = std::abs(bb); }
      else {
        const double na = std::abs(a), nr = std::hypot(na, std::abs(bb));
        cc = na / nr;
        ss = (a / na) * std::conj(bb) / nr;
        rr = (a / na) * nr;
      }
      cy.cs[(size_t)i * m + j] = cc;
      cy.sn[(size_t)i * m + j] = ss;
      Hc[(size_t)j * m + j] = rr;
      Hc[(size_t)(j + 1) * m + j] = 0;
      cd* gc = &cy.g[(size_t)i * (m + 1)];
      const cd gj = gc[j];
      gc[j] = cc * gj;
      gc[j + 1] = -std::conj(ss) * gj;
      est[i] = std::abs(gc[j + 1]);
      if (!fixed && (est[i] <= tol_abs[i] || hn == 0)) {
        done[i] = 1;
        cy.kc[i] = j + 1;
      }
      if (!done[i]) alld = false;
    }
    if (c->p.verbose && level == 0) {
      double mx = 0;
      int nact = 0;
      for (int i = 0; i < ncol; ++i)
        if (bn[i] > 0) {
          mx = std::max(mx, est[i] / bn[i]);
          nact += !done[i];
        }
      std::fprintf(stderr, "[ddamg] outer %d: max rel. residual estimate %.3e, %d columns active, "
                   "middle calls %lld (avg %.1f it), bottom calls %lld (avg %.1f it)\n", total, mx, nact,
                   c->st.middle_calls, c->st.middle_calls ? (double)c->st.middle_iters / c->st.middle_calls : 0.0,
                   c->st.bottom_calls, c->st.bottom_calls ? (double)c->st.bottom_iters / c->st.bottom_calls : 0.0);
      std::fflush(stderr);
    }
    if (!fixed && alld) break;
  }
  // per-column least squares and the update x += basis * y
  cy.coef.assign((size_t)jj * ncol * 2, 0.0);
  for (int i = 0; i < ncol; ++i) {
    const int k = cy.kc[i] >= 0 ? cy.kc[i] : jj;
    cy.kc[i] = k;
    if (k == 0) continue;
    const cd* Hc = &cy.H[(size_t)i * (m + 1) * m];
    const cd* gc = &cy.g[(size_t)i * (m + 1)];
    std::vector<cd> y(k);
    for (int q = k - 1; q >= 0; --q) {
      cd acc = gc[q];
      for (int p = q + 1; p < k; ++p) acc -= Hc[(size_t)q * m + p] * y[p];
      const cd d = Hc[(size_t)q * m + q];
      y[q] = std::abs(d) > 0 ? acc / d : cd(0);
    }
    for (int q = 0; q < k; ++q) {
      cy.coef[((size_t)q * ncol + i) * 2] = y[q].real();
      cy.coef[((size_t)q * ncol + i) * 2 + 1] = y[q].imag();
    }
  }
  if (jj > 0) {
    DD_HIP(hipMemcpyAsync(w.d_aux, cy.coef.data(), cy.coef.size() * sizeof(double), hipMemcpyHostToDevice,
                          c->stream));
    std::vector<MV> B(jj);
    for (int q = 0; q < jj; ++q)
      B[q] = pc ? basis(c, w.Z, q, level, zprec, cap, nt) : basis(c, w.V, q, level, vprec, cap, nt);
    mv_multiaxpy(c, B.data(), jj, w.d_aux, x, +1);
    DD_HIP(hipStreamSynchronize(c->stream));   // coef is a host vector reused next cycle
  }
  return jj;
}

// r = b - A x into V[0] of the workspace; beta (host) = column norms, d_n2 their squares
static void residual_norms(ddamg_ctx* c, int level, LW& w, int nt, const MV& b, const MV& x, const double* d_mu,
                           bool x_is_zero, double* d_n2, std::vector<double>& beta, bool pairs = false) {
  const int prec = b.prec, ncol = nt * c->T;
  // the residual lands where gmres_cycle normalises it: V[0], or the
  // working-precision vector when the basis is stored in FP16
  MV r = w.vprec != prec ? get(c, w.wt, level, prec, w.cap, nt) : basis(c, w.V, 0, level, prec, w.cap, nt);
  if (x_is_zero) {
    mv_copy(c, b, r);
  } else if (level == 0) {
    fine_residual(c, b, x, r, d_mu);
  } else {
    MV t = get(c, w.res, level, prec, w.cap, nt);
    operator_apply(c, level, x, t, d_mu);
    mv_sub(c, b, t, r);
  }
  mv_norm2(c, r, d_n2);
  if (pairs) pair_sum_r(c, d_n2, ncol);
  beta.resize(ncol);
  copy_to_host(c, d_n2, beta.data(), ncol * sizeof(double));
  for (int i = 0; i < ncol; ++i) beta[i] = host_norm_guard(beta[i]);
}

// ------------------------------------------------- captured GMRES steps ---
// Device-side Givens least squares of the per-column Hessenberg matrices, so
// that an unpreconditioned Arnoldi step needs no host round trip.
// H: [ncol][m+1][m] complex, cs: [ncol][m], sn: [ncol][m] complex,
// g: [ncol][m+1] complex; dots: [j+1][ncol] complex (the Gram-Schmidt
// coefficients of step j), n2: [ncol] squared norms after orthogonalisation.
__global__ void k_g_init(const double* __restrict__ n2, const double* __restrict__ tol, double* __restrict__ g,
                         int* __restrict__ kc, int* __restrict__ done, double* __restrict__ est, int m, int ncol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncol) return;
  const double beta = n2[i] > 0 ? sqrt(n2[i]) : 0.0;
  double* gi = g + (size_t)i * (m + 1) * 2;
  for (int q = 0; q <= m; ++q) gi[2 * q] = gi[2 * q + 1] = 0.0;
  gi[0] = beta;
  const int d = beta <= tol[i] ? 1 : 0;   // also zero columns (tol = beta = 0)
  done[i] = d;
  kc[i] = d ? 0 : -1;
  est[i] = beta;
}

__global__ void k_g_step(int j, int m, int ncol, const double* __restrict__ dots, const double* __restrict__ n2,
                         const double* __restrict__ osc, double* __restrict__ H, double* __restrict__ cs,
                         double* __restrict__ sn,
                         double* __restrict__ g, int* __restrict__ kc, int* __restrict__ done,
                         const double* __restrict__ tol, double* __restrict__ est) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncol) return;
  double* Hc = H + (size_t)i * (m + 1) * m * 2;
  for (int q = 0; q <= j; ++q) {
    Hc[((size_t)q * m + j) * 2] = dots[((size_t)q * ncol + i) * 2];
    Hc[((size_t)q * m + j) * 2 + 1] = dots[((size_t)q * ncol + i) * 2 + 1];
  }
  // with the one-reduction step the stored vector is (w - V h) * osc, whose
  // measured norm sqrt(n2) gives |w - V h| = sqrt(n2) / osc
  double hn = n2[i] > 0 ? sqrt(n2[i]) : 0.0;
  if (osc) hn = osc[i] > 0 ? hn / osc[i] : 0.0;
  Hc[((size_t)(j + 1) * m + j) * 2] = hn;
  Hc[((size_t)(j + 1) * m + j) * 2 + 1] = 0.0;
  if (done[i] && kc[i] >= 0) return;
  double* ci = cs + (size_t)i * m;
  double* si = sn + (size_t)i * m * 2;
  for (int q = 0; q < j; ++q) {   // previous rotations
    double* a = Hc + ((size_t)q * m + j) * 2;
    double* b = Hc + ((size_t)(q + 1) * m + j) * 2;
    const double ar = a[0], ai = a[1], br = b[0], bi = b[1];
    const double c = ci[q], sr = si[2 * q], sim = si[2 * q + 1];
    // a' = c a + s b ; b' = -conj(s) a + c b
    a[0] = c * ar + (sr * br - sim * bi);
    a[1] = c * ai + (sr * bi + sim * br);
    b[0] = -(sr * ar + sim * ai) + c * br;
    b[1] = -(sr * ai - sim * ar) + c * bi;
  }
  double* a = Hc + ((size_t)j * m + j) * 2;
  double* b = Hc + ((size_t)(j + 1) * m + j) * 2;
  const double na = hypot(a[0], a[1]), nb = hypot(b[0], b[1]);
  double c, sr, sim, rr, ri;
  if (nb == 0) { c = 1; sr = 0; sim = 0; rr = a[0]; ri = a[1]; }
  else if (na == 0) { c = 0; sr = b[0] / nb; sim = -b[1] / nb; rr = nb; ri = 0; }
  else {
    const double nr = hypot(na, nb);
    c = na / nr;
    // s = (a/|a|) conj(b) / nr
    const double ur = a[0] / na, ui = a[1] / na;
    sr = (ur * b[0] + ui * b[1]) / nr;
    sim = (ui * b[0] - ur * b[1]) / nr;
    rr = ur * nr;
    ri = ui * nr;
  }
  ci[j] = c;
  si[2 * j] = sr;
  si[2 * j + 1] = sim;
  a[0] = rr; a[1] = ri;
  b[0] = 0; b[1] = 0;
  double* gi = g + (size_t)i * (m + 1) * 2;
  const double gr = gi[2 * j], gim = gi[2 * j + 1];
  gi[2 * j] = c * gr;
  gi[2 * j + 1] = c * gim;
  gi[2 * (j + 1)] = -(sr * gr + sim * gim);       // -conj(s) g_j
  gi[2 * (j + 1) + 1] = -(sr * gim - sim * gr);
  est[i] = hypot(gi[2 * (j + 1)], gi[2 * (j + 1) + 1]);
  if (est[i] <= tol[i] || hn == 0) {
    done[i] = 1;
    kc[i] = j + 1;
  }
}

// y from the rotated triangle (k = kc or jj steps), written as update
// coefficients coef[q][i] (complex) for q < jj; kc[i] <- k
__global__ void k_g_solve(int jj, int m, int ncol, const double* __restrict__ H, const double* __restrict__ g,
                          int* __restrict__ kc, double* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncol) return;
  const int k = kc[i] >= 0 ? kc[i] : jj;
  kc[i] = k;
  const double* Hc = H + (size_t)i * (m + 1) * m * 2;
  const double* gi = g + (size_t)i * (m + 1) * 2;
  for (int q = jj - 1; q >= k; --q) coef[((size_t)q * ncol + i) * 2] = coef[((size_t)q * ncol + i) * 2 + 1] = 0.0;
  for (int q = k - 1; q >= 0; --q) {
    double vr = gi[2 * q], vi = gi[2 * q + 1];
    for (int p = q + 1; p < k; ++p) {
      const double hr = Hc[((size_t)q * m + p) * 2], hi = Hc[((size_t)q * m + p) * 2 + 1];
      const double yr = coef[((size_t)p * ncol + i) * 2], yi = coef[((size_t)p * ncol + i) * 2 + 1];
      vr -= hr * yr - hi * yi;
      vi -= hr * yi + hi * yr;
    }
    const double dr = Hc[((size_t)q * m + q) * 2], di = Hc[((size_t)q * m + q) * 2 + 1];
    const double dn = dr * dr + di * di;
    double yr = 0, yi = 0;
    if (dn > 0) {   // (vr + i vi) / (dr + i di)
      yr = (vr * dr + vi * di) / dn;
      yi = (vi * dr - vr * di) / dn;
    }
    coef[((size_t)q * ncol + i) * 2] = yr;
    coef[((size_t)q * ncol + i) * 2 + 1] = yi;
  }
}

static hipStream_t capture_stream(ddamg_ctx* c) {
  if (!c->cap_stream) DD_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  return c->cap_stream;
}

static void knob_state(ddamg_ctx* c, int (&k)[7]) {
  k[0] = c->dslash_rs[0];
  k[1] = c->dslash_rs[1];
  k[2] = c->fp32_links;
  k[3] = c->coarse_mfma;
  k[4] = c->sap_variant;
  k[5] = c->dslash_order;
  k[6] = c->gram_lowsync;
}

static GraphState& graph_state(ddamg_ctx* c, LW& w, int level, int nt, int m) {
  int k[7];
  knob_state(c, k);
  GraphState* g = w.gs;
  const int g5 = level > 0 ? c->coarse[level].g5out : 0;
  const bool same = g && g->nt == nt && g->m == m && g->g5 == g5 && std::equal(k, k + 7, g->knobs);
  if (same) return *g;
  destroy_graphs(c, g);
  g = new GraphState();
  w.gs = g;
  g->nt = nt;
  g->m = m;
  g->g5 = g5;
  g->ncol = nt * c->T;
  std::copy(k, k + 7, g->knobs);
  const size_t n = g->ncol;
  auto dal = [&](size_t cnt) { return (double*)c->pool.alloc(std::max<size_t>(cnt, 1) * sizeof(double)); };
  g->d_H = dal(n * (m + 1) * m * 2);
  g->d_cs = dal(n * m);
  g->d_sn = dal(n * m * 2);
  g->d_g = dal(n * (m + 1) * 2);
  g->d_tol = dal(n);
  g->d_est = dal(n);
  g->d_n2 = dal(n);
  g->d_cbuf = dal(2 * n);
  g->d_mu = dal(n);
  g->d_coef = dal((size_t)KMAX * n * 2);
  size_t part = 0;
  const MV v0 = basis(c, w.V, 0, level, w.prec, w.cap, nt);
  for (int q = 1; q <= m + 1; ++q) part = std::max(part, multidot_partials(v0, q));
  g->d_part = dal(part);
  g->d_osc = dal(n);
  g->d_apart = dal(multiaxpy_partials(v0));
  g->d_kc = (int*)c->pool.alloc(n * sizeof(int));
  g->d_done = (int*)c->pool.alloc(n * sizeof(int));
  g->graph.assign(m, nullptr);
  g->exec.assign(m, nullptr);
  return *g;
}

// One Arnoldi step j (operator, CGS, norm, normalisation, Givens) on the
// current stream; used for capture only, so it must not synchronise.
static void arnoldi_step_device(ddamg_ctx* c, int level, LW& w, GraphState& g, int j) {
  const int nt = g.nt, prec = w.prec, cap = w.cap;
  MV vj = basis(c, w.V, j, level, prec, cap, nt);
  MV vn = basis(c, w.V, j + 1, level, prec, cap, nt);
  operator_apply(c, level, vj, vn, g.d_mu);
  std::vector<MV> Vs(j + 2);
  for (int i = 0; i <= j; ++i) Vs[i] = basis(c, w.V, i, level, prec, cap, nt);
  const bool one_red = c->gram_lowsync != 0;
  if (one_red) {
    // one reduction: the dots with the basis and |w|^2 together; the update
    // pass stores w - V h already scaled by the predicted 1 / h_{j+1,j}
    Vs[j + 1] = vn;
    mv_multidot_buf(c, Vs.data(), j + 2, vn, w.d_h, g.d_part);
    hipLaunchKernelGGL(k_lowsync_scale, dim3((g.ncol + 63) / 64), dim3(64), 0, c->stream, j, g.ncol, w.d_h, g.d_osc);
    DD_HIP(hipGetLastError());
    mv_multiaxpy_scale_norm2(c, Vs.data(), j + 1, w.d_h, vn, -1, g.d_osc, g.d_n2, g.d_apart);
    mv_renorm(c, vn, g.d_n2, renorm_tau(c, prec));
  } else {
    mv_multidot_buf(c, Vs.data(), j + 1, vn, w.d_h, g.d_part);
    mv_multiaxpy(c, Vs.data(), j + 1, w.d_h, vn, -1);
    mv_norm2_buf(c, vn, g.d_n2, g.d_cbuf, g.d_part);
    mv_normalize(c, vn, g.d_n2);
  }
  hipLaunchKernelGGL(k_g_step, dim3((g.ncol + 63) / 64), dim3(64), 0, c->stream, j, g.m, g.ncol, w.d_h, g.d_n2,
                     one_red ? g.d_osc : (const double*)nullptr, g.d_H, g.d_cs, g.d_sn, g.d_g, g.d_kc, g.d_done,
                     g.d_tol, g.d_est);
  DD_HIP(hipGetLastError());
}

static hipGraphExec_t step_graph(ddamg_ctx* c, int level, LW& w, GraphState& g, int j) {
  if (g.exec[j]) return g.exec[j];
  // every basis vector the step touches exists before capture
  for (int i = 0; i <= j + 1; ++i) basis(c, w.V, i, level, w.prec, w.cap, g.nt);
  const hipStream_t saved = c->stream;
  // order the capture after all work already queued on the caller's stream
  DD_HIP(hipStreamSynchronize(saved));
  c->stream = capture_stream(c);
  DD_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    arnoldi_step_device(c, level, w, g, j);
  } catch (...) {
    hipStreamEndCapture(c->stream, &graph);
    if (graph) hipGraphDestroy(graph);
    c->stream = saved;
    throw;
  }
  const hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->stream = saved;
  DD_HIP(e);
  g.graph[j] = graph;
  DD_HIP(hipGraphInstantiate(&g.exec[j], graph, nullptr, nullptr, 0));
  return g.exec[j];
}

// Unpreconditioned restarted GMRES(m) whose Arnoldi steps are captured HIP
// graphs with the least squares on the device: the host only launches one
// graph per step and reads the convergence flags every few steps.
static void krylov_graph(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, bool x_zero,
                         double tol, int m, int maxit, KrylovOut* out) {
  constexpr int CHECK_EVERY = 4;
  const int nt = b.ntiles, ncol = b.ncol(), prec = b.prec;
  LW& w = lw(c, level, prec, nt);
  GraphState& g = graph_state(c, w, level, nt, m);
  DD_HIP(hipMemcpyAsync(g.d_mu, d_mu, ncol * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  std::vector<double> bn(ncol), tol_abs(ncol);
  mv_norm2(c, b, g.d_n2);
  copy_to_host(c, g.d_n2, bn.data(), ncol * sizeof(double));
  for (int i = 0; i < ncol; ++i) {
    bn[i] = host_norm_guard(bn[i]);
    tol_abs[i] = tol * bn[i];
  }
  DD_HIP(hipMemcpyAsync(g.d_tol, tol_abs.data(), ncol * sizeof(double), hipMemcpyHostToDevice, c->stream));
  std::vector<int> iters(ncol, 0), kc(ncol), done(ncol);
  std::vector<double> est(ncol);
  int total = 0;
  bool first = true;
  if (x_zero) mv_zero(c, x);
  while (true) {
    MV r = basis(c, w.V, 0, level, prec, w.cap, nt);
    if (x_zero && first) {
      mv_copy(c, b, r);
    } else {
      MV t = get(c, w.res, level, prec, w.cap, nt);
      operator_apply(c, level, x, t, d_mu);
      mv_sub(c, b, t, r);
    }
    first = false;
    mv_norm2(c, r, g.d_n2);
    mv_normalize(c, r, g.d_n2);
    hipLaunchKernelGGL(k_g_init, dim3((ncol + 63) / 64), dim3(64), 0, c->stream, g.d_n2, g.d_tol, g.d_g, g.d_kc,
                       g.d_done, g.d_est, m, ncol);
    DD_HIP(hipGetLastError());
    copy_to_host(c, g.d_done, done.data(), ncol * sizeof(int));
    if (std::all_of(done.begin(), done.end(), [](int v) { return v != 0; }) || total >= maxit) {
      copy_to_host(c, g.d_est, est.data(), ncol * sizeof(double));
      break;
    }
    int jj = 0;
    for (int j = 0; j < m && total < maxit; ++j) {
      hipGraphExec_t e = step_graph(c, level, w, g, j);
      DD_HIP(hipGraphLaunch(e, c->stream));
      ++total;
      jj = j + 1;
      if (jj % CHECK_EVERY == 0 || jj == m) {
        copy_to_host(c, g.d_done, done.data(), ncol * sizeof(int));
        if (std::all_of(done.begin(), done.end(), [](int v) { return v != 0; })) break;
      }
    }
    hipLaunchKernelGGL(k_g_solve, dim3((ncol + 63) / 64), dim3(64), 0, c->stream, jj, m, ncol, g.d_H, g.d_g,
                       g.d_kc, g.d_coef);
    DD_HIP(hipGetLastError());
    std::vector<MV> B(jj);
    for (int q = 0; q < jj; ++q) B[q] = basis(c, w.V, q, level, prec, w.cap, nt);
    mv_multiaxpy(c, B.data(), jj, g.d_coef, x, +1);
    copy_to_host(c, g.d_kc, kc.data(), ncol * sizeof(int));
    copy_to_host(c, g.d_est, est.data(), ncol * sizeof(double));
    copy_to_host(c, g.d_done, done.data(), ncol * sizeof(int));
    for (int i = 0; i < ncol; ++i) iters[i] += kc[i];
    if (std::all_of(done.begin(), done.end(), [](int v) { return v != 0; }) || total >= maxit) break;
  }
  if (out) {
    out->iters = iters;
    out->relres.resize(ncol);
    for (int i = 0; i < ncol; ++i) out->relres[i] = bn[i] > 0 ? est[i] / bn[i] : 0.0;
    out->total = total;
  }
}

// (F)GMRES(m) on level `level` for all columns of b (precision of b/x);
// preconditioner output precision zprec.  x holds the initial guess unless
// x_zero.  fixed: run exactly maxit iterations without a convergence test.
void krylov(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, bool x_zero, double tol, int m,
            int maxit, const Precond* pc, int zprec, bool fixed, KrylovOut* out, int role = 0) {
  const int nt = b.ntiles, ncol = b.ncol();
  DD_CHECK(m >= 1 && m < KMAX, DDAMG_EINVAL, "Krylov restart length must be in [1, 63]");
  // captured graphs record no timing events: a level whose stencil is being
  // timed live runs the host-driven steps (identical iterates)
  const bool timed = level == 1 && c->time_sap == TIMED_COARSE1;
  const bool f16_basis = role == 0 && level > 0 && b.prec == P32 && c->p.coarse_fp16;
  if (!pc && !fixed && role == 0 && c->p.use_graphs && !timed && !f16_basis) {
    krylov_graph(c, level, d_mu, b, x, x_zero, tol, m, maxit, out);
    return;
  }
  LW& w = lw(c, level, b.prec, nt, role);
  std::vector<double> bn(ncol), tol_abs(ncol), est(ncol), beta;
  double* d_n2 = w.d_h + (size_t)KMAX * ncol * 2;
  mv_norm2(c, b, d_n2);
  copy_to_host(c, d_n2, bn.data(), ncol * sizeof(double));
  std::vector<char> done(ncol, 0);
  for (int i = 0; i < ncol; ++i) {
    bn[i] = host_norm_guard(bn[i]);
    tol_abs[i] = tol * bn[i];
    if (bn[i] == 0) done[i] = 1;
    est[i] = bn[i];
  }
  std::vector<int> iters(ncol, 0);
  Cycle cy(ncol, m);
  int total = 0;
  bool first = true;
  if (x_zero) mv_zero(c, x);
  while (true) {
    residual_norms(c, level, w, nt, b, x, d_mu, x_zero && first, d_n2, beta);
    first = false;
    bool all = true;
    for (int i = 0; i < ncol; ++i) {
      est[i] = beta[i];
      if (!fixed && beta[i] <= tol_abs[i]) done[i] = 1;
      if (bn[i] == 0) done[i] = 1;
      if (!done[i]) all = false;
    }
    if ((all && !fixed) || total >= maxit) break;
    // the inner FGMRES's preconditioner is the fine smoother; SAP reads an FP16 basis directly
    const bool pc_f16 = role == 1 && c->nlev == 1 && c->p.smoother == DDAMG_SMOOTHER_SAP && sap_takes_f16(c);
    gmres_cycle(c, level, w, nt, x, d_mu, pc, zprec, maxit - total, fixed, beta, done, tol_abs, est, bn, cy, d_n2,
                total, pc_f16);
    for (int i = 0; i < ncol; ++i) iters[i] += cy.kc[i];
    bool all2 = true;
    for (int i = 0; i < ncol; ++i)
      if (!done[i]) all2 = false;
    if (fixed || all2 || total >= maxit) break;
  }
  if (out) {
    out->iters = iters;
    out->relres.resize(ncol);
    for (int i = 0; i < ncol; ++i) out->relres[i] = bn[i] > 0 ? est[i] / bn[i] : 0.0;
    out->total = total;
  }
}

// Plain restarted GMRES(m) on one level (no preconditioner), per column.
void level_gmres(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, double tol, int m, int maxit,
                 std::vector<int>* iters, std::vector<double>* relres, int* total) {
  KrylovOut ko;
  krylov(c, level, d_mu, b, x, true, tol, m, maxit, nullptr, b.prec, false, &ko);
  if (iters) *iters = ko.iters;
  if (relres) *relres = ko.relres;
  if (total) *total = ko.total;
}

// ------------------------------------------------ deflated restarting ---
// GMRES with deflated restarting, GMRES-DR(m, k) (section 4 and the outlook:
// deflated restarting at the coarsest level), for unpreconditioned solves on
// a level, every column with its own Arnoldi process (all columns in
// lockstep, converged ones idle).  A cycle builds the basis to m vectors; at
// a restart the k harmonic Ritz vectors of smallest harmonic Ritz value
// (host: the small eigenproblem H_m + |h_{m+1,m}|^2 f e_m^T,
// f = H_m^{-H} e_m) and the residual's coordinates c - Hbar y are
// orthonormalised into Q ((m+1) x (k+1)); the next cycle starts from the
// basis V Q (k+1 multi-axpys with per-column coefficients, on the device),
// Hbar Q^H Hbar Q[:m, :k] and the residual coordinates Q^H (c - Hbar y).  The
// least squares are kept triangular by Givens rotations (those that reduce
// the dense leading block after a restart, then one per step).
struct DrRot {
  int r0;
  double c;
  cd s;
};

static void dr_apply_rot(const DrRot& q, cd* v) {
  const cd a = v[q.r0], b = v[q.r0 + 1];
  v[q.r0] = q.c * a + q.s * b;
  v[q.r0 + 1] = -std::conj(q.s) * a + q.c * b;
}

static DrRot dr_make_rot(int r0, cd a, cd b) {
  double cc;
  cd ss;
  hess_givens(a, b, cc, ss);
  return DrRot{r0, cc, ss};
}

void krylov_dr(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, bool x_zero, double tol, int m,
               int kdr, int maxit, KrylovOut* out) {
  const int nt = b.ntiles, ncol = b.ncol();
  DD_CHECK(m >= 2 && m < KMAX && kdr >= 0 && kdr < m, DDAMG_EINVAL, "GMRES-DR: need 2 <= m <= 63 and 0 <= k < m");
  LW& w = lw(c, level, b.prec, nt, 2);   // a workspace of its own (the captured graphs keep theirs)
  const int cap = w.cap, prec = b.prec;
  std::vector<double> bn(ncol), tol_abs(ncol), est(ncol), beta;
  double* d_n2 = w.d_h + (size_t)KMAX * ncol * 2;
  mv_norm2(c, b, d_n2);
  copy_to_host(c, d_n2, bn.data(), ncol * sizeof(double));
  std::vector<char> done(ncol, 0);
  for (int i = 0; i < ncol; ++i) {
    bn[i] = host_norm_guard(bn[i]);
    tol_abs[i] = tol * bn[i];
    if (bn[i] == 0) done[i] = 1;
  }
  if (x_zero) mv_zero(c, x);
  residual_norms(c, level, w, nt, b, x, d_mu, x_zero, d_n2, beta);
  MV v0 = basis(c, w.V, 0, level, prec, cap, nt);
  mv_normalize(c, v0, d_n2);
  std::vector<int> iters(ncol, 0), kc(ncol, 0);
  // per column: Hbar and residual coordinates (unrotated), their rotated
  // forms, and the rotations
  std::vector<cd> Hb((size_t)ncol * (m + 1) * m), cv((size_t)ncol * (m + 1));
  std::vector<cd> Hr((size_t)ncol * (m + 1) * m), g((size_t)ncol * (m + 1));
  std::vector<std::vector<DrRot>> rots(ncol);
  std::vector<cd> hbuf((size_t)KMAX * ncol + ncol);
  std::vector<double> hraw((size_t)KMAX * ncol * 2 + ncol);
  for (int i = 0; i < ncol; ++i) {
    est[i] = beta[i];
    if (beta[i] <= tol_abs[i]) done[i] = 1;
    cv[(size_t)i * (m + 1)] = beta[i];
    g[(size_t)i * (m + 1)] = beta[i];
  }
  int total = 0, j0 = 0;
  auto H_ = [&](std::vector<cd>& A, int i, int r, int q) -> cd& { return A[((size_t)i * (m + 1) + r) * m + q]; };
  while (true) {
    bool alld = true;
    for (int i = 0; i < ncol; ++i) alld &= (bool)done[i];
    if (alld || total >= maxit) break;
    for (int i = 0; i < ncol; ++i) kc[i] = done[i] ? -2 : -1;   // -2: idle this cycle
    int jend = j0;
    for (int j = j0; j < m && total < maxit; ++j) {
      MV vj = basis(c, w.V, j, level, prec, cap, nt);
      MV vn = basis(c, w.V, j + 1, level, prec, cap, nt);
      operator_apply(c, level, vj, vn, d_mu);
      std::vector<MV> Vs(j + 1);
      for (int q = 0; q <= j; ++q) Vs[q] = basis(c, w.V, q, level, prec, cap, nt);
      mv_multidot(c, Vs.data(), j + 1, vn, w.d_h);
      mv_multiaxpy_norm2(c, Vs.data(), j + 1, w.d_h, vn, -1, d_n2);
      copy_to_host(c, w.d_h, hraw.data(), (size_t)(j + 1) * ncol * 2 * sizeof(double));
      copy_to_host(c, d_n2, hraw.data() + (size_t)KMAX * ncol * 2, ncol * sizeof(double));
      mv_normalize(c, vn, d_n2);
      ++total;
      jend = j + 1;
      bool all_now = true;
      for (int i = 0; i < ncol; ++i) {
        if (kc[i] != -1) continue;
        iters[i]++;
        const double hn = host_norm_guard(hraw[(size_t)KMAX * ncol * 2 + i]);
        for (int q = 0; q <= j; ++q)
          H_(Hb, i, q, j) = cd(hraw[((size_t)q * ncol + i) * 2], hraw[((size_t)q * ncol + i) * 2 + 1]);
        H_(Hb, i, j + 1, j) = hn;
        std::vector<cd> col(m + 1, cd(0));
        for (int q = 0; q <= j + 1; ++q) col[q] = H_(Hb, i, q, j);
        for (const DrRot& r : rots[i]) dr_apply_rot(r, col.data());
        const DrRot nr = dr_make_rot(j, col[j], col[j + 1]);
        dr_apply_rot(nr, col.data());
        rots[i].push_back(nr);
        cd* gi = &g[(size_t)i * (m + 1)];
        dr_apply_rot(nr, gi);
        for (int q = 0; q <= j + 1; ++q) H_(Hr, i, q, j) = col[q];
        est[i] = std::abs(gi[j + 1]);
        if (est[i] <= tol_abs[i] || hn == 0) kc[i] = j + 1;
        else all_now = false;
      }
      if (all_now) break;
    }
    // least squares and x += V y for every column that worked this cycle
    std::vector<double> coef((size_t)jend * ncol * 2, 0.0);
    std::vector<std::vector<cd>> ys(ncol);
    for (int i = 0; i < ncol; ++i) {
      if (kc[i] == -2) continue;
      const int k = kc[i] >= 0 ? kc[i] : jend;
      if (kc[i] >= 0) done[i] = 1;
      std::vector<cd> y(k);
      const cd* gi = &g[(size_t)i * (m + 1)];
      for (int q = k - 1; q >= 0; --q) {
        cd acc = gi[q];
        for (int p2 = q + 1; p2 < k; ++p2) acc -= H_(Hr, i, q, p2) * y[p2];
        const cd d = H_(Hr, i, q, q);
        y[q] = std::abs(d) > 0 ? acc / d : cd(0);
      }
      for (int q = 0; q < k; ++q) {
        coef[((size_t)q * ncol + i) * 2] = y[q].real();
        coef[((size_t)q * ncol + i) * 2 + 1] = y[q].imag();
      }
      ys[i] = std::move(y);
    }
    {
      std::vector<MV> Vs(jend);
      for (int q = 0; q < jend; ++q) Vs[q] = basis(c, w.V, q, level, prec, cap, nt);
      DD_HIP(hipMemcpyAsync(w.d_aux, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      mv_multiaxpy(c, Vs.data(), jend, w.d_aux, x, +1);
      DD_HIP(hipStreamSynchronize(c->stream));   // coef is host memory of this scope
    }
    bool alld2 = true;
    for (int i = 0; i < ncol; ++i) alld2 &= (bool)done[i];
    if (alld2 || total >= maxit) break;
    // deflated restart of the columns still working (jend == m for them)
    const int kk = std::min(kdr, m - 1);
    std::vector<double> qcoef((size_t)(kk + 1) * (m + 1) * ncol * 2, 0.0);   // [new i][old l][col] complex
    for (int i = 0; i < ncol; ++i) {
      if (done[i]) {   // idle column: keep its first vectors (nothing reads them)
        for (int q = 0; q <= kk; ++q) qcoef[(((size_t)q * (m + 1) + q) * ncol + i) * 2] = 1.0;
        continue;
      }
      const std::vector<cd>& y = ys[i];
      // rho = c - Hbar y
      std::vector<cd> rho(m + 1);
      for (int r = 0; r <= m; ++r) {
        cd acc = cv[(size_t)i * (m + 1) + r];
        for (int q = 0; q < m; ++q) acc -= H_(Hb, i, r, q) * y[q];
        rho[r] = acc;
      }
      // harmonic Ritz vectors: T = H_m + |h_{m+1,m}|^2 f e_m^T, H_m^H f = e_m
      std::vector<cd> P((size_t)(m + 1) * (kk + 1), cd(0));   // [row][col]
      if (kk > 0) {
        std::vector<cd> A((size_t)m * m), f(m, cd(0));
        for (int r = 0; r < m; ++r)
          for (int q = 0; q < m; ++q) A[(size_t)r * m + q] = std::conj(H_(Hb, i, q, r));   // H_m^H
        f[m - 1] = 1.0;
        // solve H_m^H f = e_m (lower Hessenberg) by Gaussian elimination with partial pivoting
        {
          std::vector<cd> M(A);
          std::vector<cd> rhs(f);
          for (int col = 0; col < m; ++col) {
            int piv = col;
            for (int r = col + 1; r < m; ++r)
              if (std::abs(M[(size_t)r * m + col]) > std::abs(M[(size_t)piv * m + col])) piv = r;
            if (piv != col) {
              for (int q = 0; q < m; ++q) std::swap(M[(size_t)col * m + q], M[(size_t)piv * m + q]);
              std::swap(rhs[col], rhs[piv]);
            }
            const cd d = M[(size_t)col * m + col];
            DD_CHECK(std::abs(d) > 0, DDAMG_EBREAKDOWN, "GMRES-DR: singular H_m at a restart");
            for (int r = col + 1; r < m; ++r) {
              const cd fct = M[(size_t)r * m + col] / d;
              if (fct == cd(0)) continue;
              for (int q = col; q < m; ++q) M[(size_t)r * m + q] -= fct * M[(size_t)col * m + q];
              rhs[r] -= fct * rhs[col];
            }
          }
          for (int r = m - 1; r >= 0; --r) {
            cd acc = rhs[r];
            for (int q = r + 1; q < m; ++q) acc -= M[(size_t)r * m + q] * f[q];
            f[r] = acc / M[(size_t)r * m + r];
          }
        }
        const double h2 = std::norm(H_(Hb, i, m, m - 1));
        std::vector<cd> T((size_t)m * m);
        for (int r = 0; r < m; ++r)
          for (int q = 0; q < m; ++q) T[(size_t)r * m + q] = H_(Hb, i, r, q) + (q == m - 1 ? h2 * f[r] : cd(0));
        std::vector<cd> ev, vec;
        DD_CHECK(hess_eig(m, T, ev, vec), DDAMG_EBREAKDOWN, "GMRES-DR: harmonic Ritz problem did not converge");
        std::vector<int> idx(m);
        for (int q = 0; q < m; ++q) idx[q] = q;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b2) { return std::abs(ev[a]) < std::abs(ev[b2]); });
        for (int q = 0; q < kk; ++q)
          for (int r = 0; r < m; ++r) P[(size_t)r * (kk + 1) + q] = vec[(size_t)r * m + idx[q]];
      }
      for (int r = 0; r <= m; ++r) P[(size_t)r * (kk + 1) + kk] = rho[r];
      // Q = orthonormal factor of P (modified Gram-Schmidt, twice)
      for (int q = 0; q <= kk; ++q) {
        for (int pass = 0; pass < 2; ++pass)
          for (int p2 = 0; p2 < q; ++p2) {
            cd d = 0;
            for (int r = 0; r <= m; ++r) d += std::conj(P[(size_t)r * (kk + 1) + p2]) * P[(size_t)r * (kk + 1) + q];
            for (int r = 0; r <= m; ++r) P[(size_t)r * (kk + 1) + q] -= d * P[(size_t)r * (kk + 1) + p2];
          }
        double nq = 0;
        for (int r = 0; r <= m; ++r) nq += std::norm(P[(size_t)r * (kk + 1) + q]);
        nq = std::sqrt(nq);
        DD_CHECK(nq > 0, DDAMG_EBREAKDOWN, "GMRES-DR: dependent deflation vectors");
        for (int r = 0; r <= m; ++r) P[(size_t)r * (kk + 1) + q] /= nq;
      }
      // Hbar_new = Q^H Hbar Q[:m, :kk], c_new = Q^H rho
      std::vector<cd> HQ((size_t)(m + 1) * kk, cd(0));
      for (int r = 0; r <= m; ++r)
        for (int q = 0; q < kk; ++q) {
          cd acc = 0;
          for (int l = 0; l < m; ++l) acc += H_(Hb, i, r, l) * P[(size_t)l * (kk + 1) + q];
          HQ[(size_t)r * kk + q] = acc;
        }
      for (int r = 0; r <= m; ++r)
        for (int q = 0; q < m; ++q) H_(Hb, i, r, q) = 0;
      for (int r = 0; r <= kk; ++r)
        for (int q = 0; q < kk; ++q) {
          cd acc = 0;
          for (int l = 0; l <= m; ++l) acc += std::conj(P[(size_t)l * (kk + 1) + r]) * HQ[(size_t)l * kk + q];
          H_(Hb, i, r, q) = acc;
        }
      cd* ci = &cv[(size_t)i * (m + 1)];
      std::vector<cd> cn(m + 1, cd(0));
      for (int r = 0; r <= kk; ++r) {
        cd acc = 0;
        for (int l = 0; l <= m; ++l) acc += std::conj(P[(size_t)l * (kk + 1) + r]) * rho[l];
        cn[r] = acc;
      }
      for (int r = 0; r <= m; ++r) ci[r] = cn[r];
      // rotated system: triangularise the dense (kk+1) x kk block
      rots[i].clear();
      cd* gi = &g[(size_t)i * (m + 1)];
      for (int r = 0; r <= m; ++r) gi[r] = ci[r];
      for (int r = 0; r <= m; ++r)
        for (int q = 0; q < m; ++q) H_(Hr, i, r, q) = H_(Hb, i, r, q);
      for (int q = 0; q < kk; ++q)
        for (int r = kk; r > q; --r) {
          const DrRot rt = dr_make_rot(r - 1, H_(Hr, i, r - 1, q), H_(Hr, i, r, q));
          for (int q2 = 0; q2 < kk; ++q2) {
            cd colv[2] = {H_(Hr, i, r - 1, q2), H_(Hr, i, r, q2)};
            DrRot loc{0, rt.c, rt.s};
            dr_apply_rot(loc, colv);
            H_(Hr, i, r - 1, q2) = colv[0];
            H_(Hr, i, r, q2) = colv[1];
          }
          dr_apply_rot(rt, gi);
          rots[i].push_back(rt);
        }
      est[i] = std::abs(gi[kk]);
      for (int r = 0; r <= m; ++r)
        for (int q = 0; q <= kk; ++q) {
          const cd v = P[(size_t)r * (kk + 1) + q];
          qcoef[(((size_t)q * (m + 1) + r) * ncol + i) * 2] = v.real();
          qcoef[(((size_t)q * (m + 1) + r) * ncol + i) * 2 + 1] = v.imag();
        }
    }
    // the next basis V_new_q = sum_l V_l Q_lq, formed in Z and copied back
    std::vector<MV> Vs(m + 1);
    for (int l = 0; l <= m; ++l) Vs[l] = basis(c, w.V, l, level, prec, cap, nt);
    for (int q = 0; q <= kk; ++q) {
      MV zq = basis(c, w.Z, q, level, prec, cap, nt);
      mv_zero(c, zq);
      DD_HIP(hipMemcpyAsync(w.d_aux, qcoef.data() + (size_t)q * (m + 1) * ncol * 2,
                            (size_t)(m + 1) * ncol * 2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
      mv_multiaxpy(c, Vs.data(), m + 1, w.d_aux, zq, +1);
      DD_HIP(hipStreamSynchronize(c->stream));   // w.d_aux is refilled for the next vector
    }
    for (int q = 0; q <= kk; ++q) mv_copy(c, basis(c, w.Z, q, level, prec, cap, nt), Vs[q]);
    j0 = kk;
  }
  if (out) {
    out->iters = iters;
    out->relres.resize(ncol);
    for (int i = 0; i < ncol; ++i) out->relres[i] = bn[i] > 0 ? est[i] / bn[i] : 0.0;
    out->total = total;
  }
}

void level_gmres_dr(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, double tol, int m, int k,
                    int maxit, std::vector<int>* iters) {
  KrylovOut ko;
  krylov_dr(c, level, d_mu, b, x, true, tol, m, k, maxit, &ko);
  if (iters) *iters = ko.iters;
}

// ------------------------------------------------------- outer solve ---
void mg_cycle(ddamg_ctx* c, int l, const double* d_mu, const MV& r, const MV& e);

// An independent FP64 check of every column as the caller receives it: x
// and b are read back from the canonical arrays into the outer solve's FP64
// buffers, wmax columns at a time, r = b - D(mu) x with the FP64 stencil,
// and err = ||r|| / ||b||.
static void final_check(ddamg_ctx* c, OuterJob& job, LW& w, int wmax) {
  const int T = c->T, ncol = job.ncol;
  const int cap = w.cap;
  const bool pairs = !job.eps.empty();
  for (int c0 = 0; c0 < ncol; c0 += wmax) {
    const int n = std::min(wmax, ncol - c0);
    const int ntn = (n + T - 1) / T, nc = ntn * T;
    std::vector<int> xm(nc, -1), bm(nc, -1);
    std::vector<double> mu(nc, 0.0), eps(nc, 0.0);
    for (int i = 0; i < n; ++i) {
      xm[i] = c0 + i;
      bm[i] = job.rhs_of[c0 + i];
      mu[i] = job.mu[c0 + i];
      if (pairs) eps[i] = job.eps[c0 + i];
    }
    const MV b = get(c, w.cb, 0, P64, cap, ntn), x = get(c, w.cx, 0, P64, cap, ntn);
    const MV r = get(c, w.cb2, 0, P64, cap, ntn);
    int* d_xm = w.d_map;
    int* d_bm = w.d_map + cap * T;
    DD_HIP(hipMemcpyAsync(d_xm, xm.data(), nc * sizeof(int), hipMemcpyHostToDevice, c->stream));
    DD_HIP(hipMemcpyAsync(d_bm, bm.data(), nc * sizeof(int), hipMemcpyHostToDevice, c->stream));
    DD_HIP(hipMemcpyAsync(w.d_muc, mu.data(), nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (pairs) DD_HIP(hipMemcpyAsync(w.d_epsc, eps.data(), nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    mv_zero(c, b);
    mv_zero(c, x);
    canon_cols(c, 0, b, d_bm, const_cast<double*>(job.b), 0);
    canon_cols(c, 0, x, d_xm, job.x, 0);
    {
      NDScope nd(c, pairs ? w.d_epsc : nullptr);
      fine_residual(c, b, x, r, w.d_muc);
    }
    double* d_n2 = w.d_h + (size_t)KMAX * cap * T * 2;
    std::vector<double> rn(nc), bn(nc);
    mv_norm2(c, r, d_n2);
    if (pairs) pair_sum_r(c, d_n2, nc);
    copy_to_host(c, d_n2, rn.data(), nc * sizeof(double));
    mv_norm2(c, b, d_n2);
    if (pairs) pair_sum_r(c, d_n2, nc);
    copy_to_host(c, d_n2, bn.data(), nc * sizeof(double));
    for (int i = 0; i < n; ++i) job.err[c0 + i] = bn[i] > 0 ? std::sqrt(rn[i] / bn[i]) : 0.0;
  }
}

// The top-level FP64 flexible GMRES over a batch of columns (column i: shift
// mu[i], right-hand side field rhs_of[i] of b, solution field i of x, both in
// the canonical layout on the device).  A scheduler keeps at most `max_active`
// columns in the internal layout at once.  At every restart the true FP64
// residual of each active column is recomputed; columns that meet tol (or
// have used max_outer iterations) write their solution back and leave, and
// waiting columns take their place.  When the membership changes, the active
// columns are gathered into dense tiles (ping-pong buffers), so converged
// columns cost nothing afterwards (section 3: shrinking the vector bundle).
void outer_solve(ddamg_ctx* c, OuterJob& job) {
  const int T = c->T, ncol = job.ncol;
  const int m = std::min(c->p.outer_restart, KMAX - 1);
  // doublets: the two columns of a pair are one Krylov vector of the doublet
  // operator; they enter, converge and leave together (even slot counts)
  const bool pairs = !job.eps.empty();
  DD_CHECK(!pairs || (ncol % 2 == 0 && (int)job.eps.size() == ncol), DDAMG_EINVAL, "doublet columns come in pairs");
  int wmax = std::max(1, std::min(ncol, job.max_active));
  if (pairs) wmax = std::max(2, wmax - wmax % 2);
  const int ntw = (wmax + T - 1) / T;
  const int prec = c->p.precision == DDAMG_MIXED ? P32 : P64;
  LW& w = lw(c, 0, P64, ntw);
  LW& w0 = lw(c, 0, prec, ntw);   // preconditioner-precision temporaries on level 0
  const int cap = w.cap;
  if (!w.d_map) {
    w.d_map = (int*)c->pool.alloc((size_t)cap * T * 3 * sizeof(int));
    w.d_muc = (double*)c->pool.alloc((size_t)cap * T * sizeof(double));
    w.d_epsc = (double*)c->pool.alloc((size_t)cap * T * sizeof(double));
  }
  MV Bs[2] = {get(c, w.cb, 0, P64, cap, ntw), get(c, w.cb2, 0, P64, cap, ntw)};
  MV Xs[2] = {get(c, w.cx, 0, P64, cap, ntw), get(c, w.cx2, 0, P64, cap, ntw)};
  MV vin = get(c, w0.rho, 0, prec, w0.cap, ntw);
  Precond smooth = [&](const MV& v, const MV& z, const double* dm) {
    NDScope diag(c, nullptr);   // doublets: the preconditioner is flavour diagonal (shifts +-mubar)
    if (c->nlev == 1) fine_smoother(c, v, z, dm);
    else mg_cycle(c, 0, dm, v, z);
  };
  // With inner_iters > 0 every outer step is preconditioned by an inner
  // FGMRES in the preconditioner's precision (FP32 Gram-Schmidt and stencil)
  // around the MG cycle / smoother, solved to inner_tol; the FP64 outer
  // FGMRES wins the accuracy back.
  const int mi = std::min(c->p.inner_iters, KMAX - 1);
  Precond pc = [&](const MV& v, const MV& z, const double* dm) {
    NDScope diag(c, nullptr);
    const MV in = (prec == v.prec) ? v : vin.tiles(0, v.ntiles);
    if (prec != v.prec) mv_copy(c, v, in);
    if (mi > 0) {
      KrylovOut ko;
      krylov(c, 0, dm, in, z, true, c->p.inner_tol, mi, c->p.inner_iters, &smooth, prec, false, &ko, 1);
      c->st.inner_iters += ko.total;
    } else {
      smooth(in, z, dm);
    }
  };
  job.iters.assign(ncol, 0);
  job.relres.assign(ncol, 0.0);
  job.converged.assign(ncol, 0);
  job.err.assign(ncol, 0.0);
  job.fallbacks.assign(ncol, 0);
  std::vector<double> bnorm(ncol, -1.0);
  std::vector<int> act;            // slot -> column (-1: empty)
  int next = 0, cur = 0, nt = 0, total = 0;
  double* d_n2 = w.d_h + (size_t)KMAX * cap * T * 2;
  Cycle cy(cap * T, m);
  cy.pairs = pairs;
  std::vector<double> beta, bn, tol_abs, est;
  std::vector<char> done;
  std::vector<char> leave;
  bool rebuild = true;
  while (true) {
    if (rebuild) {
      // new membership: kept columns first, then waiting ones, in dense tiles
      std::vector<int> nact, keep_map, b_map, x_map;
      for (int i = 0; i < (int)act.size(); ++i)
        if (act[i] >= 0 && !(i < (int)leave.size() && leave[i])) {
          nact.push_back(act[i]);
          keep_map.push_back(i);
        }
      const int nkeep = (int)nact.size();
      while ((int)nact.size() < wmax && next < ncol) {
        nact.push_back(next++);
        keep_map.push_back(-1);
      }
      if (nact.empty()) break;
      const int ntn = ((int)nact.size() + T - 1) / T;
      nact.resize(ntn * T, -1);
      keep_map.resize(ntn * T, -1);
      b_map.assign(ntn * T, -1);
      x_map.assign(ntn * T, -1);
      std::vector<double> nmu(ntn * T, 0.0), neps(ntn * T, 0.0);
      for (int i = 0; i < ntn * T; ++i) {
        if (nact[i] < 0) continue;
        nmu[i] = job.mu[nact[i]];
        if (pairs) neps[i] = job.eps[nact[i]];
        if (i >= nkeep) {
          b_map[i] = job.rhs_of[nact[i]];
          if (job.use_x0) x_map[i] = nact[i];
        }
      }
      int* d_keep = w.d_map;
      int* d_bmap = w.d_map + cap * T;
      int* d_xmap = w.d_map + 2 * cap * T;
      DD_HIP(hipMemcpyAsync(d_keep, keep_map.data(), ntn * T * sizeof(int), hipMemcpyHostToDevice, c->stream));
      DD_HIP(hipMemcpyAsync(d_bmap, b_map.data(), ntn * T * sizeof(int), hipMemcpyHostToDevice, c->stream));
      DD_HIP(hipMemcpyAsync(d_xmap, x_map.data(), ntn * T * sizeof(int), hipMemcpyHostToDevice, c->stream));
      DD_HIP(hipMemcpyAsync(w.d_muc, nmu.data(), ntn * T * sizeof(double), hipMemcpyHostToDevice, c->stream));
      DD_HIP(hipMemcpyAsync(w.d_epsc, neps.data(), ntn * T * sizeof(double), hipMemcpyHostToDevice, c->stream));
      const int alt = act.empty() ? cur : 1 - cur;
      const MV nb = Bs[alt].tiles(0, ntn), nx = Xs[alt].tiles(0, ntn);
      if (act.empty()) {
        mv_zero(c, nb);
        mv_zero(c, nx);
      } else {
        // kept columns move from the current buffers (empty slots become zero)
        const MV ob = Bs[cur].tiles(0, nt), ox = Xs[cur].tiles(0, nt);
        mv_gather_cols(c, ob, nb, d_keep, 0);
        mv_gather_cols(c, ox, nx, d_keep, 0);
      }
      canon_cols(c, 0, nb, d_bmap, const_cast<double*>(job.b), 0);
      if (job.use_x0) canon_cols(c, 0, nx, d_xmap, job.x, 0);
      DD_HIP(hipStreamSynchronize(c->stream));   // the host maps above are reused
      if (!act.empty()) c->st.col_removals++;
      act = nact;
      cur = alt;
      nt = ntn;
      const int nc = nt * T;
      // right-hand-side norms of the new columns
      std::vector<double> bn2(nc);
      mv_norm2(c, nb, d_n2);
      if (pairs) pair_sum_r(c, d_n2, nc);
      copy_to_host(c, d_n2, bn2.data(), nc * sizeof(double));
      bn.assign(nc, 0.0);
      tol_abs.assign(nc, 0.0);
      for (int i = 0; i < nc; ++i) {
        if (act[i] < 0) continue;
        if (bnorm[act[i]] < 0) bnorm[act[i]] = host_norm_guard(bn2[i]);
        bn[i] = bnorm[act[i]];
        tol_abs[i] = c->p.tol * bn[i];
      }
      est.assign(nc, 0.0);
      done.assign(nc, 0);
      leave.assign(nc, 0);
      rebuild = false;
      if (c->p.verbose) {
        std::fprintf(stderr, "[ddamg] outer %d: %d columns active in %d tiles, %d waiting\n", total,
                     (int)(act.size() - std::count(act.begin(), act.end(), -1)), nt, ncol - next);
        std::fflush(stderr);
      }
    }
    const MV b = Bs[cur].tiles(0, nt), x = Xs[cur].tiles(0, nt);
    const int nc = nt * T;
    NDScope nd(c, pairs ? w.d_epsc : nullptr);
    residual_norms(c, 0, w, nt, b, x, w.d_muc, false, d_n2, beta, pairs);
    bool any_leave = false;
    for (int i = 0; i < nc; ++i) {
      est[i] = beta[i];
      if (act[i] < 0) {
        done[i] = 1;
        continue;
      }
      const int col = act[i];
      const bool conv = bn[i] == 0 || beta[i] <= tol_abs[i];
      job.relres[col] = bn[i] > 0 ? beta[i] / bn[i] : 0.0;
      job.converged[col] = conv;
      done[i] = 0;
      if (conv || job.iters[col] >= c->p.max_outer) {
        leave[i] = 1;
        any_leave = true;
      }
    }
    if (any_leave) {
      // solutions of the leaving columns go back to the caller's x
      std::vector<int> out_map(nc, -1);
      for (int i = 0; i < nc; ++i)
        if (leave[i]) out_map[i] = act[i];
      int* d_out = w.d_map + cap * T;
      DD_HIP(hipMemcpyAsync(d_out, out_map.data(), nc * sizeof(int), hipMemcpyHostToDevice, c->stream));
      canon_cols(c, 0, x, d_out, job.x, 1);
      DD_HIP(hipStreamSynchronize(c->stream));
    }
    int n_stay = 0;
    for (int i = 0; i < nc; ++i) n_stay += act[i] >= 0 && !leave[i];
    if (any_leave && (next < ncol || n_stay == 0 || (n_stay + T - 1) / T < nt)) {
      rebuild = true;   // compact (and refill) before the next cycle
      continue;
    }
    if (n_stay == 0) break;
    for (int i = 0; i < nc; ++i)
      if (leave[i]) {   // left, but no tile to gain: carried as a finished slot
        done[i] = 1;
        act[i] = -1;
        leave[i] = 0;
      }
    const int fb0 = c->st.learned_fallbacks;
    gmres_cycle(c, 0, w, nt, x, w.d_muc, &pc, prec, m, false, beta, done, tol_abs, est, bn, cy, d_n2, total);
    const int dfb = c->st.learned_fallbacks - fb0;
    for (int i = 0; i < nc; ++i)
      if (act[i] >= 0) {
        job.iters[act[i]] += cy.kc[i];
        if (!done[i]) job.fallbacks[act[i]] += dfb;
      }
  }
  job.total = total;
  final_check(c, job, w, wmax);
}

// --------------------------------------------------------------- MG ---
static void mr_smooth(ddamg_ctx* c, int level, const double* d_mu, const MV& f, const MV& xo, int iters) {
  const int nt = f.ntiles, ncol = f.ncol();
  LW& w = lw(c, level, f.prec, nt);
  MV rho = get(c, w.rho, level, f.prec, w.cap, nt);
  MV q = get(c, w.q, level, f.prec, w.cap, nt);
  mv_copy(c, f, rho);
  mv_zero(c, xo);
  double* qr = w.d_aux;
  double* qq = w.d_aux + 2 * ncol;
  double* al = w.d_aux + 4 * ncol;
  for (int k = 0; k < iters; ++k) {
    operator_apply(c, level, rho, q, d_mu);
    mv_dot(c, q, rho, qr);
    mv_norm2(c, q, qq);
    hipLaunchKernelGGL(k_mr_alpha, dim3((ncol + 255) / 256), dim3(256), 0, c->stream, qr, qq, al, ncol);
    DD_HIP(hipGetLastError());
    mv_axpy(c, al, rho, xo, +1);
    mv_axpy(c, al, q, rho, -1);
  }
}

// Sets the gamma5-output flag of a coarse level for the lifetime of the
// object (restored on every exit path).
struct G5Scope {
  ddamg_ctx* c;
  int level, saved;
  G5Scope(ddamg_ctx* c_, int l, int on) : c(c_), level(l), saved(c_->coarse[l].g5out) { c->coarse[l].g5out = on; }
  ~G5Scope() { c->coarse[level].g5out = saved; }
};

// e = MG_l(r): restrict, solve the next level, prolong, post-smooth.
// With coarse_gamma5 the Krylov solves of the next level run on
// gamma5_c D_c(mu) e_c = gamma5_c r_c, whose operator Q_c + i dmu mu (Q_c the
// Hermitian gamma5_c D_c(0)) is normal: same solution and residual norm,
// but GMRES is not slowed by the non-normality of D_c.  A middle-level
// preconditioner then approximates (gamma5_c D_c)^-1 = D_c^-1 gamma5_c.
void mg_cycle(ddamg_ctx* c, int l, const double* d_mu, const MV& r, const MV& e) {
  const int nt = r.ntiles, prec = r.prec;
  LW& w = lw(c, l, prec, nt);
  MV rc = get(c, w.rc, l + 1, prec, w.cap, nt);
  MV ec = get(c, w.ec, l + 1, prec, w.cap, nt);
  restrict_mv(c, l, r, rc);
  KrylovOut ko;
  const bool bottom = (l + 2 == c->nlev);
  const bool g5 = c->p.coarse_gamma5 >= (bottom ? 1 : 2);
  if (g5) mv_gamma5(c, rc);
  if (bottom && c->p.coarsest_block) {
    G5Scope gs(c, l + 1, g5);
    int total = 0;
    block_gmres(c, l + 1, d_mu, rc, ec, true, c->p.r_b, std::min(c->p.bottom_maxit, KMAX - 1), c->p.bottom_maxit,
                nullptr, nullptr, &total);
    c->st.bottom_calls++;
    c->st.bottom_iters += total;
  } else if (bottom && c->p.bottom_dr_k > 0) {
    G5Scope gs(c, l + 1, g5);
    const int mr = c->p.bottom_restart > 0 ? c->p.bottom_restart : std::min(c->p.bottom_maxit, KMAX - 1);
    krylov_dr(c, l + 1, d_mu, rc, ec, true, c->p.r_b, mr, c->p.bottom_dr_k, c->p.bottom_maxit, &ko);
    c->st.bottom_calls++;
    c->st.bottom_iters += ko.total;
  } else if (bottom) {
    G5Scope gs(c, l + 1, g5);
    const int mr = c->p.bottom_restart > 0 ? c->p.bottom_restart : std::min(c->p.bottom_maxit, KMAX - 1);
    krylov(c, l + 1, d_mu, rc, ec, true, c->p.r_b, mr, c->p.bottom_maxit, nullptr, prec, false, &ko);
    c->st.bottom_calls++;
    c->st.bottom_iters += ko.total;
  } else {
    G5Scope gs(c, l + 1, g5);
    Precond pc = [&](const MV& v, const MV& z, const double* dm) {
      if (!g5) {
        mg_cycle(c, l + 1, dm, v, z);
        return;
      }
      // z = MG_{l+1}(gamma5 v): the cycle sees the plain operator D_{l+1};
      // v is flipped in place and restored (the cycle only reads it)
      G5Scope plain(c, l + 1, 0);
      mv_gamma5(c, v);
      mg_cycle(c, l + 1, dm, v, z);
      mv_gamma5(c, v);
    };
    krylov(c, l + 1, d_mu, rc, ec, true, c->p.r_m, std::min(c->p.middle_restart, KMAX - 1), c->p.middle_maxit, &pc,
           prec, false, &ko);
    c->st.middle_calls++;
    c->st.middle_iters += ko.total;
  }
  prolong_mv(c, l, ec, e, 0);
  MV res = get(c, w.res, l, prec, w.cap, nt);
  MV s = get(c, w.s, l, prec, w.cap, nt);
  if (l == 0) {
    fine_residual(c, r, e, res, d_mu);
    fine_smoother(c, res, s, d_mu);
  } else {
    MV t = get(c, w.q, l, prec, w.cap, nt);
    operator_apply(c, l, e, t, d_mu);
    mv_sub(c, r, t, res);
    mr_smooth(c, l, d_mu, res, s, c->p.coarse_smooth_iters);
  }
  mv_add(c, s, e);
}

// Fine-level smoother: SAP, or the learned PTC network (FP32) with SAP as the
// fallback whenever the network does not reduce the residual of every column.
void fine_smoother(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu) {
  if (c->p.smoother != DDAMG_SMOOTHER_LEARNED) {
    sap_apply(c, f, x, d_mu, x);
    return;
  }
  DD_CHECK(ptc_ready(c), DDAMG_ESTATE, "learned smoother selected but no weights set");
  if (!ptc_smooth(c, f, x, d_mu, c->p.smoother_cycles)) {
    c->st.learned_fallbacks++;
    sap_apply(c, f, x, d_mu, x);
  }
}

// ------------------------------------------------------------- setup ---
void galerkin(ddamg_ctx* c, int l) {
  const int N = c->tr[l].N;
  MV X = mv_alloc(c, l, P64, 2 * N);
  MV Y = mv_alloc(c, l, P64, 2 * N);
  MV Rc = mv_alloc(c, l + 1, P64, 2 * N);
  build_basis_field(c, l, X);
  for (int slot = 0; slot < 9; ++slot) {
    const int mode = slot == 0 ? 0 : 1;
    if (l == 0) fine_masked(c, X, Y, mode, slot - 1);
    else coarse_masked(c, l, X, Y, mode, slot - 1);
    restrict_mv(c, l, Y, Rc);
    scatter_blocks(c, l, Rc, slot);
  }
  DD_HIP(hipStreamSynchronize(c->stream));
  mv_free(c, X);
  mv_free(c, Y);
  mv_free(c, Rc);
}

// Build P (orthonormalised test vectors) of transition l and every operator
// below it.  tv: FP64 multivector of N columns on level l.
void build_transition(ddamg_ctx* c, int l, const MV& tv) {
  const LevelGeom& g = c->geom[l];
  const int N = c->tr[l].N;
  const size_t nP = (size_t)g.V * g.dof * N * 2;
  if (!c->tr[l].d_P64) {
    c->tr[l].d_P64 = (double*)c->pool.alloc(nP * sizeof(double));
    if (l == 0 && c->p.transfer_fp16 && c->p.precision == DDAMG_MIXED) {
      // the FP32 transfers of this level read the FP16 copy only: no FP32 copy
      DD_CHECK(N % 4 == 0 && (N == 24 || N == 32) && g.gsize % 64 == 0 && g.V % 256 == 0 && g.dof % 2 == 0,
               DDAMG_EINVAL, "transfer_fp16 needs N = 24 or 32 and aggregates of a multiple of 64 sites");
      c->tr[l].d_P16T = c->pool.alloc(nP * sizeof(_Float16));
    } else {
      c->tr[l].d_P32 = (float*)c->pool.alloc(nP * sizeof(float));
    }
  }
  gather_test_vectors(c, l, tv, c->tr[l].d_P64);
  orthonormalise_P(c, l, c->tr[l].d_P64);
  convert_P32(c, l);
  const LevelGeom& gc = c->geom[l + 1];
  const size_t nb = (size_t)gc.V * 9 * gc.dof * gc.dof * 2;
  if (!c->coarse[l + 1].d_blk64) {
    c->coarse[l + 1].d_blk64 = (double*)c->pool.alloc(nb * sizeof(double));
    c->coarse[l + 1].d_blk32 = (float*)c->pool.alloc(nb * sizeof(float));
  }
  c->coarse[l + 1].mu_factor = (l + 2 == c->nlev) ? c->p.coarse_mu_factor : 1.0;
  galerkin(c, l);
  convert_blocks32(c, l + 1);
  DD_HIP(hipStreamSynchronize(c->stream));
}

// Test-vector generation of transition l: random start vectors, then
// setup_rounds smoothing rounds (SAP on the fine level, fixed-length GMRES on
// a coarse level) each followed by normalisation (section 2: P from a few
// approximate low modes).
void setup_transition(ddamg_ctx* c, int l, const double* tv_init_host) {
  const LevelGeom& g = c->geom[l];
  const int N = c->tr[l].N;
  MV tv = mv_alloc(c, l, P64, N);
  MV tmp = mv_alloc(c, l, P64, N);
  if (tv_init_host) {
    const size_t n = (size_t)N * g.V * g.dof * 2;
    double* d = (double*)c->pool.alloc(n * sizeof(double));
    DD_HIP(hipMemcpy(d, tv_init_host, n * sizeof(double), hipMemcpyHostToDevice));
    to_internal(c, l, d, N, tv);
    DD_HIP(hipStreamSynchronize(c->stream));
    c->pool.release(d);
  } else {
    random_fill(c, l, tv, N, c->p.seed + 7919ULL * (l + 1));
  }
  std::vector<double> hmu(tv.ncol(), 0.0);
  for (int i = 0; i < N; ++i) hmu[i] = c->p.mu_setup;
  double* d_mu = (double*)c->pool.alloc(hmu.size() * sizeof(double));
  DD_HIP(hipMemcpy(d_mu, hmu.data(), hmu.size() * sizeof(double), hipMemcpyHostToDevice));
  double* d_n2 = (double*)c->pool.alloc(tv.ncol() * sizeof(double));
  for (int r = 0; r < c->p.setup_rounds; ++r) {
    if (l == 0 && c->p.setup_fine_iters > 0) {
      // inverse iteration: k steps of SAP-preconditioned FGMRES on D x = tv
      const int sp = c->p.precision == DDAMG_MIXED ? P32 : P64;
      LW& ws = lw(c, 0, sp, tv.ntiles);
      MV vin = get(c, ws.rho, 0, sp, ws.cap, tv.ntiles);
      Precond pc = [&](const MV& v, const MV& z, const double* dm) {
        if (sp != v.prec) {
          mv_copy(c, v, vin);
          sap_apply(c, vin, z, dm, z);
        } else {
          sap_apply(c, v, z, dm, z);
        }
      };
      krylov(c, 0, d_mu, tv, tmp, true, 0.0, c->p.setup_fine_iters, c->p.setup_fine_iters, &pc, sp, true, nullptr);
    } else if (l == 0) {
      sap_apply(c, tv, tmp, d_mu, tmp);
    } else {
      krylov(c, l, d_mu, tv, tmp, true, 0.0, c->p.setup_coarse_iters, c->p.setup_coarse_iters, nullptr, P64, true,
             nullptr);
    }
    mv_norm2(c, tmp, d_n2);
    mv_normalize(c, tmp, d_n2);
    mv_copy(c, tmp, tv);
  }
  build_transition(c, l, tv);
  c->pool.release(d_mu);
  c->pool.release(d_n2);
  mv_free(c, c->tvk[l]);
  c->tvk[l] = tv;
  mv_free(c, tmp);
}

// Bootstrap rounds: the fine test vectors are replaced by the multigrid cycle
// applied to them (an approximate inverse iteration with the current
// hierarchy), normalised, and every transition is rebuilt.
void bootstrap(ddamg_ctx* c) {
  MV& tv = c->tvk[0];
  const int N = c->tr[0].N;
  MV z = mv_alloc(c, 0, P64, N);
  std::vector<double> hmu(tv.ncol(), 0.0);
  for (int i = 0; i < N; ++i) hmu[i] = c->p.mu_setup;
  double* d_mu = (double*)c->pool.alloc(hmu.size() * sizeof(double));
  DD_HIP(hipMemcpy(d_mu, hmu.data(), hmu.size() * sizeof(double), hipMemcpyHostToDevice));
  double* d_n2 = (double*)c->pool.alloc(tv.ncol() * sizeof(double));
  for (int r = 0; r < c->p.setup_boot; ++r) {
    mg_cycle(c, 0, d_mu, tv, z);
    mv_norm2(c, z, d_n2);
    mv_normalize(c, z, d_n2);
    mv_copy(c, z, tv);
    build_transition(c, 0, tv);
    for (int l = 1; l + 1 < c->nlev; ++l) setup_transition(c, l, nullptr);
  }
  c->pool.release(d_mu);
  c->pool.release(d_n2);
  mv_free(c, z);
}

void build_hierarchy(ddamg_ctx* c, const double* const* tv_init) {
  for (int l = 0; l + 1 < c->nlev; ++l) setup_transition(c, l, tv_init ? tv_init[l] : nullptr);
  if (c->nlev > 1 && c->p.setup_boot > 0) bootstrap(c);
  // the setup smooths all N test vectors at once in FP64: its Krylov and
  // cycle workspaces are sized for N columns, far more than a solve of a
  // large lattice can afford next to its own; drop them (the solve sizes
  // its workspaces for its own column tiles)
  DD_HIP(hipStreamSynchronize(c->stream));
  free_work(c);
  free_block_work(c);
  // the smoothed test vectors served the bootstrap only (P holds their
  // orthonormalised form)
  for (int l = 0; l < 2; ++l) mv_free(c, c->tvk[l]);
}

// Rebuild from host test vectors (canonical layout) of transition l.
void rebuild_from_test_vectors(ddamg_ctx* c, int l, const double* tv_host) {
  const LevelGeom& g = c->geom[l];
  const int N = c->tr[l].N;
  MV tv = mv_alloc(c, l, P64, N);
  const size_t n = (size_t)N * g.V * g.dof * 2;
  double* d = (double*)c->pool.alloc(n * sizeof(double));
  DD_HIP(hipMemcpy(d, tv_host, n * sizeof(double), hipMemcpyHostToDevice));
  to_internal(c, l, d, N, tv);
  build_transition(c, l, tv);
  c->pool.release(d);
  mv_free(c, tv);
  // every coarser transition is rebuilt from its current P (coarse operators changed)
  for (int q = l + 1; q + 1 < c->nlev; ++q) {
    c->coarse[q + 1].mu_factor = (q + 2 == c->nlev) ? c->p.coarse_mu_factor : 1.0;
    galerkin(c, q);
    convert_blocks32(c, q + 1);
  }
  DD_HIP(hipStreamSynchronize(c->stream));
}

// ------------------------------------------------------------- solve ---
// Outer FP64 FGMRES over all columns, preconditioned by the MG cycle in the
// precision of the chosen mode.

}  // namespace ddamg
