// extern "C" entry points of libddamg (declared in include/ddamg.h).  No
// exception crosses this boundary: every entry point returns a status code
// and keeps a thread-local message for ddamg_last_error().
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>

#include "common.h"

namespace ddamg {
void build_geometry(ddamg_ctx* c, int level, const int* dims, const int* grp, int dof, bool fine);
void build_sap_lists(ddamg_ctx* c);
void upload_gauge(ddamg_ctx* c, const double* gauge, int on_device);
void build_hierarchy(ddamg_ctx* c, const double* const* tv_init);
void rebuild_from_test_vectors(ddamg_ctx* c, int l, const double* tv_host);
void free_work(ddamg_ctx* c);
void random_fill(ddamg_ctx* c, int level, const MV& X, int ncol, uint64_t seed);
void mv_normalize(ddamg_ctx* c, const MV& x, const double* d_n2);
}  // namespace ddamg

using namespace ddamg;

static thread_local std::string g_last_error;

template <typename F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DDAMG_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DDAMG_EDEVICE;
  }
}

extern "C" {

const char* ddamg_last_error(void) { return g_last_error.c_str(); }

const char* ddamg_strerror(int s) {
  switch (s) {
    case DDAMG_OK: return "ok";
    case DDAMG_NOT_CONVERGED: return "not converged: solution written, some columns above tolerance";
    case DDAMG_EINVAL: return "invalid argument";
    case DDAMG_ENOMEM: return "out of device memory";
    case DDAMG_EDEVICE: return "HIP runtime error";
    case DDAMG_EBREAKDOWN: return "unrecoverable Krylov breakdown";
    case DDAMG_ESTATE: return "object not built";
    default: return "unknown status";
  }
}

void ddamg_default_params(ddamg_params* p) {
  std::memset(p, 0, sizeof(*p));
  for (int m = 0; m < 4; ++m) {
    p->dims[m] = 4;
    p->agg[0][m] = 2;
    p->agg[1][m] = 2;
    p->sap_block[m] = 2;
  }
  p->kappa = 0.14;
  p->n_levels = 2;
  p->n_tv[0] = 8;
  p->n_tv[1] = 8;
  p->sap_cycles = 4;
  p->sap_mr_iters = 4;
  p->setup_rounds = 3;
  p->setup_coarse_iters = 10;
  p->setup_boot = 0;
  p->setup_fine_iters = 0;
  p->mu_setup = 0.0;
  p->coarse_mu_factor = 1.0;
  p->tol = 1e-10;
  p->r_m = 7e-2;
  p->r_b = 1e-1;
  p->outer_restart = 10;
  p->max_outer = 500;
  p->middle_restart = 20;
  p->middle_maxit = 50;
  p->bottom_maxit = 50;
  p->coarse_smooth_iters = 2;
  p->coarsest_block = 0;
  p->precision = DDAMG_PLAIN_FP64;
  p->smoother = DDAMG_SMOOTHER_SAP;
  p->smoother_cycles = 1;
  p->max_active_cols = 0;
  p->inner_iters = 0;
  p->use_graphs = 1;
  p->inner_tol = 1e-2;
  p->inner_fp16 = 0;
  p->col_tile = 8;
  p->seed = 12345;
  p->verbose = 0;
  p->csw = 0.0;
  p->sap_oddeven = 0;
  p->coarse_gamma5 = 0;
  p->bottom_restart = 0;
  p->bottom_dr_k = 0;
  p->coarse_fp16 = 0;
  p->transfer_fp16 = 0;
}

static void validate(const ddamg_params* p) {
  DD_CHECK(p, DDAMG_EINVAL, "null params");
  DD_CHECK(p->n_levels >= 1 && p->n_levels <= 3, DDAMG_EINVAL, "n_levels must be 1, 2 or 3");
  DD_CHECK(p->kappa > 0, DDAMG_EINVAL, "kappa must be positive");
  DD_CHECK(std::isfinite(p->csw), DDAMG_EINVAL, "csw must be finite");
  DD_CHECK(p->sap_oddeven == 0 || p->sap_oddeven == 1, DDAMG_EINVAL, "sap_oddeven must be 0 or 1");
  DD_CHECK(p->coarse_gamma5 >= 0 && p->coarse_gamma5 <= 2, DDAMG_EINVAL, "coarse_gamma5 must be 0, 1 or 2");
  DD_CHECK(!p->sap_oddeven || (p->csw == 0.0 && p->sap_block[0] == 4 && p->sap_block[1] == 4 &&
                               p->sap_block[2] == 4 && p->sap_block[3] == 4),
           DDAMG_EINVAL, "odd-even SAP needs 4^4 blocks and no clover term");
  DD_CHECK(p->col_tile == 0 || p->col_tile == 8, DDAMG_EINVAL, "col_tile must be 8");
  int dims[4];
  for (int m = 0; m < 4; ++m) {
    DD_CHECK(p->dims[m] >= 1, DDAMG_EINVAL, "lattice extents must be >= 1");
    DD_CHECK(p->sap_block[m] >= 1 && p->dims[m] % p->sap_block[m] == 0, DDAMG_EINVAL,
             "SAP block extents must divide the lattice");
    dims[m] = p->dims[m];
  }
  const int bs = p->sap_block[0] * p->sap_block[1] * p->sap_block[2] * p->sap_block[3];
  DD_CHECK(bs == 16 || bs == 256, DDAMG_EINVAL, "SAP blocks must have 16 or 256 sites");
  for (int l = 0; l + 1 < p->n_levels; ++l) {
    DD_CHECK(p->n_tv[l] >= 2 && p->n_tv[l] % 2 == 0 && p->n_tv[l] <= 64, DDAMG_EINVAL,
             "test vector counts must be even and in [2, 64]");
    for (int m = 0; m < 4; ++m) {
      DD_CHECK(p->agg[l][m] >= 1 && dims[m] % p->agg[l][m] == 0, DDAMG_EINVAL,
               "aggregate extents must divide the lattice");
      if (l == 0)
        DD_CHECK(p->agg[0][m] == p->sap_block[m], DDAMG_EINVAL, "first-level aggregates must equal the SAP blocks");
      dims[m] /= p->agg[l][m];
    }
  }
  DD_CHECK(p->sap_cycles >= 1 && p->sap_mr_iters >= 1, DDAMG_EINVAL, "SAP cycle counts must be >= 1");
  DD_CHECK(p->outer_restart >= 1 && p->outer_restart <= 63, DDAMG_EINVAL, "outer_restart in [1, 63]");
  DD_CHECK(p->middle_restart >= 1 && p->middle_restart <= 63, DDAMG_EINVAL, "middle_restart in [1, 63]");
  DD_CHECK(p->bottom_maxit >= 1, DDAMG_EINVAL, "bottom_maxit >= 1");
  DD_CHECK(p->bottom_restart >= 0 && p->bottom_restart <= 63, DDAMG_EINVAL, "bottom_restart in [0, 63]");
  DD_CHECK(p->bottom_dr_k >= 0 && (p->bottom_dr_k == 0 || p->bottom_dr_k + 1 <
                                   (p->bottom_restart > 0 ? p->bottom_restart : std::min(p->bottom_maxit, 63))),
           DDAMG_EINVAL, "bottom_dr_k must be below the coarsest restart length minus one");
  DD_CHECK(p->coarse_fp16 == 0 || p->coarse_fp16 == 1, DDAMG_EINVAL, "coarse_fp16 must be 0 or 1");
  DD_CHECK(p->transfer_fp16 == 0 || p->transfer_fp16 == 1, DDAMG_EINVAL, "transfer_fp16 must be 0 or 1");
  DD_CHECK(p->setup_fine_iters >= 0 && p->setup_fine_iters <= 63, DDAMG_EINVAL, "setup_fine_iters in [0, 63]");
  DD_CHECK(p->setup_boot >= 0 && p->setup_boot <= 16, DDAMG_EINVAL, "setup_boot in [0, 16]");
  DD_CHECK(p->setup_coarse_iters >= 1 && p->setup_coarse_iters <= 63, DDAMG_EINVAL, "setup_coarse_iters in [1, 63]");
  DD_CHECK(p->tol > 0 && p->r_m > 0 && p->r_b > 0, DDAMG_EINVAL, "tolerances must be positive");
  DD_CHECK(p->precision == DDAMG_PLAIN_FP64 || p->precision == DDAMG_MIXED, DDAMG_EINVAL, "precision mode");
  DD_CHECK(p->smoother == DDAMG_SMOOTHER_SAP || p->smoother == DDAMG_SMOOTHER_LEARNED, DDAMG_EINVAL, "smoother");
  DD_CHECK(p->smoother_cycles >= 1 && p->smoother_cycles <= 64, DDAMG_EINVAL, "smoother_cycles");
  DD_CHECK(p->max_active_cols >= 0, DDAMG_EINVAL, "max_active_cols");
  DD_CHECK(p->inner_iters >= 0 && p->inner_iters <= 10000 && p->inner_tol >= 0 && p->inner_tol < 1, DDAMG_EINVAL,
           "inner_iters / inner_tol");
}

// ------------------------------------------------ no-allocation scratch ---
// Device memory of ddamg_apply_op_noalloc: a file-scope device array (each
// GPU holds its own copy while the library is loaded).  Host code never uses
// its name as an address: the address is resolved once per device, with that
// device current, at the first setup on it, and kept per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_addr[64] = {};

static void* noalloc_scratch_address(int dev) {
  DD_CHECK(dev >= 0 && dev < 64, DDAMG_EDEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    DD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch)));
    DD_CHECK(ptr != nullptr, DDAMG_EDEVICE, "no device address for the scratch array");
    g_scratch_addr[dev] = ptr;
  }
  return g_scratch_addr[dev];
}

int ddamg_setup(const ddamg_params* p, const double* gauge, int gauge_on_device, const double* const* tv_init,
                void* hip_stream, ddamg_ctx** out) {
  return guarded([&]() -> int {
    DD_CHECK(out && gauge, DDAMG_EINVAL, "null pointer");
    *out = nullptr;
    validate(p);
    auto t0 = std::chrono::steady_clock::now();
    ddamg_ctx* c = new ddamg_ctx();
    try {
      DD_HIP(hipGetDevice(&c->device));
      c->noalloc_scratch = noalloc_scratch_address(c->device);
      c->p = *p;
      if (c->p.col_tile == 0) c->p.col_tile = 8;
      c->T = 8;
      c->stream = (hipStream_t)hip_stream;
      c->pool.stream = c->stream;
      c->nlev = p->n_levels;
      c->m0 = 1.0 / (2.0 * p->kappa) - 4.0;
      c->diag = 4.0 + c->m0;
      int dims[4] = {p->dims[0], p->dims[1], p->dims[2], p->dims[3]};
      build_geometry(c, 0, dims, p->sap_block, 12, true);
      for (int l = 1; l < c->nlev; ++l) {
        int grp[4] = {1, 1, 1, 1};
        for (int m = 0; m < 4; ++m) {
          dims[m] /= p->agg[l - 1][m];
          if (l + 1 < c->nlev) grp[m] = p->agg[l][m];
        }
        build_geometry(c, l, dims, grp, 2 * p->n_tv[l - 1], false);
        c->tr[l - 1].N = p->n_tv[l - 1];
      }
      build_sap_lists(c);
      upload_gauge(c, gauge, gauge_on_device);
      if (p->csw != 0.0) build_clover(c);
      build_hierarchy(c, tv_init);
      DD_HIP(hipStreamSynchronize(c->stream));
      c->pool.trim();
    } catch (...) {
      c->pool.clear();
      delete c;
      throw;
    }
    c->st.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = c;
    return DDAMG_OK;
  });
}

void ddamg_destroy(ddamg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_work(c);
  free_ptc(c);
  free_block_work(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  c->pool.clear();
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  for (hipEvent_t e : c->sap_ev) (void)hipEventDestroy(e);
  delete c;
}

int ddamg_level_info(ddamg_ctx* c, int level, int* volume, int* dof, int dims[4]) {
  return guarded([&]() -> int {
    DD_CHECK(c, DDAMG_EINVAL, "null context");
    DD_CHECK(level >= 0 && level < c->nlev, DDAMG_ESTATE, "level not built");
    const LevelGeom& g = c->geom[level];
    if (volume) *volume = g.V;
    if (dof) *dof = g.dof;
    if (dims)
      for (int m = 0; m < 4; ++m) dims[m] = g.dims[m];
    return DDAMG_OK;
  });
}

static double* upload_mu(ddamg_ctx* c, const double* mu, int n_col, int ncolp) {
  std::vector<double> h(ncolp, 0.0);
  for (int i = 0; i < n_col; ++i) {
    DD_CHECK(std::isfinite(mu[i]), DDAMG_EINVAL, "mu contains NaN/Inf");
    h[i] = mu[i];
  }
  double* d = (double*)c->pool.alloc(h.size() * sizeof(double));
  DD_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  DD_HIP(hipStreamSynchronize(c->stream));
  return d;
}

int ddamg_apply_op(ddamg_ctx* c, int level, int precision, const double* mu, int n_col, const double* x, double* y) {
  return guarded([&]() -> int {
    DD_CHECK(c && mu && x && y && n_col >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    DD_CHECK(level >= 0 && level < c->nlev, DDAMG_ESTATE, "level not built");
    DD_CHECK(precision == DDAMG_FP64 || precision == DDAMG_FP32, DDAMG_EINVAL, "precision");
    const int prec = precision == DDAMG_FP64 ? P64 : P32;
    MV a = mv_alloc(c, level, prec, n_col), b = mv_alloc(c, level, prec, n_col);
    double* d_mu = upload_mu(c, mu, n_col, a.ncol());
    to_internal(c, level, x, n_col, a);
    operator_apply(c, level, a, b, d_mu);
    from_internal(c, level, b, n_col, y);
    DD_HIP(hipStreamSynchronize(c->stream));
    mv_free(c, a);
    mv_free(c, b);
    c->pool.release(d_mu);
    return DDAMG_OK;
  });
}

int ddamg_apply_op_nd(ddamg_ctx* c, int precision, const double* mubar, const double* epsbar, int n_pair,
                      const double* x, double* y) {
  return guarded([&]() -> int {
    DD_CHECK(c && mubar && epsbar && x && y && n_pair >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    DD_CHECK(precision == DDAMG_FP64 || precision == DDAMG_FP32, DDAMG_EINVAL, "precision");
    const int prec = precision == DDAMG_FP64 ? P64 : P32;
    const int ncol = 2 * n_pair;
    std::vector<double> hmu(ncol), eps;
    for (int i = 0; i < n_pair; ++i) {
      DD_CHECK(std::isfinite(mubar[i]) && std::isfinite(epsbar[i]), DDAMG_EINVAL, "mubar / epsbar contain NaN/Inf");
      hmu[2 * i] = mubar[i];
      hmu[2 * i + 1] = -mubar[i];
    }
    MV a = mv_alloc(c, 0, prec, ncol), b = mv_alloc(c, 0, prec, ncol);
    eps.assign(a.ncol(), 0.0);
    for (int i = 0; i < n_pair; ++i) eps[2 * i] = eps[2 * i + 1] = epsbar[i];
    double* d_mu = upload_mu(c, hmu.data(), ncol, a.ncol());
    double* d_eps = upload_mu(c, eps.data(), a.ncol(), a.ncol());
    to_internal(c, 0, x, ncol, a);
    const double* saved = c->nd_eps;
    c->nd_eps = d_eps;
    try {
      operator_apply(c, 0, a, b, d_mu);
    } catch (...) {
      c->nd_eps = saved;
      throw;
    }
    c->nd_eps = saved;
    from_internal(c, 0, b, ncol, y);
    DD_HIP(hipStreamSynchronize(c->stream));
    mv_free(c, a);
    mv_free(c, b);
    c->pool.release(d_mu);
    c->pool.release(d_eps);
    return DDAMG_OK;
  });
}

// ddamg_apply_op without any allocation: the internal-layout input and
// output and the per-column shifts live in the device's scratch array.
int ddamg_apply_op_noalloc(ddamg_ctx* c, int level, int precision, const double* mu, int n_col, const double* x,
                           double* y) {
  return guarded([&]() -> int {
    DD_CHECK(c && mu && x && y && n_col >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    DD_CHECK(level >= 0 && level < c->nlev, DDAMG_ESTATE, "level not built");
    DD_CHECK(precision == DDAMG_FP64 || precision == DDAMG_FP32, DDAMG_EINVAL, "precision");
    DD_CHECK(c->noalloc_scratch, DDAMG_ESTATE, "scratch array not resolved for this device");
    for (int i = 0; i < n_col; ++i) DD_CHECK(std::isfinite(mu[i]), DDAMG_EINVAL, "mu contains NaN/Inf");
    const LevelGeom& g = c->geom[level];
    MV a;
    a.prec = precision == DDAMG_FP64 ? P64 : P32;
    a.T = c->T;
    a.ntiles = (n_col + a.T - 1) / a.T;
    a.dof = g.dof;
    a.nsites = g.V;
    a.nchunk = 2 * a.dof / reals_per_chunk(a.prec);
    a.owned = false;
    auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t vb = up256(a.bytes()), mb = up256((size_t)a.ncol() * sizeof(double));
    const size_t need = 2 * vb + mb;
    if (need > NOALLOC_SCRATCH_BYTES) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "batch needs %zu bytes of scratch, more than the %zu of the no-allocation entry",
                    need, NOALLOC_SCRATCH_BYTES);
      throw Error{DDAMG_EINVAL, msg};
    }
    char* base = static_cast<char*>(c->noalloc_scratch);
    MV b = a;
    a.p = base;
    b.p = base + vb;
    double* d_mu = reinterpret_cast<double*>(base + 2 * vb);
    // the padded columns of the last tile start at zero, with zero shift;
    // the array keeps the previous call's contents, so clear it (fill kernel)
    mv_zero(c, a);
    MV mupad = a;
    mupad.p = d_mu;
    mupad.prec = P64;
    mupad.nchunk = 1;
    mupad.nsites = 1;
    mupad.dof = 1;
    mupad.T = 1;
    mupad.ntiles = (int)(mb / 16);   // mb / 16 chunks of 16 bytes
    mv_zero(c, mupad);
    DD_HIP(hipMemcpyAsync(d_mu, mu, (size_t)n_col * sizeof(double), hipMemcpyHostToDevice, c->stream));
    to_internal(c, level, x, n_col, a);
    operator_apply(c, level, a, b, d_mu);
    from_internal(c, level, b, n_col, y);
    DD_HIP(hipStreamSynchronize(c->stream));
    return DDAMG_OK;
  });
}

int ddamg_apply_sap(ddamg_ctx* c, int precision, const double* mu, int n_col, const double* f, double* x) {
  return guarded([&]() -> int {
    DD_CHECK(c && mu && f && x && n_col >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    DD_CHECK(precision != DDAMG_FP16 || sap_takes_f16(c), DDAMG_EINVAL,
             "FP16 right-hand sides need 256-site SAP blocks and SAP variant 2 or 3 (or odd-even SAP)");
    const int prec = precision == DDAMG_FP64 ? P64 : P32;
    MV a = mv_alloc(c, 0, prec, n_col), b = mv_alloc(c, 0, prec, n_col);
    double* d_mu = upload_mu(c, mu, n_col, a.ncol());
    to_internal(c, 0, f, n_col, a);
    if (precision == DDAMG_FP16) {   // the right-hand sides pass through FP16 storage
      MV a16 = mv_like(c, a, P16);
      mv_copy(c, a, a16);
      mv_free(c, a);
      a = a16;
    }
    sap_apply(c, a, b, d_mu, b);
    from_internal(c, 0, b, n_col, x);
    DD_HIP(hipStreamSynchronize(c->stream));
    mv_free(c, a);
    mv_free(c, b);
    c->pool.release(d_mu);
    return DDAMG_OK;
  });
}

static int transfer(ddamg_ctx* c, int level, int precision, int n_col, const double* x, double* y, bool down) {
  DD_CHECK(c && x && y && n_col >= 1, DDAMG_EINVAL, "null pointer or empty batch");
  DD_CHECK(level >= 0 && level + 1 < c->nlev, DDAMG_ESTATE, "no such level transition");
  const int prec = precision == DDAMG_FP64 ? P64 : P32;
  const int from = down ? level : level + 1, to = down ? level + 1 : level;
  MV a = mv_alloc(c, from, prec, n_col), b = mv_alloc(c, to, prec, n_col);
  to_internal(c, from, x, n_col, a);
  if (down) restrict_mv(c, level, a, b);
  else prolong_mv(c, level, a, b, 0);
  from_internal(c, to, b, n_col, y);
  DD_HIP(hipStreamSynchronize(c->stream));
  mv_free(c, a);
  mv_free(c, b);
  return DDAMG_OK;
}

int ddamg_restrict(ddamg_ctx* c, int level, int precision, int n_col, const double* x, double* y) {
  return guarded([&]() -> int { return transfer(c, level, precision, n_col, x, y, true); });
}
int ddamg_prolong(ddamg_ctx* c, int level, int precision, int n_col, const double* x, double* y) {
  return guarded([&]() -> int { return transfer(c, level, precision, n_col, x, y, false); });
}

int ddamg_get_coarse_op(ddamg_ctx* c, int level, double* blocks) {
  return guarded([&]() -> int {
    DD_CHECK(c && blocks, DDAMG_EINVAL, "null pointer");
    DD_CHECK(level >= 1 && level < c->nlev, DDAMG_ESTATE, "no coarse operator on this level");
    const LevelGeom& g = c->geom[level];
    const int d = g.dof;
    std::vector<double> h((size_t)g.V * 9 * d * d * 2);
    DD_HIP(hipMemcpy(h.data(), c->coarse[level].d_blk64, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int a = 0; a < g.V; ++a) {
      const int ca = g.int2can[a];
      for (int slot = 0; slot < 9; ++slot)
        for (int col = 0; col < d; ++col)
          for (int row = 0; row < d; ++row) {
            const double* s = &h[((((size_t)a * 9 + slot) * d + col) * d + row) * 2];
            double* t = blocks + ((((size_t)ca * 9 + slot) * d + row) * d + col) * 2;
            t[0] = s[0];
            t[1] = s[1];
          }
    }
    return DDAMG_OK;
  });
}

int ddamg_get_test_vectors(ddamg_ctx* c, int level, double* tv) {
  return guarded([&]() -> int {
    DD_CHECK(c && tv, DDAMG_EINVAL, "null pointer");
    DD_CHECK(level >= 0 && level + 1 < c->nlev, DDAMG_ESTATE, "no such level transition");
    const LevelGeom& g = c->geom[level];
    const int N = c->tr[level].N;
    std::vector<double> h((size_t)g.V * g.dof * N * 2);
    DD_HIP(hipMemcpy(h.data(), c->tr[level].d_P64, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int s = 0; s < g.V; ++s) {
      const int cs = g.int2can[s];
      for (int k = 0; k < g.dof; ++k)
        for (int j = 0; j < N; ++j) {
          const double* q = &h[(((size_t)s * g.dof + k) * N + j) * 2];
          double* t = tv + (((size_t)j * g.V + cs) * g.dof + k) * 2;
          t[0] = q[0];
          t[1] = q[1];
        }
    }
    return DDAMG_OK;
  });
}

int ddamg_set_test_vectors(ddamg_ctx* c, int level, const double* tv) {
  return guarded([&]() -> int {
    DD_CHECK(c && tv, DDAMG_EINVAL, "null pointer");
    DD_CHECK(level >= 0 && level + 1 < c->nlev, DDAMG_ESTATE, "no such level transition");
    rebuild_from_test_vectors(c, level, tv);
    return DDAMG_OK;
  });
}

// Columns the outer solve keeps in flight: params.max_active_cols, or (0)
// as many as the free device memory holds, at the bytes per column of the
// FGMRES(m) basis, the preconditioned basis, the ping-pong right-hand sides /
// solutions and the smoother's temporaries.
static int active_columns(ddamg_ctx* c, int ncol) {
  if (c->p.max_active_cols > 0) return std::min(ncol, c->p.max_active_cols);
  // fine-level vectors per column, in units of one FP64 vector (ps: size of
  // the preconditioner precision, vs: of the inner basis):
  //   outer FGMRES: b and x ping-pong (4), basis V (m + 1), residual (1), Z (m);
  //   mixed: the FP32 input of the preconditioner and the FP64 copy of z (1 + ps);
  //   inner FGMRES: basis V (mi + 1), Z (mi), residual, and the FP32 forms of
  //   new and FP16-read vectors (up to 3).
  const double col64 = (double)c->geom[0].V * 12 * 16;
  const int m = std::min(c->p.outer_restart, 63);
  const bool mixed = c->p.precision == DDAMG_MIXED;
  const double ps = mixed ? 0.5 : 1.0;
  const int mi = std::min(c->p.inner_iters, 63);
  const bool half = mixed && c->p.inner_fp16;
  const double vs = half ? 0.25 : ps;
  const double per_col = col64 * (6 + m + m * ps + (mixed ? 1 + ps : 0.0) +
                                   (mi > 0 ? (mi + 1) * vs + (mi + 1 + (half ? 2 : 0)) * ps : 0.0));
  // workspaces come in tiles of T columns: count whole tiles, with a 10%
  // margin for the hierarchy's coarse levels and small buffers
  const double per_tile = per_col * c->T;
  size_t fre = 0, tot = 0;
  DD_HIP(hipMemGetInfo(&fre, &tot));
  const int tiles = (int)(0.9 * (double)fre / per_tile);
  DD_CHECK(tiles >= 1, DDAMG_ENOMEM,
           "device memory holds less than one tile of Krylov workspace: lower outer_restart / inner_iters");
  return std::min(ncol, tiles * c->T);
}

// Solve the columns (shift hmu[i], right-hand side b[rhs_of[i]]) together.
static int solve_columns(ddamg_ctx* c, const std::vector<double>& hmu, const std::vector<int>& rhs_of,
                         const double* b, double* x, int use_x0, ddamg_col_info* info,
                         const std::vector<double>* eps = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  c->st.middle_calls = c->st.middle_iters = c->st.bottom_calls = c->st.bottom_iters = 0;
  c->st.fine_ops = c->st.sap_calls = 0;
  c->st.learned_fallbacks = 0;
  c->st.col_removals = 0;
  c->st.inner_iters = 0;
  c->st.fp16_restores = 0;
  c->sap_ev_used = 0;
  c->sap_ev_tiles.clear();
  const int ncol = (int)hmu.size();
  for (double m : hmu) DD_CHECK(std::isfinite(m), DDAMG_EINVAL, "twisted mass is NaN/Inf");
  // NaN guard on the right-hand sides (canonical, one field per distinct rhs)
  int nb = 0;
  for (int r : rhs_of) nb = std::max(nb, r + 1);
  {
    MV Bc = mv_alloc(c, 0, P64, nb);
    to_internal(c, 0, b, nb, Bc);
    double* d_n2 = (double*)c->pool.alloc(Bc.ncol() * sizeof(double));
    mv_norm2(c, Bc, d_n2);
    std::vector<double> bn(Bc.ncol());
    copy_to_host(c, d_n2, bn.data(), bn.size() * sizeof(double));
    c->pool.release(d_n2);
    mv_free(c, Bc);
    for (int i = 0; i < nb; ++i) DD_CHECK(std::isfinite(bn[i]), DDAMG_EINVAL, "right-hand side contains NaN/Inf");
  }
  OuterJob job;
  job.ncol = ncol;
  job.mu = hmu;
  job.rhs_of = rhs_of;
  job.b = b;
  job.x = x;
  job.use_x0 = use_x0 != 0;
  if (eps) job.eps = *eps;
  job.max_active = active_columns(c, ncol);
  outer_solve(c, job);
  DD_HIP(hipStreamSynchronize(c->stream));
  c->st.outer_iters = job.total;
  int status = DDAMG_OK;
  for (int i = 0; i < ncol; ++i) {
    if (!job.converged[i]) status = DDAMG_NOT_CONVERGED;
    if (info) {
      info[i].outer_iters = job.iters[i];
      info[i].converged = job.converged[i];
      info[i].true_rel_res = job.relres[i];
      info[i].err_vs_fp64 = job.err[i];
      info[i].fallbacks = job.fallbacks[i];
    }
  }
  c->st.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  sap_timing_collect(c);
  return status;
}

int ddamg_solve(ddamg_ctx* c, const double* mu, int n_shift, const double* b, int n_rhs, double* x, int use_x0,
                ddamg_col_info* info) {
  return guarded([&]() -> int {
    DD_CHECK(c && mu && b && x && n_shift >= 1 && n_rhs >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    const int ncol = n_rhs * n_shift;
    std::vector<double> hmu(ncol);
    std::vector<int> rhs_of(ncol);
    for (int r = 0; r < n_rhs; ++r)
      for (int k = 0; k < n_shift; ++k) {
        hmu[r * n_shift + k] = mu[k];
        rhs_of[r * n_shift + k] = r;
      }
    return solve_columns(c, hmu, rhs_of, b, x, use_x0, info);
  });
}

int ddamg_solve_batch(ddamg_ctx* c, int n_sys, const int* n_rhs, const int* n_shift, const double* mu,
                      const double* b, double* x, int use_x0, ddamg_col_info* info) {
  return guarded([&]() -> int {
    DD_CHECK(c && n_rhs && n_shift && mu && b && x && n_sys >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    std::vector<double> hmu;
    std::vector<int> rhs_of;
    int r0 = 0, k0 = 0;
    for (int s = 0; s < n_sys; ++s) {
      DD_CHECK(n_rhs[s] >= 1 && n_shift[s] >= 1, DDAMG_EINVAL, "every system needs a rhs and a shift");
      for (int r = 0; r < n_rhs[s]; ++r)
        for (int k = 0; k < n_shift[s]; ++k) {
          hmu.push_back(mu[k0 + k]);
          rhs_of.push_back(r0 + r);
        }
      r0 += n_rhs[s];
      k0 += n_shift[s];
    }
    return solve_columns(c, hmu, rhs_of, b, x, use_x0, info);
  });
}

int ddamg_solve_nd(ddamg_ctx* c, const double* mubar, const double* epsbar, int n_pair, const double* b, double* x,
                   int use_x0, ddamg_col_info* info) {
  return guarded([&]() -> int {
    DD_CHECK(c && mubar && epsbar && b && x && n_pair >= 1, DDAMG_EINVAL, "null pointer or empty batch");
    const int ncol = 2 * n_pair;
    std::vector<double> hmu(ncol), eps(ncol);
    std::vector<int> rhs_of(ncol);
    for (int i = 0; i < n_pair; ++i) {
      DD_CHECK(std::isfinite(mubar[i]) && std::isfinite(epsbar[i]), DDAMG_EINVAL, "mubar / epsbar contain NaN/Inf");
      hmu[2 * i] = mubar[i];
      hmu[2 * i + 1] = -mubar[i];
      eps[2 * i] = eps[2 * i + 1] = epsbar[i];
      rhs_of[2 * i] = 2 * i;
      rhs_of[2 * i + 1] = 2 * i + 1;
    }
    return solve_columns(c, hmu, rhs_of, b, x, use_x0, info, &eps);
  });
}

int ddamg_coarse_solve(ddamg_ctx* c, int level, int precision, int block, const double* mu, int n_col,
                       const double* b, double* x, double tol, int maxit, int* iters) {
  return guarded([&]() -> int {
    DD_CHECK(c && mu && b && x && n_col >= 1 && maxit >= 1 && tol > 0, DDAMG_EINVAL, "bad arguments");
    DD_CHECK(level >= 1 && level < c->nlev, DDAMG_ESTATE, "no such coarse level");
    DD_CHECK(precision == DDAMG_FP64 || precision == DDAMG_FP32, DDAMG_EINVAL, "precision");
    const int prec = precision == DDAMG_FP64 ? P64 : P32;
    MV b64 = mv_alloc(c, level, P64, n_col);
    to_internal(c, level, b, n_col, b64);
    MV B = prec == P64 ? b64 : mv_like(c, b64, P32);
    if (prec != P64) mv_copy(c, b64, B);
    MV X = mv_alloc(c, level, prec, n_col);
    double* d_mu = upload_mu(c, mu, n_col, B.ncol());
    const int m = std::min(maxit, 63);
    std::vector<int> it;
    if (block) {
      block_gmres(c, level, d_mu, B, X, true, tol, m, maxit, &it, nullptr, nullptr);
    } else if (c->p.bottom_dr_k > 0) {   // GMRES-DR(bottom_restart, bottom_dr_k)
      level_gmres_dr(c, level, d_mu, B, X, tol, c->p.bottom_restart > 0 ? c->p.bottom_restart : m, c->p.bottom_dr_k,
                     maxit, &it);
    } else {
      level_gmres(c, level, d_mu, B, X, tol, m, maxit, &it, nullptr, nullptr);
    }
    MV x64 = prec == P64 ? X : mv_like(c, X, P64);
    if (prec != P64) mv_copy(c, X, x64);
    from_internal(c, level, x64, n_col, x);
    DD_HIP(hipStreamSynchronize(c->stream));
    if (iters)
      for (int i = 0; i < n_col; ++i) iters[i] = it[i];
    if (prec != P64) {
      mv_free(c, B);
      mv_free(c, x64);
    }
    mv_free(c, b64);
    mv_free(c, X);
    c->pool.release(d_mu);
    return DDAMG_OK;
  });
}

int ddamg_get_stats(ddamg_ctx* c, ddamg_stats* s) {
  return guarded([&]() -> int {
    DD_CHECK(c && s, DDAMG_EINVAL, "null pointer");
    std::memset(s, 0, sizeof(*s));
    s->setup_seconds = c->st.setup_seconds;
    s->solve_seconds = c->st.solve_seconds;
    s->outer_iters = c->st.outer_iters;
    s->n_middle_solves = c->st.middle_calls;
    s->n_bottom_solves = c->st.bottom_calls;
    s->avg_middle_iters = c->st.middle_calls ? (double)c->st.middle_iters / c->st.middle_calls : 0.0;
    s->avg_bottom_iters = c->st.bottom_calls ? (double)c->st.bottom_iters / c->st.bottom_calls : 0.0;
    s->n_fine_ops = c->st.fine_ops;
    s->n_sap_calls = c->st.sap_calls;
    s->learned_fallbacks = c->st.learned_fallbacks;
    s->col_removals = c->st.col_removals;
    s->n_inner_iters = c->st.inner_iters;
    s->n_fp16_restores = c->st.fp16_restores;
    s->sap_kernel_ms = c->st.sap_kernel_ms;
    s->n_sap_kernels = c->st.sap_kernel_launches;
    s->n_sap_kernel_tiles = c->st.sap_kernel_tiles;
    s->device_bytes = (long long)c->pool.held;
    s->device_bytes_peak = (long long)c->pool.peak;
    return DDAMG_OK;
  });
}

// Time `n_iter` back-to-back launches of one operator on resident internal
// vectors with HIP events on the context's stream (the stream the kernels are
// launched on).  op: 0 = fine stencil, 1 = SAP smoother, 2 = coarse stencil of
// `level`, 3 = restriction from `level`, 4 = prolongation to `level`.
// Returns the mean seconds per launch in *sec.
int ddamg_time_op(ddamg_ctx* c, int op, int level, int precision, int n_col, int n_iter, double* sec) {
  return guarded([&]() -> int {
    DD_CHECK(c && sec && n_col >= 1 && n_iter >= 1, DDAMG_EINVAL, "bad arguments");
    DD_CHECK(level >= 0 && level < c->nlev, DDAMG_ESTATE, "level not built");
    const int prec = precision == DDAMG_FP64 ? P64 : P32;
    const int lin = (op == 4) ? level + 1 : level;
    const int lout = (op == 3) ? level + 1 : level;
    DD_CHECK(!(op == 3 || op == 4) || level + 1 < c->nlev, DDAMG_ESTATE, "no such transition");
    DD_CHECK(!(op == 2) || level >= 1, DDAMG_EINVAL, "coarse stencil needs level >= 1");
    DD_CHECK(op >= 0 && op <= 6, DDAMG_EINVAL, "unknown op");
    DD_CHECK(op != 6 || (prec == P32 && level == 0 && sap_takes_f16(c)), DDAMG_EINVAL,
             "the FP16-input smoother needs FP32, level 0, 256-site SAP blocks and SAP variant 2 or 3 (or odd-even SAP)");
    MV a64 = mv_alloc(c, lin, P64, n_col);
    random_fill(c, lin, a64, a64.ncol(), 99);
    MV a = (prec == P64) ? a64 : mv_like(c, a64, P32);
    if (prec != P64) mv_copy(c, a64, a);
    if (op == 6) {  // FP64 -> FP32 -> scaled FP16
      MV a16 = mv_like(c, a64, P16);
      mv_copy(c, a, a16);
      mv_free(c, a);
      a = a16;
    }
    MV b = mv_alloc(c, lout, prec, n_col);
    std::vector<double> hm(a.ncol(), 0.01);
    double* d_mu = upload_mu(c, hm.data(), a.ncol(), a.ncol());
    auto run = [&]() {
      switch (op) {
        case 0: fine_dslash(c, a, b, d_mu); break;
        case 1:
        case 6: sap_apply(c, a, b, d_mu, b); break;
        case 2: coarse_apply(c, level, a, b, d_mu); break;
        case 3: restrict_mv(c, level, a, b); break;
        case 4: prolong_mv(c, level, a, b, 0); break;
        default: mv_copy_kernel(c, a, b); break;
      }
    };
    run();
    DD_HIP(hipStreamSynchronize(c->stream));
    hipEvent_t e0, e1;
    DD_HIP(hipEventCreate(&e0));
    DD_HIP(hipEventCreate(&e1));
    DD_HIP(hipEventRecord(e0, c->stream));
    for (int i = 0; i < n_iter; ++i) run();
    DD_HIP(hipEventRecord(e1, c->stream));
    DD_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DD_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *sec = (double)ms * 1e-3 / n_iter;
    if (prec != P64) mv_free(c, a);
    mv_free(c, a64);
    mv_free(c, b);
    c->pool.release(d_mu);
    return DDAMG_OK;
  });
}

static int* knob_slot(ddamg_ctx* c, int knob) {
  switch (knob) {
    case DDAMG_KNOB_DSLASH_SITES_FP64: return &c->dslash_rs[P64];
    case DDAMG_KNOB_DSLASH_SITES_FP32: return &c->dslash_rs[P32];
    case DDAMG_KNOB_FP32_LINKS: return &c->fp32_links;
    case DDAMG_KNOB_COARSE_MFMA: return &c->coarse_mfma;
    case DDAMG_KNOB_SAP_VARIANT: return &c->sap_variant;
    case DDAMG_KNOB_DSLASH_ORDER: return &c->dslash_order;
    case DDAMG_KNOB_WALK_SEGMENTS: return &c->walk_seg;
    case DDAMG_KNOB_FP16_RESCALE: return &c->fp16_rescale;
    case DDAMG_KNOB_TIME_SAP: return &c->time_sap;
    case DDAMG_KNOB_GRAM_ONE_REDUCTION: return &c->gram_lowsync;
    default: throw Error{DDAMG_EINVAL, "unknown knob"};
  }
}

static bool knob_valid(int knob, int value) {
  switch (knob) {
    case DDAMG_KNOB_DSLASH_SITES_FP64: return dslash_rs_valid(P64, value);
    case DDAMG_KNOB_DSLASH_SITES_FP32: return dslash_rs_valid(P32, value);
    case DDAMG_KNOB_FP32_LINKS: return value == 0 || value == 1;
    case DDAMG_KNOB_COARSE_MFMA: return value == 0 || value == 1;
    case DDAMG_KNOB_SAP_VARIANT: return value >= 0 && value <= 3;
    case DDAMG_KNOB_DSLASH_ORDER: return value >= 0 && value <= 3;
    case DDAMG_KNOB_WALK_SEGMENTS: return value == 1 || value == 2 || value == 4 || value == 8;
    case DDAMG_KNOB_FP16_RESCALE: return value >= 1 && value <= 1024;
    case DDAMG_KNOB_TIME_SAP: return value >= 0 && value <= 5;
    case DDAMG_KNOB_GRAM_ONE_REDUCTION: return value >= 0 && value <= 2;
    default: return false;
  }
}

int ddamg_set_tuning(ddamg_ctx* c, int knob, int value) {
  return guarded([&]() -> int {
    DD_CHECK(c, DDAMG_EINVAL, "null context");
    int* slot = knob_slot(c, knob);
    DD_CHECK(knob_valid(knob, value), DDAMG_EINVAL, "inadmissible knob value");
    *slot = value;
    return DDAMG_OK;
  });
}

int ddamg_get_tuning(ddamg_ctx* c, int knob, int* value) {
  return guarded([&]() -> int {
    DD_CHECK(c && value, DDAMG_EINVAL, "null pointer");
    *value = *knob_slot(c, knob);
    return DDAMG_OK;
  });
}

int ddamg_autotune(ddamg_ctx* c, int n_col, int* values) {
  return guarded([&]() -> int {
    DD_CHECK(c && n_col >= 1, DDAMG_EINVAL, "bad arguments");
    // Stencil scheme (LDS-staged site ranges in storage or time-slice order,
    // or the t-walk with 4 / 8 columns and 1..8 t segments) x FP64 sites per
    // workgroup x FP32 (link storage, sites per workgroup); the scheme is
    // shared by both precisions, so it is chosen on the sum of their best times.
    {
      std::vector<std::pair<int, int>> schemes = {{0, c->walk_seg}, {1, c->walk_seg}};
      if (c->geom[0].gsize == 256 && c->d_walk_blk)
        for (int ord : {2, 3})
          for (int seg : {1, 2, 4, 8})
            if (c->geom[0].dims[3] % seg == 0) schemes.push_back({ord, seg});
      double best_all = 1e30;
      int bo = c->dslash_order, bseg = c->walk_seg, b64 = c->dslash_rs[P64], bl = c->fp32_links,
          b32 = c->dslash_rs[P32];
      for (auto [ord, seg] : schemes) {
        c->dslash_order = ord;
        c->walk_seg = seg;
        const bool walk = ord >= 2;
        double best64 = 1e30, best32 = 1e30;
        int v64 = b64, l32 = bl, v32 = b32;
        for (int v : {16, 32, 64}) {
          if (walk && v != 16) break;       // sites per workgroup do not apply to the t-walk
          c->dslash_rs[P64] = walk ? b64 : v;
          double sec = 0;
          const int st = ddamg_time_op(c, 0, 0, DDAMG_FP64, n_col, 10, &sec);
          if (st != DDAMG_OK) return st;
          if (sec < best64) { best64 = sec; v64 = c->dslash_rs[P64]; }
        }
        for (int lk : {0, 1})
          for (int v : {32, 64, 128}) {
            if (walk && v != 32) break;
            c->fp32_links = lk;
            c->dslash_rs[P32] = walk ? b32 : v;
            double sec = 0;
            const int st = ddamg_time_op(c, 0, 0, DDAMG_FP32, n_col, 10, &sec);
            if (st != DDAMG_OK) return st;
            if (sec < best32) { best32 = sec; l32 = lk; v32 = c->dslash_rs[P32]; }
          }
        if (best64 + best32 < best_all) {
          best_all = best64 + best32;
          bo = ord;
          bseg = seg;
          b64 = v64;
          bl = l32;
          b32 = v32;
        }
      }
      c->dslash_order = bo;
      c->walk_seg = bseg;
      c->dslash_rs[P64] = b64;
      c->fp32_links = bl;
      c->dslash_rs[P32] = b32;
    }
    // FP32 SAP on 4^4 blocks: columns per workgroup x links in LDS or through the caches
    if (c->geom[0].gsize == 256) {
      double best = 1e30;
      int bv = c->sap_variant;
      for (int v : {0, 1, 2, 3}) {
        c->sap_variant = v;
        double sec = 0;
        const int st = ddamg_time_op(c, 1, 0, DDAMG_FP32, n_col, 4, &sec);
        if (st != DDAMG_OK) return st;
        if (sec < best) { best = sec; bv = v; }
      }
      c->sap_variant = bv;
    }
    // the timing runs sized the Krylov and smoother workspaces for n_col
    // columns at once; a solve that holds fewer columns in flight (large
    // lattices) sizes its own
    DD_HIP(hipStreamSynchronize(c->stream));
    free_work(c);
    c->pool.trim();
    if (values)
      for (int k = 0; k < DDAMG_N_KNOBS; ++k) values[k] = *knob_slot(c, k);
    return DDAMG_OK;
  });
}

// ---------------------------------------------------------- learned smoother ---
int ddamg_smoother_set_weights(ddamg_ctx* c, const double* w1, const double* w2) {
  return guarded([&]() -> int {
    DD_CHECK(c && w1 && w2, DDAMG_EINVAL, "null pointer");
    ptc_set_weights(c, w1, w2);
    return DDAMG_OK;
  });
}

int ddamg_smoother_get_weights(ddamg_ctx* c, double* w1, double* w2) {
  return guarded([&]() -> int {
    DD_CHECK(c && w1 && w2, DDAMG_EINVAL, "null pointer");
    ptc_get_weights(c, w1, w2);
    return DDAMG_OK;
  });
}

static const char kPtcMagic[8] = {'D', 'D', 'A', 'M', 'G', 'P', 'T', 'C'};
constexpr int kPtcVersion = 1;
constexpr size_t kPtcW = 9 * 2 * 1 * 4 * 4 * 2;   // reals per layer

int ddamg_load_smoother(ddamg_ctx* c, const char* path) {
  return guarded([&]() -> int {
    DD_CHECK(c && path, DDAMG_EINVAL, "null pointer");
    FILE* f = std::fopen(path, "rb");
    DD_CHECK(f, DDAMG_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t version = 0;
    std::vector<double> w1(kPtcW), w2(kPtcW);
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&version, sizeof version, 1, f) == 1 &&
                    std::fread(w1.data(), sizeof(double), kPtcW, f) == kPtcW &&
                    std::fread(w2.data(), sizeof(double), kPtcW, f) == kPtcW;
    const bool extra = ok && std::fgetc(f) != EOF;
    std::fclose(f);
    DD_CHECK(ok, DDAMG_EINVAL, std::string("short smoother file ") + path);
    DD_CHECK(std::memcmp(magic, kPtcMagic, 8) == 0, DDAMG_EINVAL, std::string("not a smoother file: ") + path);
    DD_CHECK(version == kPtcVersion, DDAMG_EINVAL, "unsupported smoother file version");
    DD_CHECK(!extra, DDAMG_EINVAL, std::string("trailing bytes in smoother file ") + path);
    for (double v : w1) DD_CHECK(std::isfinite(v), DDAMG_EINVAL, "smoother weights contain NaN/Inf");
    for (double v : w2) DD_CHECK(std::isfinite(v), DDAMG_EINVAL, "smoother weights contain NaN/Inf");
    ptc_set_weights(c, w1.data(), w2.data());
    return DDAMG_OK;
  });
}

int ddamg_save_smoother(ddamg_ctx* c, const char* path) {
  return guarded([&]() -> int {
    DD_CHECK(c && path, DDAMG_EINVAL, "null pointer");
    DD_CHECK(ptc_ready(c), DDAMG_ESTATE, "smoother weights not set");
    std::vector<double> w1(kPtcW), w2(kPtcW);
    ptc_get_weights(c, w1.data(), w2.data());
    FILE* f = std::fopen(path, "wb");
    DD_CHECK(f, DDAMG_EINVAL, std::string("cannot create ") + path);
    const int32_t version = kPtcVersion;
    const bool ok = std::fwrite(kPtcMagic, 1, 8, f) == 8 && std::fwrite(&version, sizeof version, 1, f) == 1 &&
                    std::fwrite(w1.data(), sizeof(double), kPtcW, f) == kPtcW &&
                    std::fwrite(w2.data(), sizeof(double), kPtcW, f) == kPtcW;
    const bool closed = std::fclose(f) == 0;
    DD_CHECK(ok && closed, DDAMG_EINVAL, std::string("cannot write ") + path);
    return DDAMG_OK;
  });
}

int ddamg_smoother_apply(ddamg_ctx* c, int n_col, const double* x, double* y) {
  return guarded([&]() -> int {
    DD_CHECK(c && x && y && n_col >= 1, DDAMG_EINVAL, "bad arguments");
    DD_CHECK(ptc_ready(c), DDAMG_ESTATE, "smoother weights not set");
    MV a = mv_alloc(c, 0, P32, n_col), b = mv_alloc(c, 0, P32, n_col);
    to_internal(c, 0, x, n_col, a);
    ptc_apply(c, a, b);
    from_internal(c, 0, b, n_col, y);
    DD_HIP(hipStreamSynchronize(c->stream));
    mv_free(c, a);
    mv_free(c, b);
    return DDAMG_OK;
  });
}

static const int PTC_CIN[2] = {1, 2}, PTC_COUT[2] = {2, 1};

int ddamg_ptc_layer(ddamg_ctx* c, int layer, int adjoint, int n_col, const double* in, double* out) {
  return guarded([&]() -> int {
    DD_CHECK(c && in && out && n_col >= 1 && (layer == 1 || layer == 2), DDAMG_EINVAL, "bad arguments");
    const int l = layer - 1;
    const int cin = adjoint ? PTC_COUT[l] : PTC_CIN[l], cout = adjoint ? PTC_CIN[l] : PTC_COUT[l];
    const size_t chan = (size_t)n_col * c->geom[0].V * 12 * 2;
    MV a[2], b[2];
    for (int i = 0; i < cin; ++i) {
      a[i] = mv_alloc(c, 0, P32, n_col);
      to_internal(c, 0, in + i * chan, n_col, a[i]);
    }
    for (int o = 0; o < cout; ++o) b[o] = mv_alloc(c, 0, P32, n_col);
    ptc_layer(c, l, adjoint != 0, a, b);
    for (int o = 0; o < cout; ++o) from_internal(c, 0, b[o], n_col, out + o * chan);
    DD_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < cin; ++i) mv_free(c, a[i]);
    for (int o = 0; o < cout; ++o) mv_free(c, b[o]);
    return DDAMG_OK;
  });
}

int ddamg_ptc_weight_grad(ddamg_ctx* c, int layer, int n_col, const double* in, const double* gout, double* g) {
  return guarded([&]() -> int {
    DD_CHECK(c && in && gout && g && n_col >= 1 && (layer == 1 || layer == 2), DDAMG_EINVAL, "bad arguments");
    const int l = layer - 1;
    const int cin = PTC_CIN[l], cout = PTC_COUT[l];
    const size_t chan = (size_t)n_col * c->geom[0].V * 12 * 2;
    MV a[2], b[2];
    for (int i = 0; i < cin; ++i) {
      a[i] = mv_alloc(c, 0, P32, n_col);
      to_internal(c, 0, in + i * chan, n_col, a[i]);
    }
    for (int o = 0; o < 2; ++o) {
      b[o] = mv_alloc(c, 0, P32, n_col);
      if (o < cout) to_internal(c, 0, gout + o * chan, n_col, b[o]);
    }
    ptc_wgrad(c, l, a, b, g);
    for (int i = 0; i < cin; ++i) mv_free(c, a[i]);
    for (int o = 0; o < 2; ++o) mv_free(c, b[o]);
    return DDAMG_OK;
  });
}

int ddamg_train_smoother(ddamg_ctx* c, const double* mus, int n_mu, int steps, int batch, double lr, int sap_sweeps,
                         uint64_t seed, double* loss_history) {
  return guarded([&]() -> int {
    DD_CHECK(c && mus && n_mu >= 1 && steps >= 1 && batch >= 1 && lr > 0 && sap_sweeps >= 0, DDAMG_EINVAL,
             "bad arguments");
    ptc_train(c, mus, n_mu, steps, batch, lr, sap_sweeps, seed, loss_history);
    return DDAMG_OK;
  });
}

}  // extern "C"
