// Internal declarations of the gfx950 multigrid library.
//
// Internal vector layout ("column-tiled SoA"): a multivector of n columns on a
// lattice level with `dof` complex components per site is stored as
//     [tile][chunk][site][T][RW]
// with T columns per tile, RW reals per 16-byte lane chunk (2 for FP64 = one
// complex, 4 for FP32 = two complexes) and nchunk = 2*dof/RW chunks per site.
// A wavefront lane handles one (site, column); a row of T lanes of one site
// reads T*16 contiguous bytes, consecutive sites are contiguous, and a link
// or coarse block loaded once serves all T columns of the tile.  This is the
// GPU form of the paper's vector bundle with the vector index running fastest
// (section 3, Fig. 2 right), chunked by the tile width as the paper chunks by
// num_loop.
//
// Sites are stored in block-major order: the lattice is cut into the blocks
// of the level's grouping (SAP blocks = first-level aggregates on the fine
// level, the next aggregates on a coarse level), blocks in lexicographic
// order, sites lexicographic inside a block.  SAP blocks, aggregates and
// restriction/prolongation therefore touch contiguous site ranges.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/ddamg.h"

namespace ddamg {

struct Error {
  int code;
  std::string msg;
};

#define DD_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::ddamg::Error{e_ == hipErrorOutOfMemory ? DDAMG_ENOMEM : DDAMG_EDEVICE,  \
                           std::string(#call) + ": " + hipGetErrorString(e_)};        \
  } while (0)

#define DD_CHECK(cond, code, msg)                        \
  do {                                                   \
    if (!(cond)) throw ::ddamg::Error{(code), (msg)};    \
  } while (0)

// P16: FP16 storage in the FP32 layout (two complexes per chunk, 8-byte
// chunks), used for Krylov bases only; a P16 multivector stores v * hscale.
enum Prec { P64 = 0, P32 = 1, P16 = 2 };

inline int reals_per_chunk(int prec) { return prec == P64 ? 2 : 4; }
inline size_t real_size(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// One multivector in the column-tiled layout.
struct MV {
  void* p = nullptr;
  int prec = P64;
  int ntiles = 0;
  int T = 8;
  int nchunk = 0;   // 2*dof / RW
  int nsites = 0;
  int dof = 0;      // complex components per site
  bool owned = false;
  double hscale = 1.0;   // P16: stored value = value * hscale

  int ncol() const { return ntiles * T; }
  size_t tile_reals() const { return (size_t)nchunk * nsites * T * reals_per_chunk(prec); }
  size_t reals() const { return tile_reals() * ntiles; }
  size_t bytes() const { return reals() * real_size(prec); }
  template <typename R> R* as() const { return static_cast<R*>(p); }
  // view of tiles [t0, t0+nt)
  MV tiles(int t0, int nt) const {
    MV v = *this;
    v.p = (char*)p + (size_t)t0 * tile_reals() * real_size(prec);
    v.ntiles = nt;
    v.owned = false;
    return v;
  }
};

// Geometry of one lattice level in the internal ordering.
struct LevelGeom {
  int dims[4] = {0, 0, 0, 0};
  int V = 0;
  int dof = 0;
  int grp[4] = {1, 1, 1, 1};   // grouping block of the internal order
  int gsize = 1;
  std::vector<int> int2can, can2int;   // host permutations
  int* d_nbr = nullptr;                // [8][V]; fine level: bit 31 = boundary sign
  int* d_int2can = nullptr;            // [V]
  int* d_can2int = nullptr;            // [V]
  std::vector<int> blk_num, blk_lex;   // lexicographic block index <-> block number (Morton rank)
  int* d_coarse_of_blk = nullptr;      // [V/gsize] internal site on the next level of each block
  int* d_blk_of_coarse = nullptr;      // [V] block number on the previous level (coarse levels)
};

// Transfer between level l and l+1.
struct Transfer {
  int N = 0;                 // test vectors; coarse dof = 2N
  double* d_P64 = nullptr;   // [V_l][dof_l][N] complex, orthonormal per (aggregate, chirality)
  float* d_P32 = nullptr;
  // level 0 with transfer_fp16: P in FP16, [k/2][2 rows x N/4 chunks][V] chunks of
  // 4 complexes (16 bytes): consecutive sites contiguous for each (row pair, chunk)
  void* d_P16T = nullptr;
};

struct Coarse {
  double* d_blk64 = nullptr;  // [V][9][d col][d row] complex (column-major blocks)
  float* d_blk32 = nullptr;
  void* d_blk16 = nullptr;    // BF16 blocks in the MFMA operand layout (d % 16 == 0)
  double mu_factor = 1.0;
  int g5out = 0;              // 1: the stencil applies gamma5_c D_c(mu) (Hermitian form + i dmu mu)
};

// Device allocation pool.  Released buffers are kept for reuse by a later
// request of about the same size (the workspaces of one solve serve the next
// one: a fresh hipMalloc of a multi-GB buffer costs hundreds of ms).  A
// reused buffer may still be read by work queued before its release, so
// reuse first waits for `stream`.  When hipMalloc runs out of memory the
// cached buffers are freed and the request is tried once more.
struct DevPool {
  std::vector<std::pair<void*, size_t>> blocks;   // live
  std::multimap<size_t, void*> cache;             // released, kept
  size_t cached_bytes = 0;
  size_t held = 0, peak = 0;                      // bytes in use or cached, and their maximum
  hipStream_t stream = nullptr;
  void* alloc(size_t bytes);
  void release(void* p);
  void trim();    // free every cached buffer
  void clear();   // free everything
};

struct Stats {
  double setup_seconds = 0, solve_seconds = 0;
  int outer_iters = 0;
  long long middle_calls = 0, middle_iters = 0, bottom_calls = 0, bottom_iters = 0;
  long long fine_ops = 0, sap_calls = 0;
  int learned_fallbacks = 0;
  int col_removals = 0;
  long long inner_iters = 0;
  long long fp16_restores = 0;
  long long orth_fallbacks = 0;      // aggregate groups orthonormalised by Gram-Schmidt (setup)
  double sap_kernel_ms = 0;          // HIP-event time of the SAP kernels (when timed)
  long long sap_kernel_launches = 0, sap_kernel_tiles = 0;
};

}  // namespace ddamg

struct ddamg_ctx {
  ddamg_params p;
  hipStream_t stream = nullptr;
  int device = 0;                     // device current at setup
  const double* nd_eps = nullptr;     // set while the fine operator is the doublet operator: epsbar per column
  void* noalloc_scratch = nullptr;    // that device's address of the no-allocation scratch array
  hipStream_t cap_stream = nullptr;   // private stream for graph capture (default priority)
  int T = 8;
  int nlev = 1;
  double m0 = 0, diag = 0;
  ddamg::LevelGeom geom[3];
  ddamg::Transfer tr[2];
  ddamg::Coarse coarse[3];
  double* d_U64 = nullptr;    // [4 mu][9 chunk][V] double2
  float* d_U32 = nullptr;     // [4 mu][3 chunk][V] float4, rows 0 and 1 (no boundary sign)
  float* d_U32f = nullptr;    // [4 mu][5 chunk][V] float4, full links, boundary sign folded in
  double* d_clov64 = nullptr; // clover site term (c_sw != 0): [36 chunk][V] double2, two packed 6x6 blocks
  float* d_clov32 = nullptr;  // the same in FP32: [18 chunk][V] float4
  int* d_sap_list[2] = {nullptr, nullptr};   // block ids of each colour
  int n_sap[2] = {0, 0};
  double* d_scratch = nullptr;  // reduction partials
  size_t scratch_bytes = 0;
  double* d_small = nullptr;    // small temporary results
  int small_n = 0;
  double* h_pinned = nullptr;   // pinned host staging of small results
  size_t pinned_bytes = 0;
  ddamg::DevPool pool;
  ddamg::Stats st;
  void* work = nullptr;         // solver workspaces (solve.hip)
  void* ptc = nullptr;          // learned smoother state (ptc.hip)
  void* bwork = nullptr;        // block GMRES workspaces (block.hip)
  ddamg::MV tvk[2];             // smoothed (not orthonormalised) test vectors of each transition
  int dslash_rs[2] = {32, 32};  // fine stencil sites per workgroup, per precision (autotuned)
  int fp32_links = 0;           // FP32 fine stencil links: 0 = full 3x3, 1 = 2-row compressed
  int coarse_mfma = 1;          // FP32 coarse stencil on BF16 MFMA (d % 16 == 0)
  int dslash_order = 0;         // fine stencil scheme: 0 storage order, 1 time-slice order, 2/3 t-walk (4/8 columns)
  int* d_walk_blk = nullptr;    // [xyz block column][t block] block numbers (4^4 site blocks)
  int walk_seg = 2;             // t-walk stencil: segments of the t direction (one workgroup each)
  int fp16_rescale = 4;         // FP16 Arnoldi basis: bound on the entry scales of the stored vectors
  int time_sap = 0;             // kernel class timed with HIP events at every launch of a solve (0 off)
  int gram_lowsync = 1;         // Arnoldi steps with one reduction (DDAMG_KNOB_GRAM_ONE_REDUCTION)
  std::vector<hipEvent_t> sap_ev;   // event pool, (start, stop) pairs, reused by every solve
  std::vector<int> sap_ev_tiles;    // column tiles of each timed launch
  size_t sap_ev_used = 0;
  int* d_dslash_order[4] = {nullptr, nullptr, nullptr, nullptr};   // per sites-per-workgroup 16..128
  int sap_variant = 0;          // FP32 SAP on 4^4 blocks: 0 = 2 columns/WG, links in LDS; 1 = 2 columns, links
                                // through L1/L2; 2 = 1 column/WG, 2-row links through L1/L2; 3 = 1 column/WG,
                                // full links through L1/L2
};

namespace ddamg {

// ---- multivector management (blas.hip) ----
MV mv_alloc(ddamg_ctx* c, int level, int prec, int ncol_min);
MV mv_like(ddamg_ctx* c, const MV& a, int prec);
void mv_free(ddamg_ctx* c, MV& a);
void mv_zero(ddamg_ctx* c, const MV& a);
void mv_copy(ddamg_ctx* c, const MV& src, const MV& dst);          // any precisions
void mv_axpy(ddamg_ctx* c, const double* d_alpha, const MV& x, const MV& y, int sign);  // y += sign*alpha_c x_c
void mv_xpay(ddamg_ctx* c, const MV& x, const double* d_alpha, const MV& y);  // y = x + alpha_c y
void mv_scale(ddamg_ctx* c, const double* d_alpha, const MV& x);  // x *= alpha_c (complex)
void mv_sub(ddamg_ctx* c, const MV& a, const MV& b, const MV& out);   // out = a - b
void mv_add(ddamg_ctx* c, const MV& x, const MV& y);                  // y += x
void mv_gamma5(ddamg_ctx* c, const MV& x);                            // x <- gamma5 x (in place)
void mv_copy_kernel(ddamg_ctx* c, const MV& s, const MV& d);          // plain copy kernel
void mv_gather_cols(ddamg_ctx* c, const MV& full, const MV& comp, const int* d_map, int dir);
// per-column complex dots <V_j, w> for j < k, written to d_out[j*ncol + c] (complex)
void mv_multidot(ddamg_ctx* c, const MV* Vs, int k, const MV& w, double* d_out);
// w -= sum_j coef[j*ncol+c] V_j   (coef complex, device)
void mv_multiaxpy(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign);
void mv_norm2(ddamg_ctx* c, const MV& a, double* d_out);          // per column, real
// mv_multiaxpy followed by mv_norm2 of w, fused into one pass where possible
void mv_multiaxpy_norm2(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign,
                        double* d_n2);
// the same for an unnormalised FP16 basis, writing the result into an FP16 vector
void mv_multiaxpy_norm2_into_f16(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const double* d_cinv2,
                                 const MV& w, const MV& out, const double* d_osc, double* d_n2);
// variants on caller-owned buffers (no context scratch: safe to capture in a graph)
size_t multidot_partials(const MV& w, int k);
void mv_multidot_buf(ddamg_ctx* c, const MV* Vs, int k, const MV& w, double* d_out, double* part);
// w <- (w + sign * sum_j coef_j V_j) * osc[col] and d_n2[col] = |result|^2 in
// one pass (same-precision FP32 or FP64 bases); part: partial sums buffer of
// multiaxpy_partials(w) doubles, or null for the context scratch
void mv_multiaxpy_scale_norm2(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign,
                              const double* d_osc, double* d_n2, double* part);
size_t multiaxpy_partials(const MV& w);
void mv_norm2_buf(ddamg_ctx* c, const MV& a, double* d_out, double* cbuf, double* part);
void mv_dot(ddamg_ctx* c, const MV& a, const MV& b, double* d_out);  // per column complex
// masked scaling: columns with mask==0 are zeroed
// canonical <-> internal conversion (fine or coarse level)
void to_internal(ddamg_ctx* c, int level, const double* canon, int n_col, const MV& out);
void from_internal(ddamg_ctx* c, int level, const MV& in, int n_col, double* canon);
// dir 0: mv column j <- canon field map[j]; dir 1: canon field map[j] <- mv column j (map[j] < 0: skipped)
void canon_cols(ddamg_ctx* c, int level, const MV& mv, const int* d_map, double* canon, int dir);

// ---- fine-level kernels (fine.hip) ----
void fine_dslash(ddamg_ctx* c, const MV& x, const MV& y, const double* d_mu);
void fine_residual(ddamg_ctx* c, const MV& b, const MV& x, const MV& r, const double* d_mu);
void fine_masked(ddamg_ctx* c, const MV& x, const MV& y, int mode, int hop);
void sap_apply(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, const MV& work);
bool sap_takes_f16(ddamg_ctx* c);
void build_clover(ddamg_ctx* c);   // clover site term from the FP64 links (c_sw != 0)   // sap_apply accepts an FP16 right-hand side
bool dslash_rs_valid(int prec, int rs);

// ---- coarse kernels (coarse.hip) ----
void coarse_apply(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu);
void coarse_masked(ddamg_ctx* c, int level, const MV& x, const MV& y, int mode, int hop);
void restrict_mv(ddamg_ctx* c, int level, const MV& x, const MV& y);
void prolong_mv(ddamg_ctx* c, int level, const MV& x, const MV& y, int accumulate);
void build_basis_field(ddamg_ctx* c, int level, const MV& X);   // X[s*N+j] = P restricted to chirality s
void gather_test_vectors(ddamg_ctx* c, int level, const MV& tv, double* d_P);   // tv -> [V][d][N]
void orthonormalise_P(ddamg_ctx* c, int level, double* d_P);
void scatter_blocks(ddamg_ctx* c, int level, const MV& R, int slot);  // coarse level = level+1
void convert_P32(ddamg_ctx* c, int level);
void convert_blocks32(ddamg_ctx* c, int level);

// ---- learned smoother (ptc.hip) ----
void ptc_set_weights(ddamg_ctx* c, const double* w1, const double* w2);
void ptc_get_weights(ddamg_ctx* c, double* w1, double* w2);
bool ptc_ready(ddamg_ctx* c);
void ptc_layer(ddamg_ctx* c, int layer, bool adjoint, const MV* in, const MV* out);
void ptc_wgrad(ddamg_ctx* c, int layer, const MV* in, const MV* gout, double* g_host);
void ptc_apply(ddamg_ctx* c, const MV& v, const MV& z);
bool ptc_smooth(ddamg_ctx* c, const MV& v, const MV& z, const double* d_mu, int cycles);
void ptc_train(ddamg_ctx* c, const double* mus, int n_mu, int steps, int batch, double lr, int sap_sweeps,
               uint64_t seed, double* loss_hist);
void free_ptc(ddamg_ctx* c);
// fine-level smoother of the preconditioner: SAP, or the learned network with SAP fallback
void fine_smoother(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu);

// A batch of fine-level systems for the outer solve: column i has shift mu[i],
// right-hand side field rhs_of[i] of b and solution field i of x (canonical
// layout, device).  At most max_active columns are in flight at once.
struct OuterJob {
  int ncol = 0;
  std::vector<double> mu;
  std::vector<int> rhs_of;
  const double* b = nullptr;
  double* x = nullptr;
  bool use_x0 = false;
  int max_active = 0;
  // results per column
  std::vector<int> iters;
  std::vector<double> relres;   // true FP64 relative residual when the column left
  std::vector<char> converged;
  std::vector<double> eps;      // doublet solves: epsbar per column (pairs of columns), empty otherwise
  std::vector<double> err;      // FP64 relative residual of the caller's x, recomputed after the solve
  std::vector<int> fallbacks;   // learned-smoother fallbacks while the column was in flight
  int total = 0;                // outer iterations (cycles x steps) of the whole batch
};
void outer_solve(ddamg_ctx* c, OuterJob& job);
// restarted block GMRES(m) on a level, columns grouped by equal shift
void block_gmres(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, bool x_zero, double tol,
                 int m, int maxit, std::vector<int>* iters, std::vector<double>* relres, int* total);
void free_block_work(ddamg_ctx* c);
void level_gmres(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, double tol, int m, int maxit,
                 std::vector<int>* iters, std::vector<double>* relres, int* total);
// the same with deflated restarting, GMRES-DR(m, k)
void level_gmres_dr(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, double tol, int m, int k,
                    int maxit, std::vector<int>* iters);

// ---- host helpers ----
void operator_apply(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu);
bool coarse_takes_f16(ddamg_ctx* c, int level, int ntiles);
double* scratch(ddamg_ctx* c, size_t bytes);          // reduction partials (grows)
double* small_buffer(ddamg_ctx* c, int n_doubles);    // short-lived small device results (grows)
void mv_convert(ddamg_ctx* c, const MV& s, const MV& d);
void mv_normalize(ddamg_ctx* c, const MV& x, const double* d_norm2);   // x_c /= sqrt(norm2_c)
void copy_to_host(ddamg_ctx* c, const void* d, void* h, size_t bytes);
// HIP events around a SAP kernel launch (no-ops unless the time_sap knob is
// set or the stream is being captured); collect sums them after a
// synchronisation of the stream
void sap_timing_begin(ddamg_ctx* c);
void sap_timing_end(ddamg_ctx* c, int ntiles);
void sap_timing_collect(ddamg_ctx* c);
// the same for one kernel class (the value of the time_sap knob): HIP events
// around every launch of that class
enum { TIMED_SAP = 1, TIMED_COARSE1 = 2, TIMED_RESTRICT0 = 3, TIMED_PROLONG0 = 4, TIMED_DSLASH = 5 };
void kernel_timing_begin(ddamg_ctx* c, int cls);
void kernel_timing_end(ddamg_ctx* c, int cls, int ntiles);

}  // namespace ddamg
