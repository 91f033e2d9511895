// Block GMRES with block Gram-Schmidt and Cholesky QR (paper section 4: block
// Krylov solvers on the coarsest level, where the columns that share a twisted
// mass share the operator D_c(mu)).
//
// Columns of a batch are grouped by equal shift; every group runs its own
// block Arnoldi, all groups in lockstep so one operator launch serves the
// whole batch.  For a group of s columns:
//   V_0 S_0 = B - A X                      (Cholesky QR, twice)
//   W = A V_j;  H_ij = V_i^H W, W -= V_i H_ij  for i <= j   (block CGS)
//   V_{j+1} H_{j+1,j} = W                  (Cholesky QR, twice)
// and X += sum_j V_j Y_j with Y minimising ||E_1 S_0 - Hbar Y||_F per column,
// the least-squares problem kept in upper-triangular form by Givens rotations
// on the host as the Hessenberg grows.  The block inner products are FP64
// reductions over the vectors (one workgroup per column pair and basis
// block); the block updates mix the columns of a group with s x s
// coefficients.  A direction that Cholesky finds (numerically) dependent is
// dropped: its column of V is zero and its row of H_{j+1,j} vanishes.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <vector>

#include "common.h"
#include "device.h"

namespace ddamg {

using cd = std::complex<double>;
constexpr int BKMAX = 64;   // basis blocks per cycle (restart length + 1)

struct BPtrs {
  const void* p[BKMAX];
};

// out[(i * npairs + p)] (complex) = sum conj(X_i[ca[p]]) W[cb[p]]
template <typename R>
__global__ void __launch_bounds__(256) k_bdot(BPtrs Xs, const R* __restrict__ W, const int* __restrict__ ca,
                                              const int* __restrict__ cb, int npairs, size_t nslot, int T,
                                              size_t tile_reals, double* __restrict__ out) {
  constexpr int RW = Chunk<R>::RW;
  const int p = blockIdx.x, i = blockIdx.y;
  const R* X = static_cast<const R*>(Xs.p[i]);
  const int a = ca[p], b = cb[p];
  const R* xa = X + (size_t)(a / T) * tile_reals + (size_t)(a % T) * RW;
  const R* wb = W + (size_t)(b / T) * tile_reals + (size_t)(b % T) * RW;
  double re = 0, im = 0;
  for (size_t q = threadIdx.x; q < nslot; q += blockDim.x) {
    const size_t o = q * T * RW;
#pragma unroll
    for (int k = 0; k < RW; k += 2) {
      const double xr = xa[o + k], xi = xa[o + k + 1], wr = wb[o + k], wi = wb[o + k + 1];
      re += xr * wr + xi * wi;
      im += xr * wi - xi * wr;
    }
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[((size_t)i * npairs + p) * 2] = sr[0];
    out[((size_t)i * npairs + p) * 2 + 1] = si[0];
  }
}

// Y[b] = beta Y[b] + sum_i sum_{a in group(b)} X_i[a] C[i][pair(a, b)]
// One thread per 16-byte chunk of Y in the layout order; columns outside
// every group are zeroed when beta == 0 and left alone otherwise.
template <typename R>
__global__ void k_bupdate(BPtrs Xs, int nvec, R* __restrict__ Y, double beta, const double* __restrict__ C,
                          int npairs, const int* __restrict__ grp, const int* __restrict__ pos,
                          const int* __restrict__ gstart, const int* __restrict__ gcols,
                          const int* __restrict__ pbase, size_t nslot, int T, int ntiles, size_t tile_reals) {
  constexpr int RW = Chunk<R>::RW;
  const size_t n = (size_t)ntiles * nslot * T;
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < n; u += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(u % T);
    const size_t q = (u / T) % nslot;
    const int tile = (int)(u / ((size_t)T * nslot));
    const int b = tile * T + t;
    R* y = Y + (size_t)tile * tile_reals + (q * T + t) * RW;
    const int g = grp[b];
    if (g < 0) {
      if (beta == 0.0) {
#pragma unroll
        for (int k = 0; k < RW; ++k) y[k] = (R)0;
      }
      continue;
    }
    const int s = gstart[g + 1] - gstart[g], bi = pos[b];
    double acc[RW];
#pragma unroll
    for (int k = 0; k < RW; ++k) acc[k] = beta == 0.0 ? 0.0 : beta * (double)y[k];
    for (int i = 0; i < nvec; ++i) {
      const R* X = static_cast<const R*>(Xs.p[i]);
      const double* Ci = C + ((size_t)i * npairs + pbase[g] + bi) * 2;
      for (int ai = 0; ai < s; ++ai) {
        const int a = gcols[gstart[g] + ai];
        const double cr = Ci[(size_t)ai * s * 2], ci = Ci[(size_t)ai * s * 2 + 1];
        const R* x = X + (size_t)(a / T) * tile_reals + (q * T + (a % T)) * RW;
#pragma unroll
        for (int k = 0; k < RW; k += 2) {
          const double xr = x[k], xi = x[k + 1];
          acc[k] += xr * cr - xi * ci;
          acc[k + 1] += xr * ci + xi * cr;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RW; ++k) y[k] = (R)acc[k];
  }
}

static inline dim3 gridn(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

// Column groups of one batch (equal shift), with the device tables the
// kernels read.
struct Groups {
  int ng = 0, npairs = 0, ncol = 0;
  std::vector<int> gstart, gcols, pbase, grp, pos;
  int *d_grp = nullptr, *d_pos = nullptr, *d_gstart = nullptr, *d_gcols = nullptr, *d_pbase = nullptr;
  int *d_ca = nullptr, *d_cb = nullptr;
  int size(int g) const { return gstart[g + 1] - gstart[g]; }
};

static int* upload_ints(ddamg_ctx* c, const std::vector<int>& v) {
  int* d = (int*)c->pool.alloc(std::max<size_t>(v.size(), 1) * sizeof(int));
  if (!v.empty()) DD_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  return d;
}

static Groups make_groups(ddamg_ctx* c, const std::vector<double>& mu, const std::vector<double>& bn) {
  Groups G;
  G.ncol = (int)mu.size();
  std::map<double, std::vector<int>> by;
  for (int i = 0; i < G.ncol; ++i)
    if (bn[i] > 0) by[mu[i]].push_back(i);
  G.grp.assign(G.ncol, -1);
  G.pos.assign(G.ncol, 0);
  G.gstart.push_back(0);
  std::vector<int> ca, cb;
  for (auto& kv : by) {
    const int g = G.ng++;
    const int s = (int)kv.second.size();
    G.pbase.push_back(G.npairs);
    for (int k = 0; k < s; ++k) {
      G.grp[kv.second[k]] = g;
      G.pos[kv.second[k]] = k;
      G.gcols.push_back(kv.second[k]);
    }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        ca.push_back(kv.second[a]);
        cb.push_back(kv.second[b]);
      }
    G.npairs += s * s;
    G.gstart.push_back((int)G.gcols.size());
  }
  G.d_grp = upload_ints(c, G.grp);
  G.d_pos = upload_ints(c, G.pos);
  G.d_gstart = upload_ints(c, G.gstart);
  G.d_gcols = upload_ints(c, G.gcols);
  G.d_pbase = upload_ints(c, G.pbase);
  G.d_ca = upload_ints(c, ca);
  G.d_cb = upload_ints(c, cb);
  return G;
}

static void free_groups(ddamg_ctx* c, Groups& G) {
  int* all[] = {G.d_grp, G.d_pos, G.d_gstart, G.d_gcols, G.d_pbase, G.d_ca, G.d_cb};
  for (int* p : all)
    if (p) c->pool.release(p);
}

// H[i][pair] = X_i^H W for the given basis blocks (host result, complex)
static void block_dots(ddamg_ctx* c, const Groups& G, const std::vector<MV>& Xs, const MV& W, double* d_out,
                       std::vector<double>& host) {
  const int nvec = (int)Xs.size();
  if (G.npairs == 0) return;
  BPtrs P{};
  for (int i = 0; i < nvec; ++i) P.p[i] = Xs[i].p;
  const size_t nslot = (size_t)W.nchunk * W.nsites;
  dim3 grid(G.npairs, nvec);
  if (W.prec == P64)
    hipLaunchKernelGGL(k_bdot<double>, grid, dim3(256), 0, c->stream, P, W.as<double>(), G.d_ca, G.d_cb, G.npairs,
                       nslot, W.T, W.tile_reals(), d_out);
  else
    hipLaunchKernelGGL(k_bdot<float>, grid, dim3(256), 0, c->stream, P, W.as<float>(), G.d_ca, G.d_cb, G.npairs,
                       nslot, W.T, W.tile_reals(), d_out);
  DD_HIP(hipGetLastError());
  host.resize((size_t)nvec * G.npairs * 2);
  copy_to_host(c, d_out, host.data(), host.size() * sizeof(double));
}

// Y = beta Y + sum_i X_i C_i (C on the device, [nvec][npairs] complex)
static void block_update(ddamg_ctx* c, const Groups& G, const std::vector<MV>& Xs, const MV& Y, double beta,
                         const double* d_C) {
  const int nvec = (int)Xs.size();
  BPtrs P{};
  for (int i = 0; i < nvec; ++i) P.p[i] = Xs[i].p;
  const size_t nslot = (size_t)Y.nchunk * Y.nsites;
  const size_t n = (size_t)Y.ntiles * nslot * Y.T;
  if (Y.prec == P64)
    hipLaunchKernelGGL(k_bupdate<double>, gridn(n), dim3(256), 0, c->stream, P, nvec, Y.as<double>(), beta, d_C,
                       G.npairs, G.d_grp, G.d_pos, G.d_gstart, G.d_gcols, G.d_pbase, nslot, Y.T, Y.ntiles,
                       Y.tile_reals());
  else
    hipLaunchKernelGGL(k_bupdate<float>, gridn(n), dim3(256), 0, c->stream, P, nvec, Y.as<float>(), beta, d_C,
                       G.npairs, G.d_grp, G.d_pos, G.d_gstart, G.d_gcols, G.d_pbase, nslot, Y.T, Y.ntiles,
                       Y.tile_reals());
  DD_HIP(hipGetLastError());
}

// Per group: R (upper triangular, s x s, row-major) with G = R^H R from the
// Gram matrix; dependent directions (pivot <= eps * largest diagonal) get a
// zero row.  Rinv (as update coefficients, [pair(a, b)] = (R^+)[a][b]) maps W
// to the orthonormal V = W R^+.
static void chol_factor(const Groups& G, const std::vector<double>& gram, double eps, std::vector<cd>& R,
                        std::vector<double>& rinv_pairs) {
  R.assign((size_t)G.npairs, cd(0));
  rinv_pairs.assign((size_t)G.npairs * 2, 0.0);
  for (int g = 0; g < G.ng; ++g) {
    const int s = G.size(g), pb = G.pbase[g];
    auto gm = [&](int a, int b) { return cd(gram[(size_t)(pb + a * s + b) * 2], gram[(size_t)(pb + a * s + b) * 2 + 1]); };
    double dmax = 0;
    for (int a = 0; a < s; ++a) dmax = std::max(dmax, gm(a, a).real());
    std::vector<cd> U((size_t)s * s, cd(0));   // upper triangular, G = U^H U
    std::vector<char> live(s, 0);
    for (int k = 0; k < s; ++k) {
      // U[k][k]^2 = G[k][k] - sum_{i<k} |U[i][k]|^2 ; U[k][j] = (G[k][j] - sum_i conj(U[i][k]) U[i][j]) / U[k][k]
      double d = gm(k, k).real();
      for (int i = 0; i < k; ++i) d -= std::norm(U[(size_t)i * s + k]);
      if (!(d > eps * dmax) || dmax <= 0) continue;   // dependent direction: row k stays zero
      live[k] = 1;
      const double ukk = std::sqrt(d);
      U[(size_t)k * s + k] = ukk;
      for (int j = k + 1; j < s; ++j) {
        cd v = gm(k, j);
        for (int i = 0; i < k; ++i) v -= std::conj(U[(size_t)i * s + k]) * U[(size_t)i * s + j];
        U[(size_t)k * s + j] = v / ukk;
      }
    }
    // pseudo-inverse of U on its live rows / columns (back substitution)
    std::vector<cd> Ui((size_t)s * s, cd(0));
    for (int j = 0; j < s; ++j) {
      if (!live[j]) continue;
      for (int i = j; i >= 0; --i) {
        if (!live[i]) continue;
        cd v = (i == j) ? cd(1) : cd(0);
        for (int k = i + 1; k <= j; ++k)
          if (live[k]) v -= U[(size_t)i * s + k] * Ui[(size_t)k * s + j];
        Ui[(size_t)i * s + j] = v / U[(size_t)i * s + i];
      }
    }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        R[(size_t)pb + a * s + b] = U[(size_t)a * s + b];
        rinv_pairs[(size_t)(pb + a * s + b) * 2] = Ui[(size_t)a * s + b].real();
        rinv_pairs[(size_t)(pb + a * s + b) * 2 + 1] = Ui[(size_t)a * s + b].imag();
      }
  }
}

// Cholesky QR twice: V = W R^+ with R the product of both factors.
static void chol_qr2(ddamg_ctx* c, const Groups& G, const MV& W, const MV& V, double eps, double* d_buf,
                     double* d_coef, std::vector<cd>& R) {
  std::vector<double> gram, rinv;
  std::vector<cd> R1, R2;
  block_dots(c, G, {W}, W, d_buf, gram);
  chol_factor(G, gram, eps, R1, rinv);
  DD_HIP(hipMemcpyAsync(d_coef, rinv.data(), rinv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  block_update(c, G, {W}, V, 0.0, d_coef);
  block_dots(c, G, {V}, V, d_buf, gram);
  chol_factor(G, gram, eps, R2, rinv);
  DD_HIP(hipMemcpyAsync(d_coef, rinv.data(), rinv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  block_update(c, G, {V}, W, 0.0, d_coef);   // W <- V R2^+ (orthonormal again)
  mv_copy(c, W, V);
  DD_HIP(hipStreamSynchronize(c->stream));   // host coefficient vectors are reused
  // R = R2 R1 per group
  R.assign((size_t)G.npairs, cd(0));
  for (int g = 0; g < G.ng; ++g) {
    const int s = G.size(g), pb = G.pbase[g];
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        cd v = 0;
        for (int k = 0; k < s; ++k) v += R2[(size_t)pb + a * s + k] * R1[(size_t)pb + k * s + b];
        R[(size_t)pb + a * s + b] = v;
      }
  }
}

// Upper-triangular least squares of one group's block Hessenberg, grown one
// block column at a time with Givens rotations.
struct GroupLS {
  int s = 0, m = 0;
  std::vector<cd> H;     // [(m+1)s][m s] row-major, rotated in place
  std::vector<cd> E;     // [(m+1)s][s] right-hand sides, rotated in place
  struct Rot { int p, q; double c; cd sn; };
  std::vector<Rot> rots;
  void init(int s_, int m_, const std::vector<cd>& S0, int pb) {
    s = s_;
    m = m_;
    H.assign((size_t)(m + 1) * s * m * s, cd(0));
    E.assign((size_t)(m + 1) * s * s, cd(0));
    rots.clear();
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) E[(size_t)a * s + b] = S0[(size_t)pb + a * s + b];
  }
  cd& h(int r, int col) { return H[(size_t)r * m * s + col]; }
  static void apply(const Rot& r, cd& x, cd& y) {   // [x; y] <- [c s; -conj(s) c] [x; y]
    const cd a = x, b = y;
    x = r.c * a + r.sn * b;
    y = -std::conj(r.sn) * a + r.c * b;
  }
  // block column j: Hij (i <= j) from the block Gram-Schmidt, Hj1 = R of the QR
  void add_block_column(int j, const std::vector<double>& hdots, int npairs, int pb, const std::vector<cd>& Rn) {
    for (int bcol = 0; bcol < s; ++bcol) {
      const int col = j * s + bcol;
      for (int i = 0; i <= j; ++i)
        for (int a = 0; a < s; ++a) {
          const size_t k = ((size_t)i * npairs + pb + a * s + bcol) * 2;
          h(i * s + a, col) = cd(hdots[k], hdots[k + 1]);
        }
      for (int a = 0; a < s; ++a) h((j + 1) * s + a, col) = Rn[(size_t)pb + a * s + bcol];
      // previous rotations
      for (const Rot& r : rots) apply(r, h(r.p, col), h(r.q, col));
      // zero the entries below the diagonal of this column
      for (int q = col + 1; q <= (j + 1) * s + s - 1; ++q) {
        cd& x = h(col, col);
        cd& y = h(q, col);
        if (std::abs(y) == 0) continue;
        Rot r{col, q, 0, 0};
        if (std::abs(x) == 0) {
          r.c = 0;
          r.sn = std::conj(y) / std::abs(y);
        } else {
          const double nx = std::abs(x), nr = std::hypot(nx, std::abs(y));
          r.c = nx / nr;
          r.sn = (x / nx) * std::conj(y) / nr;
        }
        apply(r, x, y);
        y = 0;
        for (int b = 0; b < s; ++b) apply(r, E[(size_t)r.p * s + b], E[(size_t)r.q * s + b]);
        rots.push_back(r);
      }
    }
  }
  // residual norm of right-hand side b after block columns 0..j
  double resid(int j, int b) const {
    double v = 0;
    for (int r = (j + 1) * s; r < (j + 2) * s; ++r) v += std::norm(E[(size_t)r * s + b]);
    return std::sqrt(v);
  }
  // Y ((j+1)s x s) by back substitution; zero pivots (dropped directions) give zero rows
  std::vector<cd> solve(int j) const {
    const int n = (j + 1) * s;
    std::vector<cd> Y((size_t)n * s, cd(0));
    const double hmax = [&] {
      double v = 0;
      for (int r = 0; r < n; ++r) v = std::max(v, std::abs(H[(size_t)r * m * s + r]));
      return v;
    }();
    for (int b = 0; b < s; ++b)
      for (int r = n - 1; r >= 0; --r) {
        cd v = E[(size_t)r * s + b];
        for (int k = r + 1; k < n; ++k) v -= H[(size_t)r * m * s + k] * Y[(size_t)k * s + b];
        const cd d = H[(size_t)r * m * s + r];
        Y[(size_t)r * s + b] = std::abs(d) > 1e-14 * hmax ? v / d : cd(0);
      }
    return Y;
  }
};

struct BlockWork {
  int cap = 0;
  std::vector<MV> V;
  MV W, T;
  double* d_buf = nullptr;   // block dots
  double* d_coef = nullptr;  // update coefficients
  size_t nbuf = 0, ncoef = 0;
};

using BlockWorkMap = std::map<std::pair<int, int>, BlockWork>;   // (level, precision)

static BlockWork& block_work(ddamg_ctx* c, int level, int prec, int nt, int m, size_t npairs) {
  if (!c->bwork) c->bwork = new BlockWorkMap();
  BlockWork& w = (*static_cast<BlockWorkMap*>(c->bwork))[{level, prec}];
  if (nt > w.cap) {
    for (MV& v : w.V) mv_free(c, v);
    w.V.clear();
    mv_free(c, w.W);
    mv_free(c, w.T);
    w.cap = nt;
  }
  while ((int)w.V.size() < m + 1) w.V.push_back(mv_alloc(c, level, prec, w.cap * c->T));
  if (!w.W.p) w.W = mv_alloc(c, level, prec, w.cap * c->T);
  if (!w.T.p) w.T = mv_alloc(c, level, prec, w.cap * c->T);
  const size_t need = (size_t)(m + 1) * std::max<size_t>(npairs, 1) * 2;
  if (need > w.nbuf) {
    if (w.d_buf) c->pool.release(w.d_buf);
    if (w.d_coef) c->pool.release(w.d_coef);
    w.nbuf = w.ncoef = need;
    w.d_buf = (double*)c->pool.alloc(need * sizeof(double));
    w.d_coef = (double*)c->pool.alloc(need * sizeof(double));
  }
  return w;
}

void free_block_work(ddamg_ctx* c) {
  if (!c->bwork) return;
  for (auto& kv : *static_cast<BlockWorkMap*>(c->bwork)) {
    BlockWork& w = kv.second;
    for (MV& v : w.V) mv_free(c, v);
    mv_free(c, w.W);
    mv_free(c, w.T);
    if (w.d_buf) c->pool.release(w.d_buf);
    if (w.d_coef) c->pool.release(w.d_coef);
  }
  delete static_cast<BlockWorkMap*>(c->bwork);
  c->bwork = nullptr;
}

// Restarted block GMRES(m) on level `level` for every column of b (x: initial
// guess unless x_zero).  Stops when every column's residual estimate is below
// tol * ||b_c||, or after maxit block steps.  iters / relres per column.
void block_gmres(ddamg_ctx* c, int level, const double* d_mu, const MV& b, const MV& x, bool x_zero, double tol,
                 int m, int maxit, std::vector<int>* iters_out, std::vector<double>* relres_out, int* total_out) {
  DD_CHECK(m >= 1 && m < BKMAX, DDAMG_EINVAL, "block GMRES restart length must be in [1, 63]");
  const int nt = b.ntiles, ncol = b.ncol(), prec = b.prec;
  const double eps = prec == P64 ? 1e-24 : 1e-12;   // relative pivot (squared norm) of a dropped direction
  std::vector<double> mu(ncol), bn(ncol);
  copy_to_host(c, d_mu, mu.data(), ncol * sizeof(double));
  {
    double* d = small_buffer(c, 4 * ncol);
    mv_norm2(c, b, d + 2 * ncol);
    copy_to_host(c, d + 2 * ncol, bn.data(), ncol * sizeof(double));
    for (double& v : bn) v = v > 0 ? std::sqrt(v) : 0.0;
  }
  Groups G = make_groups(c, mu, bn);
  BlockWork& w = block_work(c, level, prec, nt, m, G.npairs);
  std::vector<int> iters(ncol, 0);
  std::vector<double> est(ncol, 0.0);
  int total = 0;
  if (x_zero) mv_zero(c, x);
  bool first = true;
  std::vector<GroupLS> ls(G.ng);
  while (G.ng > 0) {
    // block residual and its QR
    MV W = w.W.tiles(0, nt), Tm = w.T.tiles(0, nt);
    if (first && x_zero) {
      mv_copy(c, b, W);
    } else {
      operator_apply(c, level, x, Tm, d_mu);
      mv_sub(c, b, Tm, W);
    }
    first = false;
    std::vector<cd> S0;
    MV V0 = w.V[0].tiles(0, nt);
    chol_qr2(c, G, W, V0, eps, w.d_buf, w.d_coef, S0);
    bool all = true;
    for (int g = 0; g < G.ng; ++g) {
      const int s = G.size(g), pb = G.pbase[g];
      ls[g].init(s, m, S0, pb);
      for (int bi = 0; bi < s; ++bi) {
        const int col = G.gcols[G.gstart[g] + bi];
        double v = 0;
        for (int a = 0; a < s; ++a) v += std::norm(S0[(size_t)pb + a * s + bi]);
        est[col] = std::sqrt(v);
        if (est[col] > tol * bn[col]) all = false;
      }
    }
    if (all || total >= maxit) break;
    int jj = 0;
    for (int j = 0; j < m && total < maxit; ++j) {
      MV Vj = w.V[j].tiles(0, nt);
      operator_apply(c, level, Vj, W, d_mu);
      std::vector<MV> Vs;
      for (int i = 0; i <= j; ++i) Vs.push_back(w.V[i].tiles(0, nt));
      std::vector<double> hd;
      block_dots(c, G, Vs, W, w.d_buf, hd);
      std::vector<double> neg(hd.size());
      for (size_t k = 0; k < hd.size(); ++k) neg[k] = -hd[k];
      DD_HIP(hipMemcpyAsync(w.d_coef, neg.data(), neg.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      block_update(c, G, Vs, W, 1.0, w.d_coef);
      std::vector<cd> Rn;
      MV Vn = w.V[j + 1].tiles(0, nt);
      chol_qr2(c, G, W, Vn, eps, w.d_buf, w.d_coef, Rn);   // synchronises (neg is reused)
      ++total;
      jj = j + 1;
      bool alld = true;
      for (int g = 0; g < G.ng; ++g) {
        ls[g].add_block_column(j, hd, G.npairs, G.pbase[g], Rn);
        for (int bi = 0; bi < G.size(g); ++bi) {
          const int col = G.gcols[G.gstart[g] + bi];
          est[col] = ls[g].resid(j, bi);
          if (est[col] > tol * bn[col]) alld = false;
        }
      }
      if (alld) break;
    }
    // x += sum_j V_j Y_j
    std::vector<double> coef((size_t)jj * G.npairs * 2, 0.0);
    for (int g = 0; g < G.ng; ++g) {
      const int s = G.size(g), pb = G.pbase[g];
      const std::vector<cd> Y = ls[g].solve(jj - 1);
      for (int i = 0; i < jj; ++i)
        for (int a = 0; a < s; ++a)
          for (int bi = 0; bi < s; ++bi) {
            const cd v = Y[(size_t)(i * s + a) * s + bi];
            coef[((size_t)i * G.npairs + pb + a * s + bi) * 2] = v.real();
            coef[((size_t)i * G.npairs + pb + a * s + bi) * 2 + 1] = v.imag();
          }
    }
    std::vector<MV> Vs;
    for (int i = 0; i < jj; ++i) Vs.push_back(w.V[i].tiles(0, nt));
    DD_HIP(hipMemcpyAsync(w.d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    block_update(c, G, Vs, x, 1.0, w.d_coef);
    DD_HIP(hipStreamSynchronize(c->stream));
    for (int col = 0; col < ncol; ++col)
      if (G.grp[col] >= 0) iters[col] += jj;
    bool conv = true;
    for (int col = 0; col < ncol; ++col)
      if (G.grp[col] >= 0 && est[col] > tol * bn[col]) conv = false;
    if (conv || total >= maxit) break;
  }
  free_groups(c, G);
  if (iters_out) *iters_out = iters;
  if (relres_out) {
    relres_out->assign(ncol, 0.0);
    for (int col = 0; col < ncol; ++col) (*relres_out)[col] = bn[col] > 0 ? est[col] / bn[col] : 0.0;
  }
  if (total_out) *total_out = total;
}

}  // namespace ddamg
