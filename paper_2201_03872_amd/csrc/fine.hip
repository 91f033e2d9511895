// Fine-level kernels: the batched twisted-mass Wilson stencil (FP64 with full
// links, FP32 with 2-row compressed links), its masked form used by the
// Galerkin setup, and the fused red-black SAP half-sweep.
//
// Operator (the paper's D_TM = D_W + i mu gamma5, Fig. 6 caption, in the m0
// normalisation):
//   (D x)(s) = (4+m0) x(s) + i mu gamma5 x(s)
//              - 1/2 sum_nu [(1-g_nu) U_nu(s) x(s+nu) + (1+g_nu) U_nu(s-nu)^dag x(s-nu)]
// In the chiral basis g_nu = [[0, A_nu], [A_nu^dag, 0]] with A = -i s1, -i s2,
// -i s3, 1 for nu = x, y, z, t; (1 -+ g_nu) x = [h; -+A^dag h] with
// h = x_up -+ A x_down, so every hop moves a two-spin half spinor through one
// SU(3) multiplication.  The antiperiodic time boundary is a sign on the hop
// (bit 31 of the neighbour table), never folded into the links: with 2-row
// compression the third row is rebuilt as conj(row0 x row1), which would lose
// a sign stored in the link.
#include "common.h"
#include "device.h"

namespace ddamg {

constexpr int TT = 8;                 // columns per tile
constexpr int SPW = 256 / TT;         // sites per 256-lane workgroup

// ---------------------------------------------------------------- links ---
template <typename R, bool C2>
__device__ __forceinline__ void load_link(const void* __restrict__ Uv, int mu, int s, int V, cx<R> (&u)[9]) {
  if constexpr (!C2) {
    const double2* U = reinterpret_cast<const double2*>(Uv) + (size_t)mu * 9 * V;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 c = U[(size_t)k * V + s];
      u[k] = {(R)c.x, (R)c.y};
    }
  } else {
    const float4* U = reinterpret_cast<const float4*>(Uv) + (size_t)mu * 3 * V;
    float4 a = U[s], b = U[(size_t)V + s], c = U[2 * (size_t)V + s];
    u[0] = {(R)a.x, (R)a.y}; u[1] = {(R)a.z, (R)a.w}; u[2] = {(R)b.x, (R)b.y};
    u[3] = {(R)b.z, (R)b.w}; u[4] = {(R)c.x, (R)c.y}; u[5] = {(R)c.z, (R)c.w};
    // row 2 = conj(row 0 x row 1)  (det U = 1)
    u[6] = conj_(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj_(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj_(u[0] * u[4] - u[1] * u[3]);
  }
}

// ------------------------------------------------------- spin structure ---
// h = x_up - A x_down (forward) or x_up + A x_down (backward), for colour c
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void project(const cx<R> (&p)[12], cx<R> (&h)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> p2 = p[6 + c], p3 = p[9 + c], a0, a1;
    if constexpr (MU == 0) { a0 = mul_mi(p3); a1 = mul_mi(p2); }
    else if constexpr (MU == 1) { a0 = (R)-1 * p3; a1 = p2; }
    else if constexpr (MU == 2) { a0 = mul_mi(p2); a1 = mul_i(p3); }
    else { a0 = p2; a1 = p3; }
    if constexpr (FWD) { h[c] = p[c] - a0; h[3 + c] = p[3 + c] - a1; }
    else { h[c] = p[c] + a0; h[3 + c] = p[3 + c] + a1; }
  }
}

// acc_up += g ; acc_down -= A^dag g (forward) or += A^dag g (backward)
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void reconstruct(cx<R> (&acc)[12], const cx<R> (&g)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> g0 = g[c], g1 = g[3 + c], b0, b1;
    if constexpr (MU == 0) { b0 = mul_i(g1); b1 = mul_i(g0); }
    else if constexpr (MU == 1) { b0 = g1; b1 = (R)-1 * g0; }
    else if constexpr (MU == 2) { b0 = mul_i(g0); b1 = mul_mi(g1); }
    else { b0 = g0; b1 = g1; }
    acc[c] = acc[c] + g0;
    acc[3 + c] = acc[3 + c] + g1;
    if constexpr (FWD) { acc[6 + c] = acc[6 + c] - b0; acc[9 + c] = acc[9 + c] - b1; }
    else { acc[6 + c] = acc[6 + c] + b0; acc[9 + c] = acc[9 + c] + b1; }
  }
}

template <bool FWD, typename R>
__device__ __forceinline__ void colour(const cx<R> (&u)[9], const cx<R> (&h)[6], cx<R> (&g)[6]) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> r = {0, 0};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (FWD) cmac(r, u[a * 3 + b], h[sp * 3 + b]);
        else cmac_conj(r, u[b * 3 + a], h[sp * 3 + b]);
      }
      g[sp * 3 + a] = r;
    }
}

// One hop term accumulated into acc (without the -1/2).  `ld(h, nb, p)` loads
// the neighbour spinor of hop h (0..3 forward, 4..7 backward) and returns
// false to drop the hop.
template <int MU, bool FWD, typename R, bool C2, typename Loader>
__device__ __forceinline__ void hop(cx<R> (&acc)[12], const void* __restrict__ U, const int* __restrict__ nbr,
                                    int V, int s, Loader&& ld) {
  constexpr int H = FWD ? MU : 4 + MU;
  const int e = nbr[(size_t)H * V + s];
  const int nb = e & 0x7fffffff;
  cx<R> p[12];
  if (!ld(H, nb, p)) return;
  cx<R> h[6];
  project<MU, FWD>(p, h);
  if (e < 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = (R)-1 * h[k];
  }
  cx<R> u[9];
  load_link<R, C2>(U, MU, FWD ? s : nb, V, u);
  cx<R> g[6];
  colour<FWD>(u, h, g);
  reconstruct<MU, FWD>(acc, g);
}

// The eight hops one after the other: a non-unrolled loop over a uniform
// switch keeps only one neighbour spinor and one link live at a time.
template <typename R, bool C2, typename Loader>
__device__ __forceinline__ void all_hops(cx<R> (&acc)[12], const void* U, const int* nbr, int V, int s, Loader&& ld) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    switch (h) {
      case 0: hop<0, true, R, C2>(acc, U, nbr, V, s, ld); break;
      case 1: hop<1, true, R, C2>(acc, U, nbr, V, s, ld); break;
      case 2: hop<2, true, R, C2>(acc, U, nbr, V, s, ld); break;
      case 3: hop<3, true, R, C2>(acc, U, nbr, V, s, ld); break;
      case 4: hop<0, false, R, C2>(acc, U, nbr, V, s, ld); break;
      case 5: hop<1, false, R, C2>(acc, U, nbr, V, s, ld); break;
      case 6: hop<2, false, R, C2>(acc, U, nbr, V, s, ld); break;
      default: hop<3, false, R, C2>(acc, U, nbr, V, s, ld); break;
    }
  }
}

// out = diag x + i mu gamma5 x - 1/2 acc
template <typename R>
__device__ __forceinline__ void site_diag(cx<R> (&out)[12], const cx<R> (&x)[12], const cx<R> (&acc)[12], R diag, R mu) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const R g = k < 6 ? mu : -mu;
    out[k].re = diag * x[k].re - g * x[k].im - (R)0.5 * acc[k].re;
    out[k].im = diag * x[k].im + g * x[k].re - (R)0.5 * acc[k].im;
  }
}

// ------------------------------------------------------------ dslash ---
// MODE 0: y = D x ; MODE 1: y = b - D x
template <typename R, bool C2, int MODE>
__global__ void __launch_bounds__(256) k_dslash(const R* __restrict__ x, R* __restrict__ y, const R* __restrict__ b,
                                                const void* __restrict__ U, const int* __restrict__ nbr,
                                                const double* __restrict__ mu, int V, size_t tile_reals, R diag,
                                                int nsb) {
  const int t = threadIdx.x % TT, sl = threadIdx.x / TT;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = wg / nsb;
  const int s = (wg % nsb) * SPW + sl;
  if (s >= V) return;
  const R* xt = x + (size_t)tile * tile_reals;
  auto ld = [&](int, int nb, cx<R>(&p)[12]) {
    load_cx<R, 12>(xt, V, TT, nb, t, p);
    return true;
  };
  cx<R> acc[12];
  all_hops<R, C2>(acc, U, nbr, V, s, ld);
  cx<R> xs[12], out[12];
  load_cx<R, 12>(xt, V, TT, s, t, xs);
  site_diag(out, xs, acc, diag, (R)mu[tile * TT + t]);
  if constexpr (MODE == 1) {
    cx<R> bs[12];
    load_cx<R, 12>(b + (size_t)tile * tile_reals, V, TT, s, t, bs);
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = bs[k] - out[k];
  }
  store_cx<R, 12>(y + (size_t)tile * tile_reals, V, TT, s, t, out);
}

// Masked stencil for the Galerkin construction (FP64):
//   mode 0: y = (4+m0) x + sum of the hops that stay inside the aggregate of s
//   mode 1: y = the single hop `hopi` (0..3 forward, 4..7 backward) if it
//           leaves the aggregate of s, else 0.
// Aggregates are the gsize-site groups of the internal order.
__global__ void __launch_bounds__(256) k_dslash_masked(const double* __restrict__ x, double* __restrict__ y,
                                                       const void* __restrict__ U, const int* __restrict__ nbr,
                                                       int V, size_t tile_reals, double diag, int nsb, int gsize,
                                                       int mode, int hopi) {
  using R = double;
  const int t = threadIdx.x % TT, sl = threadIdx.x / TT;
  const int wg = blockIdx.x;
  const int tile = wg / nsb;
  const int s = (wg % nsb) * SPW + sl;
  if (s >= V) return;
  const R* xt = x + (size_t)tile * tile_reals;
  const int ag = s / gsize;
  cx<R> acc[12];
  auto ld = [&](int h, int nb, cx<R>(&p)[12]) {
    const bool inside = (nb / gsize) == ag;
    const bool keep = mode == 0 ? inside : (h == hopi && !inside);
    if (!keep) return false;
    load_cx<R, 12>(xt, V, TT, nb, t, p);
    return true;
  };
  all_hops<R, false>(acc, U, nbr, V, s, ld);
  cx<R> out[12];
  cx<R> xs[12];
  load_cx<R, 12>(xt, V, TT, s, t, xs);
  const double dg = mode == 0 ? diag : 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) out[k] = dg * xs[k] - 0.5 * acc[k];
  store_cx<R, 12>(y + (size_t)tile * tile_reals, V, TT, s, t, out);
}

// ---------------------------------------------------------------- SAP ---
// One colour half-sweep of red-black SAP (paper section 2): every workgroup
// owns one block of that colour and K columns of a tile.
//   1. r = f - D x on the block's sites (full stencil, neighbours in global memory);
//   2. k_MR minimal-residual steps on D_BB (hops leaving the block dropped),
//      rho kept in LDS for the in-block neighbour exchange, the two inner
//      products per column reduced over the block with wavefront shuffles;
//   3. x += delta on the block.
// Blocks of one colour never neighbour each other, so the in-place update of
// x is race free.
template <typename R, bool C2, int K, int BS>
__global__ void __launch_bounds__(BS * K) k_sap_half(const R* __restrict__ f, R* __restrict__ x,
                                                     const void* __restrict__ U, const int* __restrict__ nbr,
                                                     const double* __restrict__ mu, const int* __restrict__ blist,
                                                     int V, int ntiles, size_t tile_reals, R diag, int mr_iters) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW;
  constexpr int NCH = 24 / RW;
  constexpr int NT = BS * K;
  constexpr int NSUB = TT / K;
  constexpr int NW = NT >= 64 ? NT / 64 : 1;
  constexpr int WL = NT >= 64 ? 64 : NT;    // lanes per wave actually used
  __shared__ C lds[NCH * BS * K];
  __shared__ R red[NW][K][3];

  int wg = blockIdx.x;
  const int sub = wg % NSUB;
  wg /= NSUB;
  const int tile = wg % ntiles;
  const int bi = wg / ntiles;
  const int kk = threadIdx.x % K, sl = threadIdx.x / K;
  const int t = sub * K + kk;
  const int blk = blist[bi];
  const int s = blk * BS + sl;
  const R* ft = f + (size_t)tile * tile_reals;
  R* xt = x + (size_t)tile * tile_reals;
  const R m = (R)mu[tile * TT + t];

  // 1. block residual
  cx<R> rho[12], dl[12], q[12];
  {
    auto ldg = [&](int, int nb, cx<R>(&p)[12]) {
      load_cx<R, 12>(xt, V, TT, nb, t, p);
      return true;
    };
    cx<R> acc[12], xs[12], fs[12];
    all_hops<R, C2>(acc, U, nbr, V, s, ldg);
    load_cx<R, 12>(xt, V, TT, s, t, xs);
    load_cx<R, 12>(ft, V, TT, s, t, fs);
    site_diag(q, xs, acc, diag, m);
#pragma unroll
    for (int k = 0; k < 12; ++k) { rho[k] = fs[k] - q[k]; dl[k] = {0, 0}; }
  }

  // 2. block MR
  auto ldl = [&](int, int nb, cx<R>(&p)[12]) {
    if (nb / BS != blk) return false;
    const int l = nb - blk * BS;
    if constexpr (RW == 2) {
#pragma unroll
      for (int k = 0; k < NCH; ++k) { C c = lds[(k * BS + l) * K + kk]; p[k] = {c.x, c.y}; }
    } else {
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        C c = lds[(k * BS + l) * K + kk];
        p[2 * k] = {c.x, c.y};
        p[2 * k + 1] = {c.z, c.w};
      }
    }
    return true;
  };
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int it = 0; it < mr_iters; ++it) {
    if constexpr (RW == 2) {
#pragma unroll
      for (int k = 0; k < NCH; ++k) lds[(k * BS + sl) * K + kk] = C{rho[k].re, rho[k].im};
    } else {
#pragma unroll
      for (int k = 0; k < NCH; ++k)
        lds[(k * BS + sl) * K + kk] = C{rho[2 * k].re, rho[2 * k].im, rho[2 * k + 1].re, rho[2 * k + 1].im};
    }
    __syncthreads();
    cx<R> acc[12];
    all_hops<R, C2>(acc, U, nbr, V, s, ldl);
    site_diag(q, rho, acc, diag, m);
    R nr = 0, ni = 0, dd = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      nr += q[k].re * rho[k].re + q[k].im * rho[k].im;
      ni += q[k].re * rho[k].im - q[k].im * rho[k].re;
      dd += q[k].re * q[k].re + q[k].im * q[k].im;
    }
#pragma unroll
    for (int off = K; off < WL; off <<= 1) {
      nr += __shfl_xor(nr, off, WL);
      ni += __shfl_xor(ni, off, WL);
      dd += __shfl_xor(dd, off, WL);
    }
    if (lane < K) { red[wave][lane][0] = nr; red[wave][lane][1] = ni; red[wave][lane][2] = dd; }
    __syncthreads();
    nr = 0; ni = 0; dd = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) { nr += red[w][kk][0]; ni += red[w][kk][1]; dd += red[w][kk][2]; }
    cx<R> a = dd > 0 ? cx<R>{nr / dd, ni / dd} : cx<R>{0, 0};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      dl[k] = dl[k] + a * rho[k];
      rho[k] = rho[k] - a * q[k];
    }
  }
  // 3. update
  cx<R> xs[12];
  load_cx<R, 12>(xt, V, TT, s, t, xs);
#pragma unroll
  for (int k = 0; k < 12; ++k) xs[k] = xs[k] + dl[k];
  store_cx<R, 12>(xt, V, TT, s, t, xs);
}

// ------------------------------------------------------------ wrappers ---
static inline int nsb_of(int V) { return (V + SPW - 1) / SPW; }

void fine_dslash(ddamg_ctx* c, const MV& x, const MV& y, const double* d_mu) {
  const int V = c->geom[0].V;
  const int nsb = nsb_of(V);
  dim3 grid(nsb * x.ntiles), blk(256);
  if (x.prec == P64)
    hipLaunchKernelGGL((k_dslash<double, false, 0>), grid, blk, 0, c->stream, x.as<double>(), y.as<double>(),
                       nullptr, c->d_U64, c->geom[0].d_nbr, d_mu, V, x.tile_reals(), c->diag, nsb);
  else
    hipLaunchKernelGGL((k_dslash<float, true, 0>), grid, blk, 0, c->stream, x.as<float>(), y.as<float>(), nullptr,
                       c->d_U32, c->geom[0].d_nbr, d_mu, V, x.tile_reals(), (float)c->diag, nsb);
  DD_HIP(hipGetLastError());
  c->st.fine_ops++;
}

void fine_residual(ddamg_ctx* c, const MV& b, const MV& x, const MV& r, const double* d_mu) {
  const int V = c->geom[0].V;
  const int nsb = nsb_of(V);
  dim3 grid(nsb * x.ntiles), blk(256);
  if (x.prec == P64)
    hipLaunchKernelGGL((k_dslash<double, false, 1>), grid, blk, 0, c->stream, x.as<double>(), r.as<double>(),
                       b.as<double>(), c->d_U64, c->geom[0].d_nbr, d_mu, V, x.tile_reals(), c->diag, nsb);
  else
    hipLaunchKernelGGL((k_dslash<float, true, 1>), grid, blk, 0, c->stream, x.as<float>(), r.as<float>(),
                       b.as<float>(), c->d_U32, c->geom[0].d_nbr, d_mu, V, x.tile_reals(), (float)c->diag, nsb);
  DD_HIP(hipGetLastError());
  c->st.fine_ops++;
}

void fine_masked(ddamg_ctx* c, const MV& x, const MV& y, int mode, int hopi) {
  DD_CHECK(x.prec == P64, DDAMG_EINVAL, "masked stencil is FP64 only");
  const int V = c->geom[0].V;
  const int nsb = nsb_of(V);
  dim3 grid(nsb * x.ntiles), blk(256);
  hipLaunchKernelGGL(k_dslash_masked, grid, blk, 0, c->stream, x.as<double>(), y.as<double>(), c->d_U64,
                     c->geom[0].d_nbr, V, x.tile_reals(), c->diag, nsb, c->geom[0].gsize, mode, hopi);
  DD_HIP(hipGetLastError());
}

template <typename R, bool C2, int K, int BS>
static void launch_sap(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, int colour) {
  const int nb = c->n_sap[colour];
  dim3 grid(nb * x.ntiles * (TT / K)), blk(BS * K);
  hipLaunchKernelGGL((k_sap_half<R, C2, K, BS>), grid, blk, 0, c->stream, f.as<R>(), x.as<R>(),
                     C2 ? (const void*)c->d_U32 : (const void*)c->d_U64, c->geom[0].d_nbr, d_mu,
                     c->d_sap_list[colour], c->geom[0].V, x.ntiles, x.tile_reals(), (R)c->diag,
                     c->p.sap_mr_iters);
  DD_HIP(hipGetLastError());
}

void sap_apply(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, const MV&) {
  mv_zero(c, x);
  const int BS = c->geom[0].gsize;
  for (int cyc = 0; cyc < c->p.sap_cycles; ++cyc)
    for (int colour = 0; colour < 2; ++colour) {
      if (x.prec == P64) {
        if (BS == 256) launch_sap<double, false, 1, 256>(c, f, x, d_mu, colour);
        else if (BS == 16) launch_sap<double, false, 4, 16>(c, f, x, d_mu, colour);
        else throw Error{DDAMG_EINVAL, "SAP block must have 16 or 256 sites"};
      } else {
        if (BS == 256) launch_sap<float, true, 2, 256>(c, f, x, d_mu, colour);
        else if (BS == 16) launch_sap<float, true, 8, 16>(c, f, x, d_mu, colour);
        else throw Error{DDAMG_EINVAL, "SAP block must have 16 or 256 sites"};
      }
    }
  c->st.sap_calls++;
}

}  // namespace ddamg
