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
#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"
#include "device.h"

namespace ddamg {

constexpr int TT = 8;                 // columns per tile
constexpr int SPW = 256 / TT;         // sites per 256-lane workgroup

// ---------------------------------------------------------------- links ---
// Link storage kinds:
//   LK_D  FP64 full 3x3, [mu][9][V] double2, boundary sign folded into the
//         t-links that cross the boundary;
//   LK_F  FP32 full 3x3, [mu][5][V] float4 (last half chunk unused), sign folded;
//   LK_C  FP32 2-row, [mu][3][V] float4, no sign (row 3 = conj(row1 x row2)
//         cannot carry one): the sign comes from bit 31 of the neighbour table.
constexpr int LK_D = 0, LK_F = 1, LK_C = 2;

template <typename R>
__device__ __forceinline__ void unpack_2row(float4 a, float4 b, float4 c, cx<R> (&u)[9]) {
  u[0] = {(R)a.x, (R)a.y}; u[1] = {(R)a.z, (R)a.w}; u[2] = {(R)b.x, (R)b.y};
  u[3] = {(R)b.z, (R)b.w}; u[4] = {(R)c.x, (R)c.y}; u[5] = {(R)c.z, (R)c.w};
  u[6] = conj_(u[1] * u[5] - u[2] * u[4]);
  u[7] = conj_(u[2] * u[3] - u[0] * u[5]);
  u[8] = conj_(u[0] * u[4] - u[1] * u[3]);
}

template <typename R, int LK>
__device__ __forceinline__ void load_link(const void* __restrict__ Uv, int mu, int s, int V, cx<R> (&u)[9]) {
  if constexpr (LK == LK_D) {
    const double2* U = reinterpret_cast<const double2*>(Uv) + (size_t)mu * 9 * V;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 c = U[(size_t)k * V + s];
      u[k] = {(R)c.x, (R)c.y};
    }
  } else if constexpr (LK == LK_F) {
    const float4* U = reinterpret_cast<const float4*>(Uv) + (size_t)mu * 5 * V;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float4 c = U[(size_t)k * V + s];
      u[2 * k] = {(R)c.x, (R)c.y};
      u[2 * k + 1] = {(R)c.z, (R)c.w};
    }
    float4 c = U[4 * (size_t)V + s];
    u[8] = {(R)c.x, (R)c.y};
  } else {
    const float4* U = reinterpret_cast<const float4*>(Uv) + (size_t)mu * 3 * V;
    unpack_2row(U[s], U[(size_t)V + s], U[2 * (size_t)V + s], u);
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

// Accumulate one hop term into acc (without the -1/2) from a loaded
// neighbour spinor p and link u; e is the neighbour-table entry (bit 31 =
// boundary sign).
template <int MU, bool FWD, bool TSIGN, typename R>
__device__ __forceinline__ void hop_apply(cx<R> (&acc)[12], const cx<R> (&p)[12], const cx<R> (&u)[9], int e) {
  cx<R> h[6];
  project<MU, FWD>(p, h);
  if (TSIGN && e < 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = (R)-1 * h[k];
  }
  cx<R> g[6];
  colour<FWD>(u, h, g);
  reconstruct<MU, FWD>(acc, g);
}

// One hop: the neighbour spinor and the link are requested together (the
// neighbour index is already in a register), so each hop costs one memory
// round trip.  `ld(h, nb, p)` loads the neighbour spinor of hop h (0..3
// forward, 4..7 backward) and returns false to drop the hop.
template <int MU, bool FWD, typename R, typename Loader, typename LinkLoader>
__device__ __forceinline__ void hop_one(cx<R> (&acc)[12], const LinkLoader& ll, const int (&e)[8], int s,
                                        Loader&& ld) {
  constexpr int H = FWD ? MU : 4 + MU;
  const int eh = e[H];
  int nb = eh & 0x7fffffff;
  int ls = FWD ? s : nb;
  // opaque to the optimiser: address arithmetic stays inside this hop instead
  // of being hoisted (64-bit addresses of all hops would not fit in registers)
  asm volatile("" : "+v"(nb), "+v"(ls));
  cx<R> p[12], u[9];
  if (!ld(H, nb, p)) return;
  ll(MU, ls, u);
  hop_apply<MU, FWD, LinkLoader::table_sign>(acc, p, u, eh);
}

template <typename R, int LK>
struct GlobalLinks {
  static constexpr bool table_sign = (LK == LK_C);
  const void* U;
  int V;
  __device__ __forceinline__ void operator()(int mu, int site, cx<R> (&u)[9]) const { load_link<R, LK>(U, mu, site, V, u); }
};

__device__ __forceinline__ void load_nbrs(const int* __restrict__ nbr, int V, int s, int (&e)[8]) {
#pragma unroll
  for (int h = 0; h < 8; ++h) e[h] = nbr[(size_t)h * V + s];
}

// The eight hops one after the other: a non-unrolled loop over a uniform
// switch keeps one neighbour spinor and one link live at a time.
template <typename R, int LK, typename Loader, typename LinkLoader>
__device__ __forceinline__ void all_hops_e(cx<R> (&acc)[12], const LinkLoader& U, const int (&e)[8], int s,
                                           Loader&& ld) {
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    // keeps the compiler from hoisting the loads of later hops (which would
    // hold all eight neighbour spinors in registers at once)
    asm volatile("" ::: "memory");
    switch (h) {
      case 0: hop_one<0, true, R>(acc, U, e, s, ld); break;
      case 1: hop_one<1, true, R>(acc, U, e, s, ld); break;
      case 2: hop_one<2, true, R>(acc, U, e, s, ld); break;
      case 3: hop_one<3, true, R>(acc, U, e, s, ld); break;
      case 4: hop_one<0, false, R>(acc, U, e, s, ld); break;
      case 5: hop_one<1, false, R>(acc, U, e, s, ld); break;
      case 6: hop_one<2, false, R>(acc, U, e, s, ld); break;
      default: hop_one<3, false, R>(acc, U, e, s, ld); break;
    }
  }
}

template <typename R, int LK, typename Loader, typename LinkLoader>
__device__ __forceinline__ void all_hops_ll(cx<R> (&acc)[12], const LinkLoader& U, const int* nbr, int V, int s,
                                            Loader&& ld) {
  int e[8];
  load_nbrs(nbr, V, s, e);
  all_hops_e<R, LK>(acc, U, e, s, ld);
}

template <typename R, int LK, typename Loader>
__device__ __forceinline__ void all_hops(cx<R> (&acc)[12], const void* U, const int* nbr, int V, int s, Loader&& ld) {
  all_hops_ll<R, LK>(acc, GlobalLinks<R, LK>{U, V}, nbr, V, s, ld);
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

// ------------------------------------------------------- clover term ---
// Site term with a clover (Sheikholeslami-Wohlert form, the reading taken for
// the twisted-mass clover operator): A(x) = (4 + m0) + c_sw (i/4)
// sum_{mu != nu} sigma_{mu nu} F_{mu nu}(x), sigma_{mu nu} = (i/2)[gamma_mu,
// gamma_nu], F = (Q - Q^dagger) / 8 with Q the four plaquettes at x.  In the
// chiral basis sigma_{kl} = -eps_{klm} diag(s_m, s_m) and sigma_{k4} =
// diag(s_k, -s_k) (s = Pauli matrices), so A has one 6x6 block per chirality
// c = +1 (spins 0, 1) and c = -1 (spins 2, 3), with row 3 * spin + colour:
//   A_c = (4 + m0) + c_sw (i/2) [[E3, E1 - i E2], [E1 + i E2, -E3]],
//   E1 = -F_yz + c F_xt,  E2 = F_xz + c F_yt,  E3 = -F_xy + c F_zt.
// Each Hermitian block is packed as its 6 real diagonal entries and the 15
// complex entries above the diagonal, row by row (36 reals); a site's 72 reals
// are stored as chunks of the working precision, [72 / RW][V] like the links.
constexpr int CLOV_REALS = 72;

__host__ __device__ constexpr int clov_upper(int i, int j) { return 6 + 2 * (i * (11 - i) / 2 + (j - i - 1)); }

// y = A(x) v at site s, streamed chunk by chunk (one chunk of the packed
// block live at a time; complexes never straddle a chunk since the 6 diagonal
// reals are an even count)
__device__ constexpr int CLOV_I[15] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4};
__device__ constexpr int CLOV_J[15] = {1, 2, 3, 4, 5, 2, 3, 4, 5, 3, 4, 5, 4, 5, 5};
template <typename R>
__device__ __forceinline__ void clover_mul(const R* __restrict__ clov, int V, int s, const cx<R> (&v)[12],
                                           cx<R> (&y)[12]) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW, NB = 36 / RW;
  const C* cc = reinterpret_cast<const C*>(clov);
#pragma unroll
  for (int k = 0; k < 12; ++k) y[k] = {0, 0};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int o = 6 * b;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const C ch = cc[(size_t)(b * NB + k) * V + s];
      R e[RW];
      if constexpr (RW == 2) {
        e[0] = ch.x;
        e[1] = ch.y;
      } else {
        e[0] = ch.x;
        e[1] = ch.y;
        e[2] = ch.z;
        e[3] = ch.w;
      }
#pragma unroll
      for (int h = 0; h < RW; h += 2) {
        const int r = k * RW + h;
        if (r < 6) {   // two real diagonal entries
          y[o + r] = y[o + r] + e[h] * v[o + r];
          y[o + r + 1] = y[o + r + 1] + e[h + 1] * v[o + r + 1];
        } else {       // A_ij (i < j): y_i += A_ij v_j, y_j += conj(A_ij) v_i
          const int q = (r - 6) / 2, i = CLOV_I[q], j = CLOV_J[q];
          const cx<R> u{e[h], e[h + 1]};
          cmac(y[o + i], u, v[o + j]);
          cmac_conj(y[o + j], u, v[o + i]);
        }
      }
    }
  }
}

// out = A(x) x + i mu gamma5 x - 1/2 acc
template <typename R>
__device__ __forceinline__ void site_diag_cl(cx<R> (&out)[12], const cx<R> (&x)[12], const cx<R> (&acc)[12],
                                             const R* __restrict__ clov, int V, int s, R mu) {
  clover_mul(clov, V, s, x, out);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const R g = k < 6 ? mu : -mu;
    out[k].re += -g * x[k].im - (R)0.5 * acc[k].re;
    out[k].im += g * x[k].re - (R)0.5 * acc[k].im;
  }
}

// The packed clover term of every site from the FP64 links (the boundary sign
// folded into them cancels: a closed loop crosses the time boundary an even
// number of times).  One thread per site; writes FP64 and FP32 copies.
__device__ __forceinline__ void m3_load(const double* __restrict__ U, int mu, int s, int V, cx<double> (&m)[9]) {
  const double2* u = reinterpret_cast<const double2*>(U);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 e = u[((size_t)mu * 9 + k) * V + s];
    m[k] = {e.x, e.y};
  }
}
__device__ __forceinline__ void m3_mul(const cx<double> (&a)[9], const cx<double> (&b)[9], bool da, bool db,
                                       cx<double> (&c)[9]) {
  // c = op(a) op(b), op = dagger when flagged
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> acc{0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const cx<double> x = da ? conj_(a[k * 3 + i]) : a[i * 3 + k];
        const cx<double> y = db ? conj_(b[j * 3 + k]) : b[k * 3 + j];
        acc = acc + x * y;
      }
      c[i * 3 + j] = acc;
    }
}

__global__ void __launch_bounds__(128) k_clover_build(const double* __restrict__ U, const int* __restrict__ nbr, int V,
                                                      double csw, double diag, double* __restrict__ out64,
                                                      float* __restrict__ out32) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  auto nb = [&](int h, int site) { return nbr[(size_t)h * V + site] & 0x7fffffff; };
  // F[p] for the planes xy, xz, xt, yz, yt, zt
  cx<double> F[6][9];
  const int PM[6] = {0, 0, 0, 1, 1, 2}, PN[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll 1
  for (int p = 0; p < 6; ++p) {
    const int mu = PM[p], nu = PN[p];
    const int xpm = nb(mu, s), xpn = nb(nu, s), xmm = nb(4 + mu, s), xmn = nb(4 + nu, s);
    const int xpn_mm = nb(4 + mu, xpn), xmm_mn = nb(4 + nu, xmm), xmn_pm = nb(mu, xmn);
    cx<double> A[9], B[9], T1[9], T2[9], Q[9];
    for (int k = 0; k < 9; ++k) Q[k] = {0, 0};
    // leaf (+mu, +nu, -mu, -nu): U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    m3_load(U, mu, s, V, A); m3_load(U, nu, xpm, V, B); m3_mul(A, B, false, false, T1);
    m3_load(U, mu, xpn, V, A); m3_mul(T1, A, false, true, T2);
    m3_load(U, nu, s, V, A); m3_mul(T2, A, false, true, T1);
    for (int k = 0; k < 9; ++k) Q[k] = Q[k] + T1[k];
    // leaf (+nu, -mu, -nu, +mu): U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    m3_load(U, nu, s, V, A); m3_load(U, mu, xpn_mm, V, B); m3_mul(A, B, false, true, T1);
    m3_load(U, nu, xmm, V, A); m3_mul(T1, A, false, true, T2);
    m3_load(U, mu, xmm, V, A); m3_mul(T2, A, false, false, T1);
    for (int k = 0; k < 9; ++k) Q[k] = Q[k] + T1[k];
    // leaf (-mu, -nu, +mu, +nu): U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    m3_load(U, mu, xmm, V, A); m3_load(U, nu, xmm_mn, V, B); m3_mul(A, B, true, true, T1);
    m3_load(U, mu, xmm_mn, V, A); m3_mul(T1, A, false, false, T2);
    m3_load(U, nu, xmn, V, A); m3_mul(T2, A, false, false, T1);
    for (int k = 0; k < 9; ++k) Q[k] = Q[k] + T1[k];
    // leaf (-nu, +mu, +nu, -mu): U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    m3_load(U, nu, xmn, V, A); m3_load(U, mu, xmn, V, B); m3_mul(A, B, true, false, T1);
    m3_load(U, nu, xmn_pm, V, A); m3_mul(T1, A, false, false, T2);
    m3_load(U, mu, s, V, A); m3_mul(T2, A, false, true, T1);
    for (int k = 0; k < 9; ++k) Q[k] = Q[k] + T1[k];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const cx<double> q = Q[i * 3 + j], qt = conj_(Q[j * 3 + i]);
        F[p][i * 3 + j] = {(q.re - qt.re) / 8.0, (q.im - qt.im) / 8.0};
      }
  }
  enum { XY = 0, XZ = 1, XT = 2, YZ = 3, YT = 4, ZT = 5 };
  for (int b = 0; b < 2; ++b) {
    const double c = b == 0 ? 1.0 : -1.0;
    cx<double> E1[9], E2[9], E3[9];
    for (int k = 0; k < 9; ++k) {
      E1[k] = (-1.0) * F[YZ][k] + c * F[XT][k];
      E2[k] = F[XZ][k] + c * F[YT][k];
      E3[k] = (-1.0) * F[XY][k] + c * F[ZT][k];
    }
    // the 6x6 block M = c_sw (i/2) [[E3, E1 - i E2], [E1 + i E2, -E3]] + diag
    auto elem = [&](int r, int q) {
      const int sr = r / 3, cr = r % 3, sq = q / 3, cq = q % 3, k = cr * 3 + cq;
      cx<double> m;
      if (sr == 0 && sq == 0) m = E3[k];
      else if (sr == 1 && sq == 1) m = {-E3[k].re, -E3[k].im};
      else if (sr == 0) m = E1[k] - mul_i(E2[k]);
      else m = E1[k] + mul_i(E2[k]);
      m = (0.5 * csw) * mul_i(m);
      if (r == q) m.re += diag;
      return m;
    };
    double a[36];
    for (int i = 0; i < 6; ++i) a[i] = elem(i, i).re;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        const cx<double> m = elem(i, j);
        a[clov_upper(i, j)] = m.re;
        a[clov_upper(i, j) + 1] = m.im;
      }
    for (int r = 0; r < 36; ++r) {
      const int g = 36 * b + r;
      out64[((size_t)(g / 2) * V + s) * 2 + g % 2] = a[r];
      out32[((size_t)(g / 4) * V + s) * 4 + g % 4] = (float)a[r];
    }
  }
}

// Links of the fine stencil: the forward links of the workgroup's site range
// staged in LDS (2-row FP32), the others (backward hops that leave the
// range) from global memory.
template <typename R, int LK, int RS>
struct RangeLinks {
  static constexpr bool table_sign = (LK == LK_C);
  const float4* ulds;
  const void* U;
  int V;
  int base;
  __device__ __forceinline__ void operator()(int mu, int site, cx<R> (&u)[9]) const {
    const unsigned l = (unsigned)(site - base);
    if (l < (unsigned)RS)
      unpack_2row(ulds[(mu * 3) * RS + l], ulds[(mu * 3 + 1) * RS + l], ulds[(mu * 3 + 2) * RS + l], u);
    else
      load_link<R, LK>(U, mu, site, V, u);
  }
};

// ------------------------------------------------------------ dslash ---
// The fine stencil, MODE 0: y = D x ; MODE 1: y = b - D x.
// With LDS staging: a workgroup owns RS consecutive sites of the
// internal (block-major) order for one column tile, copies their spinors
// into LDS once, and reads every neighbour that falls inside its range from
// LDS; only the neighbours outside the range go through L1/L2.  A site's
// spinor is then fetched from the cache hierarchy about 3.5 times instead of
// 9, which is what lets the kernel run at HBM speed rather than L2 speed.
template <typename R, int LK, int MODE, int RS, bool CL = false>
__global__ void __launch_bounds__(RS * TT) k_dslash_lds(const R* __restrict__ x, R* __restrict__ y,
                                                        const R* __restrict__ b, const void* __restrict__ U,
                                                        const int* __restrict__ nbr, const double* __restrict__ mu,
                                                        int V, size_t tile_reals, R diag, int nsb,
                                                        const int* __restrict__ order, const R* __restrict__ clov) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW, NCH = 24 / RW;
  __shared__ C lds[NCH * RS * TT];
  __shared__ float4 ulds[LK == LK_C ? 12 * RS : 1];
  const int t = threadIdx.x % TT, sl = threadIdx.x / TT;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = wg / nsb;
  // site ranges in storage order, or (order) sorted by time slice so that the
  // ranges in flight on an XCD form a thin t-slab whose neighbours stay in L2
  const int r0 = order ? order[wg % nsb] : (wg % nsb) * RS;
  const int s = r0 + sl;
  const bool active = s < V;
  const R* xt = x + (size_t)tile * tile_reals;
  const C* xc = reinterpret_cast<const C*>(xt);
  if (active) {
#pragma unroll
    for (int k = 0; k < NCH; ++k) lds[(k * RS + sl) * TT + t] = xc[((size_t)k * V + s) * TT + t];
  }
  if constexpr (LK == LK_C) {   // the range's forward links, each loaded once
    const float4* Ug = reinterpret_cast<const float4*>(U);
    for (int i = threadIdx.x; i < 12 * RS; i += RS * TT) {
      const int q = i / RS, l = i % RS;
      if (r0 + l < V) ulds[i] = Ug[(size_t)q * V + r0 + l];
    }
  }
  __syncthreads();
  if (!active) return;
  auto from_lds = [&](int l, cx<R>(&p)[12]) {
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const C v = lds[(k * RS + l) * TT + t];
      if constexpr (RW == 2) p[k] = {v.x, v.y};
      else { p[2 * k] = {v.x, v.y}; p[2 * k + 1] = {v.z, v.w}; }
    }
  };
  auto ld = [&](int, int nb, cx<R>(&p)[12]) {
    const unsigned l = (unsigned)(nb - r0);
    if (l < (unsigned)RS) from_lds((int)l, p);
    else load_cx<R, 12>(xt, V, TT, nb, t, p);
    return true;
  };
  cx<R> acc[12], out[12], xs[12];
  if constexpr (LK == LK_C) all_hops_ll<R, LK>(acc, RangeLinks<R, LK, RS>{ulds, U, V, r0}, nbr, V, s, ld);
  else all_hops<R, LK>(acc, U, nbr, V, s, ld);
  from_lds(sl, xs);
  if constexpr (CL) site_diag_cl(out, xs, acc, clov, V, s, (R)mu[tile * TT + t]);
  else site_diag(out, xs, acc, diag, (R)mu[tile * TT + t]);
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
                                                       int mode, int hopi, const double* __restrict__ clov) {
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
  all_hops<R, LK_D>(acc, U, nbr, V, s, ld);
  cx<R> out[12];
  cx<R> xs[12];
  load_cx<R, 12>(xt, V, TT, s, t, xs);
  if (mode == 0 && clov) {
    clover_mul(clov, V, s, xs, out);
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = out[k] - 0.5 * acc[k];
  } else {
    const double dg = mode == 0 ? diag : 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = dg * xs[k] - 0.5 * acc[k];
  }
  store_cx<R, 12>(y + (size_t)tile * tile_reals, V, TT, s, t, out);
}

// ---------------------------------------------------------------- SAP ---
// Links of the in-block MR steps: FP32 2-row links staged in LDS (ULDS; sign
// from the neighbour table), or read through the caches from global memory
// (FP32 2-row, FP32 full with the boundary sign folded in, or FP64 full).
template <typename R, int LK, int BS, bool ULDS>
struct SapLinks {
  static constexpr bool table_sign = (LK == LK_C);
  const float4* ulds;
  const void* U;
  int V;
  int base;
  __device__ __forceinline__ void operator()(int mu, int site, cx<R> (&u)[9]) const {
    if constexpr (LK == LK_C && ULDS) {
      const int l = site - base;
      unpack_2row(ulds[(mu * 3) * BS + l], ulds[(mu * 3 + 1) * BS + l], ulds[(mu * 3 + 2) * BS + l], u);
    } else {
      load_link<R, LK>(U, mu, site, V, u);
    }
  }
};

// The hops in direction MU that leave a SAP block of BS sites, from global
// memory: where the block is at least 2 sites wide in MU a site lies on at
// most one face, so the forward and backward cases share one load of the
// neighbour spinor and one of the link (the lanes of a wave take either;
// lanes inside the block idle).
template <int MU, int BS, typename R, int LK>
__device__ __forceinline__ void leaving_hops(cx<R> (&acc)[12], const int (&e)[8], int s, int blk,
                                             const R* __restrict__ xt, int V, int t, const GlobalLinks<R, LK>& gl) {
  const int ef = e[MU], eb = e[4 + MU];
  const int nf = ef & 0x7fffffff, nbk = eb & 0x7fffffff;
  const bool fo = nf / BS != blk, bo = nbk / BS != blk;
  if (!fo && !bo) return;
  int nb = fo ? nf : nbk;
  int ls = fo ? s : nbk;
  asm volatile("" : "+v"(nb), "+v"(ls));
  cx<R> p[12], u[9];
  load_cx<R, 12>(xt, V, TT, nb, t, p);
  gl(MU, ls, u);
  if (fo) hop_apply<MU, true, GlobalLinks<R, LK>::table_sign>(acc, p, u, ef);
  else hop_apply<MU, false, GlobalLinks<R, LK>::table_sign>(acc, p, u, eb);
  if (fo && bo) {   // both faces: a block one site wide in this direction
    int nb2 = nbk;
    asm volatile("" : "+v"(nb2));
    load_cx<R, 12>(xt, V, TT, nb2, t, p);
    gl(MU, nb2, u);
    hop_apply<MU, false, GlobalLinks<R, LK>::table_sign>(acc, p, u, eb);
  }
}

// One colour half-sweep of red-black SAP (paper section 2): every workgroup
// owns one block of that colour and K columns of a tile.
//   1. r = f - D x on the block's sites (full stencil, neighbours in global memory);
//   2. k_MR minimal-residual steps on D_BB (hops leaving the block dropped),
//      rho kept in LDS for the in-block neighbour exchange, the two inner
//      products per column reduced over the block with wavefront shuffles;
//   3. x += delta on the block.
// Blocks of one colour never neighbour each other, so the in-place update of
// x is race free.
// FP32 one-column form: at least 4 waves per SIMD (128 VGPRs, a few spilled),
// measured 3% faster on the whole solve than the 3 waves of 134 VGPRs; with a
// clover term 3 waves (3% faster than the 2 of the unconstrained build)
template <typename R, int LK, int K, int BS, bool ULDS, typename FIN = R, bool CL = false>
__global__ void __launch_bounds__(BS * K, (sizeof(R) == 4 && K == 1) ? (CL ? 3 : 4) : 1) k_sap_half(const FIN* __restrict__ f, R* __restrict__ x,
                                                     const void* __restrict__ U, const int* __restrict__ nbr,
                                                     const double* __restrict__ mu, const int* __restrict__ blist,
                                                     int V, int ntiles, size_t tile_reals, R diag, int mr_iters,
                                                     int x_zero, float fscale, const R* __restrict__ clov) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW;
  constexpr int NCH = 24 / RW;
  constexpr int NT = BS * K;
  constexpr int NSUB = TT / K;
  constexpr int NW = NT >= 64 ? NT / 64 : 1;
  constexpr int WL = NT >= 64 ? 64 : NT;    // lanes per wave actually used
  __shared__ C lds[NCH * BS * K];
  __shared__ R red[NW][K][3];
  __shared__ float4 ulds[(LK == LK_C && ULDS) ? 12 * BS : 1];

  // the NSUB workgroups of one block read the same 128-byte rows: keep them
  // on one XCD (shared L2) by numbering workgroups XCD-contiguously
  int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int sub = wg % NSUB;
  wg /= NSUB;
  const int tile = wg % ntiles;
  const int bi = wg / ntiles;
  const int kk = threadIdx.x % K, sl = threadIdx.x / K;
  const int t = sub * K + kk;
  const int blk = blist[bi];
  const int s = blk * BS + sl;
  const FIN* ft = f + (size_t)tile * tile_reals;   // FP16 right-hand sides: same layout, stored * 1/fscale
  auto load_f = [&](cx<R>(&v)[12]) {
    if constexpr (std::is_same<FIN, R>::value) load_cx<R, 12>(ft, V, TT, s, t, v);
    else load_cx_f16<12>(ft, V, TT, s, t, fscale, v);
  };
  R* xt = x + (size_t)tile * tile_reals;
  const R m = (R)mu[tile * TT + t];

  // 1. block residual.  x_zero 1: the first half-sweep of a call, x = 0
  // everywhere, so the residual is f; x_zero 2: the second one, x = 0 on the
  // blocks of this colour (not yet visited), so in-block hops and the site's
  // own x drop out and x is never read there.
  int e8[8];
  load_nbrs(nbr, V, s, e8);
  cx<R> rho[12], dl[12], q[12];
  if (x_zero == 1) {
    load_f(rho);
#pragma unroll
    for (int k = 0; k < 12; ++k) dl[k] = {0, 0};
  } else {
    auto ldg = [&](int, int nb, cx<R>(&p)[12]) {
      if (x_zero == 2 && nb / BS == blk) return false;
      load_cx<R, 12>(xt, V, TT, nb, t, p);
      return true;
    };
    cx<R> acc[12], xs[12], fs[12];
    if (x_zero == 2) {   // x is zero on the block: only the hops that leave it
      const GlobalLinks<R, LK> gl{U, V};
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
#pragma unroll 1
      for (int d = 0; d < 4; ++d) {
        asm volatile("" ::: "memory");
        switch (d) {
          case 0: leaving_hops<0, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          case 1: leaving_hops<1, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          case 2: leaving_hops<2, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          default: leaving_hops<3, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
        }
      }
    } else {
      all_hops_e<R, LK>(acc, GlobalLinks<R, LK>{U, V}, e8, s, ldg);
    }
    if (x_zero == 2) {
#pragma unroll
      for (int k = 0; k < 12; ++k) xs[k] = {0, 0};
    } else {
      load_cx<R, 12>(xt, V, TT, s, t, xs);
    }
    load_f(fs);
    if constexpr (CL) site_diag_cl(q, xs, acc, clov, V, s, m);
    else site_diag(q, xs, acc, diag, m);
#pragma unroll
    for (int k = 0; k < 12; ++k) { rho[k] = fs[k] - q[k]; dl[k] = {0, 0}; }
  }

  // the block's forward links (2-row FP32) staged in LDS for the MR steps;
  // the backward link of an in-block hop is the forward link of an in-block site
  if constexpr (LK == LK_C && ULDS) {
    const float4* Ug = reinterpret_cast<const float4*>(U);
    for (int i = threadIdx.x; i < 12 * BS; i += NT) {
      const int mu_q = i / BS, l = i % BS;
      ulds[i] = Ug[(size_t)mu_q * V + blk * BS + l];
    }
  }
  const SapLinks<R, LK, BS, ULDS> lll{ulds, U, V, blk * BS};

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
    all_hops_e<R, LK>(acc, lll, e8, s, ldl);
    if constexpr (CL) site_diag_cl(q, rho, acc, clov, V, s, m);
    else site_diag(q, rho, acc, diag, m);
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
  // 3. update (x = 0 on this block before the half-sweep: store the correction)
  if (x_zero) {
    store_cx<R, 12>(xt, V, TT, s, t, dl);
  } else {
    cx<R> xs[12];
    load_cx<R, 12>(xt, V, TT, s, t, xs);
#pragma unroll
    for (int k = 0; k < 12; ++k) xs[k] = xs[k] + dl[k];
    store_cx<R, 12>(xt, V, TT, s, t, xs);
  }
}

// --------------------------------------------------- odd-even SAP ---
// One colour half-sweep of red-black SAP whose block solves run MR on the
// odd-even reduced block systems (4^4 blocks, no clover term).  Inside a
// block every hop joins an even and an odd site, so with the site term
// D_ee, D_oo = (4 + m0) + i mu gamma5 and the hop parts D_eo, D_oe of D_BB:
//   S x_o = r_o - D_oe D_ee^{-1} r_e,   S = D_oo - D_oe D_ee^{-1} D_eo,
//   x_e = D_ee^{-1} (r_e - D_eo x_o).
// A workgroup of 128 K lanes owns one block and K columns of a tile (the
// column index runs fastest over the lanes, so the K lanes of one site touch
// adjacent bytes of every chunk); the lanes of site pair i own the i-th even
// and the i-th odd site of the block (local site 2i + b, with b fixing the
// parity), so neither half of an MR step leaves lanes idle.  Per
// step the even half gathers the odd in-block neighbours (D_eo, then
// D_ee^{-1}) and the odd half the even ones (D_oe), both from LDS; one
// reduction per column and block follows.  The first cycle of a call uses
// that x is zero as the plain kernel does (x_zero 1 and 2).
template <typename R, int LK, typename FIN = R, int K = 1>
__global__ void __launch_bounds__(128 * K, sizeof(R) == 4 ? 3 : 1) k_sap_oe(const FIN* __restrict__ f, R* __restrict__ x,
                                                const void* __restrict__ U, const int* __restrict__ nbr,
                                                const double* __restrict__ mu, const int* __restrict__ blist, int V,
                                                int ntiles, size_t tile_reals, R diag, int mr_iters, int x_zero,
                                                float fscale) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW, NCH = 24 / RW, BS = 256, NH = 128, NW = 2 * K;
  static_assert(TT % K == 0 && 64 % K == 0, "columns per workgroup");
  __shared__ C lodd[NCH * NH * K];    // odd-site vectors by parity index, [chunk][pair][column]
  __shared__ C leven[NCH * NH * K];   // even-site vectors
  __shared__ R red[NW][K][3];

  int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int kk = threadIdx.x % K;
  const int t = (wg % (TT / K)) * K + kk;
  wg /= TT / K;
  const int tile = wg % ntiles;
  const int bi = wg / ntiles;
  const int i = threadIdx.x / K;
  const int blk = blist[bi];
  const int par = ((i >> 1) ^ (i >> 3) ^ (i >> 5)) & 1;   // parity of y + z + t of local sites 2i, 2i+1
  const int se = blk * BS + 2 * i + par, so = blk * BS + 2 * i + (par ^ 1);
  const FIN* ft = f + (size_t)tile * tile_reals;
  R* xt = x + (size_t)tile * tile_reals;
  const R m = (R)mu[tile * TT + t];
  // D_ee^-1 = (diag - i mu gamma5) / (diag^2 + mu^2): one reciprocal per
  // lane instead of a division per component and call
  const R inv_den = R(1) / (diag * diag + m * m);
  const GlobalLinks<R, LK> gl{U, V};

  // (diag + i mu gamma5) v and its inverse, in place
  auto site_mul = [&](cx<R>(&v)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const R g = k < 6 ? m : -m;
      v[k] = {diag * v[k].re - g * v[k].im, diag * v[k].im + g * v[k].re};
    }
  };
  auto site_inv = [&](cx<R>(&v)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const R g = k < 6 ? -m : m;
      v[k] = {(diag * v[k].re - g * v[k].im) * inv_den, (diag * v[k].im + g * v[k].re) * inv_den};
    }
  };
  auto to_lds = [&](C* arr, const cx<R>(&v)[12]) {
    if constexpr (RW == 2) {
#pragma unroll
      for (int k = 0; k < NCH; ++k) arr[(k * NH + i) * K + kk] = C{v[k].re, v[k].im};
    } else {
#pragma unroll
      for (int k = 0; k < NCH; ++k)
        arr[(k * NH + i) * K + kk] = C{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
    }
  };
  auto from_lds = [&](const C* arr, int pi, cx<R>(&p)[12]) {
    if constexpr (RW == 2) {
#pragma unroll
      for (int k = 0; k < NCH; ++k) { const C c = arr[(k * NH + pi) * K + kk]; p[k] = {c.x, c.y}; }
    } else {
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        const C c = arr[(k * NH + pi) * K + kk];
        p[2 * k] = {c.x, c.y};
        p[2 * k + 1] = {c.z, c.w};
      }
    }
  };
  // in-block neighbours from an LDS array of the other parity; hops that
  // leave the block are dropped (Dirichlet block)
  auto gather = [&](const C* arr, const int (&e8)[8], int s, cx<R>(&acc)[12]) {
    auto ld = [&](int, int nb, cx<R>(&p)[12]) {
      if (nb / BS != blk) return false;
      from_lds(arr, (nb - blk * BS) >> 1, p);
      return true;
    };
    all_hops_e<R, LK>(acc, gl, e8, s, ld);
  };
  // block residual at one site, as in the plain kernel, except that the
  // right-hand side is loaded after the hops (it holds no registers while
  // they run)
  auto residual = [&](int s, const int (&e8)[8], cx<R>(&r)[12]) {
    auto load_f = [&]() {
      if constexpr (std::is_same<FIN, R>::value) load_cx<R, 12>(ft, V, TT, s, t, r);
      else load_cx_f16<12>(ft, V, TT, s, t, fscale, r);
    };
    if (x_zero == 1) {
      load_f();
      return;
    }
    auto ldg = [&](int, int nb, cx<R>(&p)[12]) {
      if (x_zero == 2 && nb / BS == blk) return false;
      load_cx<R, 12>(xt, V, TT, nb, t, p);
      return true;
    };
    cx<R> acc[12], xs[12], q[12];
    if (x_zero == 2) {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
#pragma unroll 1
      for (int d = 0; d < 4; ++d) {
        asm volatile("" ::: "memory");
        switch (d) {
          case 0: leaving_hops<0, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          case 1: leaving_hops<1, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          case 2: leaving_hops<2, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
          default: leaving_hops<3, BS, R, LK>(acc, e8, s, blk, xt, V, t, gl); break;
        }
      }
    } else {
      all_hops_e<R, LK>(acc, gl, e8, s, ldg);
    }
    asm volatile("" ::: "memory");
    if (x_zero == 2) {
#pragma unroll
      for (int k = 0; k < 12; ++k) xs[k] = {0, 0};
    } else {
      load_cx<R, 12>(xt, V, TT, s, t, xs);
    }
    site_diag(q, xs, acc, diag, m);
    load_f();
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] = r[k] - q[k];
  };

  int ee[8], eo[8];
  load_nbrs(nbr, V, se, ee);
  load_nbrs(nbr, V, so, eo);
  cx<R> rho[12], dl[12], q[12], acc[12];
  residual(se, ee, q);
  site_inv(q);                    // D_ee^{-1} r_e
  to_lds(leven, q);
  // second half sweep of the first cycle: x is zero on the block, so
  // D_ee^{-1} r_e waits where x_e goes for the back substitution (its block-
  // leaving hops are not gathered twice)
  if (x_zero == 2) store_cx<R, 12>(xt, V, TT, se, t, q);
  residual(so, eo, rho);
  to_lds(lodd, rho);   // parked in LDS (not yet in use) during the gather
  __syncthreads();
  // right-hand side of the Schur system: r_o - D_oe D_ee^{-1} r_e (D_oe = -1/2 hops)
  gather(leven, eo, so, acc);
  from_lds(lodd, i, rho);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    rho[k] = rho[k] + (R)0.5 * acc[k];
    dl[k] = {0, 0};
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int it = 0; it < mr_iters; ++it) {
    to_lds(lodd, rho);
    __syncthreads();
    // even half: u = D_ee^{-1} D_eo rho
    gather(lodd, ee, se, acc);
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = (R)-0.5 * acc[k];
    site_inv(q);
    to_lds(leven, q);
    __syncthreads();
    // odd half: q = S rho = D_oo rho - D_oe u (rho is read back from LDS,
    // where it waits unchanged since the step began, so that it holds no
    // registers through the two gathers)
    gather(leven, eo, so, acc);
    from_lds(lodd, i, rho);
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = rho[k];
    site_mul(q);
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = q[k] + (R)0.5 * acc[k];
    R nr = 0, ni = 0, dd = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      nr += q[k].re * rho[k].re + q[k].im * rho[k].im;
      ni += q[k].re * rho[k].im - q[k].im * rho[k].re;
      dd += q[k].re * q[k].re + q[k].im * q[k].im;
    }
#pragma unroll
    for (int off = K; off < 64; off <<= 1) {
      nr += __shfl_xor(nr, off, 64);
      ni += __shfl_xor(ni, off, 64);
      dd += __shfl_xor(dd, off, 64);
    }
    if (lane < K) { red[wave][lane][0] = nr; red[wave][lane][1] = ni; red[wave][lane][2] = dd; }
    __syncthreads();
    nr = 0;
    ni = 0;
    dd = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      nr += red[w][kk][0];
      ni += red[w][kk][1];
      dd += red[w][kk][2];
    }
    const cx<R> a = dd > 0 ? cx<R>{nr / dd, ni / dd} : cx<R>{0, 0};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      dl[k] = dl[k] + a * rho[k];
      rho[k] = rho[k] - a * q[k];
    }
  }
  // back substitution: x_e = D_ee^{-1} r_e - D_ee^{-1} D_eo x_o (the even
  // residual is recomputed unless it was kept: x is unchanged so far)
  to_lds(lodd, dl);
  // the even residual first (it reads x, which the barrier below then orders
  // before every write of x on the block), the gather after it, so that
  // neither holds registers during the other
  cx<R> xe[12];
  if (x_zero != 2) residual(se, ee, xe);
  __syncthreads();
  gather(lodd, ee, se, acc);
  if (x_zero == 2) {
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = (R)0.5 * acc[k];
    site_inv(q);
    load_cx<R, 12>(xt, V, TT, se, t, xe);
#pragma unroll
    for (int k = 0; k < 12; ++k) xe[k] = xe[k] + q[k];
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) xe[k] = xe[k] + (R)0.5 * acc[k];
    site_inv(xe);
  }
  from_lds(lodd, i, dl);   // x_o waited in LDS through the back substitution
  if (x_zero) {
    store_cx<R, 12>(xt, V, TT, so, t, dl);
    store_cx<R, 12>(xt, V, TT, se, t, xe);
  } else {
    cx<R> xs[12];
    load_cx<R, 12>(xt, V, TT, so, t, xs);
#pragma unroll
    for (int k = 0; k < 12; ++k) xs[k] = xs[k] + dl[k];
    store_cx<R, 12>(xt, V, TT, so, t, xs);
    load_cx<R, 12>(xt, V, TT, se, t, xs);
#pragma unroll
    for (int k = 0; k < 12; ++k) xs[k] = xs[k] + xe[k];
    store_cx<R, 12>(xt, V, TT, se, t, xs);
  }
}

// ------------------------------------------------------------ wrappers ---
static inline int nsb_of(int V) { return (V + SPW - 1) / SPW; }

// Sites per workgroup of the LDS-staged stencil: a tile-shape knob chosen by
// the autotuner (more sites = more neighbours served from LDS, fewer
// workgroups resident per CU).
// t-walk stencil (4^4 site blocks only): a workgroup owns one 4x4x4 xyz patch
// of a column of blocks along t and TC columns of a tile, and walks the whole
// time direction.  psi(t-1), psi(t), psi(t+1) of its own sites stay in
// registers (the t hops), the current slice is exchanged through LDS (x, y, z
// hops inside the patch); only the x, y, z faces of the patch are read from
// global memory, while the neighbouring patches, which walk in step, hold the
// same slice in L2.  Every spinor is thus read from HBM about once.
template <typename R, int LK, int MODE, int TC>
__global__ void __launch_bounds__(64 * TC) k_dslash_walk(const R* __restrict__ x, R* __restrict__ y,
                                                        const R* __restrict__ b, const void* __restrict__ U,
                                                        const int* __restrict__ nbr, const double* __restrict__ mu,
                                                        const int* __restrict__ walk_blk, int V, int nbt,
                                                        int npatch, int nseg, size_t tile_reals, R diag) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW, NCH = 24 / RW, NH = TT / TC;
  __shared__ C lds[NCH * 64 * TC];
  const int tc = threadIdx.x % TC, l = threadIdx.x / TC;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int patch = wg % npatch;
  const int seg = (wg / npatch) % nseg;     // segment of the t direction walked
  const int th = wg / npatch / nseg;        // tile * NH + half
  const int tile = th / NH, t = (th % NH) * TC + tc;
  const R* xt = x + (size_t)tile * tile_reals;
  R* yt = y + (size_t)tile * tile_reals;
  const int* wb = walk_blk + (size_t)patch * nbt;
  const int Lt = 4 * nbt, len = Lt / nseg, g0 = seg * len, g1 = g0 + len;
  auto site = [&](int gt) { return wb[gt >> 2] * 256 + l + 64 * (gt & 3); };
  const R m = (R)mu[tile * TT + t];
  cx<R> prev[12], cur[12], nxt[12];
  load_cx<R, 12>(xt, V, TT, site((g0 + Lt - 1) % Lt), t, prev);
  load_cx<R, 12>(xt, V, TT, site(g0), t, cur);
  load_cx<R, 12>(xt, V, TT, site((g0 + 1) % Lt), t, nxt);
  const GlobalLinks<R, LK> ll{U, V};
  for (int gt = g0; gt < g1; ++gt) {
    const int s = site(gt);
    const int base = s - l;                 // first site of this patch slice
    // the current slice of the patch to LDS
    if constexpr (RW == 2) {
#pragma unroll
      for (int k = 0; k < NCH; ++k) lds[(k * 64 + l) * TC + tc] = C{cur[k].re, cur[k].im};
    } else {
#pragma unroll
      for (int k = 0; k < NCH; ++k)
        lds[(k * 64 + l) * TC + tc] = C{cur[2 * k].re, cur[2 * k].im, cur[2 * k + 1].re, cur[2 * k + 1].im};
    }
    __syncthreads();
    int e8[8];
    load_nbrs(nbr, V, s, e8);
    auto ld = [&](int h, int nb, cx<R>(&p)[12]) {
      if (h == 3) {
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k] = nxt[k];
        return true;
      }
      if (h == 7) {
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k] = prev[k];
        return true;
      }
      const unsigned q = (unsigned)(nb - base);
      if (q < 64u) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
          const C v = lds[(k * 64 + (int)q) * TC + tc];
          if constexpr (RW == 2) p[k] = {v.x, v.y};
          else { p[2 * k] = {v.x, v.y}; p[2 * k + 1] = {v.z, v.w}; }
        }
      } else {
        load_cx<R, 12>(xt, V, TT, nb, t, p);
      }
      return true;
    };
    cx<R> acc[12], out[12];
    all_hops_e<R, LK>(acc, ll, e8, s, ld);
    site_diag(out, cur, acc, diag, m);
    if constexpr (MODE == 1) {
      cx<R> bs[12];
      load_cx<R, 12>(b + (size_t)tile * tile_reals, V, TT, s, t, bs);
#pragma unroll
      for (int k = 0; k < 12; ++k) out[k] = bs[k] - out[k];
    }
    store_cx<R, 12>(yt, V, TT, s, t, out);
    __syncthreads();   // the slice in LDS is replaced next step
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      prev[k] = cur[k];
      cur[k] = nxt[k];
    }
    if (gt + 1 < g1) load_cx<R, 12>(xt, V, TT, site((gt + 2) % Lt), t, nxt);
  }
}

template <typename R, int LK, int MODE, int TC>
static void launch_walk(ddamg_ctx* c, const MV& x, const MV& y, const MV* b, const double* d_mu, const void* U) {
  const LevelGeom& g = c->geom[0];
  const int npatch = (g.dims[0] / 4) * (g.dims[1] / 4) * (g.dims[2] / 4);
  const int nbt = g.dims[3] / 4;
  const int nseg = g.dims[3] % c->walk_seg == 0 ? c->walk_seg : 1;
  hipLaunchKernelGGL((k_dslash_walk<R, LK, MODE, TC>), dim3(npatch * nseg * x.ntiles * (TT / TC)), dim3(64 * TC), 0,
                     c->stream, x.as<R>(), y.as<R>(), b ? b->as<R>() : nullptr, U, g.d_nbr, d_mu, c->d_walk_blk, g.V,
                     nbt, npatch, nseg, x.tile_reals(), (R)c->diag);
}

bool dslash_walk_ok(ddamg_ctx* c) { return c->geom[0].gsize == 256 && c->d_walk_blk != nullptr; }

// Start sites of the RS-site ranges sorted by the time coordinate of their
// first site (stable, so block order is kept within a time slice).
static const int* dslash_order(ddamg_ctx* c, int RS) {
  int slot = 0;
  while ((16 << slot) < RS) ++slot;
  if (!c->d_dslash_order[slot]) {
    const LevelGeom& g = c->geom[0];
    const int nsb = (g.V + RS - 1) / RS;
    std::vector<std::pair<int, int>> key(nsb);
    for (int q = 0; q < nsb; ++q) {
      const int can = g.int2can[(size_t)q * RS];
      const int tcoord = can / (g.dims[0] * g.dims[1] * g.dims[2]);
      key[q] = {tcoord, q};
    }
    std::stable_sort(key.begin(), key.end());
    std::vector<int> r0(nsb);
    for (int q = 0; q < nsb; ++q) r0[q] = key[q].second * RS;
    int* d = (int*)c->pool.alloc(nsb * sizeof(int));
    DD_HIP(hipMemcpy(d, r0.data(), nsb * sizeof(int), hipMemcpyHostToDevice));
    c->d_dslash_order[slot] = d;
  }
  return c->d_dslash_order[slot];
}

template <typename R, int LK, int MODE, int RS, bool CL = false>
static void launch_rs(ddamg_ctx* c, const MV& x, const MV& y, const MV* b, const double* d_mu, const void* U) {
  const int V = c->geom[0].V;
  const int nsb = (V + RS - 1) / RS;
  const int* order = (c->dslash_order && !CL) ? dslash_order(c, RS) : nullptr;
  const R* clov = nullptr;
  if constexpr (CL) clov = (const R*)(sizeof(R) == 8 ? (const void*)c->d_clov64 : (const void*)c->d_clov32);
  hipLaunchKernelGGL((k_dslash_lds<R, LK, MODE, RS, CL>), dim3(nsb * x.ntiles), dim3(RS * TT), 0, c->stream,
                     x.as<R>(), y.as<R>(), b ? b->as<R>() : nullptr, U, c->geom[0].d_nbr, d_mu, V, x.tile_reals(),
                     (R)c->diag, nsb, order, clov);
}

bool dslash_rs_valid(int prec, int rs) {
  if (prec == P64) return rs == 16 || rs == 32 || rs == 64;
  return rs == 32 || rs == 64 || rs == 128;
}

template <int MODE, int LK>
static void launch_f32(ddamg_ctx* c, const MV& x, const MV& y, const MV* b, const double* d_mu, const void* U) {
  switch (c->dslash_rs[P32]) {
    case 32: launch_rs<float, LK, MODE, 32>(c, x, y, b, d_mu, U); break;
    case 64: launch_rs<float, LK, MODE, 64>(c, x, y, b, d_mu, U); break;
    default: launch_rs<float, LK, MODE, 128>(c, x, y, b, d_mu, U); break;
  }
}

template <int MODE>
static void launch_dslash(ddamg_ctx* c, const MV& x, const MV& y, const MV* b, const double* d_mu) {
  if (c->d_clov64) {   // with a clover term: the LDS-range kernel, 32 sites per workgroup, storage order
    if (x.prec == P64) launch_rs<double, LK_D, MODE, 32, true>(c, x, y, b, d_mu, c->d_U64);
    else if (c->fp32_links == 0) launch_rs<float, LK_F, MODE, 32, true>(c, x, y, b, d_mu, c->d_U32f);
    else launch_rs<float, LK_C, MODE, 32, true>(c, x, y, b, d_mu, c->d_U32);
    DD_HIP(hipGetLastError());
    c->st.fine_ops++;
    return;
  }
  if (c->dslash_order >= 2 && dslash_walk_ok(c)) {   // t-walk kernel, 4 or 8 columns per workgroup
    const bool tc8 = c->dslash_order == 3;
    if (x.prec == P64) {
      if (tc8) launch_walk<double, LK_D, MODE, 8>(c, x, y, b, d_mu, c->d_U64);
      else launch_walk<double, LK_D, MODE, 4>(c, x, y, b, d_mu, c->d_U64);
    } else if (c->fp32_links == 0) {
      if (tc8) launch_walk<float, LK_F, MODE, 8>(c, x, y, b, d_mu, c->d_U32f);
      else launch_walk<float, LK_F, MODE, 4>(c, x, y, b, d_mu, c->d_U32f);
    } else {
      if (tc8) launch_walk<float, LK_C, MODE, 8>(c, x, y, b, d_mu, c->d_U32);
      else launch_walk<float, LK_C, MODE, 4>(c, x, y, b, d_mu, c->d_U32);
    }
    DD_HIP(hipGetLastError());
    c->st.fine_ops++;
    return;
  }
  if (x.prec == P64) {
    switch (c->dslash_rs[P64]) {
      case 16: launch_rs<double, LK_D, MODE, 16>(c, x, y, b, d_mu, c->d_U64); break;
      case 32: launch_rs<double, LK_D, MODE, 32>(c, x, y, b, d_mu, c->d_U64); break;
      default: launch_rs<double, LK_D, MODE, 64>(c, x, y, b, d_mu, c->d_U64); break;
    }
  } else if (c->fp32_links == 0) {
    launch_f32<MODE, LK_F>(c, x, y, b, d_mu, c->d_U32f);
  } else {
    launch_f32<MODE, LK_C>(c, x, y, b, d_mu, c->d_U32);
  }
  DD_HIP(hipGetLastError());
  c->st.fine_ops++;
}

// Flavour coupling of the non-degenerate doublet operator: the two flavours
// of a doublet are the columns t and t^1 of one tile, so the partner of a
// 16-byte unit is the unit next to it (u ^ 1): y += sign * epsbar_col * x(partner).
template <typename C>
__global__ void k_flavour_mix(const C* __restrict__ x, C* __restrict__ y, const double* __restrict__ eps,
                              size_t nunits, int T, size_t tile_units, double sign) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const size_t col = (u / tile_units) * T + u % T;
    const C p = x[u ^ 1];
    C v = y[u];
    if constexpr (sizeof(v.x) == 8) {
      const double e = sign * eps[col];
      v.x += e * p.x; v.y += e * p.y;
    } else {
      const float e = (float)(sign * eps[col]);
      v.x += e * p.x; v.y += e * p.y; v.z += e * p.z; v.w += e * p.w;
    }
    y[u] = v;
  }
}

static void flavour_mix(ddamg_ctx* c, const MV& x, const MV& y, double sign) {
  DD_CHECK(x.prec == y.prec && x.reals() == y.reals() && x.T % 2 == 0, DDAMG_EINVAL, "flavour mix: shape");
  const size_t tile_units = (size_t)x.nchunk * x.nsites * x.T, nunits = tile_units * x.ntiles;
  size_t g = (nunits + 255) / 256;
  if (g > 65536) g = 65536;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_flavour_mix<double2>, dim3((unsigned)g), dim3(256), 0, c->stream, (const double2*)x.p,
                       (double2*)y.p, c->nd_eps, nunits, x.T, tile_units, sign);
  else if (x.prec == P32)
    hipLaunchKernelGGL(k_flavour_mix<float4>, dim3((unsigned)g), dim3(256), 0, c->stream, (const float4*)x.p,
                       (float4*)y.p, c->nd_eps, nunits, x.T, tile_units, sign);
  else
    throw Error{DDAMG_EINVAL, "flavour mix: FP64 or FP32"};
  DD_HIP(hipGetLastError());
}

// With c->nd_eps set (the outer solve of doublets, ddamg_apply_op_nd) the
// fine operator is the doublet operator: D(+-mubar) per column (the shifts
// carry the signs) and - epsbar tau1.
void fine_dslash(ddamg_ctx* c, const MV& x, const MV& y, const double* d_mu) {
  kernel_timing_begin(c, TIMED_DSLASH);
  launch_dslash<0>(c, x, y, nullptr, d_mu);
  kernel_timing_end(c, TIMED_DSLASH, x.ntiles);
  if (c->nd_eps) flavour_mix(c, x, y, -1.0);
}

void fine_residual(ddamg_ctx* c, const MV& b, const MV& x, const MV& r, const double* d_mu) {
  launch_dslash<1>(c, x, r, &b, d_mu);
  if (c->nd_eps) flavour_mix(c, x, r, +1.0);
}

void fine_masked(ddamg_ctx* c, const MV& x, const MV& y, int mode, int hopi) {
  DD_CHECK(x.prec == P64, DDAMG_EINVAL, "masked stencil is FP64 only");
  const int V = c->geom[0].V;
  const int nsb = nsb_of(V);
  dim3 grid(nsb * x.ntiles), blk(256);
  hipLaunchKernelGGL(k_dslash_masked, grid, blk, 0, c->stream, x.as<double>(), y.as<double>(), c->d_U64,
                     c->geom[0].d_nbr, V, x.tile_reals(), c->diag, nsb, c->geom[0].gsize, mode, hopi,
                     c->d_clov64);
  DD_HIP(hipGetLastError());
}

template <typename R, int LK, int K, int BS, bool ULDS = true, typename FIN = R, bool CL = false>
static void launch_sap(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, int colour, int x_zero) {
  const int nb = c->n_sap[colour];
  dim3 grid(nb * x.ntiles * (TT / K)), blk(BS * K);
  const void* U = LK == LK_C ? (const void*)c->d_U32 : LK == LK_F ? (const void*)c->d_U32f : (const void*)c->d_U64;
  const R* clov = nullptr;
  if constexpr (CL) clov = (const R*)(sizeof(R) == 8 ? (const void*)c->d_clov64 : (const void*)c->d_clov32);
  sap_timing_begin(c);
  hipLaunchKernelGGL((k_sap_half<R, LK, K, BS, ULDS, FIN, CL>), grid, blk, 0, c->stream, f.as<FIN>(), x.as<R>(), U,
                     c->geom[0].d_nbr, d_mu, c->d_sap_list[colour], c->geom[0].V, x.ntiles, x.tile_reals(),
                     (R)c->diag, c->p.sap_mr_iters, x_zero, (float)(1.0 / f.hscale), clov);
  DD_HIP(hipGetLastError());
  sap_timing_end(c, x.ntiles);
}

// SAP with a clover term: one column per workgroup on 4^4 blocks (full or
// 2-row FP32 links by the variant knob), the 16-site forms otherwise
static void sap_clover(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu) {
  const int BS = c->geom[0].gsize;
  const bool full = c->sap_variant == 3;
  DD_CHECK(BS == 256 || BS == 16, DDAMG_EINVAL, "SAP block must have 16 or 256 sites");
  for (int cyc = 0; cyc < c->p.sap_cycles; ++cyc)
    for (int colour = 0; colour < 2; ++colour) {
      const int xz = cyc == 0 ? 1 + colour : 0;
      if (f.prec == P16) {
        if (full) launch_sap<float, LK_F, 1, 256, false, _Float16, true>(c, f, x, d_mu, colour, xz);
        else launch_sap<float, LK_C, 1, 256, false, _Float16, true>(c, f, x, d_mu, colour, xz);
      } else if (x.prec == P64) {
        if (BS == 256) launch_sap<double, LK_D, 1, 256, true, double, true>(c, f, x, d_mu, colour, xz);
        else launch_sap<double, LK_D, 4, 16, true, double, true>(c, f, x, d_mu, colour, xz);
      } else if (BS == 256) {
        if (full) launch_sap<float, LK_F, 1, 256, false, float, true>(c, f, x, d_mu, colour, xz);
        else launch_sap<float, LK_C, 1, 256, false, float, true>(c, f, x, d_mu, colour, xz);
      } else {
        launch_sap<float, LK_C, 8, 16, true, float, true>(c, f, x, d_mu, colour, xz);
      }
    }
  c->st.sap_calls++;
}

// Columns per workgroup of the FP32 odd-even SAP kernel (LDS: 24.6 KB per
// column, so three workgroups of two columns fit a CU).
constexpr int SAP_OE_COLS = 2;

// x is fully written by the first cycle (each site belongs to one block of
// one colour), so it needs no clearing beforehand.
template <typename R, int LK, typename FIN = R>
static void launch_sap_oe(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, int colour, int x_zero) {
  constexpr int K = sizeof(R) == 4 ? SAP_OE_COLS : 1;   // FP64: the LDS of one column already limits residency
  const int nb = c->n_sap[colour];
  const void* U = LK == LK_C ? (const void*)c->d_U32 : LK == LK_F ? (const void*)c->d_U32f : (const void*)c->d_U64;
  sap_timing_begin(c);
  hipLaunchKernelGGL((k_sap_oe<R, LK, FIN, K>), dim3(nb * x.ntiles * (TT / K)), dim3(128 * K), 0, c->stream, f.as<FIN>(),
                     x.as<R>(), U, c->geom[0].d_nbr, d_mu, c->d_sap_list[colour], c->geom[0].V, x.ntiles,
                     x.tile_reals(), (R)c->diag, c->p.sap_mr_iters, x_zero, (float)(1.0 / f.hscale));
  DD_HIP(hipGetLastError());
  sap_timing_end(c, x.ntiles);
}

// SAP with odd-even reduced block solves (4^4 blocks).  FP32 takes the 2-row
// links: measured 5% faster here than full links, and fixed so that the
// kernel does not change with the SAP variant knob (which selects among
// forms that differ by a few percent and from run to run).
static void sap_oddeven(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu) {
  DD_CHECK(c->geom[0].gsize == 256 && !c->d_clov64, DDAMG_EINVAL, "odd-even SAP needs 4^4 blocks and no clover term");
  for (int cyc = 0; cyc < c->p.sap_cycles; ++cyc)
    for (int colour = 0; colour < 2; ++colour) {
      const int xz = cyc == 0 ? 1 + colour : 0;
      if (f.prec == P16) launch_sap_oe<float, LK_C, _Float16>(c, f, x, d_mu, colour, xz);
      else if (x.prec == P64) launch_sap_oe<double, LK_D>(c, f, x, d_mu, colour, xz);
      else launch_sap_oe<float, LK_C>(c, f, x, d_mu, colour, xz);
    }
  c->st.sap_calls++;
}

void build_clover(ddamg_ctx* c) {
  const int V = c->geom[0].V;
  c->d_clov64 = (double*)c->pool.alloc((size_t)V * CLOV_REALS * sizeof(double));
  c->d_clov32 = (float*)c->pool.alloc((size_t)V * CLOV_REALS * sizeof(float));
  hipLaunchKernelGGL(k_clover_build, dim3((V + 127) / 128), dim3(128), 0, c->stream, c->d_U64, c->geom[0].d_nbr, V,
                     c->p.csw, c->diag, c->d_clov64, c->d_clov32);
  DD_HIP(hipGetLastError());
}

bool sap_takes_f16(ddamg_ctx* c) {
  return c->geom[0].gsize == 256 && (c->p.sap_oddeven || c->sap_variant == 2 || c->sap_variant == 3);
}

void sap_apply(ddamg_ctx* c, const MV& f, const MV& x, const double* d_mu, const MV&) {
  const int BS = c->geom[0].gsize;
  if (c->d_clov64 || c->p.sap_oddeven) {
    DD_CHECK(f.prec != P16 || (x.prec == P32 && sap_takes_f16(c)), DDAMG_EINVAL,
             "SAP: FP16 input needs the FP32 one-column variant");
    if (c->p.sap_oddeven) sap_oddeven(c, f, x, d_mu);
    else sap_clover(c, f, x, d_mu);
    return;
  }
  if (f.prec == P16) {   // right-hand sides read straight from an FP16 Krylov basis
    DD_CHECK(x.prec == P32 && sap_takes_f16(c), DDAMG_EINVAL, "SAP: FP16 input needs the FP32 one-column variant");
    for (int cyc = 0; cyc < c->p.sap_cycles; ++cyc)
      for (int colour = 0; colour < 2; ++colour) {
        const int xz = cyc == 0 ? 1 + colour : 0;
        if (c->sap_variant == 3) launch_sap<float, LK_F, 1, 256, false, _Float16>(c, f, x, d_mu, colour, xz);
        else launch_sap<float, LK_C, 1, 256, false, _Float16>(c, f, x, d_mu, colour, xz);
      }
    c->st.sap_calls++;
    return;
  }
  for (int cyc = 0; cyc < c->p.sap_cycles; ++cyc)
    for (int colour = 0; colour < 2; ++colour) {
      // first cycle: x = 0 everywhere (colour 0), then on the colour-1 blocks
      const int xz = cyc == 0 ? 1 + colour : 0;
      if (x.prec == P64) {
        if (BS == 256) launch_sap<double, LK_D, 1, 256>(c, f, x, d_mu, colour, xz);
        else if (BS == 16) launch_sap<double, LK_D, 4, 16>(c, f, x, d_mu, colour, xz);
        else throw Error{DDAMG_EINVAL, "SAP block must have 16 or 256 sites"};
      } else {
        if (BS == 256 && c->sap_variant == 0) launch_sap<float, LK_C, 2, 256, true>(c, f, x, d_mu, colour, xz);
        else if (BS == 256 && c->sap_variant == 1) launch_sap<float, LK_C, 2, 256, false>(c, f, x, d_mu, colour, xz);
        else if (BS == 256 && c->sap_variant == 3) launch_sap<float, LK_F, 1, 256, false>(c, f, x, d_mu, colour, xz);
        else if (BS == 256) launch_sap<float, LK_C, 1, 256, false>(c, f, x, d_mu, colour, xz);
        else if (BS == 16) launch_sap<float, LK_C, 8, 16>(c, f, x, d_mu, colour, xz);
        else throw Error{DDAMG_EINVAL, "SAP block must have 16 or 256 sites"};
      }
    }
  c->st.sap_calls++;
}

}  // namespace ddamg
