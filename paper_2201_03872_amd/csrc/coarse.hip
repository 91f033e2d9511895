// Coarse-level kernels: restriction R = P^dag and prolongation P (paper
// section 2: built from approximate low modes, chirality preserving), the
// batched coarse stencil, and the pieces of the Galerkin setup.
//
// Coarse operator on level l+1 (blocks d x d, d = 2N):
//   y(a) = A0(a) x(a) + i dmu mu gamma5_c x(a) + sum_nu [F_nu(a) x(a+nu) + B_nu(a) x(a-nu)]
// Blocks are stored column-major, [site][slot][col j][row i], slot 0 = A0,
// 1+nu = F_nu, 5+nu = B_nu, so the lanes of one column j that own
// consecutive rows i read consecutive addresses, and one block element serves
// all T columns of the tile.
#include "common.h"
#include "device.h"

namespace ddamg {

constexpr int TC = 8;

static inline dim3 grid1(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

template <typename R>
__device__ __forceinline__ void store_one(R* __restrict__ tile, int nsites, int T, int s, int t, int k, cx<R> v) {
  constexpr int RW = Chunk<R>::RW;
  constexpr int CPC = RW / 2;
  R* q = tile + (((size_t)(k / CPC) * nsites + s) * T + t) * RW + (k % CPC) * 2;
  q[0] = v.re;
  q[1] = v.im;
}

// ------------------------------------------------------- coarse stencil ---
// MODE 0: full operator with twist; MODE 1: self block + hops internal to the
// grouping of this level (no twist); MODE 2: single hop `hopi` if it leaves
// the group of the site.  g5o = 1 (MODE 0 only) applies gamma5_c to the
// result: y = gamma5_c D_c(mu) x = gamma5_c D_c(0) x + i dmu mu x, the
// Hermitian form of the coarse operator shifted by i dmu mu.
template <typename R, int MODE>
__global__ void k_coarse(const R* __restrict__ x, R* __restrict__ y, const R* __restrict__ blk,
                         const int* __restrict__ nbr, const double* __restrict__ mu, double muf, int V, int d,
                         size_t tile_reals, int gsize, int hopi, int g5o) {
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int s = wg % V;
  const int tile = wg / V;
  const int i = threadIdx.x / TC, t = threadIdx.x % TC;
  const R* xt = x + (size_t)tile * tile_reals;
  cx<R> acc = {0, 0};
  const int g = s / gsize;
  for (int slot = 0; slot < 9; ++slot) {
    int nb = s;
    if (slot > 0) nb = nbr[(size_t)(slot - 1) * V + s];
    if constexpr (MODE == 1) {
      if (slot > 0 && nb / gsize != g) continue;
    } else if constexpr (MODE == 2) {
      if (slot != 1 + hopi || nb / gsize == g) continue;
    }
    const cx<R>* A = reinterpret_cast<const cx<R>*>(blk) + ((size_t)s * 9 + slot) * d * d + i;
    for (int j = 0; j < d; ++j) cmac(acc, A[(size_t)j * d], load_one(xt, V, TC, nb, t, j));
  }
  if constexpr (MODE == 0) {
    const cx<R> xs = load_one(xt, V, TC, s, t, i);
    const R g5 = i < d / 2 ? (R)1 : (R)-1;
    if (g5o) acc = g5 * acc;
    const R m = (R)(muf * mu[tile * TC + t]) * (g5o ? (R)1 : g5);
    acc.re -= m * xs.im;
    acc.im += m * xs.re;
  }
  store_one(y + (size_t)tile * tile_reals, V, TC, s, t, i, acc);
}

// ------------------------------------------------- MFMA coarse stencil ---
// The coarse stencil is a dense contraction per coarse site: Y (d x n) =
// sum_p A_p (d x d) X_{n_p} (d x n) over the 9 blocks, all complex.  In real
// form, with A' = [Re A | Im A] (d x 2d),
//   Re Y = A' [Re X; -Im X],   Im Y = A' [Im X; Re X],
// so one real product of depth 18d per site serves both halves.  It runs on
// v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation.  A workgroup
// owns one coarse site and up to four 16-column groups (two tiles each), so
// each block operand is loaded once for up to 64 columns; wave w computes the
// rows [16w, 16w+16) of both halves.  Lane layout of the instruction (A 16x32,
// B 32x16, D 16x16): lane l holds A[l%16][8(l/16)+e], B[8(l/16)+e][l%16]
// (e = 0..7) and D[4(l/16)+r][l%16] (r = 0..3).  The blocks are stored once in
// that A layout, [site][p][row tile][k step][lane][8], so every operand is one
// coalesced 16-byte load per lane.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// blocks (column-major complex [site][9][col][row], FP64) -> BF16 A layout
__global__ void k_blocks_bf16(const double* __restrict__ blk, bf16x8* __restrict__ out, int V, int d) {
  const int MT = d / 16, KS = d / 16;
  const size_t n = (size_t)V * 9 * MT * KS * 64;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const int lane = (int)(q % 64);
    const int ks = (int)((q / 64) % KS);
    const int mt = (int)((q / (64 * KS)) % MT);
    const size_t sp = q / ((size_t)64 * KS * MT);       // site * 9 + p
    const int i = 16 * mt + lane % 16;
    const int k0 = 32 * ks + 8 * (lane / 16);
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      const int jj = k < d ? k : k - d;
      const double* a = blk + ((sp * d + jj) * d + i) * 2;
      v[e] = (__bf16)(float)(k < d ? a[0] : a[1]);
    }
    out[q] = v;
  }
}

// GPW = 16-column groups per workgroup: 4 reads each block once for 64
// columns (large coarse lattices); 1 gives four times the workgroups, which
// wins on small coarse lattices where the stencil is latency bound.
template <int MFMA_GPW>
__global__ void __launch_bounds__(256) k_coarse_mfma(const float* __restrict__ x, float* __restrict__ y,
                                                     const bf16x8* __restrict__ A, const int* __restrict__ nbr,
                                                     const double* __restrict__ mu, double muf, int V, int d,
                                                     size_t tile_reals, int ntiles, int g5o) {
  const int ngrp = (ntiles + 1) / 2;
  const int nwgc = (ngrp + MFMA_GPW - 1) / MFMA_GPW;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int s = wg % V, g0 = (wg / V) * MFMA_GPW;
  const int ng = min(MFMA_GPW, ngrp - g0);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int KS = d / 16, MT = d / 16;
  const int j = lane % 16, kb = lane / 16;
  f32x4 accr[MFMA_GPW], acci[MFMA_GPW];
#pragma unroll
  for (int g = 0; g < MFMA_GPW; ++g) {
    accr[g] = f32x4{0, 0, 0, 0};
    acci[g] = f32x4{0, 0, 0, 0};
  }
  const bf16x8* Aw = A + ((size_t)s * 9 * MT + w) * KS * 64 + lane;
  for (int p = 0; p < 9; ++p) {
    const int nb = p == 0 ? s : nbr[(size_t)(p - 1) * V + s];
    const bf16x8* Ap = Aw + (size_t)p * MT * KS * 64;
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = 32 * ks + 8 * kb;
      const bool re_part = k0 < d;
      const int c0 = re_part ? k0 : k0 - d;
      const bf16x8 a = Ap[(size_t)ks * 64];
#pragma unroll
      for (int g = 0; g < MFMA_GPW; ++g) {
        if (g >= ng) break;
        const int col = 16 * (g0 + g) + j;
        const int tile = col / TC, t = col % TC;
        bf16x8 b1, b2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (tile < ntiles)
            v = *reinterpret_cast<const float4*>(x + (size_t)tile * tile_reals +
                                                 (((size_t)(c0 / 2 + q) * V + nb) * TC + t) * 4);
          // v = (re, im) of complex c0+2q and c0+2q+1
          if (re_part) {
            b1[2 * q] = (__bf16)v.x; b1[2 * q + 1] = (__bf16)v.z;
            b2[2 * q] = (__bf16)v.y; b2[2 * q + 1] = (__bf16)v.w;
          } else {
            b1[2 * q] = (__bf16)(-v.y); b1[2 * q + 1] = (__bf16)(-v.w);
            b2[2 * q] = (__bf16)v.x; b2[2 * q + 1] = (__bf16)v.z;
          }
        }
        accr[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, accr[g], 0, 0, 0);
        acci[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b2, acci[g], 0, 0, 0);
      }
    }
  }
  // twist i dmu mu gamma5_c on the site's own x (FP32), then store; with
  // g5o the rows of chirality -1 change sign and the twist becomes i dmu mu
  // on every row (the Hermitian form gamma5_c D_c)
#pragma unroll
  for (int g = 0; g < MFMA_GPW; ++g) {
    if (g >= ng) break;
    const int col = 16 * (g0 + g) + j;
    const int tile = col / TC, t = col % TC;
    if (tile >= ntiles) continue;
    const float m = (float)(muf * mu[tile * TC + t]);
    const float* xt = x + (size_t)tile * tile_reals;
    float* yt = y + (size_t)tile * tile_reals;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + 4 * kb + r;
      const size_t o = (((size_t)(i / 2) * V + s) * TC + t) * 4 + (i % 2) * 2;
      const float sg = (g5o && i >= d / 2) ? -1.f : 1.f;
      const float gm = (g5o || i < d / 2) ? m : -m;
      yt[o] = sg * accr[g][r] - gm * xt[o + 1];
      yt[o + 1] = sg * acci[g][r] + gm * xt[o];
    }
  }
  (void)nwgc;
}

// One tile (T = 8 columns) per workgroup, for coarse lattices where the
// batch in flight is a single tile: the real and imaginary halves of the 8
// columns share one 16-wide B operand, B = [[Re X, Im X]; [-Im X, Re X]]
// (rows 0..d-1 against Re A, d..2d-1 against Im A), so one MFMA per k step
// yields [Re Y | Im Y] and no lane computes a padded column.  The x of the
// site and its 8 neighbours (9 d complexes per column) is staged in LDS once
// by coalesced 16-byte loads and shared by the d/16 waves (each owns 16
// rows); the A operand streams from memory once per workgroup.
// XT = _Float16: x is an FP16 Krylov basis vector (the FP32 layout with
// 2-byte reals, entries stored times 1/xscale), read and scaled on the way
// into LDS, so the coarse GMRES with an FP16 basis needs no FP32 copy first.
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

template <int D, typename XT>
__global__ void __launch_bounds__(64 * (D / 16)) k_coarse_mfma_t1(const XT* __restrict__ x, float* __restrict__ y,
                                                                 const bf16x8* __restrict__ A,
                                                                 const int* __restrict__ nbr,
                                                                 const double* __restrict__ mu, double muf, int V,
                                                                 int g5o, float xscale) {
  constexpr int MT = D / 16, KS = D / 16, NCH = D / 2;   // row tiles, k steps, 2-complex chunks per site
  constexpr int NT = 64 * MT;
  __shared__ float4 xs[9][NCH][TC];
  const int s = xcd_remap(blockIdx.x, gridDim.x);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  int nb[9];
  nb[0] = s;
#pragma unroll
  for (int p = 1; p < 9; ++p) nb[p] = nbr[(size_t)(p - 1) * V + s];
  for (int q = threadIdx.x; q < 9 * NCH * TC; q += NT) {
    const int t = q % TC, c = (q / TC) % NCH, p = q / (TC * NCH);
    const size_t src = ((size_t)c * V + nb[p]) * TC + t;
    if constexpr (sizeof(XT) == 4) {
      xs[p][c][t] = reinterpret_cast<const float4*>(x)[src];
    } else {
      const h4v h = reinterpret_cast<const h4v*>(x)[src];
      xs[p][c][t] = float4{(float)h.x * xscale, (float)h.y * xscale, (float)h.z * xscale, (float)h.w * xscale};
    }
  }
  __syncthreads();
  const int n = lane % 16, kb = lane / 16;
  const int t = n % 8;
  const bool imh = n >= 8;
  f32x4 acc = f32x4{0, 0, 0, 0};
  const bf16x8* Aw = A + ((size_t)s * 9 * MT + w) * KS * 64 + lane;
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    bf16x8 a[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = Aw[((size_t)p * MT * KS + ks) * 64];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = 32 * ks + 8 * kb;          // 8 consecutive k of one half
      const bool re_part = k0 < D;
      const int c0 = re_part ? k0 : k0 - D;
      bf16x8 b;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = xs[p][c0 / 2 + q][t];   // (re, im) of complexes c0+2q, c0+2q+1
        float e0, e1;
        if (!imh) {   // real half of the output: [Re X; -Im X]
          e0 = re_part ? v.x : -v.y;
          e1 = re_part ? v.z : -v.w;
        } else {      // imaginary half: [Im X; Re X]
          e0 = re_part ? v.y : v.x;
          e1 = re_part ? v.w : v.z;
        }
        b[2 * q] = (__bf16)e0;
        b[2 * q + 1] = (__bf16)e1;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b, acc, 0, 0, 0);
    }
  }
  // lane (n, kb) holds rows 16w + 4kb + r of column t: the real part (n < 8)
  // or the imaginary part (n >= 8); twist i dmu mu gamma5_c on the site's own
  // x (with g5o: gamma5_c on the stencil part, i dmu mu on every row)
  const float m = (float)(muf * mu[t]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * w + 4 * kb + r;
    const float sg = (g5o && i >= D / 2) ? -1.f : 1.f;
    const float gm = (g5o || i < D / 2) ? m : -m;
    const float4 v = xs[0][i / 2][t];
    const float xr = (i % 2) ? v.z : v.x, xi = (i % 2) ? v.w : v.y;
    const size_t o = (((size_t)(i / 2) * V + s) * TC + t) * 4 + (i % 2) * 2;
    if (!imh) y[o] = sg * acc[r] - gm * xi;
    else y[o + 1] = sg * acc[r] + gm * xr;
  }
}

static bool use_mfma(ddamg_ctx* c, int level, const MV& x) {
  const int d = c->geom[level].dof;
  return x.prec == P32 && c->coarse_mfma && d % 16 == 0 && d <= 64 && c->coarse[level].d_blk16 != nullptr;
}

// The coarse stencil takes an FP16 input directly (one-tile MFMA form).
bool coarse_takes_f16(ddamg_ctx* c, int level, int ntiles) {
  const int d = c->geom[level].dof;
  return level > 0 && ntiles == 1 && c->coarse_mfma && d % 16 == 0 && d >= 16 && d <= 64 &&
         c->coarse[level].d_blk16 != nullptr;
}

static void coarse_apply_launch(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu);

void coarse_apply(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu) {
  if (level == 1) kernel_timing_begin(c, TIMED_COARSE1);
  coarse_apply_launch(c, level, x, y, d_mu);
  if (level == 1) kernel_timing_end(c, TIMED_COARSE1, x.ntiles);
}

static void coarse_apply_launch(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu) {
  const LevelGeom& g = c->geom[level];
  const int d = g.dof;
  DD_CHECK(x.prec != P16 || x.ntiles == 1, DDAMG_EINVAL, "coarse stencil: FP16 input needs one column tile");
  if ((use_mfma(c, level, x) || x.prec == P16) && x.ntiles == 1) {
    DD_CHECK(x.prec == P32 || (x.prec == P16 && y.prec == P32 && coarse_takes_f16(c, level, 1)), DDAMG_EINVAL,
             "coarse stencil: FP16 input needs the one-tile MFMA form");
    const bf16x8* A = (const bf16x8*)c->coarse[level].d_blk16;
    const double muf = c->coarse[level].mu_factor;
    const int g5o = c->coarse[level].g5out;
#define DD_T1(DD, XT, NTH)                                                                                     \
  hipLaunchKernelGGL((k_coarse_mfma_t1<DD, XT>), dim3(g.V), dim3(NTH), 0, c->stream, x.as<XT>(), y.as<float>(), A, \
                     g.d_nbr, d_mu, muf, g.V, g5o, xs)
    const float xs = x.prec == P16 ? (float)(1.0 / x.hscale) : 1.0f;
    if (x.prec == P16) {
      switch (d) {
        case 16: DD_T1(16, _Float16, 64); break;
        case 32: DD_T1(32, _Float16, 128); break;
        case 48: DD_T1(48, _Float16, 192); break;
        default: DD_T1(64, _Float16, 256); break;
      }
    } else {
      switch (d) {
        case 16: DD_T1(16, float, 64); break;
        case 32: DD_T1(32, float, 128); break;
        case 48: DD_T1(48, float, 192); break;
        default: DD_T1(64, float, 256); break;
      }
    }
#undef DD_T1
    DD_HIP(hipGetLastError());
    return;
  }
  if (use_mfma(c, level, x)) {
    const int ngrp = (x.ntiles + 1) / 2;
    if ((size_t)g.V * ngrp >= 8192) {
      const int nwgc = (ngrp + 3) / 4;
      hipLaunchKernelGGL(k_coarse_mfma<4>, dim3(g.V * nwgc), dim3(64 * (d / 16)), 0, c->stream, x.as<float>(),
                         y.as<float>(), (const bf16x8*)c->coarse[level].d_blk16, g.d_nbr, d_mu,
                         c->coarse[level].mu_factor, g.V, d, x.tile_reals(), x.ntiles, c->coarse[level].g5out);
    } else {
      hipLaunchKernelGGL(k_coarse_mfma<1>, dim3(g.V * ngrp), dim3(64 * (d / 16)), 0, c->stream, x.as<float>(),
                         y.as<float>(), (const bf16x8*)c->coarse[level].d_blk16, g.d_nbr, d_mu,
                         c->coarse[level].mu_factor, g.V, d, x.tile_reals(), x.ntiles, c->coarse[level].g5out);
    }
    DD_HIP(hipGetLastError());
    return;
  }
  dim3 grid(g.V * x.ntiles), blk(d * TC);
  if (x.prec == P64)
    hipLaunchKernelGGL((k_coarse<double, 0>), grid, blk, 0, c->stream, x.as<double>(), y.as<double>(),
                       c->coarse[level].d_blk64, g.d_nbr, d_mu, c->coarse[level].mu_factor, g.V, d, x.tile_reals(),
                       g.gsize, 0, c->coarse[level].g5out);
  else
    hipLaunchKernelGGL((k_coarse<float, 0>), grid, blk, 0, c->stream, x.as<float>(), y.as<float>(),
                       c->coarse[level].d_blk32, g.d_nbr, d_mu, c->coarse[level].mu_factor, g.V, d, x.tile_reals(),
                       g.gsize, 0, c->coarse[level].g5out);
  DD_HIP(hipGetLastError());
}

void coarse_masked(ddamg_ctx* c, int level, const MV& x, const MV& y, int mode, int hopi) {
  DD_CHECK(x.prec == P64, DDAMG_EINVAL, "masked coarse stencil is FP64 only");
  const LevelGeom& g = c->geom[level];
  const int d = g.dof;
  dim3 grid(g.V * x.ntiles), blk(d * TC);
  if (mode == 0)
    hipLaunchKernelGGL((k_coarse<double, 1>), grid, blk, 0, c->stream, x.as<double>(), y.as<double>(),
                       c->coarse[level].d_blk64, g.d_nbr, nullptr, 0.0, g.V, d, x.tile_reals(), g.gsize, 0, 0);
  else
    hipLaunchKernelGGL((k_coarse<double, 2>), grid, blk, 0, c->stream, x.as<double>(), y.as<double>(),
                       c->coarse[level].d_blk64, g.d_nbr, nullptr, 0.0, g.V, d, x.tile_reals(), g.gsize, hopi, 0);
  DD_HIP(hipGetLastError());
}

// ------------------------------------------------------------ restrict ---
// y(a)[s*N + j] = sum_{x in A_a} sum_{k of chirality s} conj(P[x][k][j]) x(x)[k]
// A dense contraction per aggregate, Y (2N x T) = P_a^dag X_a, streaming P
// once: one workgroup of four waves per (aggregate, tile); lane (s, j) of a
// wave owns row s*N + j for all T columns of the tile.  The aggregate's sites
// are taken in batches whose vector chunks (all T columns) the workgroup
// first stages in LDS with coalesced 16-byte loads (one distinct chunk per
// lane); the waves then take every fourth site of the batch, each lane
// reading its P entries from memory (consecutive j: coalesced) and the
// chunks of the site from LDS (the same address on every lane of a
// chirality: a broadcast), and their partial sums meet in LDS at the end.
template <typename R>
__global__ void __launch_bounds__(256) k_restrict(const R* __restrict__ x, R* __restrict__ y, const R* __restrict__ P,
                                                  const int* __restrict__ blk_of_coarse, int Vf, int dof, int N, int gs,
                                                  int Vc, size_t tile_f, size_t tile_c) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW;
  constexpr int CPC = RW / 2;
  constexpr int NWR = 4;          // waves per aggregate, each over every NWR-th site of a batch
  constexpr int XS = 1536;        // staged chunks (24 KB)
  __shared__ C xs[XS];
  __shared__ cx<R> part[NWR - 1][TC][64];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int a = wg % Vc, tile = wg / Vc;
  const int r = threadIdx.x % 64, wv = threadIdx.x / 64;
  const bool live = r < 2 * N;
  const int sig = live ? r / N : 0, j = live ? r % N : 0;
  const int h = dof / 2;
  const int b = blk_of_coarse[a];
  const C* xt = reinterpret_cast<const C*>(x + (size_t)tile * tile_f);
  const cx<R>* Pc = reinterpret_cast<const cx<R>*>(P);
  const int nchs = dof / CPC;                 // chunks per site
  const int per_site = nchs * TC;             // staged units per site
  const int sb = XS / per_site;               // sites per batch
  cx<R> acc[TC];
#pragma unroll
  for (int t = 0; t < TC; ++t) acc[t] = {0, 0};
  const int c0 = sig * h / CPC, nch = h / CPC;
  for (int q0 = 0; q0 < gs; q0 += sb) {
    const int nsb = gs - q0 < sb ? gs - q0 : sb;
    // stage: unit u = (chunk ch, site qq, column t), site fastest after t so
    // that consecutive lanes read consecutive 16-byte chunks of memory
    for (int u = threadIdx.x; u < nsb * per_site; u += blockDim.x) {
      const int t = u % TC, rest = u / TC;
      const int qq = rest % nsb, ch = rest / nsb;
      xs[(qq * nchs + ch) * TC + t] = xt[((size_t)ch * Vf + (size_t)b * gs + q0 + qq) * TC + t];
    }
    __syncthreads();
    for (int qq = wv; qq < nsb; qq += NWR) {
      const int s = b * gs + q0 + qq;
      for (int cc = 0; cc < nch; ++cc) {
        const int ch = c0 + cc;
        cx<R> pv[CPC];
#pragma unroll
        for (int e = 0; e < CPC; ++e) pv[e] = Pc[((size_t)s * dof + ch * CPC + e) * N + j];
        const C* xc = xs + (qq * nchs + ch) * TC;
#pragma unroll
        for (int t = 0; t < TC; ++t) {
          const C v = xc[t];
          if constexpr (CPC == 1) {
            cmac_conj(acc[t], pv[0], cx<R>{v.x, v.y});
          } else {
            cmac_conj(acc[t], pv[0], cx<R>{v.x, v.y});
            cmac_conj(acc[t], pv[1], cx<R>{v.z, v.w});
          }
        }
      }
    }
    __syncthreads();
  }
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < TC; ++t) part[wv - 1][t][r] = acc[t];
  }
  __syncthreads();
  if (wv > 0 || !live) return;
#pragma unroll
  for (int t = 0; t < TC; ++t)
#pragma unroll
    for (int w = 0; w < NWR - 1; ++w) acc[t] = acc[t] + part[w][t][r];
  R* yt = y + (size_t)tile * tile_c;
#pragma unroll
  for (int t = 0; t < TC; ++t) store_one(yt, Vc, TC, a, t, r, acc[t]);
}

// ---- FP16 P (transfer_fp16, level 0): layout P16T[k/2][q][site][4] with
// q = (k % 2) * N/4 + j/4 and 4 consecutive j per 16-byte chunk, so that the
// lanes of consecutive sites read consecutive chunks (prolongation) and the
// lanes j of one site read 4-byte entries of a few chunks (restriction).
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ size_t p16t_index(int k, int j, int s, int N, int Vf) {
  return ((((size_t)(k / 2) * (N / 2) + (k % 2) * (N / 4) + j / 4) * Vf + s) * 4 + j % 4);
}

__global__ void k_to_p16t(const double* __restrict__ P, h2v* __restrict__ out, int Vf, int dof, int N) {
  const size_t total = (size_t)Vf * dof * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % N);
    const int k = (int)((i / N) % dof);
    const int s = (int)(i / ((size_t)N * dof));
    h2v v;
    v.x = (_Float16)P[i * 2];
    v.y = (_Float16)P[i * 2 + 1];
    out[p16t_index(k, j, s, N, Vf)] = v;
  }
}

// The restriction of k_restrict<float> with P read from P16T.
__global__ void __launch_bounds__(256) k_restrict16(const float* __restrict__ x, float* __restrict__ y,
                                                    const h2v* __restrict__ P, const int* __restrict__ blk_of_coarse,
                                                    int Vf, int dof, int N, int gs, int Vc, size_t tile_f,
                                                    size_t tile_c) {
  using C = float4;
  constexpr int NWR = 4;
  constexpr int XS = 1536;
  __shared__ C xs[XS];
  __shared__ cx<float> part[NWR - 1][TC][64];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int a = wg % Vc, tile = wg / Vc;
  const int r = threadIdx.x % 64, wv = threadIdx.x / 64;
  const bool live = r < 2 * N;
  const int sig = live ? r / N : 0, j = live ? r % N : 0;
  const int h = dof / 2;
  const int b = blk_of_coarse[a];
  const C* xt = reinterpret_cast<const C*>(x + (size_t)tile * tile_f);
  const int nchs = dof / 2;
  const int per_site = nchs * TC;
  const int sb = XS / per_site;
  cx<float> acc[TC];
#pragma unroll
  for (int t = 0; t < TC; ++t) acc[t] = {0, 0};
  const int c0 = sig * h / 2, nch = h / 2;
  for (int q0 = 0; q0 < gs; q0 += sb) {
    const int nsb = gs - q0 < sb ? gs - q0 : sb;
    for (int u = threadIdx.x; u < nsb * per_site; u += blockDim.x) {
      const int t = u % TC, rest = u / TC;
      const int qq = rest % nsb, ch = rest / nsb;
      xs[(qq * nchs + ch) * TC + t] = xt[((size_t)ch * Vf + (size_t)b * gs + q0 + qq) * TC + t];
    }
    __syncthreads();
    for (int qq = wv; qq < nsb; qq += NWR) {
      const int s = b * gs + q0 + qq;
      for (int cc = 0; cc < nch; ++cc) {
        const int ch = c0 + cc;
        cx<float> pv[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const h2v v = P[p16t_index(ch * 2 + e, j, s, N, Vf)];
          pv[e] = cx<float>{(float)v.x, (float)v.y};
        }
        const C* xc = xs + (qq * nchs + ch) * TC;
#pragma unroll
        for (int t = 0; t < TC; ++t) {
          const C v = xc[t];
          cmac_conj(acc[t], pv[0], cx<float>{v.x, v.y});
          cmac_conj(acc[t], pv[1], cx<float>{v.z, v.w});
        }
      }
    }
    __syncthreads();
  }
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < TC; ++t) part[wv - 1][t][r] = acc[t];
  }
  __syncthreads();
  if (wv > 0 || !live) return;
#pragma unroll
  for (int t = 0; t < TC; ++t)
#pragma unroll
    for (int w = 0; w < NWR - 1; ++w) acc[t] = acc[t] + part[w][t][r];
  float* yt = y + (size_t)tile * tile_c;
#pragma unroll
  for (int t = 0; t < TC; ++t) store_one(yt, Vc, TC, a, t, r, acc[t]);
}

// y(x)[k] (+)= sum_j P[x][k][j] xc(a(x))[s(k)*N + j] with P from P16T: one
// lane per (row pair c, fine site) computing both rows of the pair for the T
// columns of a tile.  Each wave's 64 sites lie in one aggregate (aggregates of
// a multiple of 64 sites), whose coarse vector half (N complexes x T columns)
// the wave stages in LDS; the lane then streams its 2 x N/4 chunks of P
// (consecutive sites: consecutive chunks) and reads the coarse values from
// LDS (one address per wave: a broadcast).
template <int NN>
__global__ void __launch_bounds__(256) k_prolong16(const float* __restrict__ xc, float* __restrict__ y,
                                                   const h2v* __restrict__ P, const int* __restrict__ coarse_of_blk,
                                                   int Vf, int dof, int gs, int Vc, size_t tile_f, size_t tile_c,
                                                   int accumulate) {
  __shared__ float4 xs[4][NN / 2][TC];   // per wave: pairs of complexes (j, j+1) per column
  const int npair = dof / 2;
  const int nsblk = Vf / 256;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int sbk = blk % nsblk;
  const int c = (blk / nsblk) % npair;
  const int tile = blk / (nsblk * npair);
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int s = sbk * 256 + threadIdx.x;
  const int a = coarse_of_blk[(sbk * 256 + wv * 64) / gs];
  const int sig = (2 * c) / (dof / 2);
  const float4* ct = reinterpret_cast<const float4*>(xc + (size_t)tile * tile_c);
  for (int u = lane; u < (NN / 2) * TC; u += 64) {
    const int t = u % TC, jp = u / TC;
    xs[wv][jp][t] = ct[((size_t)(sig * (NN / 2) + jp) * Vc + a) * TC + t];
  }
  __syncthreads();
  cx<float> acc[2][TC];
#pragma unroll
  for (int rr = 0; rr < 2; ++rr)
#pragma unroll
    for (int t = 0; t < TC; ++t) acc[rr][t] = {0, 0};
  const uint4* Pc = reinterpret_cast<const uint4*>(P);
#pragma unroll
  for (int rr = 0; rr < 2; ++rr) {
#pragma unroll 3
    for (int q4 = 0; q4 < NN / 4; ++q4) {
      const uint4 raw = Pc[((size_t)c * (NN / 2) + rr * (NN / 4) + q4) * Vf + s];
      const h2v* pe = reinterpret_cast<const h2v*>(&raw);
#pragma unroll
      for (int e = 0; e < 4; e += 2) {
        const cx<float> p0{(float)pe[e].x, (float)pe[e].y}, p1{(float)pe[e + 1].x, (float)pe[e + 1].y};
        const int jp = (q4 * 4 + e) / 2;
#pragma unroll
        for (int t = 0; t < TC; ++t) {
          const float4 v = xs[wv][jp][t];
          cmac(acc[rr][t], p0, cx<float>{v.x, v.y});
          cmac(acc[rr][t], p1, cx<float>{v.z, v.w});
        }
      }
    }
  }
  float4* yt = reinterpret_cast<float4*>(y + (size_t)tile * tile_f);
#pragma unroll
  for (int t = 0; t < TC; ++t) {
    float4* out = yt + ((size_t)c * Vf + s) * TC + t;
    float4 o = {acc[0][t].re, acc[0][t].im, acc[1][t].re, acc[1][t].im};
    if (accumulate) {
      const float4 p = *out;
      o.x += p.x; o.y += p.y; o.z += p.z; o.w += p.w;
    }
    *out = o;
  }
}

void convert_P16T(ddamg_ctx* c, int level) {
  const LevelGeom& g = c->geom[level];
  const size_t n = (size_t)g.V * g.dof * c->tr[level].N;
  hipLaunchKernelGGL(k_to_p16t, grid1(n), dim3(256), 0, c->stream, c->tr[level].d_P64, (h2v*)c->tr[level].d_P16T,
                     g.V, g.dof, c->tr[level].N);
  DD_HIP(hipGetLastError());
}

void restrict_mv(ddamg_ctx* c, int level, const MV& x, const MV& y) {
  const LevelGeom& gf = c->geom[level];
  const LevelGeom& gc = c->geom[level + 1];
  const int N = c->tr[level].N;
  DD_CHECK(x.prec == y.prec && x.ntiles == y.ntiles && x.nsites == gf.V && y.nsites == gc.V, DDAMG_EINVAL,
           "restrict: shape");
  DD_CHECK(2 * N <= 64 && gf.dof % (2 * reals_per_chunk(x.prec) / 2) == 0, DDAMG_EINVAL,
           "restrict: at most 32 test vectors, chirality halves of whole chunks");
  dim3 grid(gc.V * x.ntiles), blk(256);
  if (level == 0) kernel_timing_begin(c, TIMED_RESTRICT0);
  if (x.prec == P64)
    hipLaunchKernelGGL(k_restrict<double>, grid, blk, 0, c->stream, x.as<double>(), y.as<double>(), c->tr[level].d_P64,
                       gc.d_blk_of_coarse, gf.V, gf.dof, N, gf.gsize, gc.V, x.tile_reals(), y.tile_reals());
  else if (c->tr[level].d_P16T)
    hipLaunchKernelGGL(k_restrict16, grid, blk, 0, c->stream, x.as<float>(), y.as<float>(),
                       (const h2v*)c->tr[level].d_P16T, gc.d_blk_of_coarse, gf.V, gf.dof, N, gf.gsize, gc.V,
                       x.tile_reals(), y.tile_reals());
  else
    hipLaunchKernelGGL(k_restrict<float>, grid, blk, 0, c->stream, x.as<float>(), y.as<float>(), c->tr[level].d_P32,
                       gc.d_blk_of_coarse, gf.V, gf.dof, N, gf.gsize, gc.V, x.tile_reals(), y.tile_reals());
  DD_HIP(hipGetLastError());
  if (level == 0) kernel_timing_end(c, TIMED_RESTRICT0, x.ntiles);
}

// ------------------------------------------------------------- prolong ---
// y(x)[k] (+)= sum_j P[x][k][j] xc(a(x))[s(k)*N + j]
// One lane per (fine site, column of the tile) computing every component of
// its site.  The lane first holds its column of the coarse vector (2N
// complexes; the T lanes of a site read one line per chunk), then walks its
// P rows in storage order, each row (N complexes) loaded as consecutive
// 16-byte chunks (the same for the T lanes of a site), so every P line is used
// up at once instead of being revisited from the caches; its output chunks of
// consecutive columns form one line per chunk.  DOF is the fine dof (12 on the
// fine level, 2N' on a coarse one), NN the number N of test vectors.
template <typename R, int DOF, int NN>
__global__ void __launch_bounds__(256) k_prolong(const R* __restrict__ xc, R* __restrict__ y, const R* __restrict__ P,
                                                 const int* __restrict__ coarse_of_blk, int Vf, int gs, int Vc,
                                                 size_t tile_f, size_t tile_c, int accumulate, int ntiles) {
  using C = typename Chunk<R>::type;
  constexpr int RW = Chunk<R>::RW;
  constexpr int CPC = RW / 2;
  constexpr int H = DOF / 2;
  constexpr int NCH = NN / CPC;    // chunks of a P row and of one chirality of the coarse vector
  const size_t lane_id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int t = (int)(lane_id % TC);
  const size_t st = lane_id / TC;
  const int s = (int)(st % Vf), tile = (int)(st / Vf);
  if (tile >= ntiles) return;
  const int a = coarse_of_blk[s / gs];
  const C* ct = reinterpret_cast<const C*>(xc + (size_t)tile * tile_c);
  C* yt = reinterpret_cast<C*>(y + (size_t)tile * tile_f);
  const C* Ps = reinterpret_cast<const C*>(P + (size_t)s * DOF * NN * 2);
  C xv[2][NCH];
#pragma unroll
  for (int sg = 0; sg < 2; ++sg)
#pragma unroll
    for (int q = 0; q < NCH; ++q) xv[sg][q] = ct[((size_t)(sg * NCH + q) * Vc + a) * TC + t];
  cx<R> acc[CPC];
#pragma unroll
  for (int k = 0; k < DOF; ++k) {
    const int sg = k / H;
    cx<R> v = {0, 0};
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const C pv = Ps[(size_t)k * NCH + q];
      const C x = xv[sg][q];
      if constexpr (CPC == 1) {
        cmac(v, cx<R>{pv.x, pv.y}, cx<R>{x.x, x.y});
      } else {
        cmac(v, cx<R>{pv.x, pv.y}, cx<R>{x.x, x.y});
        cmac(v, cx<R>{pv.z, pv.w}, cx<R>{x.z, x.w});
      }
    }
    acc[k % CPC] = v;
    if (k % CPC == CPC - 1) {
      C* out = yt + ((size_t)(k / CPC) * Vf + s) * TC + t;
      if constexpr (CPC == 1) {
        if (accumulate) { const C o = *out; acc[0].re += o.x; acc[0].im += o.y; }
        *out = C{acc[0].re, acc[0].im};
      } else {
        if (accumulate) {
          const C o = *out;
          acc[0].re += o.x; acc[0].im += o.y; acc[1].re += o.z; acc[1].im += o.w;
        }
        *out = C{acc[0].re, acc[0].im, acc[1].re, acc[1].im};
      }
    }
  }
}

template <typename R, int DOF, int NN>
static void launch_prolong(ddamg_ctx* c, const R* xc, R* y, const R* P, const LevelGeom& gf, const LevelGeom& gc,
                           size_t tile_f, size_t tile_c, int accumulate, int ntiles) {
  const size_t lanes = (size_t)gf.V * TC * ntiles;
  hipLaunchKernelGGL((k_prolong<R, DOF, NN>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, c->stream, xc, y,
                     P, gf.d_coarse_of_blk, gf.V, gf.gsize, gc.V, tile_f, tile_c, accumulate, ntiles);
}

// the fine dof and N of every level transition the library builds: the
// fine level (12) to N = 4..32, and coarse levels (2N') to N = 4..32
template <typename R>
static void prolong_dispatch(ddamg_ctx* c, const R* xc, R* y, const R* P, const LevelGeom& gf, const LevelGeom& gc,
                             int N, size_t tile_f, size_t tile_c, int accumulate, int ntiles) {
#define DD_PROLONG_N(D)                                                                                   \
  switch (N) {                                                                                           \
    case 2: launch_prolong<R, D, 2>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return;   \
    case 4: launch_prolong<R, D, 4>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return;   \
    case 6: launch_prolong<R, D, 6>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return;   \
    case 8: launch_prolong<R, D, 8>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return;   \
    case 12: launch_prolong<R, D, 12>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return; \
    case 16: launch_prolong<R, D, 16>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return; \
    case 24: launch_prolong<R, D, 24>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return; \
    case 32: launch_prolong<R, D, 32>(c, xc, y, P, gf, gc, tile_f, tile_c, accumulate, ntiles); return; \
    default: break;                                                                                      \
  }
  switch (gf.dof) {
    case 12: DD_PROLONG_N(12) break;
    case 8: DD_PROLONG_N(8) break;
    case 16: DD_PROLONG_N(16) break;
    case 24: DD_PROLONG_N(24) break;
    case 32: DD_PROLONG_N(32) break;
    case 48: DD_PROLONG_N(48) break;
    case 64: DD_PROLONG_N(64) break;
    default: break;
  }
#undef DD_PROLONG_N
  throw Error{DDAMG_EINVAL, "prolong: unsupported (dof, N): dof in {8, 12, 16, 24, 32, 48, 64}, N in {2, 4, 6, 8, "
                            "12, 16, 24, 32}"};
}

void prolong_mv(ddamg_ctx* c, int level, const MV& x, const MV& y, int accumulate) {
  const LevelGeom& gf = c->geom[level];
  const LevelGeom& gc = c->geom[level + 1];
  const int N = c->tr[level].N;
  DD_CHECK(x.prec == y.prec && x.ntiles == y.ntiles && y.nsites == gf.V && x.nsites == gc.V, DDAMG_EINVAL,
           "prolong: shape");
  const int cpc = reals_per_chunk(x.prec) / 2;
  DD_CHECK(N % cpc == 0, DDAMG_EINVAL, "prolong: N must be whole chunks");
  DD_CHECK(x.prec == P64 || c->tr[level].d_P32 || (c->tr[level].d_P16T && (N == 24 || N == 32)), DDAMG_ESTATE,
           "prolong: no FP32 or FP16 P for this level");
  if (level == 0) kernel_timing_begin(c, TIMED_PROLONG0);
  if (x.prec == P64)
    prolong_dispatch<double>(c, x.as<double>(), y.as<double>(), c->tr[level].d_P64, gf, gc, N, y.tile_reals(),
                             x.tile_reals(), accumulate, x.ntiles);
  else if (c->tr[level].d_P16T && N == 24)
    hipLaunchKernelGGL(k_prolong16<24>, dim3((unsigned)((size_t)x.ntiles * (gf.dof / 2) * (gf.V / 256))), dim3(256),
                       0, c->stream, x.as<float>(), y.as<float>(), (const h2v*)c->tr[level].d_P16T,
                       gf.d_coarse_of_blk, gf.V, gf.dof, gf.gsize, gc.V, y.tile_reals(), x.tile_reals(), accumulate);
  else if (c->tr[level].d_P16T && N == 32)
    hipLaunchKernelGGL(k_prolong16<32>, dim3((unsigned)((size_t)x.ntiles * (gf.dof / 2) * (gf.V / 256))), dim3(256),
                       0, c->stream, x.as<float>(), y.as<float>(), (const h2v*)c->tr[level].d_P16T,
                       gf.d_coarse_of_blk, gf.V, gf.dof, gf.gsize, gc.V, y.tile_reals(), x.tile_reals(), accumulate);
  else
    prolong_dispatch<float>(c, x.as<float>(), y.as<float>(), c->tr[level].d_P32, gf, gc, N, y.tile_reals(),
                            x.tile_reals(), accumulate, x.ntiles);
  DD_HIP(hipGetLastError());
  if (level == 0) kernel_timing_end(c, TIMED_PROLONG0, x.ntiles);
}

// ------------------------------------------------------------- setup ---
// X[col = s*N + j](x)[k] = P[x][k][j] if chirality(k) == s else 0   (FP64)
__global__ void k_basis_field(const double* __restrict__ P, double* __restrict__ X, int V, int dof, int N,
                              size_t tile_reals) {
  const size_t total = (size_t)2 * N * V * dof;
  const int h = dof / 2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % dof);
    const size_t r = i / dof;
    const int s = (int)(r % V);
    const int col = (int)(r / V);
    const int sig = col / N, j = col % N;
    cx<double> v = {0, 0};
    if (k / h == sig) {
      const double* p = P + (((size_t)s * dof + k) * N + j) * 2;
      v = {p[0], p[1]};
    }
    store_one(X + (size_t)(col / TC) * tile_reals, V, TC, s, col % TC, k, v);
  }
}

void build_basis_field(ddamg_ctx* c, int level, const MV& X) {
  const LevelGeom& g = c->geom[level];
  const int N = c->tr[level].N;
  DD_CHECK(X.prec == P64 && X.ncol() >= 2 * N && X.nsites == g.V, DDAMG_EINVAL, "basis field: shape");
  const size_t n = (size_t)2 * N * g.V * g.dof;
  hipLaunchKernelGGL(k_basis_field, grid1(n), dim3(256), 0, c->stream, c->tr[level].d_P64, X.as<double>(), g.V, g.dof,
                     N, X.tile_reals());
  DD_HIP(hipGetLastError());
}

// P[s][k][j] = tv_j(s)[k]
__global__ void k_gather_tv(const double* __restrict__ tv, double* __restrict__ P, int V, int dof, int N,
                            size_t tile_reals) {
  const size_t total = (size_t)V * dof * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % N);
    const size_t r = i / N;
    const int k = (int)(r % dof);
    const int s = (int)(r / dof);
    const cx<double> v = load_one(tv + (size_t)(j / TC) * tile_reals, V, TC, s, j % TC, k);
    P[2 * i] = v.re;
    P[2 * i + 1] = v.im;
  }
}

void gather_test_vectors(ddamg_ctx* c, int level, const MV& tv, double* d_P) {
  const LevelGeom& g = c->geom[level];
  const int N = c->tr[level].N;
  DD_CHECK(tv.prec == P64 && tv.ncol() >= N && tv.nsites == g.V, DDAMG_EINVAL, "gather tv: shape");
  const size_t n = (size_t)g.V * g.dof * N;
  hipLaunchKernelGGL(k_gather_tv, grid1(n), dim3(256), 0, c->stream, tv.as<double>(), d_P, g.V, g.dof, N,
                     tv.tile_reals());
  DD_HIP(hipGetLastError());
}

// Block reduction of a complex value over 256 threads (result in every thread).
__device__ __forceinline__ cx<double> block_sum(cx<double> v, cx<double>* red) {
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  const int w = threadIdx.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  cx<double> r = red[0];
  for (int q = 1; q < (int)(blockDim.x / 64); ++q) r = r + red[q];
  return r;
}

// Orthonormalise, per (group of gs sites, chirality), the N columns of the
// (gs * dof/2) x N matrix P by modified Gram-Schmidt applied twice; the
// diagonal of R comes out real and positive, so the result equals any other
// QR of full-rank input with that convention.
__device__ void mgs_group(double* __restrict__ P, int dof, int N, int gs, int b, int sig, cx<double>* red) {
  const int h = dof / 2;
  const int nrows = gs * h;
  cx<double>* Pc = reinterpret_cast<cx<double>*>(P);
  auto at = [&](int row, int j) -> cx<double>& {
    const int s = b * gs + row / h, k = sig * h + row % h;
    return Pc[((size_t)s * dof + k) * N + j];
  };
  for (int j = 0; j < N; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        cx<double> part = {0, 0};
        for (int row = threadIdx.x; row < nrows; row += blockDim.x) cmac_conj(part, at(row, i), at(row, j));
        const cx<double> rij = block_sum(part, red);
        for (int row = threadIdx.x; row < nrows; row += blockDim.x) {
          cx<double>& q = at(row, j);
          q = q - rij * at(row, i);
        }
        __syncthreads();
      }
    cx<double> part = {0, 0};
    for (int row = threadIdx.x; row < nrows; row += blockDim.x) {
      const cx<double> q = at(row, j);
      part.re += q.re * q.re + q.im * q.im;
    }
    const double nrm = sqrt(block_sum(part, red).re);
    const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
    for (int row = threadIdx.x; row < nrows; row += blockDim.x) {
      cx<double>& q = at(row, j);
      q = inv * q;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_orthonormalise(double* __restrict__ P, int dof, int N, int gs) {
  __shared__ cx<double> red[4];
  mgs_group(P, dof, N, gs, blockIdx.x / 2, blockIdx.x % 2, red);
}

// The same orthonormalisation by Cholesky QR applied twice: per (group,
// chirality) one pass forms the Gram matrix G = A^H A (rows staged in LDS in
// chunks, one or more (i, j) entries per lane), a wave factors G = R^H R
// (Cholesky, real positive diagonal) and every lane then replaces its rows a
// by a R^-1 (forward substitution against R in LDS).  Two passes give
// orthonormal columns to rounding for test vectors far from dependent, and
// the same Q as Gram-Schmidt (the QR with a real positive diagonal is unique).
// A group whose Gram matrix has a pivot that is not safely positive (nearly
// dependent vectors) orthonormalises its current rows by Gram-Schmidt instead
// (same span, same unique Q); *fallbacks counts such groups.
constexpr int OQ_NMAX = 32;
constexpr int OQ_CH = 64;   // staged rows per chunk
__global__ void __launch_bounds__(256) k_orthonormalise_cq(double* __restrict__ P, int dof, int N, int gs,
                                                           int* __restrict__ fallbacks) {
  __shared__ cx<double> rows[OQ_CH][OQ_NMAX];
  __shared__ cx<double> G[OQ_NMAX][OQ_NMAX + 1];
  __shared__ cx<double> red[4];
  __shared__ int bad;
  const int b = blockIdx.x / 2, sig = blockIdx.x % 2;
  const int h = dof / 2;
  const int nrows = gs * h;
  const int npair = N * (N + 1) / 2;
  cx<double>* Pc = reinterpret_cast<cx<double>*>(P);
  auto rowp = [&](int row) -> cx<double>* {
    const int s = b * gs + row / h, k = sig * h + row % h;
    return Pc + ((size_t)s * dof + k) * N;
  };
  if (threadIdx.x == 0) bad = 0;
  for (int pass = 0; pass < 2; ++pass) {
    // Gram matrix: lane entries e = threadIdx.x, threadIdx.x + 256, ... of the upper triangle
    cx<double> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    int ei[3], ej[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      int e = threadIdx.x + q * 256, i = 0;
      while (e >= N - i && i < N) { e -= N - i; ++i; }
      ei[q] = i;
      ej[q] = i + e;
    }
    for (int r0 = 0; r0 < nrows; r0 += OQ_CH) {
      const int nr = nrows - r0 < OQ_CH ? nrows - r0 : OQ_CH;
      __syncthreads();
      for (int u = threadIdx.x; u < nr * N; u += blockDim.x) rows[u / N][u % N] = rowp(r0 + u / N)[u % N];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (threadIdx.x + q * 256 >= npair) break;
        for (int r = 0; r < nr; ++r) cmac_conj(acc[q], rows[r][ei[q]], rows[r][ej[q]]);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (threadIdx.x + q * 256 < npair) {
        G[ei[q]][ej[q]] = acc[q];
        G[ej[q]][ei[q]] = cx<double>{acc[q].re, -acc[q].im};
      }
    __syncthreads();
    // Cholesky G = R^H R on wave 0 (R upper, kept in the upper triangle of G)
    // (one wave: its LDS accesses complete in issue order; wave_barrier only
    // keeps the compiler from moving them across the steps)
    if (threadIdx.x < 64) {
      const int ln = threadIdx.x;
      double gmax = 0;
      for (int k = 0; k < N; ++k) gmax = G[k][k].re > gmax ? G[k][k].re : gmax;
      for (int k = 0; k < N; ++k) {
        const double dkk = G[k][k].re;
        // a pivot below 1e-13 of the largest diagonal: the condition number
        // is beyond what Cholesky QR twice orthonormalises to rounding
        if (!(dkk > 1e-13 * gmax)) {
          if (ln == 0) bad = 1;
          break;
        }
        const double d = sqrt(dkk);
        // row k of R: R_kj = G_kj / d (j >= k)
        for (int j = k + ln; j < N; j += 64) G[k][j] = cx<double>{G[k][j].re / d, G[k][j].im / d};
        __builtin_amdgcn_wave_barrier();
        // trailing update G_ij -= conj(R_ki) R_kj for k < i <= j
        for (int ij = ln; ij < (N - k - 1) * (N - k - 1); ij += 64) {
          const int i = k + 1 + ij / (N - k - 1), j = k + 1 + ij % (N - k - 1);
          if (j < i) continue;
          const cx<double> rki = G[k][i], rkj = G[k][j];
          G[i][j] = cx<double>{G[i][j].re - (rki.re * rkj.re + rki.im * rkj.im),
                               G[i][j].im - (rki.re * rkj.im - rki.im * rkj.re)};
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    if (bad) {   // uniform: written before the barrier above
      mgs_group(P, dof, N, gs, b, sig, red);
      if (threadIdx.x == 0) atomicAdd(fallbacks, 1);
      return;
    }
    // rows: a <- a R^-1 (a R_new = a_old, forward substitution over the columns)
    for (int row = threadIdx.x; row < nrows; row += blockDim.x) {
      cx<double>* a = rowp(row);
      cx<double> v[OQ_NMAX];
      for (int j = 0; j < N; ++j) v[j] = a[j];
      for (int j = 0; j < N; ++j) {
        cx<double> t = v[j];
        for (int p = 0; p < j; ++p) {
          const cx<double> rpj = G[p][j];
          t = cx<double>{t.re - (v[p].re * rpj.re - v[p].im * rpj.im), t.im - (v[p].re * rpj.im + v[p].im * rpj.re)};
        }
        const double d = G[j][j].re;
        v[j] = cx<double>{t.re / d, t.im / d};
      }
      for (int j = 0; j < N; ++j) a[j] = v[j];
    }
  }
}

void orthonormalise_P(ddamg_ctx* c, int level, double* d_P) {
  const LevelGeom& g = c->geom[level];
  const int nblk = g.V / g.gsize;
  const int N = c->tr[level].N;
  if (N <= OQ_NMAX) {
    int* d_fb = (int*)c->pool.alloc(sizeof(int));
    DD_HIP(hipMemsetAsync(d_fb, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_orthonormalise_cq, dim3(2 * nblk), dim3(256), 0, c->stream, d_P, g.dof, N, g.gsize, d_fb);
    DD_HIP(hipGetLastError());
    int fb = 0;
    DD_HIP(hipMemcpyAsync(&fb, d_fb, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(hipStreamSynchronize(c->stream));
    c->pool.release(d_fb);
    c->st.orth_fallbacks += fb;
    return;
  }
  hipLaunchKernelGGL(k_orthonormalise, dim3(2 * nblk), dim3(256), 0, c->stream, d_P, g.dof, N, g.gsize);
  DD_HIP(hipGetLastError());
}

// blocks(level+1)[a][slot][col][row] = Rc[col](a)[row]
__global__ void k_scatter_blocks(const double* __restrict__ Rc, double* __restrict__ blk, int Vc, int d,
                                 size_t tile_reals, int slot) {
  const size_t total = (size_t)Vc * d * d;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(i % d);
    const size_t r = i / d;
    const int col = (int)(r % d);
    const int a = (int)(r / d);
    const cx<double> v = load_one(Rc + (size_t)(col / TC) * tile_reals, Vc, TC, a, col % TC, row);
    double* q = blk + ((((size_t)a * 9 + slot) * d + col) * d + row) * 2;
    q[0] = v.re;
    q[1] = v.im;
  }
}

void scatter_blocks(ddamg_ctx* c, int level, const MV& Rc, int slot) {
  const LevelGeom& gc = c->geom[level + 1];
  const int d = gc.dof;
  const size_t n = (size_t)gc.V * d * d;
  hipLaunchKernelGGL(k_scatter_blocks, grid1(n), dim3(256), 0, c->stream, Rc.as<double>(),
                     c->coarse[level + 1].d_blk64, gc.V, d, Rc.tile_reals(), slot);
  DD_HIP(hipGetLastError());
}

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

void convert_P32(ddamg_ctx* c, int level) {
  const LevelGeom& g = c->geom[level];
  const size_t n = (size_t)g.V * g.dof * c->tr[level].N * 2;
  if (c->tr[level].d_P32) {
    hipLaunchKernelGGL(k_d2f, grid1(n), dim3(256), 0, c->stream, c->tr[level].d_P64, c->tr[level].d_P32, n);
    DD_HIP(hipGetLastError());
  }
  if (c->tr[level].d_P16T) convert_P16T(c, level);
  DD_HIP(hipGetLastError());
}

void convert_blocks32(ddamg_ctx* c, int level) {
  const LevelGeom& g = c->geom[level];
  const size_t n = (size_t)g.V * 9 * g.dof * g.dof * 2;
  hipLaunchKernelGGL(k_d2f, grid1(n), dim3(256), 0, c->stream, c->coarse[level].d_blk64, c->coarse[level].d_blk32, n);
  DD_HIP(hipGetLastError());
  // BF16 copy in the MFMA operand layout (same number of reals, 2 bytes each)
  if (g.dof % 16 == 0 && g.dof <= 256) {
    if (!c->coarse[level].d_blk16) c->coarse[level].d_blk16 = c->pool.alloc(n * 2);
    const size_t nv = (size_t)g.V * 9 * (g.dof / 16) * (g.dof / 16) * 64;
    hipLaunchKernelGGL(k_blocks_bf16, grid1(nv), dim3(256), 0, c->stream, c->coarse[level].d_blk64,
                       (bf16x8*)c->coarse[level].d_blk16, g.V, g.dof);
    DD_HIP(hipGetLastError());
  }
}

}  // namespace ddamg
