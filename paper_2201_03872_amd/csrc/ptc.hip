// Learned smoother: gauge-covariant parallel-transport convolution (PTC)
// network, forward / input-gradient / weight-gradient kernels and training.
//
// Layer:  out_o(x) = sum_i sum_p W[p][o][i] (T_p in_i)(x)
// paths p = 0 (identity), 1..4 = +mu, 5..8 = -mu with
//   T_{+mu} phi(x) = U_mu(x) phi(x+mu),  T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu)
// (FP32 full links with the antiperiodic sign folded in), W[p][o][i] a 4x4
// complex spin matrix.  The network is two layers, 1 -> 2 -> 1 channels, no
// activation; weights are stored in BF16 on the device and used with FP32
// accumulation.  The input gradient of a layer is the same layer with the
// adjoint weights W'[p'][i][o] = W[p][o][i]^dag on the reversed path p'.
#include <cmath>
#include <cstring>
#include <random>

#include "common.h"
#include "device.h"

namespace ddamg {

constexpr int TP = 8;   // columns per tile

// ---------------------------------------------------------------- BF16 ---
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;                                                   // round to nearest even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// full FP32 link (sign folded): [mu][5][V] float4
__device__ __forceinline__ void ptc_link(const float4* __restrict__ U, int mu, int s, int V, cx<float> (&u)[9]) {
  const float4* b = U + (size_t)mu * 5 * V;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 c = b[(size_t)k * V + s];
    u[2 * k] = {c.x, c.y};
    u[2 * k + 1] = {c.z, c.w};
  }
  const float4 c = b[4 * (size_t)V + s];
  u[8] = {c.x, c.y};
}

// t = T_p in(at neighbour), all four spins
__device__ __forceinline__ void ptc_transport(int p, const float4* __restrict__ U, const int* __restrict__ nbr, int V,
                                              int s, const float* __restrict__ tile, int t, cx<float> (&out)[12]) {
  int site = s;
  if (p > 0) site = nbr[(size_t)(p - 1) * V + s] & 0x7fffffff;
  asm volatile("" : "+v"(site));
  cx<float> in[12];
  load_cx<float, 12>(tile, V, TP, site, t, in);
  if (p == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = in[k];
    return;
  }
  const bool fwd = p <= 4;
  const int mu = (p - 1) & 3;
  cx<float> u[9];
  ptc_link(U, mu, fwd ? s : site, V, u);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<float> r = {0, 0};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (fwd) cmac(r, u[a * 3 + b], in[sp * 3 + b]);
        else cmac_conj(r, u[b * 3 + a], in[sp * 3 + b]);
      }
      out[sp * 3 + a] = r;
    }
}

struct ChanPtrs {
  const float* in[2];
  float* out[2];
};

// out_o = sum_{p,i} W[p][o][i] T_p in_i   (W: BF16 complex [9][COUT][CIN][4][4])
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_ptc_layer(ChanPtrs ch, const uint16_t* __restrict__ Wb, const float4* __restrict__ U,
                                                   const int* __restrict__ nbr, int V, size_t tile_reals, int nsb) {
  constexpr int NW = 9 * COUT * CIN * 16;
  __shared__ cx<float> W[NW];
  for (int k = threadIdx.x; k < NW; k += blockDim.x) W[k] = {bf16_to_f32(Wb[2 * k]), bf16_to_f32(Wb[2 * k + 1])};
  __syncthreads();
  const int t = threadIdx.x % TP, sl = threadIdx.x / TP;
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = wg / nsb;
  const int s = (wg % nsb) * (256 / TP) + sl;
  if (s >= V) return;
  cx<float> acc[COUT][12];
#pragma unroll
  for (int o = 0; o < COUT; ++o)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[o][k] = {0, 0};
#pragma unroll 1
  for (int p = 0; p < 9; ++p) {
#pragma unroll
    for (int i = 0; i < CIN; ++i) {
      cx<float> tr[12];
      ptc_transport(p, U, nbr, V, s, ch.in[i] + (size_t)tile * tile_reals, t, tr);
#pragma unroll
      for (int o = 0; o < COUT; ++o) {
        const cx<float>* w = W + ((p * COUT + o) * CIN + i) * 16;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int tq = 0; tq < 4; ++tq) {
            const cx<float> wv = w[sp * 4 + tq];
#pragma unroll
            for (int c = 0; c < 3; ++c) cmac(acc[o][sp * 3 + c], wv, tr[tq * 3 + c]);
          }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < COUT; ++o) store_cx<float, 12>(ch.out[o] + (size_t)tile * tile_reals, V, TP, s, t, acc[o]);
}

// Weight gradient partials: part[wg][p][o][i][s][t] = sum over this workgroup's
// (site, column) lanes of gout_o[s][c] conj((T_p in_i)[t][c]).
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_ptc_wgrad(ChanPtrs ch, const float* __restrict__ g0, const float* __restrict__ g1,
                                                   const float4* __restrict__ U, const int* __restrict__ nbr, int V,
                                                   size_t tile_reals, int nsb, int ntiles, double* __restrict__ part) {
  constexpr int NG = COUT * CIN * 16;
  __shared__ float red[4][NG][2];
  const int t = threadIdx.x % TP, sl = threadIdx.x / TP;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int nwg = gridDim.x;
  for (int p = 0; p < 9; ++p) {
    cx<float> acc[COUT][CIN][16];
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
      for (int i = 0; i < CIN; ++i)
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[o][i][k] = {0, 0};
    for (int item = blockIdx.x; item < nsb * ntiles; item += nwg) {
      const int tile = item / nsb;
      const int s = (item % nsb) * (256 / TP) + sl;
      if (s >= V) continue;
      cx<float> go[COUT][12];
      load_cx<float, 12>(g0 + (size_t)tile * tile_reals, V, TP, s, t, go[0]);
      if (COUT > 1) load_cx<float, 12>(g1 + (size_t)tile * tile_reals, V, TP, s, t, go[COUT - 1]);
#pragma unroll
      for (int i = 0; i < CIN; ++i) {
        cx<float> tr[12];
        ptc_transport(p, U, nbr, V, s, ch.in[i] + (size_t)tile * tile_reals, t, tr);
#pragma unroll
        for (int o = 0; o < COUT; ++o)
#pragma unroll
          for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int tq = 0; tq < 4; ++tq)
#pragma unroll
              for (int c = 0; c < 3; ++c) cmac_conj(acc[o][i][sp * 4 + tq], tr[tq * 3 + c], go[o][sp * 3 + c]);
      }
    }
    // cmac_conj(a, b, c): a += conj(b) c, so acc = sum gout_o[s][c] conj(tr[t][c])
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
      for (int i = 0; i < CIN; ++i)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          float a = acc[o][i][k].re, b = acc[o][i][k].im;
#pragma unroll
          for (int off = 1; off < 64; off <<= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
          }
          if (lane == 0) {
            red[wave][(o * CIN + i) * 16 + k][0] = a;
            red[wave][(o * CIN + i) * 16 + k][1] = b;
          }
        }
    __syncthreads();
    for (int k = threadIdx.x; k < NG; k += blockDim.x) {
      double a = 0, b = 0;
      for (int w4 = 0; w4 < 4; ++w4) { a += red[w4][k][0]; b += red[w4][k][1]; }
      double* q = part + (((size_t)blockIdx.x * 9 + p) * NG + k) * 2;
      q[0] = a;
      q[1] = b;
    }
    __syncthreads();
  }
}

__global__ void k_sum_partials(const double* __restrict__ part, double* __restrict__ out, int nwg, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double a = 0, b = 0;
  for (int w = 0; w < nwg; ++w) {
    a += part[((size_t)w * n + k) * 2];
    b += part[((size_t)w * n + k) * 2 + 1];
  }
  out[2 * k] = a;
  out[2 * k + 1] = b;
}

// per column: scale = a[c] (real), x *= scale
__global__ void k_scale_real(float* __restrict__ x, const double* __restrict__ a, size_t npairs, int T, int RWp,
                             size_t tile_pairs, int mode) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npairs; i += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(i / tile_pairs);
    const int t = (int)((i / RWp) % T);
    const double v = a[tile * T + t];
    const double s = mode == 0 ? (v > 0 ? 1.0 / sqrt(v) : 0.0) : (v > 0 ? 1.0 / v : 0.0);
    x[2 * i] = (float)(x[2 * i] * s);
    x[2 * i + 1] = (float)(x[2 * i + 1] * s);
  }
}

// -------------------------------------------------------------- state ---
struct PtcState {
  std::vector<double> w[2];      // FP64 master weights (host), complex interleaved
  uint16_t* d_w[2] = {nullptr, nullptr};    // BF16 forward weights
  uint16_t* d_wadj[2] = {nullptr, nullptr}; // BF16 adjoint weights (input gradient)
  bool set = false;
  // smoother workspace (FP32 fine multivectors, `cap` tiles each):
  // hidden channels h0, h1, residual, correction, FP32 copies of input / output
  int cap = 0;
  MV ws[6];
  double* d_coef = nullptr;   // per-column MR dots and coefficients, 10 doubles per column
  int coef_cap = 0;
};

static const int CIN_OF[2] = {1, 2}, COUT_OF[2] = {2, 1};

static PtcState& state(ddamg_ctx* c) {
  if (!c->ptc) c->ptc = new PtcState();
  return *static_cast<PtcState*>(c->ptc);
}

void free_ptc(ddamg_ctx* c) {
  if (!c->ptc) return;
  PtcState* st = static_cast<PtcState*>(c->ptc);
  for (MV& m : st->ws) mv_free(c, m);
  if (st->d_coef) c->pool.release(st->d_coef);
  delete st;
  c->ptc = nullptr;
}

// the smoother workspace, grown to at least nt tiles
static MV* workspace(ddamg_ctx* c, int nt) {
  PtcState& st = state(c);
  if (nt > st.cap) {
    for (MV& m : st.ws) mv_free(c, m);
    for (MV& m : st.ws) m = mv_alloc(c, 0, P32, nt * c->T);
    st.cap = nt;
  }
  if (nt * c->T > st.coef_cap) {
    if (st.d_coef) c->pool.release(st.d_coef);
    st.coef_cap = nt * c->T;
    st.d_coef = (double*)c->pool.alloc((size_t)10 * st.coef_cap * sizeof(double));
  }
  return st.ws;
}

static size_t nweights(int layer) { return (size_t)9 * COUT_OF[layer] * CIN_OF[layer] * 16; }

// upload BF16 forward and adjoint weights from the FP64 masters
static void upload_weights(ddamg_ctx* c) {
  PtcState& st = state(c);
  for (int l = 0; l < 2; ++l) {
    const int co = COUT_OF[l], ci = CIN_OF[l];
    const size_t n = nweights(l);
    std::vector<uint16_t> fw(2 * n), ad(2 * n);
    auto at = [&](int p, int o, int i, int a, int b) { return (((size_t)p * co + o) * ci + i) * 16 + a * 4 + b; };
    auto atT = [&](int p, int i, int o, int a, int b) { return (((size_t)p * ci + i) * co + o) * 16 + a * 4 + b; };
    for (int p = 0; p < 9; ++p) {
      const int pa = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
      for (int o = 0; o < co; ++o)
        for (int i = 0; i < ci; ++i)
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
              const size_t k = at(p, o, i, a, b);
              const double re = st.w[l][2 * k], im = st.w[l][2 * k + 1];
              fw[2 * k] = f32_to_bf16((float)re);
              fw[2 * k + 1] = f32_to_bf16((float)im);
              // adjoint: W'[pa][i][o][b][a] = conj(W[p][o][i][a][b])
              const size_t ka = atT(pa, i, o, b, a);
              ad[2 * ka] = f32_to_bf16((float)re);
              ad[2 * ka + 1] = f32_to_bf16((float)-im);
            }
    }
    if (!st.d_w[l]) {
      st.d_w[l] = (uint16_t*)c->pool.alloc(2 * n * sizeof(uint16_t));
      st.d_wadj[l] = (uint16_t*)c->pool.alloc(2 * n * sizeof(uint16_t));
    }
    DD_HIP(hipMemcpy(st.d_w[l], fw.data(), fw.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    DD_HIP(hipMemcpy(st.d_wadj[l], ad.data(), ad.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  st.set = true;
}

void ptc_set_weights(ddamg_ctx* c, const double* w1, const double* w2) {
  PtcState& st = state(c);
  st.w[0].assign(w1, w1 + 2 * nweights(0));
  st.w[1].assign(w2, w2 + 2 * nweights(1));
  for (double v : st.w[0]) DD_CHECK(std::isfinite(v), DDAMG_EINVAL, "weights contain NaN/Inf");
  for (double v : st.w[1]) DD_CHECK(std::isfinite(v), DDAMG_EINVAL, "weights contain NaN/Inf");
  upload_weights(c);
}

void ptc_get_weights(ddamg_ctx* c, double* w1, double* w2) {
  PtcState& st = state(c);
  DD_CHECK(st.set, DDAMG_ESTATE, "smoother weights not set");
  std::memcpy(w1, st.w[0].data(), st.w[0].size() * sizeof(double));
  std::memcpy(w2, st.w[1].data(), st.w[1].size() * sizeof(double));
}

bool ptc_ready(ddamg_ctx* c) { return c->ptc && state(c).set; }

// one layer (layer 0 or 1) or its adjoint; in/out: FP32 fine multivectors
void ptc_layer(ddamg_ctx* c, int layer, bool adjoint, const MV* in, const MV* out) {
  PtcState& st = state(c);
  DD_CHECK(st.set, DDAMG_ESTATE, "smoother weights not set");
  const int cin = adjoint ? COUT_OF[layer] : CIN_OF[layer];
  const int cout = adjoint ? CIN_OF[layer] : COUT_OF[layer];
  const MV& x = in[0];
  DD_CHECK(x.prec == P32 && x.nsites == c->geom[0].V, DDAMG_EINVAL, "ptc: FP32 fine vectors expected");
  const int V = c->geom[0].V;
  const int nsb = (V + 256 / TP - 1) / (256 / TP);
  ChanPtrs ch{};
  for (int i = 0; i < cin; ++i) ch.in[i] = in[i].as<float>();
  for (int o = 0; o < cout; ++o) ch.out[o] = out[o].as<float>();
  const uint16_t* W = adjoint ? st.d_wadj[layer] : st.d_w[layer];
  dim3 grid(nsb * x.ntiles), blk(256);
  if (cin == 1 && cout == 2)
    hipLaunchKernelGGL((k_ptc_layer<1, 2>), grid, blk, 0, c->stream, ch, W, (const float4*)c->d_U32f,
                       c->geom[0].d_nbr, V, x.tile_reals(), nsb);
  else
    hipLaunchKernelGGL((k_ptc_layer<2, 1>), grid, blk, 0, c->stream, ch, W, (const float4*)c->d_U32f,
                       c->geom[0].d_nbr, V, x.tile_reals(), nsb);
  DD_HIP(hipGetLastError());
}

// g (host, complex [9][cout][cin][16]) = 2 sum gout conj(T_p in)
void ptc_wgrad(ddamg_ctx* c, int layer, const MV* in, const MV* gout, double* g_host) {
  const int cin = CIN_OF[layer], cout = COUT_OF[layer];
  const MV& x = in[0];
  const int V = c->geom[0].V;
  const int nsb = (V + 256 / TP - 1) / (256 / TP);
  const int nwg = std::min(1024, nsb * x.ntiles);
  const int NG = cout * cin * 16;
  double* part = scratch(c, (size_t)nwg * 9 * NG * 2 * sizeof(double));
  double* d_out = small_buffer(c, 9 * NG * 2);
  ChanPtrs ch{};
  for (int i = 0; i < cin; ++i) ch.in[i] = in[i].as<float>();
  if (cin == 1)
    hipLaunchKernelGGL((k_ptc_wgrad<1, 2>), dim3(nwg), dim3(256), 0, c->stream, ch, gout[0].as<float>(),
                       gout[1].as<float>(), (const float4*)c->d_U32f, c->geom[0].d_nbr, V, x.tile_reals(), nsb,
                       x.ntiles, part);
  else
    hipLaunchKernelGGL((k_ptc_wgrad<2, 1>), dim3(nwg), dim3(256), 0, c->stream, ch, gout[0].as<float>(),
                       gout[0].as<float>(), (const float4*)c->d_U32f, c->geom[0].d_nbr, V, x.tile_reals(), nsb,
                       x.ntiles, part);
  DD_HIP(hipGetLastError());
  const int n = 9 * NG;
  hipLaunchKernelGGL(k_sum_partials, dim3((n + 255) / 256), dim3(256), 0, c->stream, part, d_out, nwg, n);
  DD_HIP(hipGetLastError());
  copy_to_host(c, d_out, g_host, (size_t)n * 2 * sizeof(double));
  // dL/dRe W + i dL/dIm W = 2 sum gout conj(T_p in)
  for (int k = 0; k < 2 * n; ++k) g_host[k] *= 2.0;
}

// --------------------------------------------------------- smoother use ---
// z = f(v) for one network pass (FP32 in, FP32 out, distinct buffers).
void ptc_apply(ddamg_ctx* c, const MV& v, const MV& z) {
  MV* ws = workspace(c, v.ntiles);
  const MV h[2] = {ws[0].tiles(0, v.ntiles), ws[1].tiles(0, v.ntiles)};
  ptc_layer(c, 0, false, &v, h);
  ptc_layer(c, 1, false, h, &z);
}

// alpha = <q, r> / <q, q> per column (minimal-residual step), 0 where <q,q> = 0
__global__ void k_ptc_alpha(const double* __restrict__ qr, const double* __restrict__ qq, double* __restrict__ a,
                            int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = qq[i];
  a[2 * i] = d > 0 ? qr[2 * i] / d : 0.0;
  a[2 * i + 1] = d > 0 ? qr[2 * i + 1] / d : 0.0;
}

// The learned smoother: from z = 0, r = v, `cycles` minimal-residual steps
// with the network as search direction: p = f(r), q = D p,
// alpha = <q,r>/<q,q>, z += alpha p, r -= alpha q.  Returns false if the
// network's own first output does not reduce the residual of every column,
// ||v - D f(v)|| >= ||v||, i.e. ||q0||^2 >= 2 Re<q0, v>, for a column with
// v != 0 (the condition for using SAP instead); z then holds the smoother's
// result all the same.
// v and z may be FP32 or FP64 (converted through the workspace).
bool ptc_smooth(ddamg_ctx* c, const MV& v, const MV& z, const double* d_mu, int cycles) {
  const int nt = v.ntiles, ncol = v.ncol();
  MV* ws = workspace(c, nt);
  PtcState& st = state(c);
  const MV q = ws[2].tiles(0, nt), p = ws[3].tiles(0, nt), r = ws[4].tiles(0, nt);
  const MV z32 = z.prec == P32 ? z : ws[5].tiles(0, nt);
  double* qr0 = st.d_coef;            // [ncol] complex <q0, v>
  double* qq0 = qr0 + 2 * ncol;       // [ncol] ||q0||^2
  double* vv = qq0 + ncol;            // [ncol] ||v||^2
  double* qr = vv + ncol;             // [ncol] complex
  double* qq = qr + 2 * ncol;         // [ncol]
  double* al = qq + ncol;             // [ncol] complex
  mv_copy(c, v, r);
  mv_norm2(c, r, vv);
  mv_zero(c, z32);
  for (int k = 0; k < cycles; ++k) {
    ptc_apply(c, r, p);
    fine_dslash(c, p, q, d_mu);
    mv_dot(c, q, r, k == 0 ? qr0 : qr);
    mv_norm2(c, q, k == 0 ? qq0 : qq);
    hipLaunchKernelGGL(k_ptc_alpha, dim3((ncol + 255) / 256), dim3(256), 0, c->stream, k == 0 ? qr0 : qr,
                       k == 0 ? qq0 : qq, al, ncol);
    DD_HIP(hipGetLastError());
    mv_axpy(c, al, p, z32, +1);
    if (k + 1 < cycles) mv_axpy(c, al, q, r, -1);
  }
  if (z.prec != P32) mv_copy(c, z32, z);
  std::vector<double> h(4 * ncol);
  copy_to_host(c, qr0, h.data(), h.size() * sizeof(double));
  for (int i = 0; i < ncol; ++i)   // zero columns (padding, converged) pass
    if (h[3 * ncol + i] > 0 && !(h[2 * ncol + i] < 2.0 * h[2 * i])) return false;
  return true;
}

// ------------------------------------------------------------ training ---
void random_fill(ddamg_ctx* c, int level, const MV& X, int ncol, uint64_t seed);

// Adam on the FP64 master weights from residual -> error pairs: each step
// draws Gaussian errors e0 and lets the SAP solver iteration act on them,
// e = (1 - M_SAP D)^k e0 with k = step mod (sap_sweeps + 1), so the pairs
// range from rough errors to the smooth ones SAP leaves behind; r = D(mu_c) e,
// both scaled by 1/||r||; loss per column ||f(r) - e||^2 / ||e||^2 (mean over
// the batch).
void ptc_train(ddamg_ctx* c, const double* mus, int n_mu, int steps, int batch, double lr, int sap_sweeps,
               uint64_t seed, double* loss_hist) {
  PtcState& st = state(c);
  DD_CHECK(st.set, DDAMG_ESTATE, "smoother weights not initialised");
  DD_CHECK(steps >= 1 && batch >= 1 && n_mu >= 1 && sap_sweeps >= 0, DDAMG_EINVAL, "training sizes");
  MV e64 = mv_alloc(c, 0, P64, batch);
  const int ncol = e64.ncol();
  MV e = mv_alloc(c, 0, P32, batch), r = mv_alloc(c, 0, P32, batch);
  MV h[2] = {mv_alloc(c, 0, P32, batch), mv_alloc(c, 0, P32, batch)};
  MV y = mv_alloc(c, 0, P32, batch), gy = mv_alloc(c, 0, P32, batch);
  MV gh[2] = {mv_alloc(c, 0, P32, batch), mv_alloc(c, 0, P32, batch)};
  std::vector<double> hmu(ncol, 0.0);
  for (int i = 0; i < ncol; ++i) hmu[i] = mus[i % n_mu];
  double* d_mu = (double*)c->pool.alloc(ncol * sizeof(double));
  DD_HIP(hipMemcpy(d_mu, hmu.data(), ncol * sizeof(double), hipMemcpyHostToDevice));
  double* d_n = (double*)c->pool.alloc(2 * ncol * sizeof(double));
  const size_t n0 = 2 * nweights(0), n1 = 2 * nweights(1);
  std::vector<double> m[2] = {std::vector<double>(n0, 0.0), std::vector<double>(n1, 0.0)};
  std::vector<double> vv[2] = {std::vector<double>(n0, 0.0), std::vector<double>(n1, 0.0)};
  std::vector<double> g[2] = {std::vector<double>(n0), std::vector<double>(n1)};
  const double b1 = 0.9, b2 = 0.999, eps = 1e-12;
  const size_t np = e.reals() / 2;
  size_t gsz = (np + 255) / 256;
  if (gsz > 65536) gsz = 65536;
  for (int it = 0; it < steps; ++it) {
    random_fill(c, 0, e64, batch, seed + 1315423911ULL * (it + 1));
    mv_copy(c, e64, e);
    const int k = sap_sweeps > 0 ? it % (sap_sweeps + 1) : 0;
    for (int q = 0; q < k; ++q) {
      // e <- e - M_SAP D e  (y, gy serve as temporaries)
      fine_dslash(c, e, y, d_mu);
      sap_apply(c, y, gy, d_mu, gy);
      mv_sub(c, e, gy, e);
    }
    fine_dslash(c, e, r, d_mu);
    mv_norm2(c, r, d_n);
    hipLaunchKernelGGL(k_scale_real, dim3((unsigned)gsz), dim3(256), 0, c->stream, r.as<float>(), d_n, np, e.T, 2,
                       e.tile_reals() / 2, 0);
    hipLaunchKernelGGL(k_scale_real, dim3((unsigned)gsz), dim3(256), 0, c->stream, e.as<float>(), d_n, np, e.T, 2,
                       e.tile_reals() / 2, 0);
    // forward
    ptc_layer(c, 0, false, &r, h);
    ptc_layer(c, 1, false, h, &y);
    // gy = (y - e) / ||e||^2 ; loss
    mv_sub(c, y, e, gy);
    mv_norm2(c, e, d_n);
    mv_norm2(c, gy, d_n + ncol);
    std::vector<double> hn(2 * ncol);
    copy_to_host(c, d_n, hn.data(), hn.size() * sizeof(double));
    double loss = 0;
    int cnt = 0;
    for (int i = 0; i < ncol; ++i)
      if (hn[i] > 0) {
        loss += hn[ncol + i] / hn[i];
        ++cnt;
      }
    loss /= std::max(cnt, 1);
    if (loss_hist) loss_hist[it] = loss;
    hipLaunchKernelGGL(k_scale_real, dim3((unsigned)gsz), dim3(256), 0, c->stream, gy.as<float>(), d_n, np, e.T, 2,
                       e.tile_reals() / 2, 1);
    // backward
    ptc_wgrad(c, 1, h, &gy, g[1].data());
    ptc_layer(c, 1, true, &gy, gh);
    ptc_wgrad(c, 0, &r, gh, g[0].data());
    // Adam (mean over the batch: the loss above is averaged over cnt columns)
    const double inv = 1.0 / std::max(cnt, 1);
    for (int l = 0; l < 2; ++l)
      for (size_t k = 0; k < g[l].size(); ++k) {
        const double gk = g[l][k] * inv;
        m[l][k] = b1 * m[l][k] + (1 - b1) * gk;
        vv[l][k] = b2 * vv[l][k] + (1 - b2) * gk * gk;
        const double mh = m[l][k] / (1 - std::pow(b1, it + 1)), vh = vv[l][k] / (1 - std::pow(b2, it + 1));
        st.w[l][k] -= lr * mh / (std::sqrt(vh) + eps);
      }
    upload_weights(c);
  }
  DD_HIP(hipStreamSynchronize(c->stream));
  MV* all[] = {&e64, &e, &r, &h[0], &h[1], &y, &gy, &gh[0], &gh[1]};
  for (MV* a : all) mv_free(c, *a);
  c->pool.release(d_mu);
  c->pool.release(d_n);
}

}  // namespace ddamg
