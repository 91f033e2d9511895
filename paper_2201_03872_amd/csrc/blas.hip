// Multivector management, layout conversion and per-column BLAS on the
// column-tiled layout [tile][m][T][RW] (m runs over chunk x site).
//
// Inner products are reduced in a fixed order (per-thread partials, wavefront
// shuffles, one partial per workgroup, a second pass over the partials), with
// FP64 accumulation for both precisions: results are bitwise reproducible and
// no atomics are used.  This is the single-GPU analogue of the paper's global
// reductions (section 4: they dominate block-solver overhead); every
// orthogonalisation step issues one fused multi-dot instead of one reduction
// per inner product.
#include "common.h"
#include "device.h"

namespace ddamg {

constexpr int TTB = 8;
constexpr int MAXK = 64;

// ------------------------------------------------------------- pool ---
void* DevPool::alloc(size_t bytes) {
  size_t want = ((bytes ? bytes : 16) + 255) & ~(size_t)255;
  if (want >= ((size_t)1 << 20)) want = (want + ((size_t)2 << 20) - 1) & ~(((size_t)2 << 20) - 1);
  auto it = cache.lower_bound(want);
  if (it != cache.end() && it->first <= want + want / 4) {
    void* p = it->second;
    const size_t sz = it->first;
    cache.erase(it);
    cached_bytes -= sz;
    DD_HIP(hipStreamSynchronize(stream));
    blocks.push_back({p, sz});
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory && !cache.empty()) {
    (void)hipGetLastError();
    trim();
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess)
    throw Error{e == hipErrorOutOfMemory ? DDAMG_ENOMEM : DDAMG_EDEVICE,
                "device allocation of " + std::to_string(want) + " bytes: " + hipGetErrorString(e)};
  blocks.push_back({p, want});
  held += want;
  if (held > peak) peak = held;
  return p;
}
void DevPool::release(void* p) {
  for (size_t i = 0; i < blocks.size(); ++i)
    if (blocks[i].first == p) {
      cache.insert({blocks[i].second, p});
      cached_bytes += blocks[i].second;
      blocks.erase(blocks.begin() + i);
      return;
    }
}
void DevPool::trim() {
  for (auto& kv : cache) (void)hipFree(kv.second);
  cache.clear();
  held -= cached_bytes;
  cached_bytes = 0;
}
void DevPool::clear() {
  trim();
  for (auto& b : blocks) (void)hipFree(b.first);
  blocks.clear();
  held = 0;
}

MV mv_alloc(ddamg_ctx* c, int level, int prec, int ncol_min) {
  MV a;
  a.prec = prec;
  a.T = c->T;
  a.ntiles = (ncol_min + a.T - 1) / a.T;
  if (a.ntiles < 1) a.ntiles = 1;
  a.dof = c->geom[level].dof;
  a.nsites = c->geom[level].V;
  a.nchunk = 2 * a.dof / reals_per_chunk(prec);
  // FP16 bases hold unit vectors: scale their entries (about 1/sqrt(n)) to
  // about 1/16, far from the FP16 subnormal and overflow ranges
  if (prec == P16) a.hscale = std::sqrt((double)a.nsites * a.dof) / 16.0;
  a.p = c->pool.alloc(a.bytes());
  a.owned = true;
  mv_zero(c, a);
  return a;
}

MV mv_like(ddamg_ctx* c, const MV& a, int prec) {
  MV b = a;
  b.prec = prec;
  b.nchunk = 2 * a.dof / reals_per_chunk(prec);
  b.hscale = prec == P16 ? std::sqrt((double)a.nsites * a.dof) / 16.0 : 1.0;
  b.p = c->pool.alloc(b.bytes());
  b.owned = true;
  mv_zero(c, b);
  return b;
}

void mv_free(ddamg_ctx* c, MV& a) {
  if (a.owned && a.p) c->pool.release(a.p);
  a.p = nullptr;
}

// ----------------------------------------------------------- kernels ---
__global__ void k_fill(uint4* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = uint4{0, 0, 0, 0};
}

static inline dim3 grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

void mv_zero(ddamg_ctx* c, const MV& a) {
  const size_t n = a.bytes() / 16;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, c->stream, (uint4*)a.p, n);
  DD_HIP(hipGetLastError());
}

// canonical [col][site][dof] complex  ->  tiled internal (either precision)
template <typename R>
__global__ void k_to_internal(const double* __restrict__ src, R* __restrict__ dst, const int* __restrict__ int2can,
                              int n_col, int ncolp, int V, int dof, int T) {
  constexpr int RW = Chunk<R>::RW, CPC = RW / 2;
  const int nchunk = 2 * dof / RW;
  const size_t total = (size_t)ncolp * V * dof;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    // i = ((col * V) + s) * dof + k  with s the internal site
    const int k = (int)(i % dof);
    const size_t cs = i / dof;
    const int s = (int)(cs % V);
    const int col = (int)(cs / V);
    double re = 0, im = 0;
    if (col < n_col) {
      const double* q = src + (((size_t)col * V + int2can[s]) * dof + k) * 2;
      re = q[0]; im = q[1];
    }
    const int tile = col / T, t = col % T;
    R* d = dst + (size_t)tile * nchunk * V * T * RW + (((size_t)(k / CPC) * V + s) * T + t) * RW + (k % CPC) * 2;
    d[0] = (R)re; d[1] = (R)im;
  }
}

template <typename R>
__global__ void k_from_internal(const R* __restrict__ src, double* __restrict__ dst, const int* __restrict__ int2can,
                                int n_col, int V, int dof, int T) {
  constexpr int RW = Chunk<R>::RW, CPC = RW / 2;
  const int nchunk = 2 * dof / RW;
  const size_t total = (size_t)n_col * V * dof;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % dof);
    const size_t cs = i / dof;
    const int s = (int)(cs % V);
    const int col = (int)(cs / V);
    const int tile = col / T, t = col % T;
    const R* q = src + (size_t)tile * nchunk * V * T * RW + (((size_t)(k / CPC) * V + s) * T + t) * RW + (k % CPC) * 2;
    double* d = dst + (((size_t)col * V + int2can[s]) * dof + k) * 2;
    d[0] = (double)q[0]; d[1] = (double)q[1];
  }
}

void to_internal(ddamg_ctx* c, int level, const double* canon, int n_col, const MV& out) {
  const LevelGeom& g = c->geom[level];
  DD_CHECK(out.nsites == g.V && out.dof == g.dof && out.ncol() >= n_col, DDAMG_EINVAL, "to_internal: shape");
  const size_t n = (size_t)out.ncol() * g.V * g.dof;
  if (out.prec == P64)
    hipLaunchKernelGGL(k_to_internal<double>, grid_for(n), dim3(256), 0, c->stream, canon, out.as<double>(),
                       g.d_int2can, n_col, out.ncol(), g.V, g.dof, out.T);
  else
    hipLaunchKernelGGL(k_to_internal<float>, grid_for(n), dim3(256), 0, c->stream, canon, out.as<float>(),
                       g.d_int2can, n_col, out.ncol(), g.V, g.dof, out.T);
  DD_HIP(hipGetLastError());
}

void from_internal(ddamg_ctx* c, int level, const MV& in, int n_col, double* canon) {
  const LevelGeom& g = c->geom[level];
  DD_CHECK(in.nsites == g.V && in.dof == g.dof && in.ncol() >= n_col, DDAMG_EINVAL, "from_internal: shape");
  const size_t n = (size_t)n_col * g.V * g.dof;
  if (in.prec == P64)
    hipLaunchKernelGGL(k_from_internal<double>, grid_for(n), dim3(256), 0, c->stream, in.as<double>(), canon,
                       g.d_int2can, n_col, g.V, g.dof, in.T);
  else
    hipLaunchKernelGGL(k_from_internal<float>, grid_for(n), dim3(256), 0, c->stream, in.as<float>(), canon,
                       g.d_int2can, n_col, g.V, g.dof, in.T);
  DD_HIP(hipGetLastError());
}

// Column-mapped conversions for the outer solve's scheduler: internal column
// j of `mv` <-> canonical field map[j] of `canon` ([*][V][dof] complex);
// columns with map[j] < 0 are left untouched.
template <typename R>
__global__ void k_canon_cols(R* __restrict__ in, double* __restrict__ canon, const int* __restrict__ int2can,
                             const int* __restrict__ map, int n_col, int V, int dof, int T, int dir) {
  constexpr int RW = Chunk<R>::RW, CPC = RW / 2;
  const int nchunk = 2 * dof / RW;
  const size_t total = (size_t)n_col * V * dof;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % dof);
    const size_t cs = i / dof;
    const int s = (int)(cs % V);
    const int col = (int)(cs / V);
    const int f = map[col];
    if (f < 0) continue;
    const int tile = col / T, t = col % T;
    R* q = in + (size_t)tile * nchunk * V * T * RW + (((size_t)(k / CPC) * V + s) * T + t) * RW + (k % CPC) * 2;
    double* d = canon + (((size_t)f * V + int2can[s]) * dof + k) * 2;
    if (dir == 0) {
      q[0] = (R)d[0];
      q[1] = (R)d[1];
    } else {
      d[0] = (double)q[0];
      d[1] = (double)q[1];
    }
  }
}

// The same conversion as a transpose through LDS: one workgroup per (tile,
// group of SG internal sites) stages the T columns of its sites as
// [column][site][component] complexes, so that both sides are read and
// written in runs of consecutive addresses (the canonical side per column
// and site, the internal side per chunk across sites and columns).  Rows of
// the staging buffer are padded by two complexes against bank conflicts.
template <typename R, int SG>
__global__ void __launch_bounds__(256) k_canon_cols_lds(R* __restrict__ in, double* __restrict__ canon,
                                                        const int* __restrict__ int2can, const int* __restrict__ map,
                                                        int V, int dof, int dir) {
  constexpr int RW = Chunk<R>::RW, CPC = RW / 2, T = TTB;
  extern __shared__ double2 buf[];          // [T][SG * dof + 2]
  const int rowlen = SG * dof + 2;
  const int ngrp = (V + SG - 1) / SG;
  const int tile = blockIdx.x / ngrp, s0 = (blockIdx.x % ngrp) * SG;
  const int nchunk = 2 * dof / RW;
  R* it = in + (size_t)tile * nchunk * V * T * RW;
  const int nu = T * SG * dof;
  if (dir == 0) {   // canonical -> LDS (runs along the components of one column and site)
    for (int u = threadIdx.x; u < nu; u += blockDim.x) {
      const int k = u % dof, rest = u / dof, sl = rest % SG, t = rest / SG;
      const int f = map[tile * T + t], s = s0 + sl;
      if (f < 0 || s >= V) continue;
      const double* d = canon + (((size_t)f * V + int2can[s]) * dof + k) * 2;
      buf[t * rowlen + sl * dof + k] = double2{d[0], d[1]};
    }
    __syncthreads();
    // LDS -> internal (runs along the columns and sites of one chunk)
    for (int u = threadIdx.x; u < T * SG * nchunk; u += blockDim.x) {
      const int t = u % T, rest = u / T, sl = rest % SG, ch = rest / SG;
      const int f = map[tile * T + t], s = s0 + sl;
      if (f < 0 || s >= V) continue;
      R* q = it + (((size_t)ch * V + s) * T + t) * RW;
#pragma unroll
      for (int e = 0; e < CPC; ++e) {
        const double2 v = buf[t * rowlen + sl * dof + ch * CPC + e];
        q[2 * e] = (R)v.x;
        q[2 * e + 1] = (R)v.y;
      }
    }
  } else {          // internal -> LDS -> canonical
    for (int u = threadIdx.x; u < T * SG * nchunk; u += blockDim.x) {
      const int t = u % T, rest = u / T, sl = rest % SG, ch = rest / SG;
      const int f = map[tile * T + t], s = s0 + sl;
      if (f < 0 || s >= V) continue;
      const R* q = it + (((size_t)ch * V + s) * T + t) * RW;
#pragma unroll
      for (int e = 0; e < CPC; ++e) buf[t * rowlen + sl * dof + ch * CPC + e] = double2{(double)q[2 * e], (double)q[2 * e + 1]};
    }
    __syncthreads();
    for (int u = threadIdx.x; u < nu; u += blockDim.x) {
      const int k = u % dof, rest = u / dof, sl = rest % SG, t = rest / SG;
      const int f = map[tile * T + t], s = s0 + sl;
      if (f < 0 || s >= V) continue;
      const double2 v = buf[t * rowlen + sl * dof + k];
      double* d = canon + (((size_t)f * V + int2can[s]) * dof + k) * 2;
      d[0] = v.x;
      d[1] = v.y;
    }
  }
}

void canon_cols(ddamg_ctx* c, int level, const MV& mv, const int* d_map, double* canon, int dir) {
  const LevelGeom& g = c->geom[level];
  DD_CHECK(mv.nsites == g.V && mv.dof == g.dof, DDAMG_EINVAL, "canon_cols: shape");
  const size_t n = (size_t)mv.ncol() * g.V * g.dof;
  constexpr int SG = 32;
  const size_t lds = (size_t)TTB * (SG * g.dof + 2) * sizeof(double2);
  if (mv.T == TTB && lds <= 64 * 1024 && (mv.prec == P64 || mv.prec == P32)) {
    const int ngrp = (g.V + SG - 1) / SG;
    const dim3 grid((unsigned)(ngrp * mv.ntiles));
    if (mv.prec == P64)
      hipLaunchKernelGGL((k_canon_cols_lds<double, SG>), grid, dim3(256), lds, c->stream, mv.as<double>(), canon,
                         g.d_int2can, d_map, g.V, g.dof, dir);
    else
      hipLaunchKernelGGL((k_canon_cols_lds<float, SG>), grid, dim3(256), lds, c->stream, mv.as<float>(), canon,
                         g.d_int2can, d_map, g.V, g.dof, dir);
    DD_HIP(hipGetLastError());
    return;
  }
  if (mv.prec == P64)
    hipLaunchKernelGGL(k_canon_cols<double>, grid_for(n), dim3(256), 0, c->stream, mv.as<double>(), canon,
                       g.d_int2can, d_map, mv.ncol(), g.V, g.dof, mv.T, dir);
  else
    hipLaunchKernelGGL(k_canon_cols<float>, grid_for(n), dim3(256), 0, c->stream, mv.as<float>(), canon,
                       g.d_int2can, d_map, mv.ncol(), g.V, g.dof, mv.T, dir);
  DD_HIP(hipGetLastError());
}

// -------------------------------------------------- elementwise ops ---
// Every lane handles one real pair (complex) of one column; column index of
// real i in a tile: t = (i / RW) % T.
template <typename RS, typename RD>
__global__ void k_copy(const RS* __restrict__ a, RD* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (RD)a[i];
}

// FP32 <-> FP16 (same layout): b = a * scale
template <typename RS, typename RD>
__global__ void k_copy_scaled(const RS* __restrict__ a, RD* __restrict__ b, size_t n, float scale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (RD)((float)a[i] * scale);
}

// Column gather / scatter between a full multivector and a compacted one of
// the same level and precision.  map[j] (j < compact.ncol()) is the full
// column of compact slot j, or -1 for an empty slot.  dir 0: compact <- full
// (empty slots zeroed); dir 1: full <- compact (empty slots skipped, other
// full columns untouched).  One thread per 16-byte chunk of a compact slot.
__global__ void k_gather_cols(uint4* __restrict__ full, uint4* __restrict__ comp, const int* __restrict__ map,
                              size_t units_per_tile, size_t n_units, int T, int dir) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_units; i += (size_t)gridDim.x * blockDim.x) {
    const size_t tile = i / units_per_tile, rem = i % units_per_tile;
    const int t = (int)(rem % T);
    const size_t base = rem - t;                                  // (chunk, site) unit of slot 0
    const int col = map[tile * T + t];
    if (col < 0) {
      if (dir == 0) comp[i] = make_uint4(0, 0, 0, 0);
      continue;
    }
    const size_t f = (size_t)(col / T) * units_per_tile + base + col % T;
    if (dir == 0) comp[i] = full[f];
    else full[f] = comp[i];
  }
}

void mv_gather_cols(ddamg_ctx* c, const MV& full, const MV& comp, const int* d_map, int dir) {
  DD_CHECK(full.prec == comp.prec && full.nsites == comp.nsites && full.nchunk == comp.nchunk && full.T == comp.T,
           DDAMG_EINVAL, "column gather: shapes");
  const size_t upt = (size_t)comp.nchunk * comp.nsites * comp.T;
  const size_t n = upt * comp.ntiles;
  hipLaunchKernelGGL(k_gather_cols, grid_for(n), dim3(256), 0, c->stream, (uint4*)full.p, (uint4*)comp.p, d_map, upt,
                     n, comp.T, dir);
  DD_HIP(hipGetLastError());
}

// Plain device copy kernel (reads and writes a.bytes()); calibrates the
// memory-traffic counters against a kernel of known traffic.
void mv_copy_kernel(ddamg_ctx* c, const MV& s, const MV& d) {
  DD_CHECK(s.bytes() == d.bytes(), DDAMG_EINVAL, "copy: sizes");
  const size_t n = s.bytes() / sizeof(double);
  hipLaunchKernelGGL((k_copy<double, double>), grid_for(n), dim3(256), 0, c->stream, (const double*)s.p, (double*)d.p, n);
  DD_HIP(hipGetLastError());
}

void mv_copy(ddamg_ctx* c, const MV& s, const MV& d) {
  DD_CHECK(s.nsites == d.nsites && s.dof == d.dof && s.ntiles == d.ntiles, DDAMG_EINVAL, "mv_copy: shape");
  if (s.prec == d.prec) {
    DD_HIP(hipMemcpyAsync(d.p, s.p, s.bytes(), hipMemcpyDeviceToDevice, c->stream));
    return;
  }
  if (s.prec == P16 || d.prec == P16) {
    DD_CHECK((s.prec == P32 || d.prec == P32) && s.reals() == d.reals(), DDAMG_EINVAL, "mv_copy: FP16 needs FP32");
    const size_t n = s.reals();
    if (d.prec == P16)
      hipLaunchKernelGGL((k_copy_scaled<float, _Float16>), grid_for(n), dim3(256), 0, c->stream, s.as<float>(),
                         d.as<_Float16>(), n, (float)d.hscale);
    else
      hipLaunchKernelGGL((k_copy_scaled<_Float16, float>), grid_for(n), dim3(256), 0, c->stream, s.as<_Float16>(),
                         d.as<float>(), n, (float)(1.0 / s.hscale));
    DD_HIP(hipGetLastError());
    return;
  }
  // chunk widths differ between precisions: convert through the complex index
  mv_convert(c, s, d);
}

// FP64 <-> FP32 in the tiled layout.  An FP32 chunk holds two complexes,
// an FP64 chunk one, so FP32 chunk c of a (site, column) holds FP64 chunks 2c
// and 2c+1; one lane per FP32 chunk moves 16 bytes on the FP32 side and two
// 16-byte chunks on the FP64 side.
__global__ void k_convert_64_32(const double2* __restrict__ a, float4* __restrict__ b, size_t nunits, size_t nsT) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const size_t q = u / nsT, st = u - q * nsT;          // q = tile * ncd + c
    const size_t src = (2 * q) * nsT + st;               // tile * 2 ncd + 2c  (ncs = 2 ncd)
    const double2 v0 = a[src], v1 = a[src + nsT];
    b[u] = make_float4((float)v0.x, (float)v0.y, (float)v1.x, (float)v1.y);
  }
}

__global__ void k_convert_32_64(const float4* __restrict__ a, double2* __restrict__ b, size_t nunits, size_t nsT) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const size_t q = u / nsT, st = u - q * nsT;
    const float4 v = a[u];
    const size_t dst = (2 * q) * nsT + st;
    b[dst] = make_double2(v.x, v.y);
    b[dst + nsT] = make_double2(v.z, v.w);
  }
}

void mv_convert(ddamg_ctx* c, const MV& s, const MV& d) {
  DD_CHECK(s.dof == d.dof && s.nsites == d.nsites && s.ntiles <= d.ntiles && s.T == d.T && s.dof % 2 == 0,
           DDAMG_EINVAL, "mv_convert: shape");
  const size_t nsT = (size_t)s.nsites * s.T;
  const size_t n32 = (size_t)s.ntiles * (s.dof / 2) * nsT;   // FP32 chunks
  if (s.prec == P64 && d.prec == P32)
    hipLaunchKernelGGL(k_convert_64_32, grid_for(n32), dim3(256), 0, c->stream, (const double2*)s.p, (float4*)d.p,
                       n32, nsT);
  else if (s.prec == P32 && d.prec == P64)
    hipLaunchKernelGGL(k_convert_32_64, grid_for(n32), dim3(256), 0, c->stream, (const float4*)s.p, (double2*)d.p,
                       n32, nsT);
  else
    throw Error{DDAMG_EINVAL, "mv_convert: precisions"};
  DD_HIP(hipGetLastError());
}

// y += sign * alpha_col x  (complex alpha per column; same precision)
template <typename R>
__global__ void k_axpy(const double* __restrict__ alpha, const R* __restrict__ x, R* __restrict__ y, size_t npairs,
                       int T, int RWp, size_t tile_pairs, double sign) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npairs; i += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(i / tile_pairs);
    const int t = (int)((i / RWp) % T);
    const int col = tile * T + t;
    const double ar = sign * alpha[2 * col], ai = sign * alpha[2 * col + 1];
    const R xr = x[2 * i], xi = x[2 * i + 1];
    y[2 * i] += (R)(ar * xr - ai * xi);
    y[2 * i + 1] += (R)(ar * xi + ai * xr);
  }
}

// y = x + alpha_col y
template <typename R>
__global__ void k_xpay(const R* __restrict__ x, const double* __restrict__ alpha, R* __restrict__ y, size_t npairs,
                       int T, int RWp, size_t tile_pairs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npairs; i += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(i / tile_pairs);
    const int t = (int)((i / RWp) % T);
    const int col = tile * T + t;
    const double ar = alpha[2 * col], ai = alpha[2 * col + 1];
    const R yr = y[2 * i], yi = y[2 * i + 1];
    y[2 * i] = x[2 * i] + (R)(ar * yr - ai * yi);
    y[2 * i + 1] = x[2 * i + 1] + (R)(ar * yi + ai * yr);
  }
}

template <typename R>
__global__ void k_scale(const double* __restrict__ alpha, R* __restrict__ x, size_t npairs, int T, int RWp,
                        size_t tile_pairs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npairs; i += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(i / tile_pairs);
    const int t = (int)((i / RWp) % T);
    const int col = tile * T + t;
    const double ar = alpha[2 * col], ai = alpha[2 * col + 1];
    const R xr = x[2 * i], xi = x[2 * i + 1];
    x[2 * i] = (R)(ar * xr - ai * xi);
    x[2 * i + 1] = (R)(ar * xi + ai * xr);
  }
}

template <typename R>
__global__ void k_sub(const R* __restrict__ a, const R* __restrict__ b, R* __restrict__ o, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    o[i] = a[i] - b[i];
}

template <typename R>
__global__ void k_add(const R* __restrict__ a, R* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] += a[i];
}

__global__ void k_add4(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 u = a[i];
    float4 v = b[i];
    v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
    b[i] = v;
  }
}

__global__ void k_add2(const double2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 u = a[i];
    double2 v = b[i];
    v.x += u.x; v.y += u.y;
    b[i] = v;
  }
}

void mv_add(ddamg_ctx* c, const MV& x, const MV& y) {
  DD_CHECK(x.prec == y.prec && x.reals() == y.reals(), DDAMG_EINVAL, "mv_add: shape");
  const size_t n = x.bytes() / 16;   // whole 16-byte chunks
  if (x.prec == P64)
    hipLaunchKernelGGL(k_add2, grid_for(n), dim3(256), 0, c->stream, (const double2*)x.p, (double2*)y.p, n);
  else
    hipLaunchKernelGGL(k_add4, grid_for(n), dim3(256), 0, c->stream, (const float4*)x.p, (float4*)y.p, n);
  DD_HIP(hipGetLastError());
}

// x <- gamma5 x on any level: the complex components of chirality -1 (the
// second half of the dof of a site: spins 2, 3 on the fine level, the last N
// of the 2N coarse dof) change sign.
template <typename R>
__global__ void k_gamma5(R* __restrict__ x, size_t n, size_t plane, int RW, int dof) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const size_t in_tile = q % ((size_t)plane * (size_t)(2 * dof / RW));
    const int k = (int)(in_tile / plane);                  // chunk
    const int ci = k * (RW / 2) + (int)(q % RW) / 2;       // complex component
    if (ci >= dof / 2) x[q] = -x[q];
  }
}

void mv_gamma5(ddamg_ctx* c, const MV& x) {
  DD_CHECK(x.prec == P64 || x.prec == P32, DDAMG_EINVAL, "mv_gamma5: FP64 or FP32 only");
  const size_t n = x.reals();
  const int RW = reals_per_chunk(x.prec);
  const size_t plane = (size_t)x.nsites * x.T * RW;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_gamma5<double>, grid_for(n), dim3(256), 0, c->stream, x.as<double>(), n, plane, RW, x.dof);
  else
    hipLaunchKernelGGL(k_gamma5<float>, grid_for(n), dim3(256), 0, c->stream, x.as<float>(), n, plane, RW, x.dof);
  DD_HIP(hipGetLastError());
}

static inline size_t npairs_of(const MV& a) { return a.reals() / 2; }
static inline size_t tile_pairs_of(const MV& a) { return a.tile_reals() / 2; }

void mv_axpy(ddamg_ctx* c, const double* d_alpha, const MV& x, const MV& y, int sign) {
  DD_CHECK(x.prec == y.prec && x.reals() == y.reals(), DDAMG_EINVAL, "mv_axpy: shape");
  const size_t n = npairs_of(x);
  const int RWp = reals_per_chunk(x.prec) / 2;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_axpy<double>, grid_for(n), dim3(256), 0, c->stream, d_alpha, x.as<double>(), y.as<double>(),
                       n, x.T, RWp, tile_pairs_of(x), (double)sign);
  else
    hipLaunchKernelGGL(k_axpy<float>, grid_for(n), dim3(256), 0, c->stream, d_alpha, x.as<float>(), y.as<float>(), n,
                       x.T, RWp, tile_pairs_of(x), (double)sign);
  DD_HIP(hipGetLastError());
}

void mv_xpay(ddamg_ctx* c, const MV& x, const double* d_alpha, const MV& y) {
  DD_CHECK(x.prec == y.prec && x.reals() == y.reals(), DDAMG_EINVAL, "mv_xpay: shape");
  const size_t n = npairs_of(x);
  const int RWp = reals_per_chunk(x.prec) / 2;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_xpay<double>, grid_for(n), dim3(256), 0, c->stream, x.as<double>(), d_alpha, y.as<double>(),
                       n, x.T, RWp, tile_pairs_of(x));
  else
    hipLaunchKernelGGL(k_xpay<float>, grid_for(n), dim3(256), 0, c->stream, x.as<float>(), d_alpha, y.as<float>(), n,
                       x.T, RWp, tile_pairs_of(x));
  DD_HIP(hipGetLastError());
}

void mv_scale(ddamg_ctx* c, const double* d_alpha, const MV& x) {
  const size_t n = npairs_of(x);
  const int RWp = reals_per_chunk(x.prec) / 2;
  if (x.prec == P64)
    hipLaunchKernelGGL(k_scale<double>, grid_for(n), dim3(256), 0, c->stream, d_alpha, x.as<double>(), n, x.T, RWp,
                       tile_pairs_of(x));
  else
    hipLaunchKernelGGL(k_scale<float>, grid_for(n), dim3(256), 0, c->stream, d_alpha, x.as<float>(), n, x.T, RWp,
                       tile_pairs_of(x));
  DD_HIP(hipGetLastError());
}

void mv_sub(ddamg_ctx* c, const MV& a, const MV& b, const MV& o) {
  DD_CHECK(a.prec == b.prec && a.prec == o.prec && a.reals() == b.reals(), DDAMG_EINVAL, "mv_sub: shape");
  const size_t n = a.reals();
  if (a.prec == P64)
    hipLaunchKernelGGL(k_sub<double>, grid_for(n), dim3(256), 0, c->stream, a.as<double>(), b.as<double>(),
                       o.as<double>(), n);
  else
    hipLaunchKernelGGL(k_sub<float>, grid_for(n), dim3(256), 0, c->stream, a.as<float>(), b.as<float>(), o.as<float>(),
                       n);
  DD_HIP(hipGetLastError());
}

// ------------------------------------------------------ multi-dot ---
struct PtrPack {
  const void* p[MAXK];
};

// Stage 1: partial[bM][j][col] = sum over this workgroup's rows of conj(V_j) w.
// A workgroup is 256 lanes = 32 rows x 8 columns (lane = row*8 + t) and
// handles one group of KB basis vectors (blockIdx.z): the KB accumulators
// are statically indexed registers; w is re-read once per group.
constexpr int KB = 8;
template <typename R, typename RV = R>
__global__ void __launch_bounds__(256) k_multidot1(PtrPack Vs, int k, const R* __restrict__ w, double* __restrict__ part,
                                                   size_t M, int ntiles, int ncol, double vscale) {
  constexpr int RW = Chunk<R>::RW;
  constexpr int T = TTB;
  const int t = threadIdx.x % T, row = threadIdx.x / T;
  const int tile = blockIdx.y;
  const int j0 = blockIdx.z * KB;
  const int kk = min(KB, k - j0);
  const int nbM = gridDim.x;
  const size_t tile_reals = M * T * RW;
  double accr[KB], acci[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) { accr[j] = 0; acci[j] = 0; }
  const RV* vp[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) vp[j] = reinterpret_cast<const RV*>(Vs.p[j0 + (j < kk ? j : 0)]);
  for (size_t m = (size_t)blockIdx.x * 32 + row; m < M; m += (size_t)nbM * 32) {
    const size_t off = (size_t)tile * tile_reals + (m * T + t) * RW;
    R wv[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) wv[r] = w[off + r];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (j < kk) {
        const RV* v = vp[j] + off;
#pragma unroll
        for (int r = 0; r < RW; r += 2) {
          const double vr = v[r], vi = v[r + 1], xr = wv[r], xi = wv[r + 1];
          accr[j] += vr * xr + vi * xi;
          acci[j] += vr * xi - vi * xr;
        }
      }
    }
  }
  // reduce the 8 rows of a wave that share t, then the 4 waves
  __shared__ double red[4][T][KB][2];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    double a = accr[j], b = acci[j];
#pragma unroll
    for (int off = T; off < 64; off <<= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane < T) { red[wave][lane][j][0] = a; red[wave][lane][j][1] = b; }
  }
  __syncthreads();
  if (threadIdx.x < kk * T) {
    const int j = threadIdx.x / T, tt = threadIdx.x % T;
    double a = 0, b = 0;
#pragma unroll
    for (int w4 = 0; w4 < 4; ++w4) { a += red[w4][tt][j][0]; b += red[w4][tt][j][1]; }
    const int col = tile * T + tt;
    double* pp = part + (((size_t)blockIdx.x * k + j0 + j) * ncol + col) * 2;
    pp[0] = a * vscale;
    pp[1] = b * vscale;
  }
}

// Stage 1 for an FP16 basis against FP32 w: KH (up to 16) basis vectors per
// workgroup, so w is read once per group; each lane moves one 16-byte
// chunk of w and one 8-byte chunk of every basis vector per row.  The
// per-lane sums run in FP32 (the FP16 basis carries 2^-11 relative error, far
// above the rounding of a few dozen FP32 additions); the reduction across
// lanes and workgroups is FP64.
template <int KH>
__global__ void __launch_bounds__(256) k_multidot_h(PtrPack Vs, int k, const float* __restrict__ w,
                                                    double* __restrict__ part, size_t M, int ncol, double vscale) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  constexpr int T = TTB;
  const int t = threadIdx.x % T, row = threadIdx.x / T;
  const int tile = blockIdx.y;
  const int j0 = blockIdx.z * KH;
  const int kk = min(KH, k - j0);
  const int nbM = gridDim.x;
  const size_t tile_chunks = M * T;
  float accr[KH], acci[KH];
#pragma unroll
  for (int j = 0; j < KH; ++j) { accr[j] = 0; acci[j] = 0; }
  const float4* w4 = reinterpret_cast<const float4*>(w);
  for (size_t m = (size_t)blockIdx.x * 32 + row; m < M; m += (size_t)nbM * 32) {
    const size_t off = (size_t)tile * tile_chunks + m * T + t;
    const float4 wv = w4[off];
#pragma unroll
    for (int j = 0; j < KH; ++j) {
      if (j < kk) {
        // basis vectors stream through once per step: non-temporal loads
        // keep them from evicting w, which the other groups read again
        const h4 v = __builtin_nontemporal_load(reinterpret_cast<const h4*>(Vs.p[j0 + j]) + off);
        const float v0 = (float)v.x, v1 = (float)v.y, v2 = (float)v.z, v3 = (float)v.w;
        accr[j] += v0 * wv.x + v1 * wv.y + v2 * wv.z + v3 * wv.w;
        acci[j] += v0 * wv.y - v1 * wv.x + v2 * wv.w - v3 * wv.z;
      }
    }
  }
  // reduce the 8 rows of a wave that share t, then the 4 waves (FP64)
  __shared__ double red[4][T][KH][2];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int j = 0; j < KH; ++j) {
    double a = accr[j], b = acci[j];
#pragma unroll
    for (int off = T; off < 64; off <<= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane < T) { red[wave][lane][j][0] = a; red[wave][lane][j][1] = b; }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kk * T; i += 256) {
    const int j = i / T, tt = i % T;
    double a = 0, b = 0;
#pragma unroll
    for (int w4i = 0; w4i < 4; ++w4i) { a += red[w4i][tt][j][0]; b += red[w4i][tt][j][1]; }
    const int col = tile * T + tt;
    double* pp = part + (((size_t)blockIdx.x * k + j0 + j) * ncol + col) * 2;
    pp[0] = a * vscale;
    pp[1] = b * vscale;
  }
}

// second stage: one wavefront per output i = j*ncol + col sums the nbM
// partials (lane-strided, then a fixed shuffle tree: deterministic)
__global__ void __launch_bounds__(64) k_multidot2(const double* __restrict__ part, double* __restrict__ out, int nbM,
                                                  int k, int ncol) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  double a = 0, b = 0;
  for (int q = lane; q < nbM; q += 64) {
    a += part[((size_t)q * k * ncol + i) * 2];
    b += part[((size_t)q * k * ncol + i) * 2 + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if (lane == 0) {
    out[2 * i] = a;
    out[2 * i + 1] = b;
  }
}

// basis vectors per workgroup of the FP16 kernel
constexpr int KH_MAX = 16;

// workgroups along the vector length of the first reduction stage (about
// 4096 in all, 8192 for the FP16 kernel, whose lanes finish a row sooner)
static int multidot_nbm(const MV& w, int k, bool half) {
  const size_t M = (size_t)w.nchunk * w.nsites;
  const int kb = half ? KH_MAX : KB;
  const int ngroups = (k + kb - 1) / kb;
  int nbM = (int)std::min<size_t>((M + 31) / 32, (half ? 8192 : 4096) / ((size_t)w.ntiles * ngroups) + 1);
  return nbM < 1 ? 1 : nbM;
}

// doubles of the partial sums mv_multidot needs for k vectors shaped like w
// (sized for either basis precision)
size_t multidot_partials(const MV& w, int k) {
  return (size_t)std::max(multidot_nbm(w, k, false), multidot_nbm(w, k, true)) * k * w.ncol() * 2;
}

void mv_multidot(ddamg_ctx* c, const MV* Vs, int k, const MV& w, double* d_out) {
  mv_multidot_buf(c, Vs, k, w, d_out, nullptr);
}

// part: partial-sum buffer of at least multidot_partials(w, k) doubles, or
// nullptr for the context's scratch buffer
void mv_multidot_buf(ddamg_ctx* c, const MV* Vs, int k, const MV& w, double* d_out, double* part) {
  DD_CHECK(k >= 1 && k <= MAXK, DDAMG_EINVAL, "mv_multidot: k");
  DD_CHECK(w.T == TTB, DDAMG_EINVAL, "mv_multidot: tile width");
  PtrPack pk;
  const bool half = Vs[0].prec == P16 && w.prec == P32;
  for (int j = 0; j < k; ++j) {
    DD_CHECK((Vs[j].prec == w.prec || half) && Vs[j].prec == Vs[0].prec && Vs[j].reals() == w.reals(), DDAMG_EINVAL,
             "mv_multidot: shape");
    pk.p[j] = Vs[j].p;
  }
  const double vscale = half ? 1.0 / Vs[0].hscale : 1.0;
  const size_t M = (size_t)w.nchunk * w.nsites;
  const int ngroups = (k + (half ? KH_MAX : KB) - 1) / (half ? KH_MAX : KB);
  const int nbM = multidot_nbm(w, k, half);
  const int ncol = w.ncol();
  if (!part) part = scratch(c, multidot_partials(w, k) * sizeof(double));
  dim3 grid(nbM, w.ntiles, ngroups);
  if (half) {
    // groups of up to 16 basis vectors: 54 VGPRs, 8 waves per SIMD (a single
    // group of 40 needs 174 VGPRs and ran 10% slower than re-reading w)
    const int kh = std::min(k, KH_MAX);
    DD_CHECK(w.nchunk * 4 == 2 * w.dof, DDAMG_EINVAL, "mv_multidot: FP32 chunk width");
    if (kh <= 8)
      hipLaunchKernelGGL(k_multidot_h<8>, grid, dim3(256), 0, c->stream, pk, k, w.as<float>(), part, M, ncol, vscale);
    else
      hipLaunchKernelGGL(k_multidot_h<16>, grid, dim3(256), 0, c->stream, pk, k, w.as<float>(), part, M, ncol, vscale);
  } else if (w.prec == P64)
    hipLaunchKernelGGL(k_multidot1<double>, grid, dim3(256), 0, c->stream, pk, k, w.as<double>(), part, M, w.ntiles,
                       ncol, 1.0);
  else
    hipLaunchKernelGGL(k_multidot1<float>, grid, dim3(256), 0, c->stream, pk, k, w.as<float>(), part, M, w.ntiles,
                       ncol, 1.0);
  DD_HIP(hipGetLastError());
  const int n = k * ncol;
  hipLaunchKernelGGL(k_multidot2, dim3(n), dim3(64), 0, c->stream, part, d_out, nbM, k, ncol);
  DD_HIP(hipGetLastError());
}

void mv_dot(ddamg_ctx* c, const MV& a, const MV& b, double* d_out) { mv_multidot(c, &a, 1, b, d_out); }

__global__ void k_re_only(const double* in, double* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[2 * i];
}

void mv_norm2(ddamg_ctx* c, const MV& a, double* d_out) { mv_norm2_buf(c, a, d_out, nullptr, nullptr); }

// cbuf: 2 * ncol doubles, part: multidot_partials(a, 1) doubles (nullptr: context buffers)
void mv_norm2_buf(ddamg_ctx* c, const MV& a, double* d_out, double* cbuf, double* part) {
  if (!cbuf) cbuf = small_buffer(c, 2 * a.ncol());
  mv_multidot_buf(c, &a, 1, a, cbuf, part);
  hipLaunchKernelGGL(k_re_only, dim3((a.ncol() + 255) / 256), dim3(256), 0, c->stream, cbuf, d_out, a.ncol());
  DD_HIP(hipGetLastError());
}

// w += sign * sum_j coef[j][col] V_j, one layout chunk (RW reals of w, the
// same positions of every V_j) per thread, so each lane moves 16 bytes of w
// and 16 (FP32/FP64) or 8 (FP16) bytes of every basis vector per load.
template <typename RV, typename RWt, int RW>
__global__ void k_multiaxpy_chunk(PtrPack Vs, int k, const double* __restrict__ coef, RWt* __restrict__ w,
                                  size_t nunits, int T, size_t tile_units, int ncol, double sign) {
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < nunits; u += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(u / tile_units);
    const int col = tile * T + (int)(u % T);
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    for (int j = 0; j < k; ++j) {
      const RV* v = reinterpret_cast<const RV*>(Vs.p[j]) + u * RW;
      const double cr = coef[((size_t)j * ncol + col) * 2], ci = coef[((size_t)j * ncol + col) * 2 + 1];
      RV vv[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) vv[r] = v[r];
#pragma unroll
      for (int r = 0; r < RW; r += 2) {
        const double vr = vv[r], vi = vv[r + 1];
        acc[r] += cr * vr - ci * vi;
        acc[r + 1] += cr * vi + ci * vr;
      }
    }
    RWt* wp = w + u * RW;
#pragma unroll
    for (int r = 0; r < RW; ++r) wp[r] = (RWt)((double)wp[r] + sign * acc[r]);
  }
}

// w += sign * scale * sum_j coef[j][col] V_j fused with the squared norms of
// the updated w: workgroups of one tile (blockIdx.y) stride over its chunks,
// so each lane keeps one column (t = lane % T) and sums |w|^2 of what it
// stores; partial[bx][col] gets the workgroup's sum (FP64, fixed shuffle tree).
// The coefficients of the tile's T columns are staged in LDS in the
// accumulation type ACC (FP32 for an FP16 basis, whose 2^-11 relative error
// dominates; FP64 otherwise).
// With osc (per column, may be null) the stored result is (w + ...) * osc.
template <typename RV, typename RWt, int RW, typename ACC>
__global__ void __launch_bounds__(256) k_multiaxpy_norm(PtrPack Vs, int k, const double* __restrict__ coef,
                                                        RWt* __restrict__ w, int T, size_t tile_units, int ncol,
                                                        double scale, double* __restrict__ part,
                                                        const double* __restrict__ osc) {
  __shared__ ACC cf[MAXK][TTB][2];
  __shared__ double red[4][TTB];
  const int tile = blockIdx.y;
  for (int i = threadIdx.x; i < k * T; i += blockDim.x) {
    const int j = i / T, tt = i % T;
    const size_t ci = ((size_t)j * ncol + tile * T + tt) * 2;
    cf[j][tt][0] = (ACC)(coef[ci] * scale);
    cf[j][tt][1] = (ACC)(coef[ci + 1] * scale);
  }
  __syncthreads();
  const int t = threadIdx.x % T;
  const size_t base = (size_t)tile * tile_units;
  const ACC sc = osc ? (ACC)osc[tile * T + t] : (ACC)1;
  double n2 = 0;
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < tile_units; u += (size_t)gridDim.x * blockDim.x) {
    ACC acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0;
    for (int j = 0; j < k; ++j) {
      const RV* v = reinterpret_cast<const RV*>(Vs.p[j]) + (base + u) * RW;
      const ACC cr = cf[j][t][0], ci = cf[j][t][1];
      RV vv[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) vv[r] = v[r];
#pragma unroll
      for (int r = 0; r < RW; r += 2) {
        const ACC vr = (ACC)vv[r], vi = (ACC)vv[r + 1];
        acc[r] += cr * vr - ci * vi;
        acc[r + 1] += cr * vi + ci * vr;
      }
    }
    RWt* wp = w + (base + u) * RW;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const RWt o = osc ? (RWt)(((ACC)wp[r] + acc[r]) * sc) : (RWt)((ACC)wp[r] + acc[r]);
      wp[r] = o;
      n2 += (double)o * (double)o;
    }
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int off = T; off < 64; off <<= 1) n2 += __shfl_xor(n2, off, 64);
  if (lane < T) red[wave][lane] = n2;
  __syncthreads();
  if (threadIdx.x < T) {
    double a = 0;
#pragma unroll
    for (int w4 = 0; w4 < 4; ++w4) a += red[w4][threadIdx.x];
    part[(size_t)blockIdx.x * ncol + tile * T + threadIdx.x] = a;
  }
}

// The FP16-basis form that writes the next basis vector directly: the basis
// vectors V_j are stored unnormalised (entry scale c_j per column), so the
// coefficients are h'_j / c_j^2 with h'_j the dots with the stored vectors;
// w' = w - sum_j h_j v_j is formed in FP32 and stored as w' * osc[col] in FP16
// (osc: hscale over a norm estimate), with |w'|^2 per column as above.
__global__ void __launch_bounds__(256) k_multiaxpy_norm_h(PtrPack Vs, int k, const double* __restrict__ coef,
                                                          const double* __restrict__ cinv2,
                                                          const float* __restrict__ w, _Float16* __restrict__ out,
                                                          const double* __restrict__ osc, int T, size_t tile_units,
                                                          int ncol, double scale, double* __restrict__ part) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  __shared__ float cf[MAXK][TTB][2];
  __shared__ double red[4][TTB];
  const int tile = blockIdx.y;
  for (int i = threadIdx.x; i < k * T; i += blockDim.x) {
    const int j = i / T, tt = i % T;
    const size_t ji = (size_t)j * ncol + tile * T + tt;
    const double f = scale * cinv2[ji];
    cf[j][tt][0] = (float)(coef[2 * ji] * f);
    cf[j][tt][1] = (float)(coef[2 * ji + 1] * f);
  }
  __syncthreads();
  const int t = threadIdx.x % T;
  const float os = (float)osc[tile * T + t];
  const size_t base = (size_t)tile * tile_units;
  double n2 = 0;
  for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < tile_units; u += (size_t)gridDim.x * blockDim.x) {
    float acc[4] = {0, 0, 0, 0};
    for (int j = 0; j < k; ++j) {
      const h4 v = __builtin_nontemporal_load(reinterpret_cast<const h4*>(Vs.p[j]) + base + u);
      const float cr = cf[j][t][0], ci = cf[j][t][1];
      const float v0 = (float)v.x, v1 = (float)v.y, v2 = (float)v.z, v3 = (float)v.w;
      acc[0] += cr * v0 - ci * v1;
      acc[1] += cr * v1 + ci * v0;
      acc[2] += cr * v2 - ci * v3;
      acc[3] += cr * v3 + ci * v2;
    }
    const float4 wv = reinterpret_cast<const float4*>(w)[base + u];
    const float o0 = wv.x + acc[0], o1 = wv.y + acc[1], o2 = wv.z + acc[2], o3 = wv.w + acc[3];
    n2 += (double)o0 * o0 + (double)o1 * o1 + (double)o2 * o2 + (double)o3 * o3;
    reinterpret_cast<h4*>(out)[base + u] = h4{(_Float16)(o0 * os), (_Float16)(o1 * os), (_Float16)(o2 * os),
                                              (_Float16)(o3 * os)};
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int off = T; off < 64; off <<= 1) n2 += __shfl_xor(n2, off, 64);
  if (lane < T) red[wave][lane] = n2;
  __syncthreads();
  if (threadIdx.x < T) {
    double a = 0;
#pragma unroll
    for (int w4 = 0; w4 < 4; ++w4) a += red[w4][threadIdx.x];
    part[(size_t)blockIdx.x * ncol + tile * T + threadIdx.x] = a;
  }
}

// out[i] = sum over q < nb of part[q][i] (one wavefront per column, fixed tree)
__global__ void __launch_bounds__(64) k_sum_rows(const double* __restrict__ part, double* __restrict__ out, int nb,
                                                 int ncol) {
  const int i = blockIdx.x, lane = threadIdx.x;
  double a = 0;
  for (int q = lane; q < nb; q += 64) a += part[(size_t)q * ncol + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if (lane == 0) out[i] = a;
}

// FP64 w += sign * sum_j coef V_j with FP32 V_j (one complex per FP64 chunk,
// two per FP32 chunk: the FP32 position is recomputed from the complex index)
__global__ void k_multiaxpy_mixed(PtrPack Vs, int k, const double* __restrict__ coef, double* __restrict__ w,
                                  size_t npairs, int T, int nsites, size_t tile_pairs_w, size_t tile_pairs_v, int ncol,
                                  double sign) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < npairs; i += (size_t)gridDim.x * blockDim.x) {
    const int tile = (int)(i / tile_pairs_w);
    size_t r = i % tile_pairs_w;       // ((kc * nsites + s) * T + t)   (one complex per FP64 chunk)
    const int t = (int)(r % T);
    r /= T;
    const int s = (int)(r % nsites);
    const int kc = (int)(r / nsites);
    const size_t iv = (size_t)tile * tile_pairs_v + (((size_t)(kc / 2) * nsites + s) * T + t) * 2 + (kc % 2);
    const int col = tile * T + t;
    double ar = 0, ai = 0;
    for (int j = 0; j < k; ++j) {
      const float* v = reinterpret_cast<const float*>(Vs.p[j]);
      const double cr = coef[((size_t)j * ncol + col) * 2], ci = coef[((size_t)j * ncol + col) * 2 + 1];
      const double vr = v[2 * iv], vi = v[2 * iv + 1];
      ar += cr * vr - ci * vi;
      ai += cr * vi + ci * vr;
    }
    w[2 * i] += sign * ar;
    w[2 * i + 1] += sign * ai;
  }
}

void mv_multiaxpy(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign) {
  DD_CHECK(k >= 0 && k <= MAXK, DDAMG_EINVAL, "mv_multiaxpy: k");
  if (k == 0) return;
  PtrPack pk;
  for (int j = 0; j < k; ++j) {
    DD_CHECK(Vs[j].nsites == w.nsites && Vs[j].dof == w.dof && Vs[j].ntiles == w.ntiles && Vs[j].prec == Vs[0].prec,
             DDAMG_EINVAL, "mv_multiaxpy: shape");
    pk.p[j] = Vs[j].p;
  }
  const size_t n = npairs_of(w);
  const size_t nunits = (size_t)w.ntiles * w.nchunk * w.nsites * w.T;
  const size_t tile_units = (size_t)w.nchunk * w.nsites * w.T;
  if (Vs[0].prec == P16) {
    DD_CHECK(w.prec == P32, DDAMG_EINVAL, "mv_multiaxpy: FP16 basis needs FP32 w");
    hipLaunchKernelGGL((k_multiaxpy_chunk<_Float16, float, 4>), grid_for(nunits), dim3(256), 0, c->stream, pk, k,
                       d_coef, w.as<float>(), nunits, w.T, tile_units, w.ncol(), (double)sign / Vs[0].hscale);
    DD_HIP(hipGetLastError());
    return;
  }
  if (Vs[0].prec == w.prec) {
    if (w.prec == P64)
      hipLaunchKernelGGL((k_multiaxpy_chunk<double, double, 2>), grid_for(nunits), dim3(256), 0, c->stream, pk, k,
                         d_coef, w.as<double>(), nunits, w.T, tile_units, w.ncol(), (double)sign);
    else
      hipLaunchKernelGGL((k_multiaxpy_chunk<float, float, 4>), grid_for(nunits), dim3(256), 0, c->stream, pk, k,
                         d_coef, w.as<float>(), nunits, w.T, tile_units, w.ncol(), (double)sign);
    DD_HIP(hipGetLastError());
    return;
  }
  DD_CHECK(Vs[0].prec == P32 && w.prec == P64, DDAMG_EINVAL, "mv_multiaxpy: precisions");
  hipLaunchKernelGGL(k_multiaxpy_mixed, grid_for(n), dim3(256), 0, c->stream, pk, k, d_coef, w.as<double>(), n, w.T,
                     w.nsites, tile_pairs_of(w), tile_pairs_of(Vs[0]), w.ncol(), (double)sign);
  DD_HIP(hipGetLastError());
}

static int multiaxpy_blocks(const MV& w) {
  const size_t tile_units = (size_t)w.nchunk * w.nsites * w.T;
  return (int)std::max<size_t>(1, std::min<size_t>((tile_units + 255) / 256, 3072 / w.ntiles));
}

size_t multiaxpy_partials(const MV& w) { return (size_t)multiaxpy_blocks(w) * w.ncol(); }

static void multiaxpy_norm_launch(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign,
                                  const double* d_osc, double* d_n2, double* part) {
  PtrPack pk;
  for (int j = 0; j < k; ++j) {
    DD_CHECK(Vs[j].nsites == w.nsites && Vs[j].dof == w.dof && Vs[j].ntiles == w.ntiles && Vs[j].prec == Vs[0].prec,
             DDAMG_EINVAL, "mv_multiaxpy_norm2: shape");
    pk.p[j] = Vs[j].p;
  }
  const bool half = Vs[0].prec == P16 && w.prec == P32;
  const size_t tile_units = (size_t)w.nchunk * w.nsites * w.T;
  const int nb = multiaxpy_blocks(w);
  const int ncol = w.ncol();
  if (!part) part = scratch(c, (size_t)nb * ncol * sizeof(double));
  const dim3 grid(nb, w.ntiles);
  if (half)
    hipLaunchKernelGGL((k_multiaxpy_norm<_Float16, float, 4, float>), grid, dim3(256), 0, c->stream, pk, k, d_coef,
                       w.as<float>(), w.T, tile_units, ncol, (double)sign / Vs[0].hscale, part, d_osc);
  else if (w.prec == P64)
    hipLaunchKernelGGL((k_multiaxpy_norm<double, double, 2, double>), grid, dim3(256), 0, c->stream, pk, k, d_coef,
                       w.as<double>(), w.T, tile_units, ncol, (double)sign, part, d_osc);
  else
    hipLaunchKernelGGL((k_multiaxpy_norm<float, float, 4, double>), grid, dim3(256), 0, c->stream, pk, k, d_coef,
                       w.as<float>(), w.T, tile_units, ncol, (double)sign, part, d_osc);
  DD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_rows, dim3(ncol), dim3(64), 0, c->stream, part, d_n2, nb, ncol);
  DD_HIP(hipGetLastError());
}

// w += sign * sum_j coef V_j and d_n2[col] = ||w_col||^2 of the result in one
// pass over w (same-precision or FP16 bases; other pairs take the two-pass form)
void mv_multiaxpy_norm2(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign,
                        double* d_n2) {
  DD_CHECK(k >= 1 && k <= MAXK, DDAMG_EINVAL, "mv_multiaxpy_norm2: k");
  const bool half = Vs[0].prec == P16 && w.prec == P32;
  if (!(half || Vs[0].prec == w.prec) || w.T != TTB) {
    mv_multiaxpy(c, Vs, k, d_coef, w, sign);
    mv_norm2(c, w, d_n2);
    return;
  }
  multiaxpy_norm_launch(c, Vs, k, d_coef, w, sign, nullptr, d_n2, nullptr);
}

void mv_multiaxpy_scale_norm2(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const MV& w, int sign,
                              const double* d_osc, double* d_n2, double* part) {
  DD_CHECK(k >= 1 && k <= MAXK, DDAMG_EINVAL, "mv_multiaxpy_scale_norm2: k");
  DD_CHECK(Vs[0].prec == w.prec && (w.prec == P32 || w.prec == P64) && w.T == TTB, DDAMG_EINVAL,
           "mv_multiaxpy_scale_norm2: FP32 or FP64 basis of the vector's precision");
  multiaxpy_norm_launch(c, Vs, k, d_coef, w, sign, d_osc, d_n2, part);
}

// w' = w - sum_j (coef_j / c_j^2) V_j for an FP16 basis stored unnormalised
// (d_cinv2[j][col] = 1 / c_j^2), written into the FP16 vector `out` as
// w' * d_osc[col] (in units of out.hscale), and d_n2[col] = |w'|^2
void mv_multiaxpy_norm2_into_f16(ddamg_ctx* c, const MV* Vs, int k, const double* d_coef, const double* d_cinv2,
                                 const MV& w, const MV& out, const double* d_osc, double* d_n2) {
  DD_CHECK(k >= 1 && k <= MAXK && w.prec == P32 && out.prec == P16 && w.T == TTB, DDAMG_EINVAL,
           "mv_multiaxpy_norm2_into_f16: forms");
  PtrPack pk;
  for (int j = 0; j < k; ++j) {
    DD_CHECK(Vs[j].prec == P16 && Vs[j].reals() == w.reals(), DDAMG_EINVAL, "mv_multiaxpy_norm2_into_f16: shape");
    pk.p[j] = Vs[j].p;
  }
  DD_CHECK(out.reals() == w.reals(), DDAMG_EINVAL, "mv_multiaxpy_norm2_into_f16: output shape");
  const size_t tile_units = (size_t)w.nchunk * w.nsites * w.T;
  const int nb = (int)std::max<size_t>(1, std::min<size_t>((tile_units + 255) / 256, 3072 / w.ntiles));
  const int ncol = w.ncol();
  double* part = scratch(c, (size_t)nb * ncol * sizeof(double));
  hipLaunchKernelGGL(k_multiaxpy_norm_h, dim3(nb, w.ntiles), dim3(256), 0, c->stream, pk, k, d_coef, d_cinv2,
                     w.as<float>(), out.as<_Float16>(), d_osc, w.T, tile_units, ncol, -1.0 / Vs[0].hscale, part);
  DD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_rows, dim3(ncol), dim3(64), 0, c->stream, part, d_n2, nb, ncol);
  DD_HIP(hipGetLastError());
}

}  // namespace ddamg
