// Device helpers: complex arithmetic, tiled-layout chunk access, XCD-aware
// workgroup numbering.
#pragma once

#include <hip/hip_runtime.h>

namespace ddamg {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> conj_(cx<R> a) { return {a.re, -a.im}; }
// multiply by +i / -i
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }
// a += b * c ; a += conj(b) * c
template <typename R>
__device__ __forceinline__ void cmac(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
template <typename R>
__device__ __forceinline__ void cmac_conj(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}

// Real type -> 16-byte chunk type and reals per chunk.
template <typename R> struct Chunk;
template <> struct Chunk<double> { using type = double2; static constexpr int RW = 2; };
template <> struct Chunk<float> { using type = float4; static constexpr int RW = 4; };

// Load all `NC` complexes of one (site, column) from a tile: chunk k sits at
// ((k*nsites + s)*T + t) chunks from the tile base.
template <typename R, int NC>
__device__ __forceinline__ void load_cx(const R* __restrict__ tile, int nsites, int T, int s, int t,
                                        cx<R> (&v)[NC]) {
  using C = typename Chunk<R>::type;
  const C* b = reinterpret_cast<const C*>(tile);
  if constexpr (Chunk<R>::RW == 2) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      C c = b[((size_t)k * nsites + s) * T + t];
      v[k] = {c.x, c.y};
    }
  } else {
#pragma unroll
    for (int k = 0; k < NC / 2; ++k) {
      C c = b[((size_t)k * nsites + s) * T + t];
      v[2 * k] = {c.x, c.y};
      v[2 * k + 1] = {c.z, c.w};
    }
  }
}

// Load NC complexes of one (site, column) from an FP16 multivector in the
// FP32 layout (two complexes per 8-byte chunk), times `scale`.
template <int NC>
__device__ __forceinline__ void load_cx_f16(const _Float16* __restrict__ tile, int nsites, int T, int s, int t,
                                            float scale, cx<float> (&v)[NC]) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  const h4* b = reinterpret_cast<const h4*>(tile);
#pragma unroll
  for (int k = 0; k < NC / 2; ++k) {
    const h4 c = b[((size_t)k * nsites + s) * T + t];
    v[2 * k] = {(float)c.x * scale, (float)c.y * scale};
    v[2 * k + 1] = {(float)c.z * scale, (float)c.w * scale};
  }
}

template <typename R, int NC>
__device__ __forceinline__ void store_cx(R* __restrict__ tile, int nsites, int T, int s, int t,
                                         const cx<R> (&v)[NC]) {
  using C = typename Chunk<R>::type;
  C* b = reinterpret_cast<C*>(tile);
  if constexpr (Chunk<R>::RW == 2) {
#pragma unroll
    for (int k = 0; k < NC; ++k) b[((size_t)k * nsites + s) * T + t] = C{v[k].re, v[k].im};
  } else {
#pragma unroll
    for (int k = 0; k < NC / 2; ++k)
      b[((size_t)k * nsites + s) * T + t] = C{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
  }
}

// Single complex k of one (site, column).
template <typename R>
__device__ __forceinline__ cx<R> load_one(const R* __restrict__ tile, int nsites, int T, int s, int t, int k) {
  constexpr int RW = Chunk<R>::RW;
  constexpr int CPC = RW / 2;   // complexes per chunk
  const R* q = tile + (((size_t)(k / CPC) * nsites + s) * T + t) * RW + (k % CPC) * 2;
  return {q[0], q[1]};
}

// gfx950 dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Renumber so that every XCD works on one contiguous range
// of logical workgroups (neighbouring sites share L2 lines).
__device__ __forceinline__ int xcd_remap(int i, int G) {
  constexpr int NX = 8;
  int x = i % NX, l = i / NX;
  int per = G / NX, rem = G % NX;
  return x * per + (x < rem ? x : rem) + l;
}

}  // namespace ddamg
