// Context construction: lattice geometry of every level in the internal
// block-major order, neighbour tables, gauge field upload (FP64 full links,
// FP32 2-row compressed links), SAP colour lists, counter-based random setup
// vectors and the small device/host staging buffers.
#include <cmath>
#include <algorithm>
#include <cstring>

#include "common.h"
#include "device.h"

namespace ddamg {

static void coords(int i, const int* L, int* x) {
  x[0] = i % L[0];
  i /= L[0];
  x[1] = i % L[1];
  i /= L[1];
  x[2] = i % L[2];
  x[3] = i / L[2];
}
static int lex(const int* x, const int* L) { return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3])); }

// 4-d Morton key of block coordinates (bits interleaved, x lowest).
static uint64_t morton4(const int* b) {
  uint64_t k = 0;
  for (int bit = 0; bit < 16; ++bit)
    for (int m = 0; m < 4; ++m) k |= (uint64_t)((b[m] >> bit) & 1) << (4 * bit + m);
  return k;
}

// Internal order of a level: the lattice is cut into blocks of extent grp;
// blocks are numbered along a 4-d Morton (Z-order) curve, so that blocks
// adjacent in any direction are usually close in memory (their spinors are
// still in L2 when a neighbouring block is processed); sites are
// lexicographic inside a block.
void build_geometry(ddamg_ctx* c, int level, const int* dims, const int* grp, int dof, bool fine) {
  LevelGeom& g = c->geom[level];
  int B[4];
  for (int m = 0; m < 4; ++m) {
    DD_CHECK(dims[m] > 0 && grp[m] > 0 && dims[m] % grp[m] == 0, DDAMG_EINVAL,
             "lattice extent not divisible by the block/aggregate extent");
    g.dims[m] = dims[m];
    g.grp[m] = grp[m];
    B[m] = dims[m] / grp[m];
  }
  g.V = dims[0] * dims[1] * dims[2] * dims[3];
  g.gsize = grp[0] * grp[1] * grp[2] * grp[3];
  g.dof = dof;
  const int nblk = B[0] * B[1] * B[2] * B[3];
  std::vector<std::pair<uint64_t, int>> keys(nblk);
  for (int L = 0; L < nblk; ++L) {
    int b[4];
    coords(L, B, b);
    keys[L] = {morton4(b), L};
  }
  std::sort(keys.begin(), keys.end());
  g.blk_num.assign(nblk, 0);
  g.blk_lex.assign(nblk, 0);
  for (int r = 0; r < nblk; ++r) {
    g.blk_lex[r] = keys[r].second;
    g.blk_num[keys[r].second] = r;
  }
  // block numbers along t for every xyz column of 4^4 blocks (t-walk stencil)
  if (fine && grp[0] == 4 && grp[1] == 4 && grp[2] == 4 && grp[3] == 4) {
    std::vector<int> walk((size_t)nblk);
    for (int bz = 0; bz < B[2]; ++bz)
      for (int by = 0; by < B[1]; ++by)
        for (int bx = 0; bx < B[0]; ++bx)
          for (int bt = 0; bt < B[3]; ++bt) {
            const int bb[4] = {bx, by, bz, bt};
            walk[((size_t)(bx + B[0] * (by + B[1] * bz))) * B[3] + bt] = g.blk_num[lex(bb, B)];
          }
    c->d_walk_blk = (int*)c->pool.alloc(walk.size() * sizeof(int));
    DD_HIP(hipMemcpy(c->d_walk_blk, walk.data(), walk.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  g.int2can.assign(g.V, 0);
  g.can2int.assign(g.V, 0);
  for (int i = 0; i < g.V; ++i) {
    int x[4], b[4], l[4];
    coords(i, dims, x);
    for (int m = 0; m < 4; ++m) { b[m] = x[m] / grp[m]; l[m] = x[m] % grp[m]; }
    const int s = g.blk_num[lex(b, B)] * g.gsize + lex(l, grp);
    g.can2int[i] = s;
    g.int2can[s] = i;
  }
  std::vector<int> nbr((size_t)8 * g.V);
  for (int s = 0; s < g.V; ++s) {
    int x[4];
    coords(g.int2can[s], dims, x);
    for (int h = 0; h < 8; ++h) {
      const int mu = h % 4;
      const bool fwd = h < 4;
      int y[4] = {x[0], x[1], x[2], x[3]};
      y[mu] = (x[mu] + (fwd ? 1 : dims[mu] - 1)) % dims[mu];
      int e = g.can2int[lex(y, dims)];
      if (fine && mu == 3 && ((fwd && x[3] == dims[3] - 1) || (!fwd && x[3] == 0)))
        e |= (int)0x80000000u;   // antiperiodic time boundary
      nbr[(size_t)h * g.V + s] = e;
    }
  }
  g.d_nbr = (int*)c->pool.alloc(nbr.size() * sizeof(int));
  g.d_int2can = (int*)c->pool.alloc((size_t)g.V * sizeof(int));
  g.d_can2int = (int*)c->pool.alloc((size_t)g.V * sizeof(int));
  DD_HIP(hipMemcpy(g.d_nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(g.d_int2can, g.int2can.data(), (size_t)g.V * sizeof(int), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(g.d_can2int, g.can2int.data(), (size_t)g.V * sizeof(int), hipMemcpyHostToDevice));
  if (level > 0) {
    // a coarse site is a block of the previous level: its lexicographic block
    // index equals the coarse canonical site index
    LevelGeom& gf = c->geom[level - 1];
    std::vector<int> blk_of(g.V), coarse_of(g.V);
    for (int a = 0; a < g.V; ++a) {
      const int b = gf.blk_num[g.int2can[a]];
      blk_of[a] = b;
      coarse_of[b] = a;
    }
    g.d_blk_of_coarse = (int*)c->pool.alloc((size_t)g.V * sizeof(int));
    gf.d_coarse_of_blk = (int*)c->pool.alloc((size_t)g.V * sizeof(int));
    DD_HIP(hipMemcpy(g.d_blk_of_coarse, blk_of.data(), (size_t)g.V * sizeof(int), hipMemcpyHostToDevice));
    DD_HIP(hipMemcpy(gf.d_coarse_of_blk, coarse_of.data(), (size_t)g.V * sizeof(int), hipMemcpyHostToDevice));
  }
}

// SAP colour lists (chessboard over blocks).
void build_sap_lists(ddamg_ctx* c) {
  const LevelGeom& g = c->geom[0];
  int B[4];
  for (int m = 0; m < 4; ++m) {
    B[m] = g.dims[m] / g.grp[m];
    DD_CHECK(B[m] == 1 || B[m] % 2 == 0, DDAMG_EINVAL,
             "red-black SAP needs an even number of blocks in every direction");
  }
  std::vector<int> lists[2];
  const int nb = B[0] * B[1] * B[2] * B[3];
  for (int L = 0; L < nb; ++L) {
    int x[4];
    coords(L, B, x);
    lists[(x[0] + x[1] + x[2] + x[3]) % 2].push_back(g.blk_num[L]);
  }
  for (auto& l : lists) std::sort(l.begin(), l.end());
  for (int col = 0; col < 2; ++col) {
    c->n_sap[col] = (int)lists[col].size();
    c->d_sap_list[col] = (int*)c->pool.alloc(std::max<size_t>(1, lists[col].size()) * sizeof(int));
    if (!lists[col].empty())
      DD_HIP(hipMemcpy(c->d_sap_list[col], lists[col].data(), lists[col].size() * sizeof(int), hipMemcpyHostToDevice));
  }
}

// Gauge field: canonical [V][mu][3][3] complex -> FP64 [mu][9][V] (complex per
// chunk) and FP32 [mu][3][V] float4 holding rows 0 and 1.
void upload_gauge(ddamg_ctx* c, const double* gauge, int on_device) {
  const LevelGeom& g = c->geom[0];
  const size_t V = g.V;
  std::vector<double> host;
  const double* G = gauge;
  if (on_device) {
    host.resize(V * 4 * 9 * 2);
    DD_HIP(hipMemcpy(host.data(), gauge, host.size() * sizeof(double), hipMemcpyDeviceToHost));
    G = host.data();
  }
  for (size_t i = 0; i < V * 4 * 9 * 2; ++i)
    DD_CHECK(std::isfinite(G[i]), DDAMG_EINVAL, "gauge field contains NaN/Inf");
  std::vector<double> u64(V * 4 * 9 * 2);
  std::vector<float> u32(V * 4 * 3 * 4), u32f(V * 4 * 5 * 4, 0.0f);
  const int Lt = g.dims[3];
  const size_t V3 = (size_t)g.dims[0] * g.dims[1] * g.dims[2];
  for (size_t s = 0; s < V; ++s) {
    const size_t cs = g.int2can[s];
    const bool tedge = (cs / V3) == (size_t)(Lt - 1);
    for (int mu = 0; mu < 4; ++mu) {
      const double* src = G + ((cs * 4 + mu) * 9) * 2;
      // antiperiodic time: the t-link leaving the last time slice carries the sign
      const double sg = (mu == 3 && tedge) ? -1.0 : 1.0;
      for (int k = 0; k < 9; ++k) {
        u64[(((size_t)mu * 9 + k) * V + s) * 2] = sg * src[2 * k];
        u64[(((size_t)mu * 9 + k) * V + s) * 2 + 1] = sg * src[2 * k + 1];
        u32f[(((size_t)mu * 5 + k / 2) * V + s) * 4 + (k % 2) * 2] = (float)(sg * src[2 * k]);
        u32f[(((size_t)mu * 5 + k / 2) * V + s) * 4 + (k % 2) * 2 + 1] = (float)(sg * src[2 * k + 1]);
      }
      for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 4; ++r) u32[(((size_t)mu * 3 + q) * V + s) * 4 + r] = (float)src[4 * q + r];
    }
  }
  c->d_U64 = (double*)c->pool.alloc(u64.size() * sizeof(double));
  c->d_U32 = (float*)c->pool.alloc(u32.size() * sizeof(float));
  c->d_U32f = (float*)c->pool.alloc(u32f.size() * sizeof(float));
  DD_HIP(hipMemcpy(c->d_U64, u64.data(), u64.size() * sizeof(double), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(c->d_U32, u32.data(), u32.size() * sizeof(float), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(c->d_U32f, u32f.data(), u32f.size() * sizeof(float), hipMemcpyHostToDevice));
}

// Counter-based Gaussian numbers: splitmix64 of (seed, stream, index), Box-Muller.
__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__global__ void k_random(double* __restrict__ X, const int* __restrict__ int2can, int ncol, int V, int dof,
                         size_t tile_reals, uint64_t seed) {
  const size_t total = (size_t)ncol * V * dof;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % dof);
    const size_t r = i / dof;
    const int s = (int)(r % V);
    const int col = (int)(r / V);
    const uint64_t ctr = ((uint64_t)col * V + int2can[s]) * dof + k;
    const uint64_t a = splitmix(seed ^ splitmix(2 * ctr)), b = splitmix(seed ^ splitmix(2 * ctr + 1));
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    const double rad = sqrt(-2.0 * log(u1));
    const int tile = col / 8, t = col % 8;
    double* q = X + (size_t)tile * tile_reals + (((size_t)k * V + s) * 8 + t) * 2;
    q[0] = rad * cos(6.283185307179586 * u2);
    q[1] = rad * sin(6.283185307179586 * u2);
  }
}

void random_fill(ddamg_ctx* c, int level, const MV& X, int ncol, uint64_t seed) {
  DD_CHECK(X.prec == P64 && X.T == 8, DDAMG_EINVAL, "random_fill: FP64, T = 8");
  const LevelGeom& g = c->geom[level];
  const size_t n = (size_t)ncol * g.V * g.dof;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_random, dim3((unsigned)blocks), dim3(256), 0, c->stream, X.as<double>(), g.d_int2can, ncol, g.V,
                     g.dof, X.tile_reals(), seed);
  DD_HIP(hipGetLastError());
}

double* scratch(ddamg_ctx* c, size_t bytes) {
  if (bytes > c->scratch_bytes) {
    if (c->d_scratch) {
      DD_HIP(hipStreamSynchronize(c->stream));
      c->pool.release(c->d_scratch);
    }
    c->scratch_bytes = std::max(bytes, (size_t)1 << 20);
    c->d_scratch = (double*)c->pool.alloc(c->scratch_bytes);
  }
  return c->d_scratch;
}

double* small_buffer(ddamg_ctx* c, int n) {
  if (n > c->small_n) {
    if (c->d_small) {
      DD_HIP(hipStreamSynchronize(c->stream));
      c->pool.release(c->d_small);
    }
    c->small_n = std::max(n, 4096);
    c->d_small = (double*)c->pool.alloc((size_t)c->small_n * sizeof(double));
  }
  return c->d_small;
}

void copy_to_host(ddamg_ctx* c, const void* d, void* h, size_t bytes) {
  if (bytes > c->pinned_bytes) {
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    c->pinned_bytes = std::max(bytes, (size_t)1 << 16);
    DD_HIP(hipHostMalloc((void**)&c->h_pinned, c->pinned_bytes, hipHostMallocDefault));
  }
  DD_HIP(hipMemcpyAsync(c->h_pinned, d, bytes, hipMemcpyDeviceToHost, c->stream));
  DD_HIP(hipStreamSynchronize(c->stream));
  std::memcpy(h, c->h_pinned, bytes);
}

static bool timing_on(ddamg_ctx* c, int cls) {
  if (c->time_sap != cls) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  DD_HIP(hipStreamIsCapturing(c->stream, &cs));
  return cs == hipStreamCaptureStatusNone;
}

void kernel_timing_begin(ddamg_ctx* c, int cls) {
  if (!timing_on(c, cls)) return;
  if (c->sap_ev_used + 2 > c->sap_ev.size()) {
    hipEvent_t a, b;
    DD_HIP(hipEventCreate(&a));
    DD_HIP(hipEventCreate(&b));
    c->sap_ev.push_back(a);
    c->sap_ev.push_back(b);
  }
  DD_HIP(hipEventRecord(c->sap_ev[c->sap_ev_used], c->stream));
}

void kernel_timing_end(ddamg_ctx* c, int cls, int ntiles) {
  if (!timing_on(c, cls)) return;
  DD_HIP(hipEventRecord(c->sap_ev[c->sap_ev_used + 1], c->stream));
  c->sap_ev_used += 2;
  c->sap_ev_tiles.resize(c->sap_ev_used / 2);
  c->sap_ev_tiles.back() = ntiles;
}

void sap_timing_begin(ddamg_ctx* c) { kernel_timing_begin(c, TIMED_SAP); }
void sap_timing_end(ddamg_ctx* c, int ntiles) { kernel_timing_end(c, TIMED_SAP, ntiles); }

void sap_timing_collect(ddamg_ctx* c) {
  double ms = 0;
  long long tiles = 0;
  if (c->sap_ev_used) DD_HIP(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i + 1 < c->sap_ev_used; i += 2) {
    float e = 0;
    DD_HIP(hipEventElapsedTime(&e, c->sap_ev[i], c->sap_ev[i + 1]));
    ms += e;
    tiles += c->sap_ev_tiles[i / 2];
  }
  c->st.sap_kernel_ms = ms;
  c->st.sap_kernel_launches = (long long)(c->sap_ev_used / 2);
  c->st.sap_kernel_tiles = tiles;
  c->sap_ev_used = 0;
  c->sap_ev_tiles.clear();
}

void operator_apply(ddamg_ctx* c, int level, const MV& x, const MV& y, const double* d_mu) {
  if (level == 0) fine_dslash(c, x, y, d_mu);
  else coarse_apply(c, level, x, y, d_mu);
}

}  // namespace ddamg
