// Shared device/host helpers of the dbq library: errors, complex arithmetic, even-odd lattice
// indexing, XCD-aware block numbering and deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "dbq.h"

namespace dbq {

// ----------------------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DBQ_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::dbq::Error(DBQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define DBQ_CHECK(cond, msg)                                   \
  do {                                                         \
    if (!(cond)) throw ::dbq::Error(DBQ_EINVAL, (msg));        \
  } while (0)

// ----------------------------------------------------------------------------- complex
template <typename T>
struct cx {
  T re, im;
};
template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> ti(cx<T> a) { return {-a.im, a.re}; }
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  // Smith's algorithm keeps the intermediate quotient in range
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    T r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
typedef cx<double> zd;
typedef cx<float> zf;

// ----------------------------------------------------------------------------- fast division
// q = n / d for 0 <= n < 2^31 via a 32-bit magic multiplier (round-up method of Granlund and
// Montgomery): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, q = (umulhi(n, m) + n) >> l.
struct FastDiv {
  uint32_t d, m, l;
  FastDiv() : d(1), m(1), l(0) {}
  explicit FastDiv(uint32_t dv) : d(dv) {
    l = 0;
    while ((1ull << l) < dv) ++l;
    uint64_t t = ((1ull << 32) * ((1ull << l) - dv)) / dv;
    m = uint32_t(t + 1);
  }
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t hi = __umulhi(n, m);
#else
    uint32_t hi = uint32_t((uint64_t(n) * m) >> 32);
#endif
    return (hi + n) >> l;
  }
};

// ----------------------------------------------------------------------------- lattice geometry
// Internal site order: even-odd, blocked into 4-d tiles.  The lattice is cut into tiles of
// T0 x T1 x T2 x T3 sites (powers of two dividing the extents, so every tile origin has an even
// coordinate sum and each tile holds T/2 sites of either parity).  Site x of parity p gets
//   eo = p * V/2 + tile(x) * T/2 + (in-tile lex(x) >> 1),
// tile(x) = lexicographic index of floor(x_mu / T_mu) over the tile grid and in-tile lex the
// lexicographic index of x_mu mod T_mu inside the tile.  Consecutive indices of one parity fill
// one tile before the next, so a site's eight neighbours mostly lie in the same tile (or the
// neighbouring one in x or y) and are served by the cache that already holds it.  With a single
// tile covering the lattice this is the plain order p * V/2 + (lex >> 1).
struct Geom {
  int L[4];
  int V, Vh;
  int T[4];   // tile extents
  int lT[4];  // log2 of the tile extents
  int NT[4];  // tiles per direction
  int lTh;    // log2 of the half-sites per tile
  FastDiv dNT0, dNT1, dNT2;
};

// Tile extents for a lattice: per direction the largest power of two that divides L_mu and
// does not exceed 4 (all extents are even, so at least 2).  A tile holds at most 256 sites.
constexpr int TILE_MAX = 4;
inline void choose_tile(const int32_t L[4], int T[4]) {
  for (int i = 0; i < 4; ++i) {
    int t = 2;
    while (t * 2 <= TILE_MAX && L[i] % (t * 2) == 0) t *= 2;
    T[i] = t;
  }
}

inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline Geom make_geom(const int32_t L[4]) {
  Geom g;
  for (int i = 0; i < 4; ++i) g.L[i] = L[i];
  g.V = L[0] * L[1] * L[2] * L[3];
  g.Vh = g.V / 2;
  choose_tile(L, g.T);
  for (int i = 0; i < 4; ++i) {
    g.lT[i] = ilog2(g.T[i]);
    g.NT[i] = L[i] / g.T[i];
  }
  g.lTh = g.lT[0] + g.lT[1] + g.lT[2] + g.lT[3] - 1;
  g.dNT0 = FastDiv(uint32_t(g.NT[0]));
  g.dNT1 = FastDiv(uint32_t(g.NT[1]));
  g.dNT2 = FastDiv(uint32_t(g.NT[2]));
  return g;
}

// coordinates (x, y, z, t) and parity of internal index s
__host__ __device__ __forceinline__ void eo_coords(const Geom& g, int s, int c[4], int& p) {
  p = s >= g.Vh ? 1 : 0;
  const uint32_t h = uint32_t(s - p * g.Vh);
  const uint32_t tile = h >> g.lTh;
  // in-tile lex of the even-x member of the pair that shares this half index
  uint32_t r = (h & ((1u << g.lTh) - 1u)) << 1;
  const int ix = int(r & uint32_t(g.T[0] - 1));
  r >>= g.lT[0];
  const int iy = int(r & uint32_t(g.T[1] - 1));
  r >>= g.lT[1];
  const int iz = int(r & uint32_t(g.T[2] - 1));
  const int it = int(r >> g.lT[2]);
  const uint32_t q1 = g.dNT0.div(tile);
  const uint32_t q2 = g.dNT1.div(q1);
  const uint32_t q3 = g.dNT2.div(q2);
  c[1] = (int(q1 - q2 * uint32_t(g.NT[1])) << g.lT[1]) + iy;
  c[2] = (int(q2 - q3 * uint32_t(g.NT[2])) << g.lT[2]) + iz;
  c[3] = (int(q3) << g.lT[3]) + it;
  // tile origins have even coordinate sums: the parity of x is that of its in-tile coordinates
  c[0] = (int(tile - q1 * uint32_t(g.NT[0])) << g.lT[0]) + ix + ((p + iy + iz + it) & 1);
}

__host__ __device__ __forceinline__ int lex_index(const Geom& g, const int c[4]) {
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

__host__ __device__ __forceinline__ int eo_of_coords(const Geom& g, const int c[4]) {
  const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  const int tile = (c[0] >> g.lT[0]) +
                   g.NT[0] * ((c[1] >> g.lT[1]) + g.NT[1] * ((c[2] >> g.lT[2]) +
                                                             g.NT[2] * (c[3] >> g.lT[3])));
  const int il = (c[0] & (g.T[0] - 1)) | ((c[1] & (g.T[1] - 1)) << g.lT[0]) |
                 ((c[2] & (g.T[2] - 1)) << (g.lT[0] + g.lT[1])) |
                 ((c[3] & (g.T[3] - 1)) << (g.lT[0] + g.lT[1] + g.lT[2]));
  return p * g.Vh + (tile << g.lTh) + (il >> 1);
}

// internal index of the neighbour x + dir*mu (dir = +1 or -1), periodic
template <int MU, int DIR>
__host__ __device__ __forceinline__ int eo_neighbour(const Geom& g, const int c[4]) {
  int d[4] = {c[0], c[1], c[2], c[3]};
  int v = d[MU] + DIR;
  if (DIR > 0) v = (v == g.L[MU]) ? 0 : v;
  else v = (v < 0) ? g.L[MU] - 1 : v;
  d[MU] = v;
  return eo_of_coords(g, d);
}

// Order in which the blocks of a tile launch visit (tile, rhs chunk) pairs; memory holds the
// tiles lexicographically in every case, and a block's partial sums go to its tile's slot, so
// the order changes no result.  Blocks reach the XCDs in contiguous ranges of the logical index
// (xcd_block), and one XCD's L2 serves a staged face to the block of the neighbouring tile only
// if that block runs on the same XCD while the face is still cached.
//   0: tiles lexicographic, the rhs chunks of one tile adjacent.  The t-neighbour of a tile is a
//      whole t-slice of tiles away, far more than the blocks resident on one XCD.
//   1: the tile grid is cut in halves along x, y and z into eight regions (one per XCD when the
//      tile counts are even); inside a region tiles run lexicographically, so the t-neighbour is
//      one region slice away, and the chunks of a tile are adjacent.
//   2: the regions of 1, and inside a region every tile for one rhs chunk before the next chunk
//      (neighbouring tiles then stage the same rhs at the same time).
//   3: the tile grid cut in halves along z and in quarters along t into eight regions, each with
//      the whole x and y extent; inside a region tiles run lexicographically, so the x and y
//      neighbours of a tile (whose faces use a quarter of each line they touch) are one tile or
//      one tile row away, and its t neighbour one region slice away; the chunks of a tile adjacent.
__host__ __device__ __forceinline__ void tile_of_block(const Geom& g, int loc, int nch, int order,
                                              int (&tc)[4], int& tile, int& chunk) {
  if (order == 3) {
    const int sz = (g.NT[2] + 1) >> 1;
    int base = 0, z0 = 0, ez = 1, t0 = 0, et = 1;
    // region rho = a + 2b takes the upper z half if a and the t quarter b; uniform, so scalar
    for (int rho = 0; rho < 8; ++rho) {
      const int a = rho & 1, b = rho >> 1;
      z0 = a ? sz : 0;
      ez = a ? g.NT[2] - sz : sz;
      t0 = (b * g.NT[3]) >> 2;
      et = (((b + 1) * g.NT[3]) >> 2) - t0;
      const int n = g.NT[0] * g.NT[1] * ez * et * nch;
      if (loc < base + n) break;
      base += n;
    }
    const int local = loc - base;
    int tl = local / nch;
    chunk = local - tl * nch;
    tc[0] = tl % g.NT[0];
    tl /= g.NT[0];
    tc[1] = tl % g.NT[1];
    tl /= g.NT[1];
    tc[2] = z0 + tl % ez;
    tc[3] = t0 + tl / ez;
    tile = tc[0] + g.NT[0] * (tc[1] + g.NT[1] * (tc[2] + g.NT[2] * tc[3]));
    return;
  }
  if (order == 0) {
    tile = loc / nch;
    chunk = loc - tile * nch;
    const uint32_t q1 = g.dNT0.div(uint32_t(tile));
    const uint32_t q2 = g.dNT1.div(q1);
    const uint32_t q3 = g.dNT2.div(q2);
    tc[0] = int(uint32_t(tile) - q1 * uint32_t(g.NT[0]));
    tc[1] = int(q1 - q2 * uint32_t(g.NT[1]));
    tc[2] = int(q2 - q3 * uint32_t(g.NT[2]));
    tc[3] = int(q3);
    return;
  }
  int s[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = (g.NT[d] + 1) >> 1;
  int base = 0, rho = 0, e[3] = {s[0], s[1], s[2]};
  // region rho = a + 2b + 4c takes the upper half in x if a, in y if b, in z if c; the block
  // index is uniform, so this search is scalar
  for (rho = 0; rho < 8; ++rho) {
#pragma unroll
    for (int d = 0; d < 3; ++d) e[d] = ((rho >> d) & 1) ? g.NT[d] - s[d] : s[d];
    const int n = e[0] * e[1] * e[2] * g.NT[3] * nch;
    if (loc < base + n) break;
    base += n;
  }
  const int nt = e[0] * e[1] * e[2] * g.NT[3];
  const int local = loc - base;
  int tl;
  if (order == 1) {
    tl = local / nch;
    chunk = local - tl * nch;
  } else {
    chunk = local / nt;
    tl = local - chunk * nt;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int q = tl / e[d];
    tc[d] = (((rho >> d) & 1) ? s[d] : 0) + (tl - q * e[d]);
    tl = q;
  }
  tc[3] = tl;
  tile = tc[0] + g.NT[0] * (tc[1] + g.NT[1] * (tc[2] + g.NT[2] * tc[3]));
}

// ----------------------------------------------------------------------------- launch helpers
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each with its own L2.
// Renumber so that each XCD receives one contiguous range of logical blocks (neighbouring
// sites, and all right-hand sides of one site block, then share an L2).  A bijection of
// [0, n) for any n.
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int NX = 8;
  int q = n / NX, r = n % NX;
  int x = b % NX, loc = b / NX;
  int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return start + loc;
}

// Partial sums a finalize lane loads before adding any of them (one load latency per FIN_U
// partials instead of one per partial).
constexpr int FIN_U = 8;

// sum over a 64-lane wavefront, fixed butterfly order (deterministic)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave sums of NP values (a power of two up to 64), scattered: lane l ends with the sum over the
// wave of value l % NP.  Each halving step sends half of the values still held to the lane whose
// index differs in one bit and keeps the half that bit selects; the single value left is then
// summed over the lanes that hold the same one.  NP - 1 + log2(64 / NP) exchanges, against
// 6 NP for separate sums; the order of the additions is fixed.
template <int HALF, int NP>
__device__ __forceinline__ void scatter_halve(double (&v)[NP], int lane) {
  const bool up = (lane & HALF) != 0;
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const double lo = v[i], hi = v[i + HALF];
    const double send = up ? lo : hi;
    v[i] = (up ? hi : lo) + __shfl_xor(send, HALF, 64);
  }
  if constexpr (HALF > 1) scatter_halve<HALF / 2>(v, lane);
}
template <int NP>
__device__ __forceinline__ double wave_sum_small(double (&v)[NP]) {
  static_assert(NP >= 1 && NP <= 64 && (NP & (NP - 1)) == 0, "a power of two up to 64");
  if constexpr (NP > 1) scatter_halve<NP / 2>(v, threadIdx.x & 63);
  double s = v[0];
#pragma unroll
  for (int o = NP; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// Block-wide sum of NV doubles per thread; result valid in thread 0. Fixed order.
template <int NV, int BS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV * BS/64] */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = BS / 64;
  constexpr int NP = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16 : NV <= 32 ? 32 : 64;
  static_assert(NV <= 64, "at most 64 sums");
  double t[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) t[i] = i < NV ? v[i] : 0.0;
  const double mine = wave_sum_small<NP>(t);
  if (lane < NV) sh[lane * NW + w] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int j = 0; j < NW; ++j) s += sh[i * NW + j];
      v[i] = s;
    }
  }
}


}  // namespace dbq
