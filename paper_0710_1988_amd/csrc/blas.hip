// Tall-skinny FP64 products for the deflation projection (Sec. 2: U^H A V, U^H r0, x0 + V y with
// U = gamma5 V), the minimal-residual projection over previous solutions (Sec. 4) and the
// Gram-Schmidt steps of GMRES-DR's Arnoldi process.  All of them stream long vectors once and
// are bound by HBM bandwidth; the gamma5 of the left vectors is a sign folded into the loads.
#include <algorithm>
#include <cfloat>

#include "kernels.h"

namespace dbq {

namespace {

constexpr int G_BS = 256;
constexpr int G_EPT = 8;
constexpr int G_CHUNK = G_BS * G_EPT;

__device__ __forceinline__ double g5sign(long long e, long long V, int g5) {
  return (g5 && ((e / (6 * V)) & 1)) ? -1.0 : 1.0;
}

// Sums of NV (32 or 64) values over the 64 lanes of a wave, scattered: on return lane l holds the
// wave's sum of value l % NV.  Each step sends half of the remaining values to the lane whose
// index differs in one bit and keeps the half that bit selects (63 shuffles, against 6 NV for NV
// separate butterfly sums); the order of the additions is fixed.
template <int HALF, int NV>
__device__ __forceinline__ void step(double (&v)[NV], int lane) {
  const bool up = (lane & HALF) != 0;
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const double lo = v[i], hi = v[i + HALF];
    const double send = up ? lo : hi;
    v[i] = (up ? hi : lo) + __shfl_xor(send, HALF, 64);
  }
  if constexpr (HALF > 1) step<HALF / 2>(v, lane);
}

template <int NV>
__device__ __forceinline__ double wave_sum_scatter(double (&v)[NV]) {
  static_assert(NV == 32 || NV == 64, "32 or 64 values");
  const int lane = threadIdx.x & 63;
  if (NV == 32) {
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] += __shfl_xor(v[i], 32, 64);
  }
  step<NV / 2>(v, lane);
  return v[0];
}

// Each block: one chunk of G_CHUNK rows x one (TA x TB) tile of (i, j) pairs.  Tile index is
// the fastest-varying logical block index so that all tiles of a chunk run on one XCD and
// re-read the chunk from its L2.
template <int TA, int TB>
__global__ __launch_bounds__(G_BS) void k_gram(const double2* __restrict__ A, long long lda, int na,
                                               const double2* __restrict__ B, long long ldb, int nb,
                                               long long n, long long V, int g5, int ntA, int ntB,
                                               int nblocks, double* __restrict__ work) {
  const int lb = xcd_block(blockIdx.x, nblocks);
  const int ntiles = ntA * ntB;
  const int chunk = lb / ntiles;
  const int tile = lb - chunk * ntiles;
  const int ta = tile / ntB, tb = tile - (tile / ntB) * ntB;
  const int i0 = ta * TA, j0 = tb * TB;
  double acc[TA][TB][2];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b][0] = acc[a][b][1] = 0.0;
  for (int e = 0; e < G_EPT; ++e) {
    const long long row = (long long)chunk * G_CHUNK + e * G_BS + threadIdx.x;
    if (row >= n) break;
    const double sg = g5sign(row, V, g5);
    double2 bv[TB];
#pragma unroll
    for (int b = 0; b < TB; ++b)
      bv[b] = (j0 + b < nb) ? B[(long long)(j0 + b) * ldb + row] : make_double2(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < TA; ++a) {
      double2 av = (i0 + a < na) ? A[(long long)(i0 + a) * lda + row] : make_double2(0.0, 0.0);
      av.x *= sg;
      av.y *= sg;
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        // conj(av) * bv
        acc[a][b][0] += av.x * bv[b].x + av.y * bv[b].y;
        acc[a][b][1] += av.x * bv[b].y - av.y * bv[b].x;
      }
    }
  }
  constexpr int NV = TA * TB * 2, NW = G_BS / 64;
  __shared__ double sh[NV * NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double flat[NV];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b)
#pragma unroll
      for (int q = 0; q < 2; ++q) flat[(a * TB + b) * 2 + q] = acc[a][b][q];
  const double mine = wave_sum_scatter<NV>(flat);
  if (lane < NV) sh[lane * NW + w] = mine;
  __syncthreads();
  double* out = work + ((long long)chunk * ntiles + tile) * NV;
  for (int v = threadIdx.x; v < NV; v += G_BS) {
    double s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += sh[v * NW + k];
    out[v] = s;
  }
}

// C[i + j*na] = sum over chunks of the tile partials.  One block per tile: thread t adds the
// chunks t, t + G_BS, ... of every entry of the tile, then a fixed-order block reduction
// (deterministic, and not latency-bound on thousands of chunks).
template <int TA, int TB>
__global__ __launch_bounds__(G_BS) void k_gram_final(const double* __restrict__ work, int nchunks,
                                                     int ntA, int ntB, int na, int nb,
                                                     double2* __restrict__ C) {
  constexpr int NV = TA * TB * 2;
  const int tile = blockIdx.x, ntiles = ntA * ntB;
  const int ta = tile / ntB, tb = tile - ta * ntB;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int c = threadIdx.x; c < nchunks; c += G_BS) {
    const double* p = work + ((long long)c * ntiles + tile) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += p[v];
  }
  constexpr int NW = G_BS / 64;
  __shared__ double sh[NV * NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double mine = wave_sum_scatter<NV>(acc);
  if (lane < NV) sh[lane * NW + w] = mine;
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    double s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += sh[v * NW + k];
    const int q = v & 1, a = (v >> 1) / TB, b = (v >> 1) % TB;
    const int i = ta * TA + a, j = tb * TB + b;
    if (i < na && j < nb) ((double*)C)[2 * (i + (long long)j * na) + q] = s;
  }
}

template <int TA, int TB>
void gram_impl(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
               long long ldb, int nb, long long n, long long V, int g5, double2* C, double* work,
               size_t work_elems) {
  const int nchunks = int((n + G_CHUNK - 1) / G_CHUNK);
  const int ntA = (na + TA - 1) / TA, ntB = (nb + TB - 1) / TB;
  const long long nblocks = (long long)nchunks * ntA * ntB;
  DBQ_CHECK(size_t(nblocks) * TA * TB * 2 <= work_elems, "gram: workspace too small");
  DBQ_CHECK(nblocks < (1ll << 31), "gram: too many blocks");
  hipLaunchKernelGGL((k_gram<TA, TB>), dim3(unsigned(nblocks)), dim3(G_BS), 0, s, A, lda, na, B,
                     ldb, nb, n, V, g5, ntA, ntB, int(nblocks), work);
  DBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_gram_final<TA, TB>), dim3(unsigned(ntA * ntB)), dim3(G_BS), 0, s, work,
                     nchunks, ntA, ntB, na, nb, C);
  DBQ_HIP(hipGetLastError());
}

// ---- Gram products with several columns on both sides, on FP64 matrix cores.
// The complex product conj(a) b over the interleaved (re, im) doubles of the two vectors is two
// real inner products: Re = sum_k a[k] b[k] and Im = sum_k a[k] b'[k] with b' = (im, -re) per
// element.  v_mfma_f64_16x16x4f64 accumulates a 16 x 16 block D += X Y over 4 values of k, where
// lane l supplies X[l % 16][l / 16] and Y[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16] in
// its accumulator value v (rows interleaved across the lane groups; checked on the device).  The order of k inside a sum is free, so lane group q = l / 16
// of a wave takes the four doubles k0 + 4q .. k0 + 4q + 3 of a 16-double chunk of every column
// (a contiguous 32-byte load; the four groups cover one 128-byte line of each column) and feeds
// them to four successive instructions.  A wave keeps the whole (16 TA) x (16 TB) product of its
// chunks in accumulators, so each element of every column is read once per launch (the tiled
// FMA kernel reads each chunk once per 8 x 4 tile).  Chunks never straddle the gamma5 sign
// boundary at 12 V doubles (V, a product of four even extents, is a multiple of 16).
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int GM_BS = 256;           // 4 waves
constexpr int GM_CHUNK = 16;         // doubles per column per wave step
constexpr int GM_MAX_BLOCKS = 1024;

template <int TA, int TB>
__global__ __launch_bounds__(GM_BS) void k_gram_mfma(const double* __restrict__ A, long long lda,
                                                     int na, const double* __restrict__ B,
                                                     long long ldb, int nb, long long n2,
                                                     long long half2, int g5,
                                                     double* __restrict__ work) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, r = lane & 15;
  f64x4 accR[TA][TB], accI[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      accR[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
      accI[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
  // column of each tile this lane reads (rows past na / nb read a valid column and are dropped
  // by the final reduction)
  const double* ap[TA];
  const double* bp[TB];
#pragma unroll
  for (int a = 0; a < TA; ++a) ap[a] = A + (long long)min(16 * a + r, na - 1) * lda;
#pragma unroll
  for (int b = 0; b < TB; ++b) bp[b] = B + (long long)min(16 * b + r, nb - 1) * ldb;
  const long long nchunks = (n2 + GM_CHUNK - 1) / GM_CHUNK;
  const long long stride = (long long)gridDim.x * (GM_BS / 64);
  // this lane's four doubles of chunk ch of every column (zero past the end; negated on the
  // gamma5 = -1 half for the left vectors)
  auto load = [&](long long ch, double (&av)[TA][4], double (&bv)[TB][4]) {
    const long long k0 = ch * GM_CHUNK + 4 * q;
    if (k0 + 4 <= n2) {
#pragma unroll
      for (int a = 0; a < TA; ++a) {
        const double2 u = *(const double2*)(ap[a] + k0);
        const double2 w = *(const double2*)(ap[a] + k0 + 2);
        av[a][0] = u.x; av[a][1] = u.y; av[a][2] = w.x; av[a][3] = w.y;
      }
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const double2 u = *(const double2*)(bp[b] + k0);
        const double2 w = *(const double2*)(bp[b] + k0 + 2);
        bv[b][0] = u.x; bv[b][1] = u.y; bv[b][2] = w.x; bv[b][3] = w.y;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool in = k0 + t < n2;
#pragma unroll
        for (int a = 0; a < TA; ++a) av[a][t] = in ? ap[a][k0 + t] : 0.0;
#pragma unroll
        for (int b = 0; b < TB; ++b) bv[b][t] = in ? bp[b][k0 + t] : 0.0;
      }
    }
    if (g5 && ((k0 / half2) & 1)) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) av[a][t] = -av[a][t];
    }
  };
  auto mfma = [&](const double (&av)[TA][4], const double (&bv)[TB][4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        // b' = (im, -re): the partner double of k0 + t, negated when t is odd
        const double bi = (t & 1) ? -bv[b][t - 1] : bv[b][t + 1];
#pragma unroll
        for (int a = 0; a < TA; ++a) {
          accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][t], bv[b][t], accR[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][t], bi, accI[a][b], 0, 0, 0);
        }
      }
    }
  };
  // two chunks per step: the second chunk's loads are in flight while the first is multiplied
  long long ch = (long long)blockIdx.x * (GM_BS / 64) + wv;
  for (; ch + stride < nchunks; ch += 2 * stride) {
    double av0[TA][4], bv0[TB][4], av1[TA][4], bv1[TB][4];
    load(ch, av0, bv0);
    load(ch + stride, av1, bv1);
    mfma(av0, bv0);
    mfma(av1, bv1);
  }
  if (ch < nchunks) {
    double av0[TA][4], bv0[TB][4];
    load(ch, av0, bv0);
    mfma(av0, bv0);
  }
  // the four waves' products summed in LDS in wave order, then stored as this block's partial
  // [a][b][re, im][16 rows][16 columns]
  constexpr int NV = TA * TB * 2 * 256;
  __shared__ double sh[NV];
  for (int w = 0; w < GM_BS / 64; ++w) {
    if (wv == w) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int o = (a * TB + b) * 512 + (q + 4 * v) * 16 + r;
            if (w == 0) {
              sh[o] = accR[a][b][v];
              sh[o + 256] = accI[a][b][v];
            } else {
              sh[o] += accR[a][b][v];
              sh[o + 256] += accI[a][b][v];
            }
          }
    }
    __syncthreads();
  }
  double* out = work + (long long)blockIdx.x * NV;
  for (int v = threadIdx.x; v < NV; v += GM_BS) out[v] = sh[v];
}

// C[i + j na] = sum over the blocks' partials: one wavefront per output value, lane l adding the
// blocks l, l + 64, ... in order, then a fixed butterfly over the lanes (deterministic)
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gram_mfma_final(const double* __restrict__ work,
                                                         int nblocks, int na, int nb,
                                                         double2* __restrict__ C) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= na * nb) return;
  const int i = t % na, j = t / na;
  const int a = i >> 4, b = j >> 4;
  const int o = (a * TB + b) * 512 + (i & 15) * 16 + (j & 15);
  constexpr int NV = TA * TB * 2 * 256;
  double re = 0.0, im = 0.0;
  for (int k = lane; k < nblocks; k += 64) {
    re += work[(long long)k * NV + o];
    im += work[(long long)k * NV + o + 256];
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) C[i + (long long)j * na] = make_double2(re, im);
}

template <int TA, int TB>
void gram_mfma_impl(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
                    long long ldb, int nb, long long n, long long V, int g5, double2* C,
                    double* work, size_t work_elems) {
  const long long n2 = 2 * n;
  const long long nchunks = (n2 + GM_CHUNK - 1) / GM_CHUNK;
  const int nblocks = int(std::min<long long>(GM_MAX_BLOCKS, (nchunks + 3) / 4));
  constexpr int NV = TA * TB * 2 * 256;
  DBQ_CHECK(size_t(nblocks) * NV <= work_elems, "gram: workspace too small");
  DBQ_CHECK(na >= 1 && na <= 16 * TA && nb >= 1 && nb <= 16 * TB, "gram: tile count");
  hipLaunchKernelGGL((k_gram_mfma<TA, TB>), dim3(nblocks), dim3(GM_BS), 0, s, (const double*)A,
                     2 * lda, na, (const double*)B, 2 * ldb, nb, n2, 12 * V, g5, work);
  DBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_gram_mfma_final<TA, TB>), dim3((na * nb + 3) / 4), dim3(256), 0, s,
                     work, nblocks, na, nb, C);
  DBQ_HIP(hipGetLastError());
}

// Y_j = beta*Y_j + sum_i sg(e) A_i M_ij for a tile of TB columns (grid.y) of Y
template <int TB>
__global__ __launch_bounds__(256) void k_combine(const double2* __restrict__ A, long long lda,
                                                 int na, const double2* __restrict__ M, int ldm,
                                                 double2* __restrict__ Y, long long ldy, int nb,
                                                 long long n, long long V, int g5, int beta) {
  const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = blockIdx.y * TB;
  if (row >= n) return;
  const double sg = g5sign(row, V, g5);
  double acc[TB][2];
#pragma unroll
  for (int b = 0; b < TB; ++b) acc[b][0] = acc[b][1] = 0.0;
  for (int i = 0; i < na; ++i) {
    const double2 av = A[(long long)i * lda + row];
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      if (j0 + b < nb) {
        const double2 m = M[i + (long long)(j0 + b) * ldm];
        acc[b][0] += av.x * m.x - av.y * m.y;
        acc[b][1] += av.x * m.y + av.y * m.x;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < TB; ++b) {
    if (j0 + b >= nb) continue;
    double2* y = Y + (long long)(j0 + b) * ldy + row;
    double2 o = make_double2(sg * acc[b][0], sg * acc[b][1]);
    if (beta == 1) {
      const double2 yv = *y;
      o.x += yv.x;
      o.y += yv.y;
    } else if (beta == -1) {
      const double2 yv = *y;
      o.x = yv.x - o.x;
      o.y = yv.y - o.y;
    }
    *y = o;
  }
}

// ---- Arnoldi step with delayed reorthogonalisation (classical Gram-Schmidt twice, the second
// pass of each new vector done one step late so that both passes share the sweeps over the basis:
// two sweeps per step instead of four).
// On entry to step j, column j of the basis holds z_j, the once-orthogonalised, not yet
// normalised new vector, and column j+1 holds w = A z_j.  One Gram sweep gives
// G = [q_0 .. q_{j-1}, z_j]^H [z_j, w].  With nu = |z_j|, u = z_j / nu and Q = [q_0 .. q_{j-1}]:
//   s = Q^H u (second-pass coefficients of u), rho = sqrt(1 - |s|^2), q_j = (u - Q s) / rho;
//   previous column: A q_{j-1} = Q (h_{j-1} + nu s) + nu rho q_j;
//   t = Q^H w / nu, beta = u^H w / nu and, since A q_j = (w / nu - A Q s) / rho with
//   A Q = [Q, q_j] Hbar (Hbar: the corrected (j+1) x j Hessenberg block), the new column
//   h_j = ([t; (beta - s^H t) / rho] - Hbar s) / rho and the next vector
//   z_{j+1} = A q_j - [Q, q_j] h_j = (w / nu - Q (t - gamma s) - gamma u) / rho,
//   gamma = (beta - s^H t) / rho^2.
// The second sweep (k_arn_combine) writes q_j and z_{j+1} in place from
//   m0 = [-s / rho; 1 / (nu rho)],  m1 = [(t - gamma s) / rho; gamma / (nu rho)],
//   c1 = 1 / (nu rho):  col j = [Q, z_j] m0,  col j+1 = c1 w - [Q, z_j] m1.
// A vector that starts a cycle (v_1, or the last vector of a restart basis) is already
// orthonormal and consistent with Hbar: there s = 0 and nu = rho = 1, and no column is
// corrected.  With last = 1 column j (= m) is only reorthogonalised (G has one column) and the
// last Hessenberg column corrected.
constexpr int AC_BS = 256;
constexpr int AC_MAXJ = 128;

__global__ __launch_bounds__(AC_BS) void k_arn_coef(const double2* __restrict__ G, int j,
                                                    int start, int last, double2* __restrict__ H,
                                                    int ldh, double2* __restrict__ m0,
                                                    double2* __restrict__ m1,
                                                    double* __restrict__ c1) {
  __shared__ zd s_s[AC_MAXJ];
  __shared__ double red[3 * (AC_BS / 64)];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int na = j + 1;
  const double nu = start ? 1.0 : sqrt(G[j].x);
  const double inu = 1.0 / nu;
  double p[3] = {0.0, 0.0, 0.0};  // |s|^2, s^H t
  for (int i = t; i < j; i += AC_BS) {
    const zd si = start ? zd{0.0, 0.0} : zd{G[i].x * inu, G[i].y * inu};
    s_s[i] = si;
    p[0] += norm2(si);
    if (!last) {
      const zd st = cmulc(si, zd{G[na + i].x * inu, G[na + i].y * inu});
      p[1] += st.re;
      p[2] += st.im;
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    p[q] = wave_sum(p[q]);
    if (lane == 0) red[q * (AC_BS / 64) + wv] = p[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double v = 0.0;
    for (int w = 0; w < AC_BS / 64; ++w) v += red[q * (AC_BS / 64) + w];
    p[q] = v;
  }
  // a vector that lies (to rounding) in the span of Q leaves nothing to normalise: keep rho
  // away from zero so that the step stays finite (the Hessenberg entry nu rho is then ~0)
  const double rho = start ? 1.0 : sqrt(fmax(1.0 - p[0], DBL_EPSILON));
  const double irho = 1.0 / rho, c = inu * irho;
  if (!start && j >= 1) {
    for (int i = t; i < j; i += AC_BS) {
      const double2 h = H[i + (long long)(j - 1) * ldh];
      H[i + (long long)(j - 1) * ldh] = make_double2(h.x + nu * s_s[i].re, h.y + nu * s_s[i].im);
    }
    if (t == 0) H[j + (long long)(j - 1) * ldh] = make_double2(nu * rho, 0.0);
  }
  __syncthreads();
  if (last) {
    for (int i = t; i <= j; i += AC_BS)
      m0[i] = i < j ? make_double2(-s_s[i].re * irho, -s_s[i].im * irho) : make_double2(c, 0.0);
    if (t == 0) *c1 = c;
    return;
  }
  const zd beta{G[na + j].x * inu * inu, G[na + j].y * inu * inu};
  const zd bq{(beta.re - p[1]) * irho, (beta.im - p[2]) * irho};  // q_j^H w / nu
  const zd gam{bq.re * irho, bq.im * irho};
  for (int i = t; i <= j; i += AC_BS) {
    zd hs{0.0, 0.0};
    if (!start)
#pragma unroll 8
      for (int cc = 0; cc < j; ++cc) {
        const double2 h = H[i + (long long)cc * ldh];
        hs = hs + zd{h.x, h.y} * s_s[cc];
      }
    const zd ti = i < j ? zd{G[na + i].x * inu, G[na + i].y * inu} : bq;
    H[i + (long long)j * ldh] = make_double2((ti.re - hs.re) * irho, (ti.im - hs.im) * irho);
    if (i < j) {
      const zd si = s_s[i];
      m0[i] = make_double2(-si.re * irho, -si.im * irho);
      const zd g = gam * si;
      m1[i] = make_double2((ti.re - g.re) * irho, (ti.im - g.im) * irho);
    } else {
      m0[i] = make_double2(c, 0.0);
      m1[i] = make_double2(gam.re * c, gam.im * c);
    }
  }
  if (t == 0) *c1 = c;
}

// col j = sum_{i<=j} Q_i m0[i]; with TWO also col j+1 = c1 col(j+1) - sum_{i<=j} Q_i m1[i]
// (each thread reads its row of every column before it writes, so in place is safe)
template <bool TWO>
__global__ __launch_bounds__(256) void k_arn_combine(double2* Q, long long ld, int j, long long n,
                                                     const double2* __restrict__ m0,
                                                     const double2* __restrict__ m1,
                                                     const double* __restrict__ c1) {
  const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
#pragma unroll 4
  for (int i = 0; i <= j; ++i) {
    const double2 q = Q[(long long)i * ld + row];
    const double2 x = m0[i];
    a0r += q.x * x.x - q.y * x.y;
    a0i += q.x * x.y + q.y * x.x;
    if (TWO) {
      const double2 y = m1[i];
      a1r += q.x * y.x - q.y * y.y;
      a1i += q.x * y.y + q.y * y.x;
    }
  }
  if (TWO) {
    const double f = *c1;
    const double2 w = Q[(long long)(j + 1) * ld + row];
    Q[(long long)(j + 1) * ld + row] = make_double2(f * w.x - a1r, f * w.y - a1i);
  }
  Q[(long long)j * ld + row] = make_double2(a0r, a0i);
}

__global__ void k_scale(const double2* __restrict__ x, double2* __restrict__ y, long long n,
                        const double* __restrict__ nrm2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = 1.0 / sqrt(*nrm2);
  const double2 v = x[i];
  y[i] = make_double2(v.x * f, v.y * f);
}

__global__ __launch_bounds__(256) void k_norm2(const double2* __restrict__ x, long long ld,
                                               long long n, int nchunks,
                                               double* __restrict__ work) {
  const int vec = blockIdx.y;
  const int chunk = blockIdx.x;
  double s[1] = {0.0};
  for (int e = 0; e < G_EPT; ++e) {
    const long long row = (long long)chunk * G_CHUNK + e * G_BS + threadIdx.x;
    if (row < n) {
      const double2 v = x[(long long)vec * ld + row];
      s[0] += v.x * v.x + v.y * v.y;
    }
  }
  __shared__ double sh[G_BS / 64];
  block_sum<1, G_BS>(s, sh);
  if (threadIdx.x == 0) work[(long long)vec * nchunks + chunk] = s[0];
}

// one block per vector: strided partial sums, then a fixed-order block reduction
__global__ __launch_bounds__(G_BS) void k_norm2_final(const double* __restrict__ work, int nchunks,
                                                      double* __restrict__ out) {
  const int v = blockIdx.x;
  double s[1] = {0.0};
  for (int c = threadIdx.x; c < nchunks; c += G_BS) s[0] += work[(long long)v * nchunks + c];
  __shared__ double sh[G_BS / 64];
  block_sum<1, G_BS>(s, sh);
  if (threadIdx.x == 0) out[v] = s[0];
}

__global__ void k_copy(const double2* __restrict__ x, double2* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

__global__ void k_sub(const double2* __restrict__ a, const double2* __restrict__ b,
                      double2* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 u = a[i], v = b[i];
    y[i] = make_double2(u.x - v.x, u.y - v.y);
  }
}

__global__ void k_write_col(double2* __restrict__ M, int ld, int col, int count,
                            const double2* __restrict__ h1, const double2* __restrict__ h2,
                            const double* __restrict__ nrm2, int diag_row) {
  const int i = threadIdx.x;
  for (int r = i; r < count; r += blockDim.x) {
    const double2 a = h1[r], b = h2[r];
    M[r + (long long)col * ld] = make_double2(a.x + b.x, a.y + b.y);
  }
  if (i == 0) M[diag_row + (long long)col * ld] = make_double2(sqrt(*nrm2), 0.0);
}

__global__ void k_set_e1(double2* __restrict__ c, int len, const double* __restrict__ nrm2) {
  for (int r = threadIdx.x; r < len; r += blockDim.x)
    c[r] = make_double2(r == 0 ? sqrt(*nrm2) : 0.0, 0.0);
}

// deterministic start vector: splitmix64 of (seed, index) mapped to [-1, 1) per real component
__global__ void k_fill_hash(double2* __restrict__ x, long long n, unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const double a = double(z >> 43) * (1.0 / 1048576.0) - 1.0;            // 21 bits
  const double b = double((z >> 11) & 0xFFFFFull) * (1.0 / 524288.0) - 1.0;  // 20 bits
  x[i] = make_double2(a, b);
}

__global__ void k_zero(double2* __restrict__ x, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = make_double2(0.0, 0.0);
}

inline unsigned nb256(long long n) { return unsigned((n + 255) / 256); }

// ---- Basis combinations Y = beta Y + sg(e) A M with several output columns, on FP64 matrix
// cores.  With A and Y as real matrices over interleaved (re, im) doubles, the complex product is
// a real one: output column (j, re) takes a.re M_cj.re - a.im M_cj.im and (j, im) takes
// a.re M_cj.im + a.im M_cj.re.  A wave owns 16 rows (elements) of Y and all 8 NT complex output
// columns (NT 16-wide accumulator tiles, lane l holding D[l / 16 + 4 v][l % 16]); in a step,
// lane group q = l / 16 reads the element of its row in column c0 + q of A (one 16-byte load)
// and feeds its real part and its imaginary part to two instructions per tile, so every element
// of A is read once per launch.  The rows of M the steps need sit in LDS, CM_KC at a time.
constexpr int CM_BS = 256;  // 4 waves, 64 rows of Y per block
constexpr int CM_KC = 32;   // rows of M per LDS chunk (a multiple of 4)
constexpr int CM_U = 4;     // steps whose loads are in flight together

template <int NT>
__global__ __launch_bounds__(CM_BS) void k_combine_mfma(const double2* __restrict__ A,
                                                        long long lda, int na,
                                                        const double2* __restrict__ M, int ldm,
                                                        double2* __restrict__ Y, long long ldy,
                                                        int nb, long long n, long long V, int g5,
                                                        int beta) {
  constexpr int NC = 8 * NT;  // complex output columns held
  __shared__ double2 Ps[CM_KC * NC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, r = lane & 15, part = r & 1;
  const long long row0 = ((long long)blockIdx.x * (CM_BS / 64) + wv) * 16;
  const long long row = row0 + r;
  const bool in = row < n;
  f64x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < na; k0 += CM_KC) {
    const int kc = min(CM_KC, na - k0);
    __syncthreads();  // the previous chunk is no longer read
    for (int e = threadIdx.x; e < CM_KC * NC; e += CM_BS) {
      const int c = e / NC, j = e - c * NC;
      Ps[e] = (c < kc && j < nb) ? M[(k0 + c) + (long long)j * ldm] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // steps of 4 columns; a step's column stays below CM_KC (a multiple of 4), the rows of Ps
    // past kc are zero and so are the loads past it
    for (int c0 = 0; c0 < kc; c0 += 4 * CM_U) {
      double2 a[CM_U];
#pragma unroll
      for (int u = 0; u < CM_U; ++u) {
        const int c = c0 + 4 * u + q;
        a[u] = (in && c < kc) ? A[(long long)(k0 + c) * lda + row] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < CM_U; ++u) {
        if (c0 + 4 * u >= kc) break;  // uniform over the wave
        const int c = c0 + 4 * u + q;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const double2 p = Ps[c * NC + 8 * t + (r >> 1)];
          const double yre = part ? p.y : p.x;
          const double yim = part ? p.x : -p.y;
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, yre, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, yim, acc[t], 0, 0, 0);
        }
      }
    }
  }
  // lane l holds rows row0 + q + 4 v of output column 8 t + r / 2, the real part on even r and
  // the imaginary part on odd r: the even lane stores both
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double mine = acc[t][v];
      const double other = __shfl_xor(mine, 1, 64);
      const long long orow = row0 + q + 4 * v;
      const int j = 8 * t + (r >> 1);
      if (part == 0 && orow < n && j < nb) {
        const double sg = g5sign(orow, V, g5);
        double2* y = Y + (long long)j * ldy + orow;
        double2 o = make_double2(sg * mine, sg * other);
        if (beta == 1) {
          const double2 yv = *y;
          o.x += yv.x;
          o.y += yv.y;
        } else if (beta == -1) {
          const double2 yv = *y;
          o.x = yv.x - o.x;
          o.y = yv.y - o.y;
        }
        *y = o;
      }
    }
  }
}

}  // namespace

void write_col_f64(hipStream_t s, double2* M, int ld, int col, int count, const double2* h1,
                   const double2* h2, const double* nrm2, int diag_row) {
  hipLaunchKernelGGL(k_write_col, dim3(1), dim3(64), 0, s, M, ld, col, count, h1, h2, nrm2,
                     diag_row);
  DBQ_HIP(hipGetLastError());
}

void set_e1_f64(hipStream_t s, double2* c, int len, const double* nrm2) {
  hipLaunchKernelGGL(k_set_e1, dim3(1), dim3(64), 0, s, c, len, nrm2);
  DBQ_HIP(hipGetLastError());
}

void fill_hash_f64(hipStream_t s, double2* x, long long n, unsigned long long seed) {
  hipLaunchKernelGGL(k_fill_hash, dim3(nb256(n)), dim3(256), 0, s, x, n, seed);
  DBQ_HIP(hipGetLastError());
}

void zero_f64(hipStream_t s, double2* x, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3(nb256(n)), dim3(256), 0, s, x, n);
  DBQ_HIP(hipGetLastError());
}

size_t gram_work_elems(long long n, int na, int nb) {
  const long long nchunks = (n + G_CHUNK - 1) / G_CHUNK;
  // the largest of the tilings
  const long long t1 = nchunks * ((na + 7) / 8) * ((nb + 3) / 4) * 8 * 4 * 2;
  const long long t2 = nchunks * ((na + 15) / 16) * 16 * 2;
  const long long ta = (na + 15) / 16, tb = (nb + 15) / 16;
  const long long t3 = (ta <= 3 && tb <= 3) ? (long long)GM_MAX_BLOCKS * ta * tb * 2 * 256 : 0;
  return size_t(std::max(t1, std::max(t2, t3)));
}

// DBQ_GRAM_MFMA=0 keeps the FMA kernel for every shape (for comparison)
static bool gram_mfma_enabled() {
  const char* e = std::getenv("DBQ_GRAM_MFMA");
  return !(e && std::atoi(e) == 0);
}

void gram_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
              long long ldb, int nb, long long n, long long V, int g5, double2* C, double* work,
              size_t work_elems) {
  if (na <= 0 || nb <= 0) return;
  if (nb == 1) {
    gram_impl<16, 1>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems);
    return;
  }
  const int ta = (na + 15) / 16, tb = (nb + 15) / 16;
  if (ta <= 3 && tb <= 3 && gram_mfma_enabled()) {
    // (16 ta) x (16 tb) accumulator tiles per wave, na and nb up to 48
    switch (ta * 4 + tb) {
      case 5: gram_mfma_impl<1, 1>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 6: gram_mfma_impl<1, 2>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 7: gram_mfma_impl<1, 3>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 9: gram_mfma_impl<2, 1>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 10: gram_mfma_impl<2, 2>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 11: gram_mfma_impl<2, 3>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 13: gram_mfma_impl<3, 1>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      case 14: gram_mfma_impl<3, 2>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
      default: gram_mfma_impl<3, 3>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems); return;
    }
  }
  gram_impl<8, 4>(s, A, lda, na, B, ldb, nb, n, V, g5, C, work, work_elems);
}

void gram2_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* B,
               long long ldb, long long n, double2* C, double* work, size_t work_elems) {
  gram_impl<16, 2>(s, A, lda, na, B, ldb, 2, n, 1, 0, C, work, work_elems);
}

void arn_coef_f64(hipStream_t s, const double2* G, int j, int start, int last, double2* H, int ldh,
                  double2* m0, double2* m1, double* c1) {
  DBQ_CHECK(j >= 0 && j <= AC_MAXJ, "arn_coef: column index out of range");
  hipLaunchKernelGGL(k_arn_coef, dim3(1), dim3(AC_BS), 0, s, G, j, start, last, H, ldh, m0, m1, c1);
  DBQ_HIP(hipGetLastError());
}

void arn_combine_f64(hipStream_t s, double2* Q, long long ld, int j, long long n, const double2* m0,
                     const double2* m1, const double* c1) {
  if (m1)
    hipLaunchKernelGGL((k_arn_combine<true>), dim3(nb256(n)), dim3(256), 0, s, Q, ld, j, n, m0,
                       m1, c1);
  else
    hipLaunchKernelGGL((k_arn_combine<false>), dim3(nb256(n)), dim3(256), 0, s, Q, ld, j, n, m0,
                       m1, c1);
  DBQ_HIP(hipGetLastError());
}

// DBQ_COMBINE_MFMA=0 keeps the FMA kernel for every shape (for comparison)
static bool combine_mfma_enabled() {
  const char* e = std::getenv("DBQ_COMBINE_MFMA");
  return !(e && std::atoi(e) == 0);
}

void combine_f64(hipStream_t s, const double2* A, long long lda, int na, const double2* M, int ldm,
                 double2* Y, long long ldy, int nb, long long n, long long V, int g5, int beta) {
  if (nb <= 0) return;
  if (na <= 0 && beta != 0) return;
  // 9 to 40 columns of Y: one pass over A on the matrix cores (8 NT columns per wave)
  if (nb > 8 && nb <= 40 && na > 0 && combine_mfma_enabled()) {
    const dim3 grid(unsigned((n + CM_BS / 4 - 1) / (CM_BS / 4)));
    switch ((nb + 7) / 8) {
      case 2: hipLaunchKernelGGL((k_combine_mfma<2>), grid, dim3(CM_BS), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n, V, g5, beta); break;
      case 3: hipLaunchKernelGGL((k_combine_mfma<3>), grid, dim3(CM_BS), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n, V, g5, beta); break;
      case 4: hipLaunchKernelGGL((k_combine_mfma<4>), grid, dim3(CM_BS), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n, V, g5, beta); break;
      default: hipLaunchKernelGGL((k_combine_mfma<5>), grid, dim3(CM_BS), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n, V, g5, beta); break;
    }
    DBQ_HIP(hipGetLastError());
    return;
  }
  // up to 16 columns of Y per pass over A (one pass for the 12-source projection)
  if (nb <= 8) {
    dim3 grid(nb256(n), 1);
    hipLaunchKernelGGL((k_combine<8>), grid, dim3(256), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n, V,
                       g5, beta);
  } else {
    dim3 grid(nb256(n), (nb + 15) / 16);
    hipLaunchKernelGGL((k_combine<16>), grid, dim3(256), 0, s, A, lda, na, M, ldm, Y, ldy, nb, n,
                       V, g5, beta);
  }
  DBQ_HIP(hipGetLastError());
}

void scale_f64(hipStream_t s, const double2* x, double2* y, long long n, const double* nrm2) {
  hipLaunchKernelGGL(k_scale, dim3(nb256(n)), dim3(256), 0, s, x, y, n, nrm2);
  DBQ_HIP(hipGetLastError());
}

void norm2_f64(hipStream_t s, const double2* x, long long ld, int count, long long n, double* out,
               double* work, size_t work_elems) {
  const int nchunks = int((n + G_CHUNK - 1) / G_CHUNK);
  DBQ_CHECK(size_t(nchunks) * count <= work_elems, "norm2: workspace too small");
  hipLaunchKernelGGL(k_norm2, dim3(nchunks, count), dim3(G_BS), 0, s, x, ld, n, nchunks, work);
  DBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_norm2_final, dim3(count), dim3(G_BS), 0, s, work, nchunks, out);
  DBQ_HIP(hipGetLastError());
}

void copy_f64(hipStream_t s, const double2* x, double2* y, long long n) {
  hipLaunchKernelGGL(k_copy, dim3(nb256(n)), dim3(256), 0, s, x, y, n);
  DBQ_HIP(hipGetLastError());
}

void sub_f64(hipStream_t s, const double2* a, const double2* b, double2* y, long long n) {
  hipLaunchKernelGGL(k_sub, dim3(nb256(n)), dim3(256), 0, s, a, b, y, n);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
