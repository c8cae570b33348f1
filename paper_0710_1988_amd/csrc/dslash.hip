// Wilson / twisted-mass Dslash: out = A(mu) in, A(mu) = I - kappa*H + i*mu*gamma5 (the operator of
// Sec. 1 with the twisted term of the Sec. 4 action), or its dagger gamma5 A(-mu) gamma5.
//
// One thread per (site, right-hand side).  Each of the 8 hops spin-projects the neighbour
// spinor with (1 -+ gamma_mu) to two colour vectors (the projector has rank 2), multiplies them
// by the link (or its adjoint), and spreads the result back over four spins; with the chiral
// basis gamma_mu = [[0, B], [B^dagger, 0]] the projection is h = psi_up + S*B*psi_dn and the
// lower half of the result is S*B^dagger*chi.  Epilogues fuse the inner products BiCGStab needs
// right after an operator application, and finish them in the last block to arrive, so the
// solver's scalars never leave the GPU.
#include "kernels.h"

namespace dbq {

namespace {

template <typename T>
struct IO;

template <>
struct IO<double> {
  typedef double2 SE;
  typedef double2 LE;
  static constexpr int NSE = 12;
  // [6][V][2]: the pair of components (2k, 2k+1) of one site is one 32-byte access
  __device__ __forceinline__ static void load(const double2* __restrict__ b, int V, int s,
                                              zd (&p)[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 v0 = b[2 * (k * V + s)];
      double2 v1 = b[2 * (k * V + s) + 1];
      p[2 * k] = zd{v0.x, v0.y};
      p[2 * k + 1] = zd{v1.x, v1.y};
    }
  }
  __device__ __forceinline__ static void store(double2* __restrict__ b, int V, int s,
                                               const zd (&p)[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      b[2 * (k * V + s)] = make_double2(p[2 * k].re, p[2 * k].im);
      b[2 * (k * V + s) + 1] = make_double2(p[2 * k + 1].re, p[2 * k + 1].im);
    }
  }
  __device__ __forceinline__ static void link(const double2* __restrict__ U, int V, int mu, int s,
                                              zd (&u)[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 v = U[(mu * 9 + k) * V + s];
      u[k] = zd{v.x, v.y};
    }
  }
  static double link_bytes() { return 4.0 * 9 * 16; }
  static double spinor_bytes() { return 12.0 * 16; }
};

template <>
struct IO<float> {
  typedef float4 SE;
  typedef float4 LE;
  static constexpr int NSE = 6;
  __device__ __forceinline__ static void load(const float4* __restrict__ b, int V, int s,
                                              zf (&p)[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 v = b[k * V + s];
      p[2 * k] = zf{v.x, v.y};
      p[2 * k + 1] = zf{v.z, v.w};
    }
  }
  __device__ __forceinline__ static void store(float4* __restrict__ b, int V, int s,
                                               const zf (&p)[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      b[k * V + s] = make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im);
  }
  // two stored rows; the third row of an SU(3) matrix is the complex conjugate of the cross
  // product of the first two
  __device__ __forceinline__ static void link(const float4* __restrict__ U, int V, int mu, int s,
                                              zf (&u)[9]) {
    float4 a = U[(mu * 3 + 0) * V + s];
    float4 b = U[(mu * 3 + 1) * V + s];
    float4 c = U[(mu * 3 + 2) * V + s];
    u[0] = zf{a.x, a.y};
    u[1] = zf{a.z, a.w};
    u[2] = zf{b.x, b.y};
    u[3] = zf{b.z, b.w};
    u[4] = zf{c.x, c.y};
    u[5] = zf{c.z, c.w};
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
  }
  static double link_bytes() { return 4.0 * 12 * 4; }
  static double spinor_bytes() { return 24.0 * 4; }
};

// h = psi_up + S * B_mu * psi_dn  (index 3*spin + colour, spin 0..1)
template <typename T, int MU, int S>
__device__ __forceinline__ void project(const cx<T> (&p)[12], cx<T> (&h)[6]) {
  const T s = T(S);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if (MU == 0) {        // B = -i sigma_1
      h[c] = p0 - s * ti(p3);
      h[3 + c] = p1 - s * ti(p2);
    } else if (MU == 1) { // B = -i sigma_2
      h[c] = p0 - s * p3;
      h[3 + c] = p1 + s * p2;
    } else if (MU == 2) { // B = -i sigma_3
      h[c] = p0 - s * ti(p2);
      h[3 + c] = p1 + s * ti(p3);
    } else {              // B = 1
      h[c] = p0 + s * p2;
      h[3 + c] = p1 + s * p3;
    }
  }
}

// acc_up += chi, acc_dn += S * B_mu^dagger * chi
template <typename T, int MU, int S>
__device__ __forceinline__ void spread(cx<T> (&acc)[12], const cx<T> (&chi)[6]) {
  const T s = T(S);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> c0 = chi[c], c1 = chi[3 + c];
    acc[c] = acc[c] + c0;
    acc[3 + c] = acc[3 + c] + c1;
    if (MU == 0) {
      acc[6 + c] = acc[6 + c] + s * ti(c1);
      acc[9 + c] = acc[9 + c] + s * ti(c0);
    } else if (MU == 1) {
      acc[6 + c] = acc[6 + c] + s * c1;
      acc[9 + c] = acc[9 + c] - s * c0;
    } else if (MU == 2) {
      acc[6 + c] = acc[6 + c] + s * ti(c0);
      acc[9 + c] = acc[9 + c] - s * ti(c1);
    } else {
      acc[6 + c] = acc[6 + c] + s * c0;
      acc[9 + c] = acc[9 + c] + s * c1;
    }
  }
}

// one hop: BACK = false -> (1 + S gamma) U_mu(x) psi(x+mu); true -> (1 + S gamma) U_mu(y)^dag psi(y)
template <typename T, int MU, int S, bool BACK>
__device__ __forceinline__ void hop(const typename IO<T>::SE* __restrict__ in,
                                    const typename IO<T>::LE* __restrict__ U, int V, int site_link,
                                    int y, cx<T> (&acc)[12]) {
  cx<T> p[12];
  IO<T>::load(in, V, y, p);
  cx<T> h[6];
  project<T, MU, S>(p, h);
  cx<T> u[9];
  IO<T>::link(U, V, MU, site_link, u);
  cx<T> chi[6];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<T> z{T(0), T(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (!BACK) z = z + u[3 * a + b] * h[3 * sp + b];
        else z = z + cmulc(u[3 * b + a], h[3 * sp + b]);
      }
      chi[3 * sp + a] = z;
    }
  }
  spread<T, MU, S>(acc, chi);
}

template <typename T, bool DAG, int MU>
__device__ __forceinline__ void hops_mu(const typename IO<T>::SE* __restrict__ in,
                                        const typename IO<T>::LE* __restrict__ U, const Geom& g,
                                        int s, const int (&c)[4], cx<T> (&acc)[12]) {
  // forward hop uses (1 - gamma) (dagger: 1 + gamma), backward the opposite
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  const int yf = eo_neighbour<MU, +1>(g, c);
  const int yb = eo_neighbour<MU, -1>(g, c);
  hop<T, MU, SF, false>(in, U, g.V, s, yf, acc);
  hop<T, MU, SB, true>(in, U, g.V, yb, yb, acc);
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// Finish the reduction of one epilogue in the last block: every rhs of the batch is reduced by
// one wavefront over its per-block partials in a fixed order.
template <int EPI>
__device__ void finalize(const DsBatch& B, RhsScal* sc, const double* partials) {
  const int lane = threadIdx.x & 63;
  constexpr int NW = DS_BS / 64;
  const int w = blockIdx.x * NW + (threadIdx.x >> 6);
  const int stride = gridDim.x * NW;
  for (int rhs = w; rhs < B.nrhs_total; rhs += stride) {
    int l = 0;
    for (int i = 1; i < B.nlat; ++i)
      if (rhs >= B.lat[i].rhs_base) l = i;
    const int nsb = B.lat[l].nsb;
    double a0 = 0, a1 = 0, a2 = 0;
    const double* pp = partials + (long long)rhs * B.pstride * 3;
    for (int j = lane; j < nsb; j += 64) {
      a0 += pp[3 * j];
      a1 += pp[3 * j + 1];
      a2 += pp[3 * j + 2];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      RhsScal& q = sc[rhs];
      if (EPI == EPI_RHAT) {
        if (q.active) {
          zd d{a0, a1};
          q.dot = d;
          if (!finite_d(a0) || !finite_d(a1)) {
            q.flags |= F_NAN;
            q.active = 0;
          } else if (a0 == 0.0 && a1 == 0.0) {
            q.flags |= F_BREAK;
            q.active = 0;
          } else {
            q.alpha = cdiv(q.rho, d);
          }
        }
      } else if (EPI == EPI_TS) {
        if (q.active) {
          if (!finite_d(a0) || !finite_d(a1) || !finite_d(a2)) {
            q.flags |= F_NAN;
            q.active = 0;
          } else if (a2 == 0.0) {
            q.omega = zd{0.0, 0.0};
            q.flags |= F_OMEGA0;
          } else {
            q.omega = zd{a0 / a2, a1 / a2};
            if (a0 == 0.0 && a1 == 0.0) q.flags |= F_OMEGA0;
          }
        }
      } else if (EPI == EPI_RESID) {
        if (q.sel) q.rr_true = a0;
      }
    }
  }
}

template <typename T, bool DAG, int EPI>
__global__ __launch_bounds__(DS_BS) void k_dslash(DsBatch B, RhsScal* __restrict__ sc,
                                                  double* __restrict__ partials,
                                                  unsigned int* __restrict__ counter, int gate) {
  typedef typename IO<T>::SE SE;
  typedef typename IO<T>::LE LE;
  constexpr int NSE = IO<T>::NSE;
  const int lb = xcd_block(blockIdx.x, B.nblocks);
  int l = 0;
#pragma unroll
  for (int i = 1; i < MAXLAT; ++i)
    if (i < B.nlat && lb >= B.lat[i].blk_begin) l = i;
  const DsLat& L = B.lat[l];
  const int loc = lb - L.blk_begin;
  const int sb = loc / L.nrhs;
  const int r = loc - sb * L.nrhs;
  const int rhs = L.rhs_base + r;
  const int V = L.g.V;
  bool act = true;
  if (gate == 1) act = sc[rhs].active != 0;
  else if (gate == 2) act = sc[rhs].sel != 0;
  const int s = sb * DS_BS + threadIdx.x;
  const bool valid = act && (s < V);
  double red[3] = {0.0, 0.0, 0.0};
  if (valid) {
    const SE* in = (const SE*)L.in + (long long)r * NSE * V;
    SE* out = (SE*)L.out + (long long)r * NSE * V;
    const LE* U = (const LE*)L.links;
    int c[4], p;
    eo_coords(L.g, s, c, p);
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cx<T>{T(0), T(0)};
    hops_mu<T, DAG, 0>(in, U, L.g, s, c, acc);
    hops_mu<T, DAG, 1>(in, U, L.g, s, c, acc);
    hops_mu<T, DAG, 2>(in, U, L.g, s, c, acc);
    hops_mu<T, DAG, 3>(in, U, L.g, s, c, acc);
    cx<T> psi[12];
    IO<T>::load(in, V, s, psi);
    const T kap = T(L.kappa);
    const T tm = T(DAG ? -L.mu : L.mu);
    cx<T> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cx<T> v = psi[k] - kap * acc[k];
      const cx<T> tw = (k < 6 ? tm : -tm) * ti(psi[k]);  // i mu gamma5 psi, gamma5 = diag(1,1,-1,-1)
      o[k] = v + tw;
    }
    if (EPI == EPI_RESID) {
      cx<T> b[12];
      IO<T>::load((const SE*)L.aux + (long long)r * NSE * V, V, s, b);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        o[k] = b[k] - o[k];
        red[0] += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
      }
    } else if (EPI == EPI_RHAT) {
      cx<T> rh[12];
      IO<T>::load((const SE*)L.aux + (long long)r * NSE * V, V, s, rh);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        zd a{double(rh[k].re), double(rh[k].im)}, b{double(o[k].re), double(o[k].im)};
        zd d = cmulc(a, b);
        red[0] += d.re;
        red[1] += d.im;
      }
    } else if (EPI == EPI_TS) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        zd a{double(o[k].re), double(o[k].im)}, b{double(psi[k].re), double(psi[k].im)};
        zd d = cmulc(a, b);
        red[0] += d.re;
        red[1] += d.im;
        red[2] += a.re * a.re + a.im * a.im;
      }
    }
    IO<T>::store(out, V, s, o);
  }
  if (EPI != EPI_NONE) {
    __shared__ double sh[3 * (DS_BS / 64)];
    block_sum<3, DS_BS>(red, sh);
    if (threadIdx.x == 0) {
      double* pp = partials + ((long long)rhs * B.pstride + sb) * 3;
      pp[0] = red[0];
      pp[1] = red[1];
      pp[2] = red[2];
    }
  }
}

// The per-block partial sums are combined by a separate small launch: the kernel boundary makes
// every block's partials visible across XCDs without a device-scope fence in the streaming
// kernel (on a multi-XCD part such a fence writes back the whole L2 of the issuing XCD).
template <int EPI>
__global__ __launch_bounds__(DS_BS) void k_ds_finalize(DsBatch B, RhsScal* __restrict__ sc,
                                                       const double* __restrict__ partials) {
  finalize<EPI>(B, sc, partials);
}

template <typename T>
double launch(hipStream_t s, const DsBatch& b, int dagger, int epi, RhsScal* sc, double* partials,
              unsigned int* counter) {
  DBQ_CHECK(b.nlat >= 1 && b.nlat <= MAXLAT, "dslash: bad lattice count");
  DBQ_CHECK(epi == EPI_NONE || (sc && partials && counter), "dslash: epilogue needs scalars");
  int gate = 0;
  if (sc) gate = (epi == EPI_RESID) ? 2 : 1;
  dim3 grid(b.nblocks), block(DS_BS);
#define DBQ_DS(D, E) hipLaunchKernelGGL((k_dslash<T, D, E>), grid, block, 0, s, b, sc, partials, counter, gate)
  if (dagger) {
    switch (epi) {
      case EPI_NONE: DBQ_DS(true, EPI_NONE); break;
      case EPI_RHAT: DBQ_DS(true, EPI_RHAT); break;
      case EPI_TS: DBQ_DS(true, EPI_TS); break;
      default: DBQ_DS(true, EPI_RESID); break;
    }
  } else {
    switch (epi) {
      case EPI_NONE: DBQ_DS(false, EPI_NONE); break;
      case EPI_RHAT: DBQ_DS(false, EPI_RHAT); break;
      case EPI_TS: DBQ_DS(false, EPI_TS); break;
      default: DBQ_DS(false, EPI_RESID); break;
    }
  }
#undef DBQ_DS
  DBQ_HIP(hipGetLastError());
  if (epi != EPI_NONE) {
    // one wavefront per right-hand side, four per block
    const unsigned nb = unsigned((b.nrhs_total + DS_BS / 64 - 1) / (DS_BS / 64));
    if (epi == EPI_RHAT)
      hipLaunchKernelGGL((k_ds_finalize<EPI_RHAT>), dim3(nb), block, 0, s, b, sc, partials);
    else if (epi == EPI_TS)
      hipLaunchKernelGGL((k_ds_finalize<EPI_TS>), dim3(nb), block, 0, s, b, sc, partials);
    else
      hipLaunchKernelGGL((k_ds_finalize<EPI_RESID>), dim3(nb), block, 0, s, b, sc, partials);
    DBQ_HIP(hipGetLastError());
  }
  // algorithmic bytes: links once per lattice, each spinor read once and written once, plus
  // one epilogue operand per site (rhat or b)
  double bytes = 0;
  for (int i = 0; i < b.nlat; ++i) {
    const double V = b.lat[i].g.V;
    bytes += V * IO<T>::link_bytes();
    bytes += V * b.lat[i].nrhs * 2.0 * IO<T>::spinor_bytes();
    if (epi == EPI_RHAT || epi == EPI_RESID) bytes += V * b.lat[i].nrhs * IO<T>::spinor_bytes();
  }
  return bytes;
}

}  // namespace

double launch_dslash_f64(hipStream_t s, const DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, unsigned int* counter) {
  return launch<double>(s, b, dagger, epi, sc, partials, counter);
}
double launch_dslash_f32(hipStream_t s, const DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, unsigned int* counter) {
  return launch<float>(s, b, dagger, epi, sc, partials, counter);
}

}  // namespace dbq
