// Wilson / twisted-mass Dslash: out = A(mu) in, A(mu) = I - kappa*H + i*mu*gamma5 (the operator of
// Sec. 1 with the twisted term of the Sec. 4 action), or its dagger gamma5 A(-mu) gamma5.
//
// One thread per site and NB right-hand sides of one lattice: each link is loaded (and, in FP32,
// its third row rebuilt) once and applied to all NB spinors, so a batch of sources re-reads the
// gauge field NB times less and the index arithmetic is shared.  Each of the 8 hops
// spin-projects the neighbour spinor with (1 -+ gamma_mu) to two colour vectors (the projector
// has rank 2), multiplies them by the link or its adjoint with fused multiply-adds, and spreads
// the result back over four spins; with the chiral basis gamma_mu = [[0, B], [B^dagger, 0]] the
// projection is h = psi_up + S*B*psi_dn and the lower half of the result is S*B^dagger*chi.
// Epilogues fuse the inner products BiCGStab needs right after an operator application; the
// per-block partial sums are combined by a small follow-up launch (no device-scope fence in the
// streaming kernel: on a multi-XCD part such a fence writes back the issuing XCD's whole L2).
#include "kernels.h"

#ifndef DBQ_OCC_F32
#define DBQ_OCC_F32 0
#endif
#ifndef DBQ_OCC_F64
#define DBQ_OCC_F64 0
#endif
#ifndef DBQ_DS_CHAIN
#define DBQ_DS_CHAIN 0
#endif
#ifndef DBQ_DS_PARITY_INTERLEAVE
#define DBQ_DS_PARITY_INTERLEAVE 1
#endif
#ifndef DBQ_DS_NT_STORE
#define DBQ_DS_NT_STORE 1
#endif

namespace dbq {

namespace {

// z += a * b
template <typename T>
__device__ __forceinline__ void cmac(cx<T>& z, const cx<T>& a, const cx<T>& b) {
  z.re = fma(a.re, b.re, z.re);
  z.re = fma(-a.im, b.im, z.re);
  z.im = fma(a.re, b.im, z.im);
  z.im = fma(a.im, b.re, z.im);
}
// z += conj(a) * b
template <typename T>
__device__ __forceinline__ void cmacc(cx<T>& z, const cx<T>& a, const cx<T>& b) {
  z.re = fma(a.re, b.re, z.re);
  z.re = fma(a.im, b.im, z.re);
  z.im = fma(a.re, b.im, z.im);
  z.im = fma(-a.im, b.re, z.im);
}
// conj(a*b - c*d)
template <typename T>
__device__ __forceinline__ cx<T> cross_conj(const cx<T>& a, const cx<T>& b, const cx<T>& c,
                                            const cx<T>& d) {
  T re = c.im * d.im;
  re = fma(-c.re, d.re, re);
  re = fma(-a.im, b.im, re);
  re = fma(a.re, b.re, re);
  T im = -(c.im * d.re);
  im = fma(-c.re, d.im, im);
  im = fma(a.im, b.re, im);
  im = fma(a.re, b.im, im);
  return cx<T>{re, -im};
}

// Load / store through a uniform base pointer and a 32-bit byte offset, so that the address is
// a scalar base plus one VGPR (the global_load saddr form) instead of a 64-bit VGPR pair per load.
template <typename E>
__device__ __forceinline__ E ldo(const E* __restrict__ base, unsigned byte_off) {
  return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + byte_off);
}
// The operator's output is not read again by this launch: with DBQ_DS_NT_STORE it is written
// with the non-temporal hint so that it does not displace reusable neighbour data from L2.
typedef float nv_f4 __attribute__((ext_vector_type(4)));
typedef double nv_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(float4* p, const float4& v) {
  __builtin_nontemporal_store(nv_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nv_f4*>(p));
}
__device__ __forceinline__ void st_nt(double2* p, const double2& v) {
  __builtin_nontemporal_store(nv_d2{v.x, v.y}, reinterpret_cast<nv_d2*>(p));
}
// A load with the non-temporal hint, for operands read once per iteration (the epilogue's
// rhat), so that they do not displace the search vectors the next launches read again from the
// L2 and the last-level cache.
__device__ __forceinline__ float4 ld_nt(const float4* __restrict__ base, unsigned byte_off) {
  const nv_f4 v = __builtin_nontemporal_load(
      reinterpret_cast<const nv_f4*>(reinterpret_cast<const char*>(base) + byte_off));
  return make_float4(v.x, v.y, v.z, v.w);
}
template <typename E>
__device__ __forceinline__ void sto(E* __restrict__ base, unsigned byte_off, const E& v) {
  E* p = reinterpret_cast<E*>(reinterpret_cast<char*>(base) + byte_off);
#if DBQ_DS_NT_STORE
  st_nt(p, v);
#else
  *p = v;
#endif
}

template <typename T>
struct IO;

// Component arrays are V elements long; the base of each one is uniform, so only the site's
// byte offset lives in a vector register.
template <>
struct IO<double> {
  typedef double2 SE;
  typedef double2 LE;
  static constexpr int NSE = 12;  // double2 elements per site
  // [6][V][2]: the pair of components (2k, 2k+1) of one site is one 32-byte access
  __device__ __forceinline__ static void load(const double2* __restrict__ b, int V, int s,
                                              zd (&p)[12]) {
    const unsigned o = unsigned(s) * 32u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2* bk = b + 2ll * k * V;
      const double2 v0 = ldo(bk, o);
      const double2 v1 = ldo(bk, o + 16u);
      p[2 * k] = zd{v0.x, v0.y};
      p[2 * k + 1] = zd{v1.x, v1.y};
    }
  }
  __device__ __forceinline__ static void store(double2* __restrict__ b, int V, int s,
                                               const zd (&p)[12]) {
    const unsigned o = unsigned(s) * 32u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2* bk = b + 2ll * k * V;
      sto(bk, o, make_double2(p[2 * k].re, p[2 * k].im));
      sto(bk, o + 16u, make_double2(p[2 * k + 1].re, p[2 * k + 1].im));
    }
  }
  __device__ __forceinline__ static void link(const double2* __restrict__ U, int V, int mu, int s,
                                              zd (&u)[9]) {
    const unsigned o = unsigned(s) * 16u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = ldo(U + (long long)(mu * 9 + k) * V, o);
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
  static constexpr int NSE = 6;  // float4 elements per site
  __device__ __forceinline__ static void load(const float4* __restrict__ b, int V, int s,
                                              zf (&p)[12]) {
    const unsigned o = unsigned(s) * 16u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 v = ldo(b + (long long)k * V, o);
      p[2 * k] = zf{v.x, v.y};
      p[2 * k + 1] = zf{v.z, v.w};
    }
  }
  __device__ __forceinline__ static void load_nt(const float4* __restrict__ b, int V, int s,
                                                 zf (&p)[12]) {
    const unsigned o = unsigned(s) * 16u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 v = ld_nt(b + (long long)k * V, o);
      p[2 * k] = zf{v.x, v.y};
      p[2 * k + 1] = zf{v.z, v.w};
    }
  }
  __device__ __forceinline__ static void store(float4* __restrict__ b, int V, int s,
                                               const zf (&p)[12]) {
    const unsigned o = unsigned(s) * 16u;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      sto(b + (long long)k * V, o,
          make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im));
  }
  // two stored rows; the third row of an SU(3) matrix is the complex conjugate of the cross
  // product of the first two
  __device__ __forceinline__ static void link(const float4* __restrict__ U, int V, int mu, int s,
                                              zf (&u)[9]) {
    const unsigned o = unsigned(s) * 16u;
    const float4* b = U + (long long)mu * 3 * V;
    const float4 a = ldo(b, o);
    const float4 bb = ldo(b + V, o);
    const float4 c = ldo(b + 2ll * V, o);
    u[0] = zf{a.x, a.y};
    u[1] = zf{a.z, a.w};
    u[2] = zf{bb.x, bb.y};
    u[3] = zf{bb.z, bb.w};
    u[4] = zf{c.x, c.y};
    u[5] = zf{c.z, c.w};
    u[6] = cross_conj(u[1], u[5], u[2], u[4]);
    u[7] = cross_conj(u[2], u[3], u[0], u[5]);
    u[8] = cross_conj(u[0], u[4], u[1], u[3]);
  }
  static double link_bytes() { return 4.0 * 12 * 4; }
  static double spinor_bytes() { return 24.0 * 4; }
};

// h = psi_up + S * B_mu * psi_dn  (index 3*spin + colour, spin 0..1)
template <typename T, int MU, int S>
__device__ __forceinline__ void project(const cx<T> (&p)[12], cx<T> (&h)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if (MU == 0) {  // B = -i sigma_1: (B psi_dn) = (-i p3, -i p2)
      h[c] = S > 0 ? cx<T>{p0.re + p3.im, p0.im - p3.re} : cx<T>{p0.re - p3.im, p0.im + p3.re};
      h[3 + c] = S > 0 ? cx<T>{p1.re + p2.im, p1.im - p2.re} : cx<T>{p1.re - p2.im, p1.im + p2.re};
    } else if (MU == 1) {  // B = -i sigma_2: (B psi_dn) = (-p3, p2)
      h[c] = S > 0 ? p0 - p3 : p0 + p3;
      h[3 + c] = S > 0 ? p1 + p2 : p1 - p2;
    } else if (MU == 2) {  // B = -i sigma_3: (B psi_dn) = (-i p2, i p3)
      h[c] = S > 0 ? cx<T>{p0.re + p2.im, p0.im - p2.re} : cx<T>{p0.re - p2.im, p0.im + p2.re};
      h[3 + c] = S > 0 ? cx<T>{p1.re - p3.im, p1.im + p3.re} : cx<T>{p1.re + p3.im, p1.im - p3.re};
    } else {  // B = 1
      h[c] = S > 0 ? p0 + p2 : p0 - p2;
      h[3 + c] = S > 0 ? p1 + p3 : p1 - p3;
    }
  }
}

// acc_up += chi, acc_dn += S * B_mu^dagger * chi
template <typename T, int MU, int S>
__device__ __forceinline__ void spread(cx<T> (&acc)[12], const cx<T> (&chi)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<T> c0 = chi[c], c1 = chi[3 + c];
    acc[c] = acc[c] + c0;
    acc[3 + c] = acc[3 + c] + c1;
    // i*z = (-z.im, z.re)
    if (MU == 0) {  // B^dag = [[0, i], [i, 0]]: (i c1, i c0)
      acc[6 + c] = S > 0 ? cx<T>{acc[6 + c].re - c1.im, acc[6 + c].im + c1.re}
                         : cx<T>{acc[6 + c].re + c1.im, acc[6 + c].im - c1.re};
      acc[9 + c] = S > 0 ? cx<T>{acc[9 + c].re - c0.im, acc[9 + c].im + c0.re}
                         : cx<T>{acc[9 + c].re + c0.im, acc[9 + c].im - c0.re};
    } else if (MU == 1) {  // B^dag = [[0, 1], [-1, 0]]: (c1, -c0)
      acc[6 + c] = S > 0 ? acc[6 + c] + c1 : acc[6 + c] - c1;
      acc[9 + c] = S > 0 ? acc[9 + c] - c0 : acc[9 + c] + c0;
    } else if (MU == 2) {  // B^dag = [[i, 0], [0, -i]]: (i c0, -i c1)
      acc[6 + c] = S > 0 ? cx<T>{acc[6 + c].re - c0.im, acc[6 + c].im + c0.re}
                         : cx<T>{acc[6 + c].re + c0.im, acc[6 + c].im - c0.re};
      acc[9 + c] = S > 0 ? cx<T>{acc[9 + c].re + c1.im, acc[9 + c].im - c1.re}
                         : cx<T>{acc[9 + c].re - c1.im, acc[9 + c].im + c1.re};
    } else {  // B^dag = 1
      acc[6 + c] = S > 0 ? acc[6 + c] + c0 : acc[6 + c] - c0;
      acc[9 + c] = S > 0 ? acc[9 + c] + c1 : acc[9 + c] - c1;
    }
  }
}

// One hop for NB right-hand sides: BACK = false -> (1 + S gamma) U_mu(x) psi(x+mu);
// BACK = true -> (1 + S gamma) U_mu(y)^dag psi(y) with y = x - mu.  The link is read at site
// site_link of the full link field (V sites per component); the spinor at index ys of vectors
// with Vs sites per component (Vs = V, or V/2 for the half vectors of the even-odd reduced
// operator).
template <typename T, int MU, int S, bool BACK, int NB>
__device__ __forceinline__ void hop(const typename IO<T>::SE* __restrict__ in, long long rstride,
                                    int nval, const typename IO<T>::LE* __restrict__ U, int V,
                                    int site_link, int Vs, int ys, cx<T> (&acc)[NB][12]) {
  cx<T> u[9];
  IO<T>::link(U, V, MU, site_link, u);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (NB > 1 && j >= nval) break;
    cx<T> p[12];
    IO<T>::load(in + j * rstride, Vs, ys, p);
    cx<T> h[6];
    project<T, MU, S>(p, h);
    cx<T> chi[6];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<T> z{T(0), T(0)};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (!BACK) cmac(z, u[3 * a + b], h[3 * sp + b]);
          else cmacc(z, u[3 * b + a], h[3 * sp + b]);
        }
        chi[3 * sp + a] = z;
      }
    }
    spread<T, MU, S>(acc[j], chi);
  }
}

// Both hops in direction MU of the site with coordinates c and internal index s; the input
// spinors have Vs sites per component and a neighbour with internal index y sits at y - off
// (off = V/2 for odd-site half vectors, 0 otherwise).
template <typename T, bool DAG, int MU, int NB>
__device__ __forceinline__ void hops_mu(const typename IO<T>::SE* __restrict__ in,
                                        long long rstride, int nval,
                                        const typename IO<T>::LE* __restrict__ U, const Geom& g,
                                        int s, const int (&c)[4], cx<T> (&acc)[NB][12],
                                        int Vs, int off) {
  // forward hop uses (1 - gamma) (dagger: 1 + gamma), backward the opposite
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  const int yf = eo_neighbour<MU, +1>(g, c);
  const int yb = eo_neighbour<MU, -1>(g, c);
  hop<T, MU, SF, false, NB>(in, rstride, nval, U, g.V, s, Vs, yf - off, acc);
  hop<T, MU, SB, true, NB>(in, rstride, nval, U, g.V, yb, Vs, yb - off, acc);
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// Byte accounting of a gated launch (timing only), done by the blocks of the first site block or
// tile of a lattice: each rhs they process adds its spinor traffic, the first one of the lattice
// in this launch (its tag still clear) also the links.  The launch's finalize clears the tags
// again, so a graph that replays the launch counts its links on every replay.
__device__ __forceinline__ void account(const DsBatch& B, int l) {
  unsigned long long by = (unsigned long long)B.lat[l].g.V *
                          (unsigned long long)(B.acct.spinor_passes * B.acct.spinor_bytes);
  if (atomicExch(B.acct.tags + l, 1ull) == 0ull)
    by += (unsigned long long)B.lat[l].g.V * (unsigned long long)B.acct.link_bytes;
  atomicAdd(B.acct.bytes, by);
}

// Combine the per-block partials of one epilogue: every right-hand side of the batch is reduced
// by one wavefront over its site blocks in a fixed order.
template <int EPI>
__device__ void finalize(const DsBatch& B, RhsScal* sc, const double* partials) {
  // the accounted Dslash launch before this one has finished: clear its link tags
  if (B.acct.tags && blockIdx.x == 0 && threadIdx.x < B.nlat) B.acct.tags[threadIdx.x] = 0ull;
  const int lane = threadIdx.x & 63;
  constexpr int NW = DS_BS / 64;
  const int w = blockIdx.x * NW + (threadIdx.x >> 6);
  const int stride = gridDim.x * NW;
  for (int rhs = w; rhs < B.nrhs_total; rhs += stride) {
    int l = 0;
    for (int i = 1; i < B.nlat; ++i)
      if (rhs >= B.lat[i].rhs_base) l = i;
    const int nsb = B.lat[l].nsb;
    if (EPI == EPI_RHAT && B.xr_part) {
      // the end of the previous iteration, whose own finalize launch was left out: ||r||^2 from
      // the update step's partials in the order the update step's finalize adds them
      const int nch = (B.xr_nelem[rhs] + BL_CHUNK - 1) / BL_CHUNK;
      const double* pr = B.xr_part + (long long)rhs * B.xr_pstride * 3;
      double r2 = 0;
      for (int j0 = lane; j0 < nch; j0 += 64 * FIN_U) {
        double v[FIN_U];
#pragma unroll
        for (int u = 0; u < FIN_U; ++u)
          if (j0 + 64 * u < nch) v[u] = pr[3 * (j0 + 64 * u) + 2];
#pragma unroll
        for (int u = 0; u < FIN_U; ++u)
          if (j0 + 64 * u < nch) r2 += v[u];
      }
      r2 = wave_sum(r2);
      if (lane == 0) fin_xr(sc[rhs], r2);
    }
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0;
    const double* pp = partials + (long long)rhs * B.pstride * 3;
    const double* px = partials + (long long)B.nrhs_total * B.pstride * 3 +
                       (long long)rhs * B.pstride * 4;
    // FIN_U partials per lane are loaded before any of them is added, so their loads are in
    // flight together; the additions keep the order j = lane, lane + 64, ...
    for (int j0 = lane; j0 < nsb; j0 += 64 * FIN_U) {
      double v[FIN_U][7];
#pragma unroll
      for (int u = 0; u < FIN_U; ++u) {
        const int j = j0 + 64 * u;
        if (j < nsb) {
          v[u][0] = pp[3 * j];
          v[u][1] = pp[3 * j + 1];
          v[u][2] = pp[3 * j + 2];
          if (EPI == EPI_TS) {
            v[u][3] = px[4 * j];
            v[u][4] = px[4 * j + 1];
            v[u][5] = px[4 * j + 2];
            v[u][6] = px[4 * j + 3];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < FIN_U; ++u) {
        if (j0 + 64 * u < nsb) {
          a0 += v[u][0];
          a1 += v[u][1];
          a2 += v[u][2];
          if (EPI == EPI_TS) {
            a3 += v[u][3];
            a4 += v[u][4];
            a5 += v[u][5];
            a6 += v[u][6];
          }
        }
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (EPI == EPI_TS) {
      a3 = wave_sum(a3);
      a4 = wave_sum(a4);
      a5 = wave_sum(a5);
      a6 = wave_sum(a6);
    }
    if (lane == 0) {
      RhsScal& q = sc[rhs];
      if (EPI == EPI_RHAT) {
        if (q.active) {
          const zd d{a0, a1};
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
        // omega = <t, s> / |t|^2; the next rho = <rhat, s - omega t> = <rhat, s> - omega
        // <rhat, t> (both sums taken from the vectors, so no rounding carries over from earlier
        // iterations; <rhat, s> is small but not zero); beta = (rho_next / rho)(alpha / omega)
        // lets the update step form the next search direction in the same pass
        if (q.active) {
          if (!finite_d(a0) || !finite_d(a1) || !finite_d(a2) || !finite_d(a3) ||
              !finite_d(a4) || !finite_d(a5) || !finite_d(a6)) {
            q.flags |= F_NAN;
            q.active = 0;
          } else if (a2 == 0.0 || (a0 == 0.0 && a1 == 0.0)) {
            q.omega = zd{a2 == 0.0 ? 0.0 : a0 / a2, a2 == 0.0 ? 0.0 : a1 / a2};
            q.flags |= F_OMEGA0;
            q.rho_next = zd{0.0, 0.0};
            q.beta = zd{0.0, 0.0};
          } else {
            q.omega = zd{a0 / a2, a1 / a2};
            const zd rt{a3, a4}, rs{a5, a6};
            q.rho_next = rs - q.omega * rt;
            q.beta = cdiv(q.rho_next, q.rho) * cdiv(q.alpha, q.omega);
          }
        }
      } else if (EPI == EPI_RESID) {
        if (q.sel) {
          q.rr_true = a0;
          if (B.decide) {
            // reliable update on the device: converged rhs stop, the others keep sel for the
            // residual replacement that follows
            q.nrel += 1;
            if (a0 <= q.stop2) {
              q.flags = F_DONE;
              q.active = 0;
              q.sel = 0;
            } else if (!finite_d(a0)) {
              q.flags = F_NAN;
              q.active = 0;
              q.sel = 0;
            } else {
              // a stall: the FP32 recursion claimed a 10x drop (or ran STALL_ITERS iterations
              // without one) but the FP64 residual fell by less than 2x since the last check;
              // convergence claims just above the tolerance are not counted.  A residual grown
              // by 100x since the last check means the FP32 iteration diverges: stop at once.
              const bool slow = a0 > 0.25 * q.rr_prev;
              const bool diverged = a0 > 1e4 * q.rr_prev;
              if (!slow) q.stalls = 0;
              else if (q.rr <= 0.01 * q.rr_prev || q.since >= STALL_ITERS) q.stalls += 1;
              q.rr_prev = a0;
              if (q.stalls >= 2 || diverged) {
                q.flags = F_STALL;
                q.active = 0;
                q.sel = 0;
              }
            }
          }
        }
      }
    }
  }
}

// With DBQ_DS_CHAIN the coordinates of the next direction formally depend on the accumulator,
// so one direction's neighbour loads are issued at a time instead of all 8 hops' loads being
// hoisted to the top (which costs registers and therefore resident waves).
template <typename T, int NB>
__device__ __forceinline__ void chain(int (&c)[4], int& s, cx<T> (&acc)[NB][12]) {
#if DBQ_DS_CHAIN
  // every accumulator component of the first right-hand side passes through the barrier
  asm volatile(""
               : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(s),
                 "+v"(acc[0][0].re), "+v"(acc[0][0].im), "+v"(acc[0][1].re), "+v"(acc[0][1].im),
                 "+v"(acc[0][2].re), "+v"(acc[0][2].im), "+v"(acc[0][3].re), "+v"(acc[0][3].im),
                 "+v"(acc[0][4].re), "+v"(acc[0][4].im), "+v"(acc[0][5].re), "+v"(acc[0][5].im),
                 "+v"(acc[0][6].re), "+v"(acc[0][6].im), "+v"(acc[0][7].re), "+v"(acc[0][7].im),
                 "+v"(acc[0][8].re), "+v"(acc[0][8].im), "+v"(acc[0][9].re), "+v"(acc[0][9].im),
                 "+v"(acc[0][10].re), "+v"(acc[0][10].im), "+v"(acc[0][11].re), "+v"(acc[0][11].im));
#endif
}

// The site's result psi - kappa*acc + i*t*gamma5*psi (t = mu, or -mu for the dagger) and the
// epilogue's contributions to the per-block sums: RESID replaces the result by aux - result and
// adds its norm, RHAT adds <aux, result>, TS adds <result, psi>, |result|^2, <aux, result> and
// <aux, psi> (aux, the epilogue operand at the site: b for RESID, rhat for RHAT and TS).  rd holds
// DS_NSUM running sums.
template <typename T, int EPI>
__device__ __forceinline__ void finish_site(const cx<T> (&psi)[12], const cx<T> (&acc)[12], T kap,
                                            T tm, const cx<T> (&aux)[12], double* rd,
                                            cx<T> (&o)[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    // gamma5 = diag(1,1,-1,-1) over spins
    const T t = k < 6 ? tm : -tm;
    o[k].re = fma(-kap, acc[k].re, fma(-t, psi[k].im, psi[k].re));
    o[k].im = fma(-kap, acc[k].im, fma(t, psi[k].re, psi[k].im));
  }
  if (EPI == EPI_RESID) {
    T nn = T(0);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      o[k] = aux[k] - o[k];
      nn = fma(o[k].re, o[k].re, fma(o[k].im, o[k].im, nn));
    }
    rd[0] += double(nn);
  } else if (EPI == EPI_RHAT) {
    cx<T> d{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 12; ++k) cmacc(d, aux[k], o[k]);
    rd[0] += double(d.re);
    rd[1] += double(d.im);
  } else if (EPI == EPI_TS) {
    cx<T> d{T(0), T(0)}, h{T(0), T(0)}, g{T(0), T(0)};
    T nn = T(0);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cmacc(d, o[k], psi[k]);
      cmacc(h, aux[k], o[k]);
      cmacc(g, aux[k], psi[k]);
      nn = fma(o[k].re, o[k].re, fma(o[k].im, o[k].im, nn));
    }
    rd[0] += double(d.re);
    rd[1] += double(d.im);
    rd[2] += double(nn);
    rd[3] += double(h.re);
    rd[4] += double(h.im);
    rd[5] += double(g.re);
    rd[6] += double(g.im);
  }
}

// number of the DS_NSUM partial sums an epilogue fills (the others stay zero; 1 for the
// output-only one, which reduces nothing)
template <int EPI>
constexpr int epi_sums() {
  return EPI == EPI_TS ? 7 : (EPI == EPI_RHAT ? 2 : 1);
}

// block sums of the first epi_sums<EPI>() of the DS_NSUM sums of each of NB rhs (valid in
// thread 0)
template <int EPI, int NB, int BS>
__device__ __forceinline__ void block_sum_epi(double* red, double* sh) {
  constexpr int NS = epi_sums<EPI>();
  double t[NB * NS];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int i = 0; i < NS; ++i) t[j * NS + i] = red[j * DS_NSUM + i];
  block_sum<NB * NS, BS>(t, sh);
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int i = 0; i < NS; ++i) red[j * DS_NSUM + i] = t[j * NS + i];
}

// <rhat, t> and <rhat, s> of the <t, s> epilogue go to a second partial-sum region after the
// first (nrhs_total x pstride slots of 3 doubles), 4 doubles per slot
__device__ __forceinline__ double* ts_extra(const DsBatch& B, double* partials, long long rhs,
                                            long long slot) {
  return partials + (long long)B.nrhs_total * B.pstride * 3 + (rhs * B.pstride + slot) * 4;
}

// stores the block's sums of one rhs: 3 into the first region, the TS epilogue's other 4 into
// the second
template <int EPI>
__device__ __forceinline__ void store_sums(const DsBatch& B, double* partials, long long rhs,
                                           long long slot, const double* rd) {
  double* pp = partials + (rhs * B.pstride + slot) * 3;
  pp[0] = rd[0];
  pp[1] = rd[1];
  pp[2] = rd[2];
  if (EPI == EPI_TS) {
    double* px = ts_extra(B, partials, rhs, slot);
    px[0] = rd[3];
    px[1] = rd[4];
    px[2] = rd[5];
    px[3] = rd[6];
  }
}

// Minimum waves per SIMD the register allocation must leave room for (1: no constraint).
template <typename T, int NB>
struct Occ {
  static constexpr int value = sizeof(T) == 4 ? (DBQ_OCC_F32 > 0 ? DBQ_OCC_F32 : 1)
                                              : (DBQ_OCC_F64 > 0 ? DBQ_OCC_F64 : 1);
};
#define DBQ_DS_ATTR __attribute__((amdgpu_waves_per_eu(Occ<T, NB>::value)))

template <typename T, bool DAG, int EPI, int NB>
__global__ __launch_bounds__(DS_BS) DBQ_DS_ATTR
void k_dslash(DsBatch B, RhsScal* __restrict__ sc, double* __restrict__ partials, int gate) {
  typedef typename IO<T>::SE SE;
  typedef typename IO<T>::LE LE;
  constexpr int NSE = IO<T>::NSE;
  const int lb = xcd_block(blockIdx.x, B.nblocks);
  int l = 0;
#pragma unroll
  for (int i = 1; i < MAXLAT; ++i)
    if (i < B.nlat && lb >= B.lat[i].blk_begin) l = i;
  const DsLat& L = B.lat[l];
  const int ng = (L.nrhs + NB - 1) / NB;
  const int loc = lb - L.blk_begin;
  // block order within the lattice: chunks of G rhs groups; in a chunk, site blocks in order
  // with the chunk's rhs groups adjacent (they share the links through L2)
  const int G = (B.rgroup <= 0 || B.rgroup > ng) ? ng : B.rgroup;
  const int chunk = loc / (L.nsb * G);
  const int rem = loc - chunk * (L.nsb * G);
  const int Gc = min(G, ng - chunk * G);
  const int sb = rem / Gc;
  const int r0 = (chunk * G + (rem - sb * Gc)) * NB;
  const int nval = min(NB, L.nrhs - r0);
  const int V = L.g.V;
  const long long rstride = (long long)NSE * V;
  bool act[NB];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    bool a = j < nval;
    if (a && gate == 1) a = sc[L.rhs_base + r0 + j].active != 0;
    else if (a && gate == 2) a = sc[L.rhs_base + r0 + j].sel != 0;
    act[j] = a;
    any = any || a;
  }
  if (B.acct.bytes && sb == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (act[j]) account(B, l);
  }
#if DBQ_DS_PARITY_INTERLEAVE
  // consecutive site blocks alternate between the two parities of the same spatial range, so
  // each XCD (which receives a contiguous range of blocks) holds both halves of one slab and
  // finds a site's spinor and links in its own L2 when it is needed as centre and as neighbour
  const int Vh = V >> 1;
  const int hl = (sb >> 1) * DS_BS + threadIdx.x;
  const int s = (sb & 1) * Vh + hl;
  const bool in_range = hl < Vh;
#else
  const int s = sb * DS_BS + threadIdx.x;
  const bool in_range = s < V;
#endif
  double red[NB * DS_NSUM];
#pragma unroll
  for (int i = 0; i < NB * DS_NSUM; ++i) red[i] = 0.0;
  if (any && in_range) {
    const SE* in = (const SE*)L.in + r0 * rstride;
    SE* out = (SE*)L.out + r0 * rstride;
    const LE* U = (const LE*)L.links;
    int c[4], p;
    eo_coords(L.g, s, c, p);
    cx<T> acc[NB][12];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[j][k] = cx<T>{T(0), T(0)};
    int sl = s;  // link site of the forward hops, chained like the coordinates
    hops_mu<T, DAG, 0, NB>(in, rstride, nval, U, L.g, sl, c, acc, V, 0);
    chain(c, sl, acc);
    hops_mu<T, DAG, 1, NB>(in, rstride, nval, U, L.g, sl, c, acc, V, 0);
    chain(c, sl, acc);
    hops_mu<T, DAG, 2, NB>(in, rstride, nval, U, L.g, sl, c, acc, V, 0);
    chain(c, sl, acc);
    hops_mu<T, DAG, 3, NB>(in, rstride, nval, U, L.g, sl, c, acc, V, 0);
    const T kap = T(L.kappa);
    const T tm = T(DAG ? -L.mu : L.mu);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (!act[j]) continue;
      cx<T> psi[12];
      IO<T>::load(in + j * rstride, V, s, psi);
      cx<T> ax[12];
      if (EPI != EPI_NONE)
        IO<T>::load((const SE*)L.aux + (r0 + j) * rstride, V, s, ax);
      cx<T> o[12];
      finish_site<T, EPI>(psi, acc[j], kap, tm, ax, red + DS_NSUM * j, o);
      IO<T>::store(out + j * rstride, V, s, o);
    }
  }
  if (EPI != EPI_NONE) {
    __shared__ double sh[NB * DS_NSUM * (DS_BS / 64)];
    block_sum_epi<EPI, NB, DS_BS>(red, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j >= nval) break;
        store_sums<EPI>(B, partials, L.rhs_base + r0 + j, sb, red + DS_NSUM * j);
      }
    }
  }
}

// ============================================================================ even-odd halves
// The even-odd reduced operator of Sec. 3 and Sec. 4 on half vectors (the sites of one parity,
// [rhs][component][V/2] in the internal order minus the parity offset), as two launches of one
// kernel that computes the sites of one parity from the hop of the other parity's vector:
//   STEP 1 (odd sites):  out = D^{-1} (cen + c H_oe in),         D^{-1} = (1 - i t gamma5)/(1 + t^2)
//   STEP 2 (even sites): out = D cen - c H_eo in  (+ epilogue),  D = 1 + i t gamma5
// with c = L.kappa and t = L.mu (-mu for the dagger, whose hops use H^dagger).  cen may be null
// in STEP 1 (read as zero); c = 0 skips the hops.  The Schur complement
// Ahat = D - kappa^2 H_eo D^{-1} H_oe is STEP 1 (c = 1, no cen) followed by STEP 2 (c = kappa^2,
// cen = the vector Ahat is applied to); the same kernel forms the reduced right-hand side and
// the odd half of the solution.  The epilogues are those of the full operator.
// STEP 1's result D^{-1} (cen + c acc)
template <typename T>
__device__ __forceinline__ void finish_odd(const cx<T> (&cen)[12], const cx<T> (&acc)[12], T c,
                                           T tm, cx<T> (&o)[12]) {
  const T inv = T(1) / fma(tm, tm, T(1));
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const T t = k < 6 ? tm : -tm;
    const T wr = fma(c, acc[k].re, cen[k].re);
    const T wi = fma(c, acc[k].im, cen[k].im);
    // (1 - i t) (wr + i wi) = (wr + t wi) + i (wi - t wr)
    o[k].re = fma(t, wi, wr) * inv;
    o[k].im = fma(-t, wr, wi) * inv;
  }
}

template <typename T, bool DAG, int EPI, int NB, int STEP>
__global__ __launch_bounds__(DS_BS) DBQ_DS_ATTR
void k_dslash_half(DsBatch B, RhsScal* __restrict__ sc, double* __restrict__ partials, int gate) {
  typedef typename IO<T>::SE SE;
  typedef typename IO<T>::LE LE;
  constexpr int NSE = IO<T>::NSE;
  constexpr int P = STEP == 1 ? 1 : 0;  // parity of the output sites
  const int lb = xcd_block(blockIdx.x, B.nblocks);
  int l = 0;
#pragma unroll
  for (int i = 1; i < MAXLAT; ++i)
    if (i < B.nlat && lb >= B.lat[i].blk_begin) l = i;
  const DsLat& L = B.lat[l];
  const int ng = (L.nrhs + NB - 1) / NB;
  const int loc = lb - L.blk_begin;
  // block order as in k_dslash: chunks of G rhs groups, site blocks, rhs groups of a chunk
  const int G = (B.rgroup <= 0 || B.rgroup > ng) ? ng : B.rgroup;
  const int chunk = loc / (L.nsb * G);
  const int rem = loc - chunk * (L.nsb * G);
  const int Gc = min(G, ng - chunk * G);
  const int sb = rem / Gc;
  const int r0 = (chunk * G + (rem - sb * Gc)) * NB;
  const int nval = min(NB, L.nrhs - r0);
  const int Vh = L.g.V >> 1;
  const long long rstride = (long long)NSE * Vh;
  bool act[NB];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    bool a = j < nval;
    if (a && gate == 1) a = sc[L.rhs_base + r0 + j].active != 0;
    else if (a && gate == 2) a = sc[L.rhs_base + r0 + j].sel != 0;
    act[j] = a;
    any = any || a;
  }
  const int h = sb * DS_BS + threadIdx.x;
  double red[NB * DS_NSUM];
#pragma unroll
  for (int i = 0; i < NB * DS_NSUM; ++i) red[i] = 0.0;
  if (any && h < Vh) {
    const SE* in = (const SE*)L.in + r0 * rstride;
    SE* out = (SE*)L.out + r0 * rstride;
    const LE* U = (const LE*)L.links;
    const int s = P * Vh + h;
    int c[4], p;
    eo_coords(L.g, s, c, p);
    cx<T> acc[NB][12];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[j][k] = cx<T>{T(0), T(0)};
    const T coef = T(L.kappa);
    if (coef != T(0)) {
      const int off = (1 - P) * Vh;  // neighbours have the other parity
      hops_mu<T, DAG, 0, NB>(in, rstride, nval, U, L.g, s, c, acc, Vh, off);
      hops_mu<T, DAG, 1, NB>(in, rstride, nval, U, L.g, s, c, acc, Vh, off);
      hops_mu<T, DAG, 2, NB>(in, rstride, nval, U, L.g, s, c, acc, Vh, off);
      hops_mu<T, DAG, 3, NB>(in, rstride, nval, U, L.g, s, c, acc, Vh, off);
    }
    const T tm = T(DAG ? -L.mu : L.mu);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (!act[j]) continue;
      cx<T> ce[12];
      if (L.cen) {
        IO<T>::load((const SE*)L.cen + (r0 + j) * rstride, Vh, h, ce);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) ce[k] = cx<T>{T(0), T(0)};
      }
      cx<T> o[12];
      if (STEP == 1) {
        finish_odd<T>(ce, acc[j], coef, tm, o);
      } else {
        cx<T> ax[12];
        if (EPI != EPI_NONE)
          IO<T>::load((const SE*)L.aux + (r0 + j) * rstride, Vh, h, ax);
        finish_site<T, EPI>(ce, acc[j], coef, tm, ax, red + DS_NSUM * j, o);
      }
      IO<T>::store(out + j * rstride, Vh, h, o);
    }
  }
  if (EPI != EPI_NONE) {
    __shared__ double sh[NB * DS_NSUM * (DS_BS / 64)];
    block_sum_epi<EPI, NB, DS_BS>(red, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j >= nval) break;
        store_sums<EPI>(B, partials, L.rhs_base + r0 + j, sb, red + DS_NSUM * j);
      }
    }
  }
}

// ============================================================================ LDS-staged FP32
// One block per (site tile, chunk of right-hand sides).  The block holds the 8 links of each of
// its sites in registers for the whole chunk and, for one rhs after the other, copies the
// tile's spinors and the eight neighbouring faces into LDS with LDS-direct loads (no registers
// held while they are in flight), then every site reads its eight neighbours from LDS.  Each
// spinor of the tile therefore passes through the vector memory unit once per rhs instead of
// nine times (once as a centre, eight times as a neighbour), and each link once per chunk.
//
// LDS slots (per spinor component k = 0..5, float4 each, TL_SLOTS per component):
//   [0, Vt)       the tile: parity p = slot >= Vt/2, the slot's half index in the tile
//                 (the same order as in memory, so each parity half is one contiguous copy)
//   [Vt, Vt + H)  faces (mu, +), (mu, -) for mu = 0..3: the Vt/T_mu sites of the tile beyond
//                 this one in direction +-mu next to it, in lexicographic order of the three
//                 other in-tile coordinates
constexpr int TL_SLOTS = 768;  // 4^4 tile: 256 + 8 x 64

// rhs per block of the tile kernel: rgroup, 0 = all
__host__ __device__ __forceinline__ int tile_chunk(int rgroup, int nrhs) {
  return (rgroup <= 0 || rgroup > nrhs) ? nrhs : rgroup;
}

struct TileGeo {
  int vt, vh;        // sites per tile, per parity
  int fbase[8];      // first slot of each face
};

__device__ __forceinline__ TileGeo tile_geo(const Geom& g) {
  TileGeo t;
  t.vh = 1 << g.lTh;
  t.vt = 2 * t.vh;
  int b = t.vt;
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    t.fbase[f] = b;
    b += t.vt >> g.lT[f >> 1];
  }
  return t;
}

// in-tile coordinates of tile slot j < Vt (tile origins have even coordinate sums)
__device__ __forceinline__ void tile_coords(const Geom& g, const TileGeo& t, int j, int (&ic)[4]) {
  const int p = j >= t.vh ? 1 : 0;
  uint32_t r = uint32_t(j - p * t.vh) << 1;
  ic[0] = int(r & uint32_t(g.T[0] - 1));
  r >>= g.lT[0];
  ic[1] = int(r & uint32_t(g.T[1] - 1));
  r >>= g.lT[1];
  ic[2] = int(r & uint32_t(g.T[2] - 1));
  ic[3] = int(r >> g.lT[2]);
  ic[0] += (p + ic[1] + ic[2] + ic[3]) & 1;
}

__device__ __forceinline__ int in_tile_half(const Geom& g, const int (&ic)[4]) {
  const int il = ic[0] | (ic[1] << g.lT[0]) | (ic[2] << (g.lT[0] + g.lT[1])) |
                 (ic[3] << (g.lT[0] + g.lT[1] + g.lT[2]));
  return il >> 1;
}

// position of in-tile coordinates on the face orthogonal to MU
template <int MU>
__device__ __forceinline__ int face_index(const Geom& g, const int (&ic)[4]) {
  int q = 0, sh = 0;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == MU) continue;
    q |= ic[nu] << sh;
    sh += g.lT[nu];
  }
  return q;
}

// LDS slot of the neighbour x + DIR*MU of the tile site with in-tile coordinates ic
template <int MU, int DIR>
__device__ __forceinline__ int nbr_slot(const Geom& g, const TileGeo& t, const int (&ic)[4]) {
  const int v = ic[MU] + DIR;
  if (v >= 0 && v < g.T[MU]) {
    int d[4] = {ic[0], ic[1], ic[2], ic[3]};
    d[MU] = v;
    const int p = (d[0] + d[1] + d[2] + d[3]) & 1;
    return p * t.vh + in_tile_half(g, d);
  }
  return t.fbase[2 * MU + (DIR > 0 ? 0 : 1)] + face_index<MU>(g, ic);
}

// memory index (internal order) of the site held in LDS slot j of tile tc; slots past the last
// face repeat the tile's first site (their copies are never read)
__device__ __forceinline__ int slot_site(const Geom& g, const TileGeo& t, const int (&tc)[4],
                                         int tile, int j, int nslots) {
  if (j < t.vt) {
    const int p = j >= t.vh ? 1 : 0;
    return p * g.Vh + (tile << g.lTh) + (j - p * t.vh);
  }
  if (j >= nslots) return tile << g.lTh;
  // face f and its first slot, selected without indexing a local array by a runtime value
  // (which would place the array in scratch memory)
  int f = 0, fb = t.fbase[0];
#pragma unroll
  for (int i = 1; i < 8; ++i)
    if (j >= t.fbase[i]) {
      f = i;
      fb = t.fbase[i];
    }
  const int mu = f >> 1;
  const int dir = (f & 1) ? -1 : +1;
  uint32_t q = uint32_t(j - fb);
  int ic[4], tn[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) {
      ic[nu] = dir > 0 ? 0 : g.T[nu] - 1;
      int v = tc[nu] + dir;
      tn[nu] = v < 0 ? g.NT[nu] - 1 : (v == g.NT[nu] ? 0 : v);
    } else {
      ic[nu] = int(q & uint32_t(g.T[nu] - 1));
      q >>= g.lT[nu];
      tn[nu] = tc[nu];
    }
  }
  const int tile_n = tn[0] + g.NT[0] * (tn[1] + g.NT[1] * (tn[2] + g.NT[2] * tn[3]));
  const int p = (ic[0] + ic[1] + ic[2] + ic[3]) & 1;
  return p * g.Vh + (tile_n << g.lTh) + in_tile_half(g, ic);
}

// the spinor in LDS slot `slot` of a staging area with NS slots per component
template <int NS>
__device__ __forceinline__ void lds_spinor(const float4* lds, int slot, zf (&p)[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 v = lds[k * NS + slot];
    p[2 * k] = zf{v.x, v.y};
    p[2 * k + 1] = zf{v.z, v.w};
  }
}

__device__ __forceinline__ void rebuild(const float4 (&l)[3], zf (&u)[9]) {
  u[0] = zf{l[0].x, l[0].y};
  u[1] = zf{l[0].z, l[0].w};
  u[2] = zf{l[1].x, l[1].y};
  u[3] = zf{l[1].z, l[1].w};
  u[4] = zf{l[2].x, l[2].y};
  u[5] = zf{l[2].z, l[2].w};
  u[6] = cross_conj(u[1], u[5], u[2], u[4]);
  u[7] = cross_conj(u[2], u[3], u[0], u[5]);
  u[8] = cross_conj(u[0], u[4], u[1], u[3]);
}

// one hop from LDS: BACK = false -> (1 + S gamma) U psi(slot); BACK = true -> U^dagger instead
template <int MU, int S, bool BACK, int NS = TL_SLOTS>
__device__ __forceinline__ void hop_lds(const float4* lds, int slot, const float4 (&l)[3],
                                        zf (&acc)[12]) {
  zf u[9];
  rebuild(l, u);
  zf p[12];
  lds_spinor<NS>(lds, slot, p);
  zf h[6];
  project<float, MU, S>(p, h);
  zf chi[6];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      zf z{0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (!BACK) cmac(z, u[3 * a + b], h[3 * sp + b]);
        else cmacc(z, u[3 * b + a], h[3 * sp + b]);
      }
      chi[3 * sp + a] = z;
    }
  }
  spread<float, MU, S>(acc, chi);
}

template <bool DAG, int EPI>
__global__ __launch_bounds__(DS_BS) void k_dslash_tile(DsBatch B, RhsScal* __restrict__ sc,
                                                       double* __restrict__ partials, int gate) {
  __shared__ float4 lds[6 * TL_SLOTS];
  const int lb = xcd_block(blockIdx.x, B.nblocks);
  int l = 0;
#pragma unroll
  for (int i = 1; i < MAXLAT; ++i)
    if (i < B.nlat && lb >= B.lat[i].blk_begin) l = i;
  const DsLat& L = B.lat[l];
  const Geom& g = L.g;
  const int G = tile_chunk(B.rgroup, L.nrhs);
  const int nch = (L.nrhs + G - 1) / G;
  int tc[4], tile, chunk;
  tile_of_block(g, lb - L.blk_begin, nch, B.torder, tc, tile, chunk);
  const int r0 = chunk * G;
  const int Gc = min(G, L.nrhs - r0);
  const int V = g.V;
  const TileGeo tg = tile_geo(g);
  const int nslots = tg.fbase[7] + (tg.vt >> g.lT[3]);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // LDS-direct copies: wave wv fills the 64-slot chunks wv, wv + 4, wv + 8 of every component
  const int nck = (nslots + 63) >> 6;
  int seo[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) seo[i] = slot_site(g, tg, tc, tile, (wv + 4 * i) * 64 + lane, nslots);

  const bool own = tid < tg.vt;
  int ic[4] = {0, 0, 0, 0}, s = 0;
  int ns[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  float4 lf[4][3], lbk[4][3];
  if (own) {
    tile_coords(g, tg, tid, ic);
    const int p = tid >= tg.vh ? 1 : 0;
    s = p * g.Vh + (tile << g.lTh) + (tid - p * tg.vh);
    int c[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) c[mu] = (tc[mu] << g.lT[mu]) + ic[mu];
    ns[0] = nbr_slot<0, +1>(g, tg, ic);
    ns[1] = nbr_slot<0, -1>(g, tg, ic);
    ns[2] = nbr_slot<1, +1>(g, tg, ic);
    ns[3] = nbr_slot<1, -1>(g, tg, ic);
    ns[4] = nbr_slot<2, +1>(g, tg, ic);
    ns[5] = nbr_slot<2, -1>(g, tg, ic);
    ns[6] = nbr_slot<3, +1>(g, tg, ic);
    ns[7] = nbr_slot<3, -1>(g, tg, ic);
    int yb[4];
    yb[0] = eo_neighbour<0, -1>(g, c);
    yb[1] = eo_neighbour<1, -1>(g, c);
    yb[2] = eo_neighbour<2, -1>(g, c);
    yb[3] = eo_neighbour<3, -1>(g, c);
    const float4* U = (const float4*)L.links;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lf[mu][k] = ldo(U + (long long)(mu * 3 + k) * V, unsigned(s) * 16u);
        lbk[mu][k] = ldo(U + (long long)(mu * 3 + k) * V, unsigned(yb[mu]) * 16u);
      }
  }
  constexpr int SF = DAG ? +1 : -1;  // forward hop (1 - gamma), dagger (1 + gamma)
  constexpr int SB = -SF;
  const float kap = float(L.kappa);
  const float tm = float(DAG ? -L.mu : L.mu);
  auto active = [&](int j) {
    if (gate == 1) return sc[L.rhs_base + r0 + j].active != 0;
    if (gate == 2) return sc[L.rhs_base + r0 + j].sel != 0;
    return true;
  };
  auto next = [&](int j) {
    while (j < Gc && !active(j)) ++j;  // uniform over the block
    return j;
  };
  auto stage = [&](int j, float4* buf) {
    const float4* in = (const float4*)L.in + (long long)(r0 + j) * 6 * V;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int ck = wv + 4 * i;
      if (ck < nck) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
          __builtin_amdgcn_global_load_lds(
              (const void*)(in + (long long)k * V + seo[i]),
              (__attribute__((address_space(3))) void*)(buf + k * TL_SLOTS + ck * 64), 16, 0, 0);
      }
    }
  };
  // (A second LDS buffer to overlap the next copy with this rhs's arithmetic leaves room for
  // one block per CU instead of two; measured slower.)
  int j = next(0);
  if (j < Gc) stage(j, lds);
  while (j < Gc) {
    const int r = r0 + j;
    const float4* buf = lds;
    if (B.acct.bytes && tile == 0 && tid == 0) account(B, l);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's LDS-direct copies have landed
    __syncthreads();                // and everyone else's
    const int jn = next(j + 1);
    zf ax[12];
    if (own && EPI != EPI_NONE)
      IO<float>::load_nt((const float4*)L.aux + (long long)r * 6 * V, V, s, ax);
    double red[DS_NSUM];
#pragma unroll
    for (int i = 0; i < DS_NSUM; ++i) red[i] = 0.0;
    if (own) {
      zf acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = zf{0.f, 0.f};
      hop_lds<0, SF, false>(buf, ns[0], lf[0], acc);
      hop_lds<0, SB, true>(buf, ns[1], lbk[0], acc);
      hop_lds<1, SF, false>(buf, ns[2], lf[1], acc);
      hop_lds<1, SB, true>(buf, ns[3], lbk[1], acc);
      hop_lds<2, SF, false>(buf, ns[4], lf[2], acc);
      hop_lds<2, SB, true>(buf, ns[5], lbk[2], acc);
      hop_lds<3, SF, false>(buf, ns[6], lf[3], acc);
      hop_lds<3, SB, true>(buf, ns[7], lbk[3], acc);
      zf psi[12];
      lds_spinor<TL_SLOTS>(buf, tid, psi);
      zf o[12];
      finish_site<float, EPI>(psi, acc, kap, tm, ax, red, o);
      IO<float>::store((float4*)L.out + (long long)r * 6 * V, V, s, o);
    }
    if (EPI != EPI_NONE) {
      __shared__ double sh[DS_NSUM * (DS_BS / 64)];
      block_sum_epi<EPI, 1, DS_BS>(red, sh);
      if (tid == 0) {
        store_sums<EPI>(B, partials, L.rhs_base + r, tile, red);
      }
    }
    if (jn < Gc) {
      __syncthreads();  // every thread is done with the copy that is overwritten next
      stage(jn, lds);
    }
    j = jn;
  }
}

// ---------------------------------------------------------------------------- half-lattice tiles
// The two steps of the even-odd reduced operator (see k_dslash_half) with the LDS staging of
// k_dslash_tile: one block of TH_BS threads per (tile, rhs chunk) computes the tile's sites of the
// output parity P; it stages, per rhs, the tile's sites of the other parity Q and the parity-Q
// halves of the 8 neighbouring faces (the only neighbours those sites have), so every staged
// spinor passes through the vector memory unit once per rhs as a centre-tile site and at most
// once more per face it lies on.
//   LDS slots per component: [0, Vt/2) the tile's parity-Q sites in memory order; then per face f
//   = (mu, +-) the Vt/(2 T_mu) parity-Q sites of that face, indexed by the face's lexicographic
//   position (three other in-tile coordinates) shifted right by one (the lowest of those
//   coordinates has even extent, so each pair holds one site of each parity).
constexpr int TH_BS = 128;     // threads per block: the parity-P sites of a 4^4 tile
constexpr int TH_SLOTS = 384;  // 128 + 8 x 32

__device__ __forceinline__ TileGeo tile_geo_half(const Geom& g) {
  TileGeo t;
  t.vh = 1 << g.lTh;
  t.vt = 2 * t.vh;
  int b = t.vh;
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    t.fbase[f] = b;
    b += (t.vt >> g.lT[f >> 1]) >> 1;
  }
  return t;
}

// LDS slot of the (parity-Q) neighbour x + DIR*MU of the tile site with in-tile coordinates ic
template <int MU, int DIR>
__device__ __forceinline__ int nbr_slot_half(const Geom& g, const TileGeo& t, const int (&ic)[4]) {
  const int v = ic[MU] + DIR;
  if (v >= 0 && v < g.T[MU]) {
    int d[4] = {ic[0], ic[1], ic[2], ic[3]};
    d[MU] = v;
    return in_tile_half(g, d);
  }
  return t.fbase[2 * MU + (DIR > 0 ? 0 : 1)] + (face_index<MU>(g, ic) >> 1);
}

// index in the parity-Q half vector of the site held in LDS slot j of tile tc; slots past the
// last face repeat the tile's first site (their copies are never read)
__device__ __forceinline__ int slot_site_half(const Geom& g, const TileGeo& t, const int (&tc)[4],
                                              int tile, int j, int nslots, int Q) {
  if (j < t.vh) return (tile << g.lTh) + j;
  if (j >= nslots) return tile << g.lTh;
  int f = 0, fb = t.fbase[0];
#pragma unroll
  for (int i = 1; i < 8; ++i)
    if (j >= t.fbase[i]) {
      f = i;
      fb = t.fbase[i];
    }
  const int mu = f >> 1;
  const int dir = (f & 1) ? -1 : +1;
  uint32_t q = uint32_t(j - fb) << 1;
  int ic[4], tn[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) {
      ic[nu] = dir > 0 ? 0 : g.T[nu] - 1;
      int v = tc[nu] + dir;
      tn[nu] = v < 0 ? g.NT[nu] - 1 : (v == g.NT[nu] ? 0 : v);
    } else {
      ic[nu] = int(q & uint32_t(g.T[nu] - 1));
      q >>= g.lT[nu];
      tn[nu] = tc[nu];
    }
  }
  // the pair's parity-Q member: step the lowest other coordinate (even extent) by one
  if (((ic[0] + ic[1] + ic[2] + ic[3]) & 1) != Q) {
    if (mu == 0) ic[1] += 1;
    else ic[0] += 1;
  }
  const int tile_n = tn[0] + g.NT[0] * (tn[1] + g.NT[1] * (tn[2] + g.NT[2] * tn[3]));
  return (tile_n << g.lTh) + in_tile_half(g, ic);
}

template <bool DAG, int EPI, int STEP>
__global__ __launch_bounds__(TH_BS) void k_dslash_tile_half(DsBatch B, RhsScal* __restrict__ sc,
                                                            double* __restrict__ partials,
                                                            int gate) {
  constexpr int P = STEP == 1 ? 1 : 0;  // output parity
  constexpr int Q = 1 - P;              // parity of the hop input
  __shared__ float4 lds[6 * TH_SLOTS];
  const int lb = xcd_block(blockIdx.x, B.nblocks);
  int l = 0;
#pragma unroll
  for (int i = 1; i < MAXLAT; ++i)
    if (i < B.nlat && lb >= B.lat[i].blk_begin) l = i;
  const DsLat& L = B.lat[l];
  const Geom& g = L.g;
  const int G = tile_chunk(B.rgroup, L.nrhs);
  const int nch = (L.nrhs + G - 1) / G;
  int tc[4], tile, chunk;
  tile_of_block(g, lb - L.blk_begin, nch, B.torder, tc, tile, chunk);
  const int r0 = chunk * G;
  const int Gc = min(G, L.nrhs - r0);
  const int Vh = g.V >> 1;
  const TileGeo tg = tile_geo_half(g);
  const int nslots = tg.fbase[7] + ((tg.vt >> g.lT[3]) >> 1);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // LDS-direct copies: wave wv fills the 64-slot chunks wv, wv + 2, wv + 4 of every component
  const int nck = (nslots + 63) >> 6;
  int seo[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    seo[i] = slot_site_half(g, tg, tc, tile, (wv + 2 * i) * 64 + lane, nslots, Q);

  const bool own = tid < tg.vh;
  const int h = (tile << g.lTh) + tid;  // output index in the parity-P half vector
  int ns[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  float4 lf[4][3], lbk[4][3];
  if (own) {
    int ic[4];
    tile_coords(g, tg, P * tg.vh + tid, ic);
    const int s = P * Vh + h;
    int c[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) c[mu] = (tc[mu] << g.lT[mu]) + ic[mu];
    ns[0] = nbr_slot_half<0, +1>(g, tg, ic);
    ns[1] = nbr_slot_half<0, -1>(g, tg, ic);
    ns[2] = nbr_slot_half<1, +1>(g, tg, ic);
    ns[3] = nbr_slot_half<1, -1>(g, tg, ic);
    ns[4] = nbr_slot_half<2, +1>(g, tg, ic);
    ns[5] = nbr_slot_half<2, -1>(g, tg, ic);
    ns[6] = nbr_slot_half<3, +1>(g, tg, ic);
    ns[7] = nbr_slot_half<3, -1>(g, tg, ic);
    int yb[4];
    yb[0] = eo_neighbour<0, -1>(g, c);
    yb[1] = eo_neighbour<1, -1>(g, c);
    yb[2] = eo_neighbour<2, -1>(g, c);
    yb[3] = eo_neighbour<3, -1>(g, c);
    const float4* U = (const float4*)L.links;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lf[mu][k] = ldo(U + (long long)(mu * 3 + k) * g.V, unsigned(s) * 16u);
        lbk[mu][k] = ldo(U + (long long)(mu * 3 + k) * g.V, unsigned(yb[mu]) * 16u);
      }
  }
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  const float coef = float(L.kappa);
  const float tm = float(DAG ? -L.mu : L.mu);
  auto active = [&](int j) {
    if (gate == 1) return sc[L.rhs_base + r0 + j].active != 0;
    if (gate == 2) return sc[L.rhs_base + r0 + j].sel != 0;
    return true;
  };
  auto next = [&](int j) {
    while (j < Gc && !active(j)) ++j;  // uniform over the block
    return j;
  };
  auto stage = [&](int j) {
    const float4* in = (const float4*)L.in + (long long)(r0 + j) * 6 * Vh;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int ck = wv + 2 * i;
      if (ck < nck) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
          __builtin_amdgcn_global_load_lds(
              (const void*)(in + (long long)k * Vh + seo[i]),
              (__attribute__((address_space(3))) void*)(lds + k * TH_SLOTS + ck * 64), 16, 0, 0);
      }
    }
  };
  int j = next(0);
  if (j < Gc) stage(j);
  while (j < Gc) {
    const int r = r0 + j;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's LDS-direct copies have landed
    __syncthreads();                // and everyone else's
    const int jn = next(j + 1);
    double red[DS_NSUM];
#pragma unroll
    for (int i = 0; i < DS_NSUM; ++i) red[i] = 0.0;
    if (own) {
      zf ce[12], ax[12];
      if (L.cen) {
        IO<float>::load((const float4*)L.cen + (long long)r * 6 * Vh, Vh, h, ce);
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) ce[k] = zf{0.f, 0.f};
      }
      zf acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = zf{0.f, 0.f};
      hop_lds<0, SF, false, TH_SLOTS>(lds, ns[0], lf[0], acc);
      hop_lds<0, SB, true, TH_SLOTS>(lds, ns[1], lbk[0], acc);
      hop_lds<1, SF, false, TH_SLOTS>(lds, ns[2], lf[1], acc);
      hop_lds<1, SB, true, TH_SLOTS>(lds, ns[3], lbk[1], acc);
      hop_lds<2, SF, false, TH_SLOTS>(lds, ns[4], lf[2], acc);
      hop_lds<2, SB, true, TH_SLOTS>(lds, ns[5], lbk[2], acc);
      hop_lds<3, SF, false, TH_SLOTS>(lds, ns[6], lf[3], acc);
      hop_lds<3, SB, true, TH_SLOTS>(lds, ns[7], lbk[3], acc);
      // the epilogue operand is read after the hops (the empty asm keeps the compiler from
      // hoisting its load): loaded with the centre it holds registers through the hops and
      // halves the resident waves
      asm volatile("" ::: "memory");
      if (STEP == 2 && EPI != EPI_NONE)
        IO<float>::load_nt((const float4*)L.aux + (long long)r * 6 * Vh, Vh, h, ax);
      zf o[12];
      if (STEP == 1) finish_odd<float>(ce, acc, coef, tm, o);
      else
        finish_site<float, EPI>(ce, acc, coef, tm, ax, red, o);
      IO<float>::store((float4*)L.out + (long long)r * 6 * Vh, Vh, h, o);
    }
    if (EPI != EPI_NONE) {
      __shared__ double sh[DS_NSUM * (TH_BS / 64)];
      block_sum_epi<EPI, 1, TH_BS>(red, sh);
      if (tid == 0) {
        store_sums<EPI>(B, partials, L.rhs_base + r, tile, red);
      }
    }
    if (jn < Gc) {
      __syncthreads();  // every thread is done with the copy that is overwritten next
      stage(jn);
    }
    j = jn;
  }
}

template <int EPI>
__global__ __launch_bounds__(DS_BS) void k_ds_finalize(DsBatch B, RhsScal* __restrict__ sc,
                                                       const double* __restrict__ partials) {
  finalize<EPI>(B, sc, partials);
}

template <typename T, bool DAG, int EPI>
void launch_nb(hipStream_t s, const DsBatch& b, RhsScal* sc, double* partials, int gate) {
  dim3 grid(b.nblocks), block(DS_BS);
  switch (b.nb) {
    case 2: hipLaunchKernelGGL((k_dslash<T, DAG, EPI, 2>), grid, block, 0, s, b, sc, partials, gate); break;
    case 4: hipLaunchKernelGGL((k_dslash<T, DAG, EPI, 4>), grid, block, 0, s, b, sc, partials, gate); break;
    default: hipLaunchKernelGGL((k_dslash<T, DAG, EPI, 1>), grid, block, 0, s, b, sc, partials, gate); break;
  }
}

template <typename T, bool DAG>
void launch_epi(hipStream_t s, const DsBatch& b, int epi, RhsScal* sc, double* partials, int gate) {
  switch (epi) {
    case EPI_NONE: launch_nb<T, DAG, EPI_NONE>(s, b, sc, partials, gate); break;
    case EPI_RHAT: launch_nb<T, DAG, EPI_RHAT>(s, b, sc, partials, gate); break;
    case EPI_TS: launch_nb<T, DAG, EPI_TS>(s, b, sc, partials, gate); break;
    default: launch_nb<T, DAG, EPI_RESID>(s, b, sc, partials, gate); break;
  }
}

template <bool DAG>
void launch_tile_epi(hipStream_t s, const DsBatch& b, int epi, RhsScal* sc, double* partials,
                     int gate) {
  dim3 grid(b.nblocks), block(DS_BS);
  switch (epi) {
    case EPI_NONE: hipLaunchKernelGGL((k_dslash_tile<DAG, EPI_NONE>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_RHAT: hipLaunchKernelGGL((k_dslash_tile<DAG, EPI_RHAT>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_TS: hipLaunchKernelGGL((k_dslash_tile<DAG, EPI_TS>), grid, block, 0, s, b, sc, partials, gate); break;
    default: hipLaunchKernelGGL((k_dslash_tile<DAG, EPI_RESID>), grid, block, 0, s, b, sc, partials, gate); break;
  }
}

template <typename T>
double launch(hipStream_t s, DsBatch& b, int dagger, int epi, RhsScal* sc, double* partials,
              int nb, int rgroup) {
  DBQ_CHECK(b.nlat >= 1 && b.nlat <= MAXLAT, "dslash: bad lattice count");
  DBQ_CHECK(epi == EPI_NONE || (sc && partials), "dslash: epilogue needs scalars");
  const bool tiled = nb == 0;
  DBQ_CHECK(nb == 1 || nb == 2 || nb == 4 || (tiled && sizeof(T) == 4),
            "dslash: rhs per thread must be 1, 2 or 4 (0: LDS-staged tiles, FP32)");
  // block layout: per lattice nsb site blocks (tiles for the LDS-staged kernel) x rhs groups
  b.nb = tiled ? 1 : nb;
  b.rgroup = rgroup;
  long long blk = 0;
  for (int i = 0; i < b.nlat; ++i) {
    DsLat& L = b.lat[i];
    L.blk_begin = int(blk);
    if (tiled) {
      DBQ_CHECK(L.g.T[0] <= 4 && L.g.T[1] <= 4 && L.g.T[2] <= 4 && L.g.T[3] <= 4,
                "dslash: tile larger than 4^4");
      L.nsb = L.g.V >> (L.g.lTh + 1);
      const int G = tile_chunk(rgroup, L.nrhs);
      blk += (long long)L.nsb * ((L.nrhs + G - 1) / G);
    } else {
      L.nsb = 2 * ((L.g.Vh + DS_BS - 1) / DS_BS);
      blk += (long long)L.nsb * ((L.nrhs + nb - 1) / nb);
    }
    DBQ_CHECK(epi == EPI_NONE || L.nsb <= b.pstride, "dslash: partial-sum slots too few");
  }
  DBQ_CHECK(blk > 0 && blk < (1ll << 31), "dslash: grid size out of range");
  b.nblocks = int(blk);
  int gate = 0;
  if (sc) gate = (epi == EPI_RESID) ? 2 : 1;
  if (tiled) {
    if (dagger) launch_tile_epi<true>(s, b, epi, sc, partials, gate);
    else launch_tile_epi<false>(s, b, epi, sc, partials, gate);
  } else if (dagger) {
    launch_epi<T, true>(s, b, epi, sc, partials, gate);
  } else {
    launch_epi<T, false>(s, b, epi, sc, partials, gate);
  }
  DBQ_HIP(hipGetLastError());
  // algorithmic bytes: links once per lattice, each spinor read once and written once, plus
  // one epilogue operand per site (rhat or b)
  double bytes = 0;
  for (int i = 0; i < b.nlat; ++i) {
    const double V = b.lat[i].g.V;
    bytes += V * IO<T>::link_bytes();
    bytes += V * b.lat[i].nrhs * 2.0 * IO<T>::spinor_bytes();
    if (epi != EPI_NONE) bytes += V * b.lat[i].nrhs * IO<T>::spinor_bytes();
  }
  return bytes;
}

template <typename T, bool DAG, int NB, int STEP>
void launch_half_epi(hipStream_t s, const DsBatch& b, int epi, RhsScal* sc, double* partials,
                     int gate) {
  dim3 grid(b.nblocks), block(DS_BS);
  switch (epi) {
    case EPI_NONE: hipLaunchKernelGGL((k_dslash_half<T, DAG, EPI_NONE, NB, STEP>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_RHAT: hipLaunchKernelGGL((k_dslash_half<T, DAG, EPI_RHAT, NB, STEP>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_TS: hipLaunchKernelGGL((k_dslash_half<T, DAG, EPI_TS, NB, STEP>), grid, block, 0, s, b, sc, partials, gate); break;
    default: hipLaunchKernelGGL((k_dslash_half<T, DAG, EPI_RESID, NB, STEP>), grid, block, 0, s, b, sc, partials, gate); break;
  }
}

template <typename T, bool DAG, int NB>
void launch_half_step(hipStream_t s, const DsBatch& b, int step, int epi, RhsScal* sc,
                      double* partials, int gate) {
  if (step == 1) {
    dim3 grid(b.nblocks), block(DS_BS);
    hipLaunchKernelGGL((k_dslash_half<T, DAG, EPI_NONE, NB, 1>), grid, block, 0, s, b, sc, partials, gate);
  } else {
    launch_half_epi<T, DAG, NB, 2>(s, b, epi, sc, partials, gate);
  }
}

template <bool DAG>
void launch_tile_half(hipStream_t s, const DsBatch& b, int step, int epi, RhsScal* sc,
                      double* partials, int gate) {
  dim3 grid(b.nblocks), block(TH_BS);
  if (step == 1) {
    hipLaunchKernelGGL((k_dslash_tile_half<DAG, EPI_NONE, 1>), grid, block, 0, s, b, sc, partials, gate);
    return;
  }
  switch (epi) {
    case EPI_NONE: hipLaunchKernelGGL((k_dslash_tile_half<DAG, EPI_NONE, 2>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_RHAT: hipLaunchKernelGGL((k_dslash_tile_half<DAG, EPI_RHAT, 2>), grid, block, 0, s, b, sc, partials, gate); break;
    case EPI_TS: hipLaunchKernelGGL((k_dslash_tile_half<DAG, EPI_TS, 2>), grid, block, 0, s, b, sc, partials, gate); break;
    default: hipLaunchKernelGGL((k_dslash_tile_half<DAG, EPI_RESID, 2>), grid, block, 0, s, b, sc, partials, gate); break;
  }
}

template <typename T>
void launch_half(hipStream_t s, DsBatch& b, int step, int dagger, int epi, RhsScal* sc,
                 double* partials, int nb, int rgroup, int gate) {
  DBQ_CHECK(b.nlat >= 1 && b.nlat <= MAXLAT, "dslash (half): bad lattice count");
  DBQ_CHECK(step == 1 || step == 2, "dslash (half): step must be 1 or 2");
  DBQ_CHECK(step == 2 || epi == EPI_NONE, "dslash (half): epilogues follow step 2");
  DBQ_CHECK(epi == EPI_NONE || (sc && partials), "dslash (half): epilogue needs scalars");
  DBQ_CHECK(gate == 0 || sc, "dslash (half): gating needs scalars");
  const bool tiled = nb == 0;
  DBQ_CHECK(nb == 1 || nb == 2 || (tiled && sizeof(T) == 4),
            "dslash (half): rhs per thread must be 1 or 2 (0: LDS-staged tiles, FP32)");
  b.nb = tiled ? 1 : nb;
  b.rgroup = rgroup;
  long long blk = 0;
  for (int i = 0; i < b.nlat; ++i) {
    DsLat& L = b.lat[i];
    DBQ_CHECK(L.g.V % 2 == 0, "dslash (half): odd volume");
    DBQ_CHECK(L.in && L.out, "dslash (half): null vector");
    DBQ_CHECK(!((epi == EPI_RHAT || epi == EPI_RESID) && !L.aux), "dslash (half): null aux");
    L.blk_begin = int(blk);
    if (tiled) {
      DBQ_CHECK(L.g.T[0] <= 4 && L.g.T[1] <= 4 && L.g.T[2] <= 4 && L.g.T[3] <= 4,
                "dslash (half): tile larger than 4^4");
      L.nsb = L.g.V >> (L.g.lTh + 1);
      const int G = tile_chunk(rgroup, L.nrhs);
      blk += (long long)L.nsb * ((L.nrhs + G - 1) / G);
    } else {
      L.nsb = (L.g.V / 2 + DS_BS - 1) / DS_BS;
      blk += (long long)L.nsb * ((L.nrhs + nb - 1) / nb);
    }
    DBQ_CHECK(epi == EPI_NONE || L.nsb <= b.pstride, "dslash (half): partial-sum slots too few");
  }
  DBQ_CHECK(blk > 0 && blk < (1ll << 31), "dslash (half): grid size out of range");
  b.nblocks = int(blk);
  if (tiled) {
    if (dagger) launch_tile_half<true>(s, b, step, epi, sc, partials, gate);
    else launch_tile_half<false>(s, b, step, epi, sc, partials, gate);
  } else if (dagger) {
    if (nb == 2) launch_half_step<T, true, 2>(s, b, step, epi, sc, partials, gate);
    else launch_half_step<T, true, 1>(s, b, step, epi, sc, partials, gate);
  } else {
    if (nb == 2) launch_half_step<T, false, 2>(s, b, step, epi, sc, partials, gate);
    else launch_half_step<T, false, 1>(s, b, step, epi, sc, partials, gate);
  }
  DBQ_HIP(hipGetLastError());
}

}  // namespace

void launch_ds_finalize(hipStream_t s, const DsBatch& b, int epi, RhsScal* sc,
                        const double* partials) {
  if (epi == EPI_NONE) return;
  DBQ_CHECK(sc && partials, "dslash finalize: null scalars");
  // one wavefront per right-hand side, four per block
  const unsigned nfb = unsigned((b.nrhs_total + DS_BS / 64 - 1) / (DS_BS / 64));
  const dim3 block(DS_BS);
  if (epi == EPI_RHAT)
    hipLaunchKernelGGL((k_ds_finalize<EPI_RHAT>), dim3(nfb), block, 0, s, b, sc, partials);
  else if (epi == EPI_TS)
    hipLaunchKernelGGL((k_ds_finalize<EPI_TS>), dim3(nfb), block, 0, s, b, sc, partials);
  else
    hipLaunchKernelGGL((k_ds_finalize<EPI_RESID>), dim3(nfb), block, 0, s, b, sc, partials);
  DBQ_HIP(hipGetLastError());
}

double launch_dslash_f64(hipStream_t s, DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup) {
  return launch<double>(s, b, dagger, epi, sc, partials, nb, rgroup);
}
double launch_dslash_f32(hipStream_t s, DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup) {
  return launch<float>(s, b, dagger, epi, sc, partials, nb, rgroup);
}

void launch_dslash_half_f64(hipStream_t s, DsBatch& b, int step, int dagger, int epi,
                            RhsScal* sc, double* partials, int nb, int rgroup, int gate) {
  launch_half<double>(s, b, step, dagger, epi, sc, partials, nb, rgroup, gate);
}
void launch_dslash_half_f32(hipStream_t s, DsBatch& b, int step, int dagger, int epi,
                            RhsScal* sc, double* partials, int nb, int rgroup, int gate) {
  launch_half<float>(s, b, step, dagger, epi, sc, partials, nb, rgroup, gate);
}

}  // namespace dbq
