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
#define DBQ_OCC_F64 2
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
// BACK = true -> (1 + S gamma) U_mu(y)^dag psi(y) with y = x - mu.
template <typename T, int MU, int S, bool BACK, int NB>
__device__ __forceinline__ void hop(const typename IO<T>::SE* __restrict__ in, long long rstride,
                                    int nval, const typename IO<T>::LE* __restrict__ U, int V,
                                    int site_link, int y, cx<T> (&acc)[NB][12]) {
  cx<T> u[9];
  IO<T>::link(U, V, MU, site_link, u);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (NB > 1 && j >= nval) break;
    cx<T> p[12];
    IO<T>::load(in + j * rstride, V, y, p);
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

template <typename T, bool DAG, int MU, int NB>
__device__ __forceinline__ void hops_mu(const typename IO<T>::SE* __restrict__ in,
                                        long long rstride, int nval,
                                        const typename IO<T>::LE* __restrict__ U, const Geom& g,
                                        int s, const int (&c)[4], cx<T> (&acc)[NB][12]) {
  // forward hop uses (1 - gamma) (dagger: 1 + gamma), backward the opposite
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  const int yf = eo_neighbour<MU, +1>(g, c);
  const int yb = eo_neighbour<MU, -1>(g, c);
  hop<T, MU, SF, false, NB>(in, rstride, nval, U, g.V, s, yf, acc);
  hop<T, MU, SB, true, NB>(in, rstride, nval, U, g.V, yb, yb, acc);
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// Combine the per-block partials of one epilogue: every right-hand side of the batch is reduced
// by one wavefront over its site blocks in a fixed order.
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
      if (B.acct.bytes) {
        // the flag the Dslash kernel was gated on, read before this launch changes it
        const bool processed = (EPI == EPI_RESID) ? q.sel != 0 : q.active != 0;
        if (processed) {
          unsigned long long by = (unsigned long long)B.lat[l].g.V *
                                  (unsigned long long)(B.acct.spinor_passes * B.acct.spinor_bytes);
          if (atomicMax(B.acct.tags + l, B.acct.id) < B.acct.id)
            by += (unsigned long long)B.lat[l].g.V * (unsigned long long)B.acct.link_bytes;
          atomicAdd(B.acct.bytes, by);
        }
      }
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

#if DBQ_OCC_F32 > 0
// Minimum waves per SIMD the register allocation must leave room for.
template <typename T, int NB>
struct Occ {
  static constexpr int value = sizeof(T) == 4 ? (NB <= 2 ? DBQ_OCC_F32 : 2) : DBQ_OCC_F64;
};
#define DBQ_DS_ATTR __attribute__((amdgpu_waves_per_eu(Occ<T, NB>::value)))
#else
#define DBQ_DS_ATTR
#endif

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
  double red[NB * 3];
#pragma unroll
  for (int i = 0; i < NB * 3; ++i) red[i] = 0.0;
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
    hops_mu<T, DAG, 0, NB>(in, rstride, nval, U, L.g, sl, c, acc);
    chain(c, sl, acc);
    hops_mu<T, DAG, 1, NB>(in, rstride, nval, U, L.g, sl, c, acc);
    chain(c, sl, acc);
    hops_mu<T, DAG, 2, NB>(in, rstride, nval, U, L.g, sl, c, acc);
    chain(c, sl, acc);
    hops_mu<T, DAG, 3, NB>(in, rstride, nval, U, L.g, sl, c, acc);
    const T kap = T(L.kappa);
    const T tm = T(DAG ? -L.mu : L.mu);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (!act[j]) continue;
      cx<T> psi[12];
      IO<T>::load(in + j * rstride, V, s, psi);
      cx<T> o[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        // psi - kappa acc + i mu gamma5 psi, gamma5 = diag(1,1,-1,-1) over spins
        const T t = k < 6 ? tm : -tm;
        o[k].re = fma(-kap, acc[j][k].re, fma(-t, psi[k].im, psi[k].re));
        o[k].im = fma(-kap, acc[j][k].im, fma(t, psi[k].re, psi[k].im));
      }
      if (EPI == EPI_RESID) {
        cx<T> b[12];
        IO<T>::load((const SE*)L.aux + (r0 + j) * rstride, V, s, b);
        T nn = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          o[k] = b[k] - o[k];
          nn = fma(o[k].re, o[k].re, fma(o[k].im, o[k].im, nn));
        }
        red[3 * j] += double(nn);
      } else if (EPI == EPI_RHAT) {
        cx<T> rh[12];
        IO<T>::load((const SE*)L.aux + (r0 + j) * rstride, V, s, rh);
        cx<T> d{T(0), T(0)};
#pragma unroll
        for (int k = 0; k < 12; ++k) cmacc(d, rh[k], o[k]);
        red[3 * j] += double(d.re);
        red[3 * j + 1] += double(d.im);
      } else if (EPI == EPI_TS) {
        cx<T> d{T(0), T(0)};
        T nn = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          cmacc(d, o[k], psi[k]);
          nn = fma(o[k].re, o[k].re, fma(o[k].im, o[k].im, nn));
        }
        red[3 * j] += double(d.re);
        red[3 * j + 1] += double(d.im);
        red[3 * j + 2] += double(nn);
      }
      IO<T>::store(out + j * rstride, V, s, o);
    }
  }
  if (EPI != EPI_NONE) {
    __shared__ double sh[NB * 3 * (DS_BS / 64)];
    block_sum<NB * 3, DS_BS>(red, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j >= nval) break;
        double* pp = partials + ((long long)(L.rhs_base + r0 + j) * B.pstride + sb) * 3;
        pp[0] = red[3 * j];
        pp[1] = red[3 * j + 1];
        pp[2] = red[3 * j + 2];
      }
    }
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

template <typename T>
double launch(hipStream_t s, const DsBatch& in, int dagger, int epi, RhsScal* sc, double* partials,
              int nb, int rgroup) {
  DBQ_CHECK(in.nlat >= 1 && in.nlat <= MAXLAT, "dslash: bad lattice count");
  DBQ_CHECK(epi == EPI_NONE || (sc && partials), "dslash: epilogue needs scalars");
  DBQ_CHECK(nb == 1 || nb == 2 || nb == 4, "dslash: rhs per thread must be 1, 2 or 4");
  // block layout for nb right-hand sides per thread: per lattice nsb site blocks x rhs groups
  DsBatch b = in;
  b.nb = nb;
  b.rgroup = rgroup;
  long long blk = 0;
  for (int i = 0; i < b.nlat; ++i) {
    b.lat[i].blk_begin = int(blk);
    blk += (long long)b.lat[i].nsb * ((b.lat[i].nrhs + nb - 1) / nb);
  }
  DBQ_CHECK(blk > 0 && blk < (1ll << 31), "dslash: grid size out of range");
  b.nblocks = int(blk);
  int gate = 0;
  if (sc) gate = (epi == EPI_RESID) ? 2 : 1;
  if (dagger) launch_epi<T, true>(s, b, epi, sc, partials, gate);
  else launch_epi<T, false>(s, b, epi, sc, partials, gate);
  DBQ_HIP(hipGetLastError());
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

double launch_dslash_f64(hipStream_t s, const DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup) {
  return launch<double>(s, b, dagger, epi, sc, partials, nb, rgroup);
}
double launch_dslash_f32(hipStream_t s, const DsBatch& b, int dagger, int epi, RhsScal* sc,
                         double* partials, int nb, int rgroup) {
  return launch<float>(s, b, dagger, epi, sc, partials, nb, rgroup);
}

}  // namespace dbq
