// Fused BiCGStab vector updates and inner products for a batch of right-hand sides (Sec. 2 runs
// BiCGStab after the deflation step; Sec. 1 motivates it as a non-restarted method).
//
// One iteration:  Dslash v = A p with <rhat, v> -> alpha,  BI_S (r <- s = r - alpha v),
// Dslash t = A s with <t, s>, <t, t>, <rhat, t>, <rhat, s> -> omega, the next rho = <rhat, s> -
// omega <rhat, t> and beta,  BI_XR (x += alpha p + omega s; r = s - omega t;
// p = r + beta (p - omega v); ||r||^2 -> tests).  Folding the search-direction update into the
// XR pass saves a launch and three vector passes per iteration (the epilogue reads rhat, the XR
// pass v, instead of rhat in XR and r, p, v, p in a separate pass).  A reliable update restarts
// the recursion from the FP64 residual: r = rhat = p = b - A x, rho = ||r||^2.
// The scalars live in RhsScal on the device.  Each streaming kernel stores one partial sum per
// block; a small follow-up launch combines them per right-hand side in a fixed order, so the
// results do not depend on block scheduling and no device-scope fence stalls the stream.
#include "kernels.h"

namespace dbq {

namespace {

template <typename E>
struct ET;
typedef float f4v __attribute__((ext_vector_type(4)));
template <>
struct ET<double2> {
  typedef double R;
  static constexpr int NC = 1;
  __device__ __forceinline__ static void ld(const double2* p, long long i, zd (&z)[1]) {
    double2 v = p[i];
    z[0] = zd{v.x, v.y};
  }
  __device__ __forceinline__ static void st(double2* p, long long i, const zd (&z)[1]) {
    p[i] = make_double2(z[0].re, z[0].im);
  }
  // FP64 single-rhs working sets stay in the last-level cache: no hint
  __device__ __forceinline__ static void ld_last(const double2* p, long long i, zd (&z)[1]) {
    ld(p, i, z);
  }
  __device__ __forceinline__ static void st_far(double2* p, long long i, const zd (&z)[1]) {
    st(p, i, z);
  }
};
template <>
struct ET<float4> {
  typedef float R;
  static constexpr int NC = 2;
  __device__ __forceinline__ static void ld(const float4* p, long long i, zf (&z)[2]) {
    float4 v = p[i];
    z[0] = zf{v.x, v.y};
    z[1] = zf{v.z, v.w};
  }
  __device__ __forceinline__ static void st(float4* p, long long i, const zf (&z)[2]) {
    p[i] = make_float4(z[0].re, z[0].im, z[1].re, z[1].im);
  }
  // Non-temporal variants for operands this iteration does not read again (ld_last) or reads
  // only in the next XR pass (x, st_far): with 12 rhs the seven vectors of the FP32 recursion
  // exceed the last-level cache, and these hints leave it to the vectors read soon after.
  __device__ __forceinline__ static void ld_last(const float4* p, long long i, zf (&z)[2]) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p + i));
    z[0] = zf{v.x, v.y};
    z[1] = zf{v.z, v.w};
  }
  __device__ __forceinline__ static void st_far(float4* p, long long i, const zf (&z)[2]) {
    __builtin_nontemporal_store(f4v{z[0].re, z[0].im, z[1].re, z[1].im},
                                reinterpret_cast<f4v*>(p + i));
  }
};

template <typename R>
__device__ __forceinline__ cx<R> narrow(zd a) {
  return cx<R>{R(a.re), R(a.im)};
}

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

// reduce the partials of every rhs (one wavefront per rhs) and apply `fn(rhs, a0, a1, a2)`
template <typename Fn>
__device__ void reduce_rhs(const VecSet& vs, const double* partials, Fn fn) {
  const int lane = threadIdx.x & 63;
  constexpr int NW = BL_BS / 64;
  const int w = blockIdx.x * NW + (threadIdx.x >> 6);
  const int stride = gridDim.x * NW;
  for (int rhs = w; rhs < vs.nrhs; rhs += stride) {
    const int nch = (vs.nelem[rhs] + BL_CHUNK - 1) / BL_CHUNK;
    const double* pp = partials + (long long)rhs * vs.pstride * 3;
    double a0 = 0, a1 = 0, a2 = 0;
    // FIN_U partials per lane in flight together; additions in the order j = lane, lane + 64, ...
    for (int j0 = lane; j0 < nch; j0 += 64 * FIN_U) {
      double v[FIN_U][3];
#pragma unroll
      for (int u = 0; u < FIN_U; ++u) {
        const int j = j0 + 64 * u;
        if (j < nch) {
          v[u][0] = pp[3 * j];
          v[u][1] = pp[3 * j + 1];
          v[u][2] = pp[3 * j + 2];
        }
      }
#pragma unroll
      for (int u = 0; u < FIN_U; ++u) {
        if (j0 + 64 * u < nch) {
          a0 += v[u][0];
          a1 += v[u][1];
          a2 += v[u][2];
        }
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) fn(rhs, a0, a1, a2);
  }
}

__device__ __forceinline__ void store_partial(const VecSet& vs, double* partials, int rhs, int ch,
                                              double (&red)[3]) {
  __shared__ double sh[3 * (BL_BS / 64)];
  block_sum<3, BL_BS>(red, sh);
  if (threadIdx.x == 0) {
    double* pp = partials + ((long long)rhs * vs.pstride + ch) * 3;
    pp[0] = red[0];
    pp[1] = red[1];
    pp[2] = red[2];
  }
}

template <typename E, int OP>
__global__ __launch_bounds__(BL_BS) void k_bicg_step(VecSet vs, E* __restrict__ x,
                                                     E* __restrict__ r,
                                                     const E* __restrict__ rhat,
                                                     E* __restrict__ p, const E* __restrict__ v,
                                                     const E* __restrict__ t,
                                                     RhsScal* __restrict__ sc,
                                                     double* __restrict__ partials,
                                                     unsigned long long* __restrict__ acct) {
  typedef typename ET<E>::R R;
  constexpr int NC = ET<E>::NC;
  const int lb = xcd_block(blockIdx.x, vs.nblocks);
  const int2 bm = vs.blk[lb];
  const int rhs = bm.x, ch = bm.y;
  const bool act = sc[rhs].active != 0;
  double red[3] = {0.0, 0.0, 0.0};
  // byte accounting (timing only): reads x, p, s, t, v and writes x, r, p of an active rhs
  if (OP == BI_XR && acct && act && ch == 0 && threadIdx.x == 0)
    atomicAdd(acct, 8ull * (unsigned long long)vs.nelem[rhs] * sizeof(E));
  if (act) {
    const long long base = vs.off[rhs];
    const int ne = vs.nelem[rhs];
    const cx<R> al = narrow<R>(sc[rhs].alpha), om = narrow<R>(sc[rhs].omega),
                be = narrow<R>(sc[rhs].beta);
#pragma unroll
    for (int e = 0; e < BL_EPT; ++e) {
      const int idx = ch * BL_CHUNK + e * BL_BS + threadIdx.x;
      if (idx < ne) {
        const long long i = base + idx;
        if (OP == BI_S) {
          cx<R> rr[NC], vv[NC];
          ET<E>::ld(r, i, rr);
          ET<E>::ld(v, i, vv);
#pragma unroll
          for (int c = 0; c < NC; ++c) rr[c] = rr[c] - al * vv[c];
          ET<E>::st(r, i, rr);
        } else {
          cx<R> xx[NC], pp[NC], ss[NC], tt[NC], vv[NC];
          ET<E>::ld_last(x, i, xx);
          ET<E>::ld(p, i, pp);
          ET<E>::ld(r, i, ss);
          ET<E>::ld_last(t, i, tt);
          ET<E>::ld_last(v, i, vv);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            xx[c] = xx[c] + al * pp[c] + om * ss[c];
            ss[c] = ss[c] - om * tt[c];
            pp[c] = ss[c] + be * (pp[c] - om * vv[c]);
            const double br = double(ss[c].re), bi = double(ss[c].im);
            red[2] += br * br + bi * bi;
          }
          ET<E>::st_far(x, i, xx);
          ET<E>::st(r, i, ss);
          ET<E>::st(p, i, pp);
        }
      }
    }
  }
  if (OP == BI_XR) store_partial(vs, partials, rhs, ch, red);
}

// Partial sums are combined in a separate launch (see the Dslash epilogue for why).
__global__ __launch_bounds__(BL_BS) void k_fin_xr(VecSet vs, RhsScal* __restrict__ sc,
                                                  const double* __restrict__ partials) {
  reduce_rhs(vs, partials, [&](int j, double, double, double a2) { fin_xr(sc[j], a2); });
}

__device__ void fin_aux(int op, RhsScal& q, double a0, double a1, double a2);

template <int OP>
__global__ __launch_bounds__(BL_BS) void k_fin_aux(VecSet vs, RhsScal* __restrict__ sc,
                                                   const double* __restrict__ partials) {
  reduce_rhs(vs, partials, [&](int j, double a0, double a1, double a2) {
    fin_aux(OP, sc[j], a0, a1, a2);
  });
}

inline unsigned fin_blocks(const VecSet& vs) { return unsigned((vs.nrhs + BL_BS / 64 - 1) / (BL_BS / 64)); }

template <int OP>
void launch_fin_aux(hipStream_t s, const VecSet& vs, RhsScal* sc, const double* partials) {
  hipLaunchKernelGGL((k_fin_aux<OP>), dim3(fin_blocks(vs)), dim3(BL_BS), 0, s, vs, sc, partials);
  DBQ_HIP(hipGetLastError());
}

__device__ void fin_aux(int op, RhsScal& q, double a0, double a1, double a2) {
  if (op == AX_INIT) {
    if (!q.active) return;
    q.rho = zd{a2, 0.0};
    q.rhat2 = a2;
    q.rr = a2;
    q.rr_max = a2;
    q.rho_prev = q.alpha = q.omega = zd{1.0, 0.0};
    q.beta = zd{0.0, 0.0};
    q.iters = 0;
    q.flags = 0;
    q.since = 0;
    q.stalls = 0;
    q.rr_prev = a2;
    if (!fin(a2)) {
      q.flags = F_NAN;
      q.active = 0;
    } else if (a2 <= q.stop2) {
      q.flags = F_CONV;
      q.active = 0;
      q.sel = 1;
    }
  } else if (op == AX_RESTART) {
    if (!q.sel) return;
    q.rho = zd{a2, 0.0};
    q.rhat2 = a2;
    q.rr = a2;
    q.rho_prev = q.alpha = q.omega = zd{1.0, 0.0};
    q.beta = zd{0.0, 0.0};
    q.flags = 0;
    q.active = 1;
    q.sel = 0;
    q.since = 0;
  } else {  // AX_REPLACE: the recursion restarts from the FP64 residual (rhat = p = r)
    if (!q.sel) return;
    q.rho = zd{a2, 0.0};
    q.rhat2 = a2;
    q.rr = a2;
    q.rr_max = a2;
    q.flags = 0;
    q.active = 1;
    q.sel = 0;
    q.since = 0;
  }
}

// FP64 working vectors
template <int OP>
__global__ __launch_bounds__(BL_BS) void k_aux64(VecSet vs, const double2* __restrict__ r64,
                                                 double2* __restrict__ r,
                                                 double2* __restrict__ rhat,
                                                 double2* __restrict__ p, double2* __restrict__ v,
                                                 RhsScal* __restrict__ sc,
                                                 double* __restrict__ partials) {
  const int lb = xcd_block(blockIdx.x, vs.nblocks);
  const int2 bm = vs.blk[lb];
  const int rhs = bm.x, ch = bm.y;
  const bool act = OP == AX_INIT ? sc[rhs].active != 0 : sc[rhs].sel != 0;
  double red[3] = {0.0, 0.0, 0.0};
  if (act) {
    const long long base = vs.off[rhs];
    const int ne = vs.nelem[rhs];
    for (int e = 0; e < BL_EPT; ++e) {
      const int idx = ch * BL_CHUNK + e * BL_BS + threadIdx.x;
      if (idx >= ne) continue;
      const long long i = base + idx;
      if (OP == AX_REPLACE) {
        const double2 a = r64[i];
        r[i] = a;
        rhat[i] = a;
        p[i] = a;
        red[2] += a.x * a.x + a.y * a.y;
      } else {
        const double2 a = r[i];
        rhat[i] = a;
        p[i] = a;
        red[2] += a.x * a.x + a.y * a.y;
      }
    }
  }
  store_partial(vs, partials, rhs, ch, red);
}

// FP32 working vectors fed from / narrowed from FP64 ones (element e <-> FP64 elements 2e, 2e+1)
template <int OP>
__global__ __launch_bounds__(BL_BS) void k_aux32(VecSet vs, VecSet vs64,
                                                 const double2* __restrict__ r64,
                                                 float4* __restrict__ r, float4* __restrict__ rhat,
                                                 float4* __restrict__ p, float4* __restrict__ v,
                                                 float4* __restrict__ x32,
                                                 RhsScal* __restrict__ sc,
                                                 double* __restrict__ partials) {
  const int lb = xcd_block(blockIdx.x, vs.nblocks);
  const int2 bm = vs.blk[lb];
  const int rhs = bm.x, ch = bm.y;
  const bool act = OP == AX_INIT ? sc[rhs].active != 0 : sc[rhs].sel != 0;
  double red[3] = {0.0, 0.0, 0.0};
  if (act) {
    const long long base = vs.off[rhs];
    const long long base64 = vs64.off[rhs];
    const int ne = vs.nelem[rhs];
    for (int e = 0; e < BL_EPT; ++e) {
      const int idx = ch * BL_CHUNK + e * BL_BS + threadIdx.x;
      if (idx >= ne) continue;
      const long long i = base + idx;
      if (OP == AX_RESTART) {
        const float4 a = r[i];
        rhat[i] = a;
        p[i] = a;
        red[2] += double(a.x) * a.x + double(a.y) * a.y + double(a.z) * a.z + double(a.w) * a.w;
      } else {
        const double2 d0 = r64[base64 + 2 * (long long)idx];
        const double2 d1 = r64[base64 + 2 * (long long)idx + 1];
        const float4 a = make_float4(float(d0.x), float(d0.y), float(d1.x), float(d1.y));
        // init, or a replacement that restarts from the narrowed FP64 residual
        r[i] = a;
        rhat[i] = a;
        p[i] = a;
        if (OP == AX_INIT) x32[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        red[2] += double(a.x) * a.x + double(a.y) * a.y + double(a.z) * a.z + double(a.w) * a.w;
      }
    }
  }
  store_partial(vs, partials, rhs, ch, red);
}

__global__ __launch_bounds__(BL_BS) void k_xacc(VecSet vs, VecSet vs64, double2* __restrict__ x64,
                                                float4* __restrict__ x32,
                                                const RhsScal* __restrict__ sc) {
  const int lb = xcd_block(blockIdx.x, vs.nblocks);
  const int2 bm = vs.blk[lb];
  const int rhs = bm.x, ch = bm.y;
  if (!sc[rhs].sel) return;
  const long long base = vs.off[rhs];
  const long long base64 = vs64.off[rhs];
  const int ne = vs.nelem[rhs];
  for (int e = 0; e < BL_EPT; ++e) {
    const int idx = ch * BL_CHUNK + e * BL_BS + threadIdx.x;
    if (idx >= ne) continue;
    const long long i = base + idx;
    const float4 a = x32[i];
    double2* d = x64 + base64 + 2 * (long long)idx;
    double2 d0 = d[0], d1 = d[1];
    d0.x += a.x;
    d0.y += a.y;
    d1.x += a.z;
    d1.y += a.w;
    d[0] = d0;
    d[1] = d1;
    x32[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__global__ void k_mask_unselected(double2* __restrict__ Y, int k, int nrhs,
                                  const RhsScal* __restrict__ sc, int reproj_only) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * nrhs) return;
  const RhsScal& q = sc[i / k];
  if (!q.sel || (reproj_only && !q.reproj)) Y[i] = make_double2(0.0, 0.0);
}

template <typename E>
void step(hipStream_t s, int op, const VecSet& vs, E* x, E* r, const E* rhat, E* p, const E* v,
          const E* t, RhsScal* sc, double* partials, unsigned long long* acct) {
  dim3 g(vs.nblocks), b(BL_BS);
  switch (op) {
    case BI_S:
      hipLaunchKernelGGL((k_bicg_step<E, BI_S>), g, b, 0, s, vs, x, r, rhat, p, v, t, sc,
                         partials, nullptr);
      break;
    default:
      hipLaunchKernelGGL((k_bicg_step<E, BI_XR>), g, b, 0, s, vs, x, r, rhat, p, v, t, sc,
                         partials, acct);
      break;
  }
  DBQ_HIP(hipGetLastError());
}

}  // namespace

void bicg_step_f64(hipStream_t s, int op, const VecSet& vs, double2* x, double2* r,
                   const double2* rhat, double2* p, const double2* v, const double2* t,
                   RhsScal* sc, double* partials) {
  step<double2>(s, op, vs, x, r, rhat, p, v, t, sc, partials, nullptr);
}
void bicg_step_f32(hipStream_t s, int op, const VecSet& vs, float4* x, float4* r,
                   const float4* rhat, float4* p, const float4* v, const float4* t,
                   RhsScal* sc, double* partials, unsigned long long* acct) {
  step<float4>(s, op, vs, x, r, rhat, p, v, t, sc, partials, acct);
}
void bicg_fin_xr(hipStream_t s, const VecSet& vs, RhsScal* sc, const double* partials) {
  hipLaunchKernelGGL(k_fin_xr, dim3(fin_blocks(vs)), dim3(BL_BS), 0, s, vs, sc, partials);
  DBQ_HIP(hipGetLastError());
}

void bicg_aux_f64(hipStream_t s, int op, const VecSet& vs, const double2* r64, double2* r,
                  double2* rhat, double2* p, double2* v, RhsScal* sc, double* partials) {
  dim3 g(vs.nblocks), b(BL_BS);
  if (op == AX_INIT)
    hipLaunchKernelGGL((k_aux64<AX_INIT>), g, b, 0, s, vs, r64, r, rhat, p, v, sc, partials);
  else if (op == AX_RESTART)
    hipLaunchKernelGGL((k_aux64<AX_RESTART>), g, b, 0, s, vs, r64, r, rhat, p, v, sc, partials);
  else
    hipLaunchKernelGGL((k_aux64<AX_REPLACE>), g, b, 0, s, vs, r64, r, rhat, p, v, sc, partials);
  DBQ_HIP(hipGetLastError());
  if (op == AX_INIT) launch_fin_aux<AX_INIT>(s, vs, sc, partials);
  else if (op == AX_RESTART) launch_fin_aux<AX_RESTART>(s, vs, sc, partials);
  else launch_fin_aux<AX_REPLACE>(s, vs, sc, partials);
}

void bicg_aux_f32(hipStream_t s, int op, const VecSet& vs32, const VecSet& vs64,
                  const double2* r64, float4* r, float4* rhat, float4* p, float4* v, float4* x32,
                  RhsScal* sc, double* partials) {
  dim3 g(vs32.nblocks), b(BL_BS);
  if (op == AX_INIT)
    hipLaunchKernelGGL((k_aux32<AX_INIT>), g, b, 0, s, vs32, vs64, r64, r, rhat, p, v, x32, sc,
                       partials);
  else if (op == AX_RESTART)
    hipLaunchKernelGGL((k_aux32<AX_RESTART>), g, b, 0, s, vs32, vs64, r64, r, rhat, p, v, x32,
                       sc, partials);
  else
    hipLaunchKernelGGL((k_aux32<AX_REPLACE>), g, b, 0, s, vs32, vs64, r64, r, rhat, p, v, x32,
                       sc, partials);
  DBQ_HIP(hipGetLastError());
  if (op == AX_INIT) launch_fin_aux<AX_INIT>(s, vs32, sc, partials);
  else if (op == AX_RESTART) launch_fin_aux<AX_RESTART>(s, vs32, sc, partials);
  else launch_fin_aux<AX_REPLACE>(s, vs32, sc, partials);
}

void mask_unselected_f64(hipStream_t s, double2* Y, int k, int nrhs, const RhsScal* sc,
                         bool reproj_only) {
  hipLaunchKernelGGL(k_mask_unselected, dim3((k * nrhs + 255) / 256), dim3(256), 0, s, Y, k, nrhs,
                     sc, reproj_only ? 1 : 0);
  DBQ_HIP(hipGetLastError());
}

void bicg_xacc(hipStream_t s, const VecSet& vs32, const VecSet& vs64, double2* x64, float4* x32,
               const RhsScal* sc) {
  hipLaunchKernelGGL(k_xacc, dim3(vs32.nblocks), dim3(BL_BS), 0, s, vs32, vs64, x64, x32, sc);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
