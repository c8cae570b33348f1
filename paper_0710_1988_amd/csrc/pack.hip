// Layout conversion between the caller's lexicographic complex128 fields and the library's
// even-odd structure-of-arrays storage, plus the geometry tables.
#include "kernels.h"

namespace dbq {

namespace {

__global__ void k_geometry(Geom g, int32_t* lex_of_eo, int32_t* nbr) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  lex_of_eo[s] = lex_index(g, c);
  nbr[0 * g.V + s] = eo_neighbour<0, +1>(g, c);
  nbr[1 * g.V + s] = eo_neighbour<0, -1>(g, c);
  nbr[2 * g.V + s] = eo_neighbour<1, +1>(g, c);
  nbr[3 * g.V + s] = eo_neighbour<1, -1>(g, c);
  nbr[4 * g.V + s] = eo_neighbour<2, +1>(g, c);
  nbr[5 * g.V + s] = eo_neighbour<2, -1>(g, c);
  nbr[6 * g.V + s] = eo_neighbour<3, +1>(g, c);
  nbr[7 * g.V + s] = eo_neighbour<3, -1>(g, c);
}

// canonical [rhs][V lex][12] complex128 -> double2 [rhs][6][V eo][2]
__global__ void k_pack_sp64(Geom g, const double2* __restrict__ in, double2* __restrict__ out,
                            int nrhs) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const double2* src = in + ((long long)r * g.V + lex) * 12;
  double2* dst = out + (long long)r * 12 * g.V + 2 * s;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    dst[2 * (long long)k * g.V] = src[2 * k];
    dst[2 * (long long)k * g.V + 1] = src[2 * k + 1];
  }
}

__global__ void k_unpack_sp64(Geom g, const double2* __restrict__ in, double2* __restrict__ out,
                              int nrhs) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const double2* src = in + (long long)r * 12 * g.V + 2 * s;
  double2* dst = out + ((long long)r * g.V + lex) * 12;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    dst[2 * k] = src[2 * (long long)k * g.V];
    dst[2 * k + 1] = src[2 * (long long)k * g.V + 1];
  }
}

__global__ void k_pack_sp32(Geom g, const double2* __restrict__ in, float4* __restrict__ out,
                            int nrhs) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const double2* src = in + ((long long)r * g.V + lex) * 12;
  float4* dst = out + (long long)r * 6 * g.V + s;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double2 a = src[2 * k], b = src[2 * k + 1];
    dst[(long long)k * g.V] = make_float4(float(a.x), float(a.y), float(b.x), float(b.y));
  }
}

__global__ void k_unpack_sp32(Geom g, const float4* __restrict__ in, double2* __restrict__ out,
                              int nrhs) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (s >= g.V || r >= nrhs) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const float4* src = in + (long long)r * 6 * g.V + s;
  double2* dst = out + ((long long)r * g.V + lex) * 12;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float4 a = src[(long long)k * g.V];
    dst[2 * k] = make_double2(a.x, a.y);
    dst[2 * k + 1] = make_double2(a.z, a.w);
  }
}

// canonical links [4][V lex][3][3] -> double2 [4][9][V eo]
__global__ void k_pack_ln64(Geom g, const double2* __restrict__ in, double2* __restrict__ out) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int mu = blockIdx.y;
  if (s >= g.V) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const double2* src = in + ((long long)mu * g.V + lex) * 9;
  double2* dst = out + (long long)mu * 9 * g.V + s;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[(long long)k * g.V] = src[k];
}

// canonical links -> float4 [4][3][V eo], first two rows only
__global__ void k_pack_ln32(Geom g, const double2* __restrict__ in, float4* __restrict__ out) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int mu = blockIdx.y;
  if (s >= g.V) return;
  int c[4], p;
  eo_coords(g, s, c, p);
  long long lex = lex_index(g, c);
  const double2* src = in + ((long long)mu * g.V + lex) * 9;
  float4* dst = out + (long long)mu * 3 * g.V + s;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double2 a = src[2 * k], b = src[2 * k + 1];
    dst[(long long)k * g.V] = make_float4(float(a.x), float(a.y), float(b.x), float(b.y));
  }
}

// spins 2 and 3 (components 6..11) occupy the second half of every packed FP64 vector
__global__ void k_gamma5_f64(const double2* __restrict__ in, double2* __restrict__ out,
                             long long V, long long total) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  long long half = (e / (6 * V)) & 1;
  double2 v = in[e];
  if (half) v = make_double2(-v.x, -v.y);
  out[e] = v;
}

inline unsigned nblk(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

void launch_geometry(hipStream_t s, const Geom& g, int32_t* lex_of_eo, int32_t* nbr) {
  hipLaunchKernelGGL(k_geometry, dim3(nblk(g.V, 256)), dim3(256), 0, s, g, lex_of_eo, nbr);
  DBQ_HIP(hipGetLastError());
}

void pack_spinor_f64(hipStream_t s, const Geom& g, const void* canon, double2* out, int nrhs) {
  hipLaunchKernelGGL(k_pack_sp64, dim3(nblk(g.V, 256), nrhs), dim3(256), 0, s, g,
                     (const double2*)canon, out, nrhs);
  DBQ_HIP(hipGetLastError());
}
void unpack_spinor_f64(hipStream_t s, const Geom& g, const double2* in, void* canon, int nrhs) {
  hipLaunchKernelGGL(k_unpack_sp64, dim3(nblk(g.V, 256), nrhs), dim3(256), 0, s, g, in,
                     (double2*)canon, nrhs);
  DBQ_HIP(hipGetLastError());
}
void pack_spinor_f32(hipStream_t s, const Geom& g, const void* canon, float4* out, int nrhs) {
  hipLaunchKernelGGL(k_pack_sp32, dim3(nblk(g.V, 256), nrhs), dim3(256), 0, s, g,
                     (const double2*)canon, out, nrhs);
  DBQ_HIP(hipGetLastError());
}
void unpack_spinor_f32(hipStream_t s, const Geom& g, const float4* in, void* canon, int nrhs) {
  hipLaunchKernelGGL(k_unpack_sp32, dim3(nblk(g.V, 256), nrhs), dim3(256), 0, s, g, in,
                     (double2*)canon, nrhs);
  DBQ_HIP(hipGetLastError());
}
void pack_links_f64(hipStream_t s, const Geom& g, const void* canon, double2* out) {
  hipLaunchKernelGGL(k_pack_ln64, dim3(nblk(g.V, 256), 4), dim3(256), 0, s, g,
                     (const double2*)canon, out);
  DBQ_HIP(hipGetLastError());
}
void pack_links_f32(hipStream_t s, const Geom& g, const void* canon, float4* out) {
  hipLaunchKernelGGL(k_pack_ln32, dim3(nblk(g.V, 256), 4), dim3(256), 0, s, g,
                     (const double2*)canon, out);
  DBQ_HIP(hipGetLastError());
}
void gamma5_f64(hipStream_t s, const double2* in, double2* out, long long V, int count) {
  long long total = 12 * V * count;
  hipLaunchKernelGGL(k_gamma5_f64, dim3(nblk(total, 256)), dim3(256), 0, s, in, out, V, total);
  DBQ_HIP(hipGetLastError());
}

}  // namespace dbq
