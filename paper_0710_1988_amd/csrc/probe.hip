// Streaming probes: a plain copy, a read-only reduction and a fill over a caller buffer, the
// practical HBM ceiling against which the Dslash and vector kernels are read (every kernel on
// the solver path streams its operands once and is bound by HBM bandwidth).
#include "ctx.h"
#include "kernels.h"

namespace dbq {

namespace {

constexpr int PB_BS = 256;
constexpr int PB_U = 4;  // float4 elements in flight per thread and sweep
constexpr int PROBE_BLOCKS = 256 * 8;

// kind 0: dst = src; 1: per-block sums of src into dst (one float per block); 2: dst = fill.
template <int KIND>
__global__ __launch_bounds__(PB_BS) void k_stream(const float4* __restrict__ src,
                                                  float4* __restrict__ dst, long long n) {
  const long long step = (long long)gridDim.x * PB_BS * PB_U;
  float acc = 0.f;
  for (long long i0 = (long long)blockIdx.x * PB_BS * PB_U + threadIdx.x; i0 < n; i0 += step) {
    float4 v[PB_U];
#pragma unroll
    for (int u = 0; u < PB_U; ++u) {
      const long long i = i0 + (long long)u * PB_BS;
      if (KIND == 2) v[u] = make_float4(1.f, 2.f, 3.f, 4.f);
      else v[u] = i < n ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < PB_U; ++u) {
      const long long i = i0 + (long long)u * PB_BS;
      if (KIND == 1) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
      else if (i < n) dst[i] = v[u];
    }
  }
  if (KIND == 1) {
    __shared__ float sh[PB_BS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int w = 0; w < PB_BS / 64; ++w) s += sh[w];
      reinterpret_cast<float*>(dst)[blockIdx.x] = s;
    }
  }
}

}  // namespace

double stream_probe(dbq_ctx* c, const void* src, void* dst, long long bytes, int kind, int reps) {
  DBQ_CHECK(kind >= 0 && kind <= 2, "probe kind must be 0, 1 or 2");
  DBQ_CHECK(reps >= 1, "reps must be >= 1");
  DBQ_CHECK(bytes >= 16 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
  DBQ_CHECK((kind == 2 || src) && dst, "null buffer");
  const long long n = bytes / 16;
  // enough blocks for every CU several times over; the read probe writes one float per block
  // (PROBE_BLOCKS floats into dst)
  const unsigned grid = PROBE_BLOCKS;
  hipEvent_t e0, e1;
  DBQ_HIP(hipEventCreate(&e0));
  DBQ_HIP(hipEventCreate(&e1));
  auto run = [&]() {
    const float4* s = (const float4*)src;
    float4* d = (float4*)dst;
    if (kind == 0) hipLaunchKernelGGL(k_stream<0>, dim3(grid), dim3(PB_BS), 0, c->stream, s, d, n);
    else if (kind == 1) hipLaunchKernelGGL(k_stream<1>, dim3(grid), dim3(PB_BS), 0, c->stream, s, d, n);
    else hipLaunchKernelGGL(k_stream<2>, dim3(grid), dim3(PB_BS), 0, c->stream, s, d, n);
  };
  run();  // warm-up
  DBQ_HIP(hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r) run();
  DBQ_HIP(hipEventRecord(e1, c->stream));
  DBQ_HIP(hipGetLastError());
  DBQ_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DBQ_HIP(hipEventElapsedTime(&ms, e0, e1));
  DBQ_HIP(hipEventDestroy(e0));
  DBQ_HIP(hipEventDestroy(e1));
  return double(ms) / reps;
}

}  // namespace dbq
