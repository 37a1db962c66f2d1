// Streaming probes of the memory bandwidth a plain kernel reaches on this GPU: a copy and a
// read-only reduction over large device buffers with 16-byte vector accesses in a
// grid-stride loop. They give the practical ceiling to set the hop kernels' bandwidth
// against (the 8 TB/s peak is not reached by plain streams).
#include "internal.h"

namespace {

constexpr int kProbeThreads = 256;

template <bool NT>
__global__ __launch_bounds__(kProbeThreads) void k_stream_copy(const float4* __restrict__ src,
                                                               float4* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * kProbeThreads;
  for (long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) {
    const float4 v = src[i];
    if (NT) {
      __builtin_nontemporal_store(v.x, &dst[i].x);
      __builtin_nontemporal_store(v.y, &dst[i].y);
      __builtin_nontemporal_store(v.z, &dst[i].z);
      __builtin_nontemporal_store(v.w, &dst[i].w);
    } else {
      dst[i] = v;
    }
  }
}

// one partial sum per workgroup (keeps every load live)
__global__ __launch_bounds__(kProbeThreads) void k_stream_read(const float4* __restrict__ src, long long n,
                                                               float* __restrict__ part) {
  __shared__ float sh[kProbeThreads / 64];
  const long long stride = (long long)gridDim.x * kProbeThreads;
  float acc = 0.f;
  for (long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace

extern "C" {

int sap_stream_probe_blocks(void) { return 4096; }

int sap_stream_probe(void* dst, const void* src, size_t bytes, int mode, void* stream) {
  if (!dst || !src || bytes < 16 || bytes % 16) return SAP_E_ARG;
  if (mode < 0 || mode > 2) return SAP_E_ARG;
  if (((uintptr_t)dst | (uintptr_t)src) & 15) return SAP_E_ARG;
  const long long n = (long long)(bytes / 16);
  const int blocks = sap_stream_probe_blocks();
  hipStream_t s = (hipStream_t)stream;
  if (mode == 0)
    hipLaunchKernelGGL(k_stream_copy<false>, dim3(blocks), dim3(kProbeThreads), 0, s, (const float4*)src,
                       (float4*)dst, n);
  else if (mode == 1)
    hipLaunchKernelGGL(k_stream_copy<true>, dim3(blocks), dim3(kProbeThreads), 0, s, (const float4*)src,
                       (float4*)dst, n);
  else
    hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(kProbeThreads), 0, s, (const float4*)src, n,
                       (float*)dst);
  return hipGetLastError() == hipSuccess ? SAP_OK : SAP_E_HIP;
}

}  // extern "C"
