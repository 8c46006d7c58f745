// Streaming-bandwidth probes: the achievable HBM ceiling of plain access
// patterns on this device, to set the step kernel's roofline fraction in
// context (lbt1_probe_bandwidth in include/lbt1.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/lbt1.h"
#include "lbt1_runtime.hpp"

namespace lbt1 {

typedef float f4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ void put(float4 *p, float4 v) {
  if (NT) {
    f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f4v *>(p));
  } else {
    *p = v;
  }
}

// out_k = in_k * s for `streams` input/output pairs (streams = 1: copy; 3: the
// three-in, three-out pattern of a moments-only step).
template <bool NT, int STREAMS>
__global__ void __launch_bounds__(256) k_probe_copy(const float4 *__restrict__ in, float4 *__restrict__ out,
                                                    long n, float s) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int k = 0; k < STREAMS; ++k) {
      float4 v = in[k * n + i];
      v.x *= s;
      v.y *= s;
      v.z *= s;
      v.w *= s;
      put<NT>(out + k * n + i, v);
    }
  }
}

// The same with U independent elements per thread in flight.
template <bool NT, int STREAMS, int U>
__global__ void __launch_bounds__(256) k_probe_copy_u(const float4 *__restrict__ in, float4 *__restrict__ out,
                                                      long n, float s) {
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
#pragma unroll
    for (int k = 0; k < STREAMS; ++k) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = in[k * n + i + u * stride];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u].x *= s;
        v[u].y *= s;
        v[u].z *= s;
        v[u].w *= s;
        put<NT>(out + k * n + i + u * stride, v[u]);
      }
    }
  }
  for (; i < n; i += stride) {
#pragma unroll
    for (int k = 0; k < STREAMS; ++k) {
      float4 v = in[k * n + i];
      v.x *= s;
      put<NT>(out + k * n + i, v);
    }
  }
}

__global__ void __launch_bounds__(256) k_probe_read(const float4 *__restrict__ in, float *__restrict__ sink, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  float acc = 0.f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 v = in[i];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc == 12345.678f) sink[0] = acc;  // keeps the loads; practically never stores
}

template <bool NT>
__global__ void __launch_bounds__(256) k_probe_write(float4 *__restrict__ out, long n, float s) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) put<NT>(out + i, make_float4(s, s, s, s));
}

}  // namespace lbt1

using namespace lbt1;

extern "C" lbt1_status lbt1_probe_bandwidth(int32_t kind, size_t bytes, int32_t nontemporal, int32_t reps,
                                            double *gbps) {
  clear_error();
  if (!gbps || reps < 1 || bytes < (1u << 20) || kind < LBT1_PROBE_COPY || kind > LBT1_PROBE_3IN3OUT)
    return fail(LBT1_EINVAL, "bad probe arguments");
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess || (e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
    return hip_fail(e, "device query");
  // n float4 per stream; total traffic per launch ~ bytes
  const int streams_in = kind == LBT1_PROBE_COPY ? 1 : kind == LBT1_PROBE_3IN3OUT ? 3 : kind == LBT1_PROBE_READ ? 1 : 0;
  const int streams_out = kind == LBT1_PROBE_COPY ? 1 : kind == LBT1_PROBE_3IN3OUT ? 3 : kind == LBT1_PROBE_WRITE ? 1 : 0;
  const long n = (long)(bytes / 16 / (streams_in + streams_out));
  const size_t nb = (size_t)n * 16;
  float4 *in = nullptr, *out = nullptr;
  float *sink = nullptr;
  if (streams_in && (e = hipMalloc(&in, nb * streams_in)) != hipSuccess) return fail(LBT1_ENOMEM, "probe buffer");
  if (streams_out && (e = hipMalloc(&out, nb * streams_out)) != hipSuccess) {
    if (in) (void)hipFree(in);
    return fail(LBT1_ENOMEM, "probe buffer");
  }
  if ((e = hipMalloc(&sink, 256)) != hipSuccess) {
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    return fail(LBT1_ENOMEM, "probe buffer");
  }
  if (in) (void)hipMemset(in, 0, nb * streams_in);
  if (out) (void)hipMemset(out, 0, nb * streams_out);
  const dim3 block(256);
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  double best = 0;
  // every launch shape of the search: blocks per CU x elements in flight per thread
  const int per_cu[4] = {4, 8, 16, 32};
  for (int r = 0; r < 8 * (reps + 1); ++r) {
    const dim3 grid(prop.multiProcessorCount * per_cu[(r / (reps + 1)) % 4]);
    const bool unrolled = (r / (reps + 1)) >= 4;
    (void)hipEventRecord(a, nullptr);
    if (kind == LBT1_PROBE_COPY) {
      if (unrolled) {
        if (nontemporal)
          hipLaunchKernelGGL((k_probe_copy_u<true, 1, 4>), grid, block, 0, nullptr, in, out, n, 1.0f);
        else
          hipLaunchKernelGGL((k_probe_copy_u<false, 1, 4>), grid, block, 0, nullptr, in, out, n, 1.0f);
      } else if (nontemporal) {
        hipLaunchKernelGGL((k_probe_copy<true, 1>), grid, block, 0, nullptr, in, out, n, 1.0f);
      } else {
        hipLaunchKernelGGL((k_probe_copy<false, 1>), grid, block, 0, nullptr, in, out, n, 1.0f);
      }
    } else if (kind == LBT1_PROBE_3IN3OUT) {
      if (unrolled) {
        if (nontemporal)
          hipLaunchKernelGGL((k_probe_copy_u<true, 3, 2>), grid, block, 0, nullptr, in, out, n, 1.0f);
        else
          hipLaunchKernelGGL((k_probe_copy_u<false, 3, 2>), grid, block, 0, nullptr, in, out, n, 1.0f);
      } else if (nontemporal) {
        hipLaunchKernelGGL((k_probe_copy<true, 3>), grid, block, 0, nullptr, in, out, n, 1.0f);
      } else {
        hipLaunchKernelGGL((k_probe_copy<false, 3>), grid, block, 0, nullptr, in, out, n, 1.0f);
      }
    } else if (kind == LBT1_PROBE_READ) {
      hipLaunchKernelGGL(k_probe_read, grid, block, 0, nullptr, in, sink, n);
    } else {
      if (nontemporal)
        hipLaunchKernelGGL((k_probe_write<true>), grid, block, 0, nullptr, out, n, 1.0f);
      else
        hipLaunchKernelGGL((k_probe_write<false>), grid, block, 0, nullptr, out, n, 1.0f);
    }
    (void)hipEventRecord(b, nullptr);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    const double moved = (double)nb * (streams_in + streams_out);
    if (r % (reps + 1) != 0) best = std::max(best, moved / (ms * 1e-3) / 1e9);  // first of each shape warms up
  }
  e = hipGetLastError();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  (void)hipFree(sink);
  if (e != hipSuccess) return hip_fail(e, "probe launch");
  *gbps = best;
  return LBT1_OK;
}
