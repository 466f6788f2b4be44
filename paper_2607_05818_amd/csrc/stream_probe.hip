// HBM bandwidth probes: plain streaming kernels with 16-byte accesses and a
// grid-stride loop.  They measure what a bandwidth-bound kernel can reach
// on the device (the ceiling the Chebyshev passes and the update kernels
// are compared with); they take no part in any computation of the library.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "reff_internal.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_probe_copy(const f4* __restrict__ a, f4* __restrict__ b,
                                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_copy_nt(const f4* __restrict__ a,
                                                       f4* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

__global__ __launch_bounds__(256) void k_probe_read(const f4* __restrict__ a, int64_t n,
                                                    float* __restrict__ out) {
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const f4 v = a[i];
    s += v.x;
    s += v.y;
    s += v.z;
    s += v.w;
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_write(f4* __restrict__ b, int64_t n, float v) {
  const f4 x = {v, v, v, v};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    b[i] = x;
}

// Three reads and two writes per element, the traffic mix of a Chebyshev
// pass (z_j, z_{j-1}, R in; two iterates out).
__global__ __launch_bounds__(256) void k_probe_3r2w(const f4* __restrict__ a,
                                                    const f4* __restrict__ b,
                                                    const f4* __restrict__ c, f4* __restrict__ d,
                                                    f4* __restrict__ e, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const f4 x = a[i], y = b[i], z = c[i];
    f4 p, q;
    p.x = x.x + y.x;
    p.y = x.y + y.y;
    p.z = x.z + y.z;
    p.w = x.w + y.w;
    q.x = y.x - z.x;
    q.y = y.y - z.y;
    q.z = y.z - z.z;
    q.w = y.w - z.w;
    d[i] = p;
    e[i] = q;
  }
}

}  // namespace

extern "C" reff_status reff_stream_probe(int32_t kind, const void* src, void* dst, int64_t bytes,
                                         int32_t blocks, void* stream) {
  using namespace reff;
  if (kind < 0 || kind > 4) return host_fail(REFF_ERR_INVALID_ARG, "kind must be 0..4");
  if (bytes <= 0 || bytes % 16 != 0)
    return host_fail(REFF_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
  if (blocks < 1 || blocks > (1 << 20))
    return host_fail(REFF_ERR_INVALID_ARG, "blocks must be in 1 .. 2^20");
  if ((kind != 2 && !src) || !dst)
    return host_fail(REFF_ERR_INVALID_ARG, "NULL buffer");
  const int64_t n = bytes / 16;
  hipStream_t st = (hipStream_t)stream;
  const f4* a = (const f4*)src;
  f4* b = (f4*)dst;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st, a, b, n);
      break;
    case 1:
      // dst receives one float per thread (blocks x 256 x 4 bytes)
      hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(256), 0, st, a, n, (float*)dst);
      break;
    case 2:
      hipLaunchKernelGGL(k_probe_write, dim3(blocks), dim3(256), 0, st, b, n, 1.0f);
      break;
    case 3:
      hipLaunchKernelGGL(k_probe_3r2w, dim3(blocks), dim3(256), 0, st, a, a + n, a + 2 * n, b,
                         b + n, n);
      break;
    default:
      hipLaunchKernelGGL(k_probe_copy_nt, dim3(blocks), dim3(256), 0, st, a, b, n);
      break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return host_fail(REFF_ERR_DEVICE, std::string("probe: ") + hipGetErrorString(e));
  return REFF_OK;
}
