// Measurement utility: a streaming copy through buffer resources with the
// same vector widths as the apply pass, for the practical HBM ceiling.
#include "dev_apply.h"

namespace rc {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Two vectors in flight per thread and the apply pass's non-temporal cache
// policy: the fastest copy shape measured on MI355X for 87 MB buffers.
template <int VB>
__global__ __launch_bounds__(kThreads) void k_stream_copy(uint8_t* dst, const uint8_t* src, int bytes) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(src), (short)0, bytes, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, bytes, kRsrcWord3);
  constexpr int kU = 2;
  const int n = bytes / VB;
  const int stride = gridDim.x * kThreads;
  int i = blockIdx.x * kThreads + threadIdx.x;
  for (; i + (kU - 1) * stride < n; i += kU * stride) {
    if constexpr (VB == 16) {
      u32x4 v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (i + u * stride) * VB, 0, kLoadPolicy);
#pragma unroll
      for (int u = 0; u < kU; ++u)
        __builtin_amdgcn_raw_buffer_store_b128(v[u], rd, (i + u * stride) * VB, 0, kStorePolicy);
    } else {
      uint32_t d[kU][VB / 4];
#pragma unroll
      for (int u = 0; u < kU; ++u) load_group<VB / 4>(rs, (i + u * stride) * VB, d[u]);
#pragma unroll
      for (int u = 0; u < kU; ++u) store_group<VB / 4>(rd, (i + u * stride) * VB, d[u]);
    }
  }
  for (; i < n; i += stride) {
    uint32_t d[VB / 4];
    if constexpr (VB == 16) {
      u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, i * VB, 0, kLoadPolicy);
      __builtin_amdgcn_raw_buffer_store_b128(v, rd, i * VB, 0, kStorePolicy);
    } else {
      load_group<VB / 4>(rs, i * VB, d);
      store_group<VB / 4>(rd, i * VB, d);
    }
  }
  // Tail bytes that do not fill a vector.
  const int tail0 = n * VB;
  for (int t = tail0 + blockIdx.x * kThreads + threadIdx.x; t < bytes; t += stride)
    __builtin_amdgcn_raw_buffer_store_b8(__builtin_amdgcn_raw_buffer_load_b8(rs, t, 0, 0), rd, t, 0, 0);
}

hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, int vec_bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const dim3 grid(cus * 4), block(kThreads);
  uint8_t* d = (uint8_t*)dst;
  const uint8_t* s = (const uint8_t*)src;
  const int n = (int)bytes;
  switch (vec_bytes) {
    case 4: hipLaunchKernelGGL((k_stream_copy<4>), grid, block, 0, st, d, s, n); break;
    case 8: hipLaunchKernelGGL((k_stream_copy<8>), grid, block, 0, st, d, s, n); break;
    case 12: hipLaunchKernelGGL((k_stream_copy<12>), grid, block, 0, st, d, s, n); break;
    default: hipLaunchKernelGGL((k_stream_copy<16>), grid, block, 0, st, d, s, n); break;
  }
  return hipGetLastError();
}

}  // namespace rc
