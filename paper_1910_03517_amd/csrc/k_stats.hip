// Statistics kernels: band statistics of section 3.1 (the intensity
// distributions of the narrow bands along each seam), the zero fill used
// before atomic accumulation, and the whole-frame (n, S1, S2) finalize of
// 8-bit cameras from their exact histograms.
#include "rt_internal.h"

namespace rc {

// ---------------------------------------------------------------------------
// Zero fill (a kernel rather than hipMemsetAsync so that it is safe inside a
// captured graph).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_zero(uint8_t* p, int64_t bytes) {
  const int64_t nvec = bytes >> 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4* v = reinterpret_cast<uint4*>(p);
  for (int64_t i = t0; i < nvec; i += stride) v[i] = make_uint4(0, 0, 0, 0);
  for (int64_t i = (nvec << 4) + t0; i < bytes; i += stride) p[i] = 0;
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  int64_t nvec = (bytes + 15) >> 4;
  int grid = (int)((nvec + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, (uint8_t*)p, bytes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Band statistics: one workgroup per (camera, side, block).  The band is
// B' columns wide and the block's rows tall; every pixel of it adds one count
// per channel to an LDS histogram and its sample to exact 64-bit sums.
// ---------------------------------------------------------------------------
template <int C, int BPS>
__device__ void band_stats_unit(const Geo& g, const FramePtrs& fp, const Bufs& b, int k, int s, int j) {
  __shared__ uint32_t hist[kCS * kNB];
  __shared__ unsigned long long sums[kCS][2];
  const DevCam cam = g.cams[k];
  const int tid = threadIdx.x;
  for (int i = tid; i < kCS * kNB; i += blockDim.x) hist[i] = 0;
  if (tid < kCS * 2) (&sums[0][0])[tid] = 0;
  __syncthreads();

  const int r0 = (int)((int64_t)j * cam.height / g.n_blocks);
  const int r1 = (int)((int64_t)(j + 1) * cam.height / g.n_blocks);
  const int band = cam.band;
  const int c0 = (s == 0) ? 0 : cam.width - band;
  const int npx = (r1 - r0) * band;
  const int shift = cam.bit_depth - 8;
  const __amdgpu_buffer_rsrc_t rin = frame_rsrc(fp.in[k], cam);

  unsigned long long a1[C], a2[C];
#pragma unroll
  for (int c = 0; c < C; ++c) { a1[c] = 0; a2[c] = 0; }

  for (int i = tid; i < npx; i += blockDim.x) {
    const int row = i / band;
    const int px = i - row * band;
    const int rowoff = (int)((int64_t)(r0 + row) * cam.pitch);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int si = (c0 + px) * C + c;
      uint32_t v;
      if (BPS == 1) v = __builtin_amdgcn_raw_buffer_load_b8(rin, rowoff + si, 0, 0);
      else v = __builtin_amdgcn_raw_buffer_load_b16(rin, rowoff + 2 * si, 0, 0);
      uint32_t bin = v;
      if (BPS == 2) { bin = v >> shift; bin = bin > 255u ? 255u : bin; }
      atomicAdd(&hist[c * kNB + bin], 1u);
      a1[c] += v;
      a2[c] += (unsigned long long)v * v;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if (a1[c]) atomicAdd(&sums[c][0], a1[c]);
    if (a2[c]) atomicAdd(&sums[c][1], a2[c]);
  }
  __syncthreads();

  const int64_t u0 = unit_index(k, s, j, 0, g.n_blocks);
  uint32_t* oh = b.band_hist + u0 * kNB;
  for (int i = tid; i < kCS * kNB; i += blockDim.x) oh[i] = hist[i];
  if (tid < kCS) {
    uint64_t* os = b.band_sums + (u0 + tid) * 3;
    const bool used = tid < C;
    os[0] = used ? (uint64_t)npx : 0;
    os[1] = used ? sums[tid][0] : 0;
    os[2] = used ? sums[tid][1] : 0;
  }
}

__global__ __launch_bounds__(256) void k_band_stats(Geo g, FramePtrs fp, Bufs b) {
  const int unit = blockIdx.x;
  const int nb = g.n_blocks;
  const int k = unit / (2 * nb);
  const int s = (unit / nb) & 1;
  const int j = unit % nb;
  const DevCam& cam = g.cams[k];
  if (cam.bps == 2) band_stats_unit<1, 2>(g, fp, b, k, s, j);
  else if (cam.channels == 3) band_stats_unit<3, 1>(g, fp, b, k, s, j);
  else band_stats_unit<1, 1>(g, fp, b, k, s, j);
}

hipError_t launch_band_stats(const Geo& g, const FramePtrs& fp, const Bufs& b, hipStream_t st) {
  const int units = g.n_cams * 2 * g.n_blocks;
  hipLaunchKernelGGL(k_band_stats, dim3(units), dim3(256), 0, st, g, fp, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Whole-frame (n, S1, S2) of 8-bit cameras from their exact histograms:
// n = sum h[v], S1 = sum v h[v], S2 = sum v^2 h[v].  16-bit cameras
// accumulate their sums directly in the pass that builds the histogram.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_whole_finalize(Geo g, Bufs b) {
  const int k = blockIdx.x;
  const DevCam cam = g.cams[k];
  if (cam.bps != 1) return;
  __shared__ unsigned long long red[kCS][3];
  const int tid = threadIdx.x;
  if (tid < kCS * 3) (&red[0][0])[tid] = 0;
  __syncthreads();
  const uint32_t* h = b.whole_hist + (int64_t)k * kCS * kNB;
  for (int c = 0; c < cam.channels; ++c) {
    const unsigned long long cnt = h[c * kNB + tid];
    const unsigned long long v = (unsigned long long)tid;
    if (cnt) {
      atomicAdd(&red[c][0], cnt);
      atomicAdd(&red[c][1], cnt * v);
      atomicAdd(&red[c][2], cnt * v * v);
    }
  }
  __syncthreads();
  if (tid < kCS * 3) b.whole_sums[(int64_t)k * kCS * 3 + tid] = (&red[0][0])[tid];
}

hipError_t launch_whole_finalize(const Geo& g, const Bufs& b, hipStream_t st) {
  hipLaunchKernelGGL(k_whole_finalize, dim3(g.n_cams), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace rc
