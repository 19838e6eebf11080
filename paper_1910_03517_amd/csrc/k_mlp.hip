// Kernels of the learned surrogate's MLP (576 -> 256 -> 256 -> 6, ReLU):
// an FP32 GEMM on the matrix cores with fused bias / ReLU / ReLU-mask
// epilogues and an optional ones row for bias gradients, the MSE gradient and
// value, Adam over the whole network in one launch, and a row gather for
// mini-batches.
#include "dev_mlp.h"

namespace rc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;   // workgroup tile (rows and columns)
constexpr int kGemmK = 32;      // k-slab staged in LDS
constexpr int kWsMaxRows = 2048;  // up to this many rows, row-major products use the k-split tile kernel

enum { kEpiNone = 0, kEpiBias = 1, kEpiBiasRelu = 2, kEpiMask = 3 };

// C[M][N] (row stride ldc) = A x B with A(i, k) = A[i * sai + k * sak] and
// B(k, j) = B[k * sbk + j * sbj] (strides express transposes), then the
// epilogue: + bias[j]; + bias[j] and ReLU; or times (mask[i][j] > 0).  With
// ones_row non-NULL the product also gets a row M of A equal to all ones, so
// that row M of the result, the column sums of B, is stored to ones_row[j]
// (the bias gradient next to a weight gradient).
// Four waves each own a 32x32 sub-tile and accumulate it with
// v_mfma_f32_32x32x2_f32: lane l supplies A(i = l % 32, k = l / 32) and
// B(k = l / 32, j = l % 32) and holds D(i, j) for j = l % 32 and
// i = 8 (r / 4) + 4 (l / 32) + r % 4 in accumulator register r.  The next
// K-slab is fetched into registers while the current one is multiplied.
template <int EPI>
__device__ __forceinline__ void k_gemm_body(int M, int N, int K, const float* __restrict__ A, int64_t sai,
                                            int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbj,
                                            float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                            const float* __restrict__ mask, int ldm, float* __restrict__ ones_row) {
  constexpr int kPer = kGemmK * kGemmTile / 256;   // staged elements per thread and operand
  __shared__ float As[kGemmK][kGemmTile + 1];
  __shared__ float Bs[kGemmK][kGemmTile + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i0 = blockIdx.y * kGemmTile;
  const int j0 = blockIdx.x * kGemmTile;
  const int wi = (wave >> 1) * 32;
  const int wj = (wave & 1) * 32;
  const int MA = ones_row ? M + 1 : M;             // rows of A including the ones row
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

  float ra[kPer], rb[kPer];
  // Element e of a staged slab is (kk, ii) with kk fastest when the operand
  // is contiguous along k, ii fastest otherwise, so that consecutive threads
  // read consecutive addresses either way (coalesced loads).
  const bool a_kfast = sak == 1, b_kfast = sbk == 1 && sbj != 1;
  auto slab_pos = [](int e, bool kfast, int& kk, int& ii) {
    if (kfast) { kk = e % kGemmK; ii = e / kGemmK; }
    else { kk = e / kGemmTile; ii = e % kGemmTile; }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * 256;
      int kk, ii;
      slab_pos(e, a_kfast, kk, ii);
      const int gi = i0 + ii, gka = k0 + kk;
      float a = 0.0f;
      if (gka < K) {
        if (gi < M) a = A[(int64_t)gi * sai + (int64_t)gka * sak];
        else if (gi < MA) a = 1.0f;
      }
      ra[q] = a;
      slab_pos(e, b_kfast, kk, ii);
      const int gj = j0 + ii, gkb = k0 + kk;
      rb[q] = (gkb < K && gj < N) ? B[(int64_t)gkb * sbk + (int64_t)gj * sbj] : 0.0f;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += kGemmK) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * 256;
      int kk, ii;
      slab_pos(e, a_kfast, kk, ii);
      As[kk][ii] = ra[q];
      slab_pos(e, b_kfast, kk, ii);
      Bs[kk][ii] = rb[q];
    }
    __syncthreads();
    if (k0 + kGemmK < K) fetch(k0 + kGemmK);
#pragma unroll
    for (int kk = 0; kk < kGemmK; kk += 2) {
      const float a = As[kk + (lane >> 5)][wi + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wj + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  const int j = j0 + wj + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (j >= N) continue;
    if (i < M) {
      float v = acc[r];
      if (EPI == kEpiBias || EPI == kEpiBiasRelu) v += bias[j];
      if (EPI == kEpiBiasRelu) v = v > 0.0f ? v : 0.0f;
      if (EPI == kEpiMask) v = mask[(int64_t)i * ldm + j] > 0.0f ? v : 0.0f;
      C[(int64_t)i * ldc + j] = v;
    } else if (i == M && ones_row) {
      ones_row[j] = acc[r];
    }
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sai,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbj,
                                              float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                              const float* __restrict__ mask, int ldm,
                                              float* __restrict__ ones_row) {
  k_gemm_body<EPI>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, mask, ldm, ones_row);
}

// The same product for few output rows (every product of the network at
// inference and mini-batch sizes), where 64 x 64 tiles would leave most
// compute units idle and each wave a long serial chain of MFMAs.  A
// workgroup of W waves owns a 32 x 32 tile; wave w sums k over its own range
// [w kw, (w + 1) kw) (kw a multiple of 8) straight from global memory: per 8
// k, lane l supplies A(i, k0 + 4 g + c) and B(k0 + 4 g + c, j) for c = 0..3
// (g = l / 32, i and j = l % 32), the c-th of 4 MFMAs pairing k0 + c with
// k0 + 4 + c.  The loads of kWsChunk such steps are in flight together, and
// the next chunk's are issued before the current chunk's MFMAs.  The waves'
// tiles are added in LDS in wave order, then the epilogue; row M is the ones
// row when ones_row is given (stored without epilogue).
constexpr int kWsTile = 32;
constexpr int kWsChunk = 4;
template <int EPI, int W>
__global__ __launch_bounds__(W * 64) void k_gemm_wsplit(int M, int N, int K, int kw, const float* __restrict__ A,
                                                        int64_t sai, int64_t sak, const float* __restrict__ B,
                                                        int64_t sbk, int64_t sbj, float* __restrict__ C, int ldc,
                                                        const float* __restrict__ bias, const float* __restrict__ mask,
                                                        int ldm, float* __restrict__ ones_row) {
  __shared__ float red[W][16][64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 5;
  const int i0 = blockIdx.y * kWsTile, j0 = blockIdx.x * kWsTile;
  const int ia = i0 + (lane & 31), jb = j0 + (lane & 31);
  const bool arow = ia < M, bcol = jb < N;
  const float aone = (ones_row && ia == M) ? 1.0f : 0.0f;   // the ones row, or padding
  const float* pa = A + (int64_t)(arow ? ia : 0) * sai;
  const float* pb = B + (int64_t)(bcol ? jb : 0) * sbj;
  const int kbeg = wave * kw;
  const int kend = (K - kbeg) < kw ? K : kbeg + kw;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  float a[kWsChunk][4], b[kWsChunk][4], an[kWsChunk][4], bn[kWsChunk][4];
  // An operand contiguous along k is read 16 bytes per lane (one load for
  // the four k of a step) where the whole quad is in range.
  const bool a_vec = sak == 1, b_vec = sbk == 1;
  auto load = [&](int k0, float (*av)[4], float (*bv)[4]) {
#pragma unroll
    for (int s = 0; s < kWsChunk; ++s) {
      const int kq = k0 + 8 * s + 4 * g;
      const bool quad = kq + 3 < kend;
      if (a_vec && arow && quad) {
        f32x4 v;
        __builtin_memcpy(&v, pa + kq, sizeof v);
#pragma unroll
        for (int c = 0; c < 4; ++c) av[s][c] = v[c];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) av[s][c] = kq + c < kend ? (arow ? pa[(int64_t)(kq + c) * sak] : aone) : 0.0f;
      }
      if (b_vec && bcol && quad) {
        f32x4 v;
        __builtin_memcpy(&v, pb + kq, sizeof v);
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[s][c] = v[c];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[s][c] = (kq + c < kend && bcol) ? pb[(int64_t)(kq + c) * sbk] : 0.0f;
      }
    }
  };
  constexpr int kSpan = 8 * kWsChunk;
  if (kbeg < kend) load(kbeg, a, b);
  for (int k0 = kbeg; k0 < kend; k0 += kSpan) {
    if (k0 + kSpan < kend) load(k0 + kSpan, an, bn);
#pragma unroll
    for (int s = 0; s < kWsChunk; ++s) {
      if (k0 + 8 * s >= kend) break;                // wave-uniform
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s][c], b[s][c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int s = 0; s < kWsChunk; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a[s][c] = an[s][c];
        b[s][c] = bn[s][c];
      }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
  __syncthreads();
  for (int e = tid; e < 16 * 64; e += W * 64) {
    const int r = e >> 6, l = e & 63;
    float v = 0.0f;
#pragma unroll
    for (int w = 0; w < W; ++w) v += red[w][r][l];
    const int i = i0 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    const int j = j0 + (l & 31);
    if (j >= N) continue;
    if (i < M) {
      if (EPI == kEpiBias || EPI == kEpiBiasRelu) v += bias[j];
      if (EPI == kEpiBiasRelu) v = v > 0.0f ? v : 0.0f;
      if (EPI == kEpiMask) v = mask[(int64_t)i * ldm + j] > 0.0f ? v : 0.0f;
      C[(int64_t)i * ldc + j] = v;
    } else if (i == M && ones_row) {
      ones_row[j] = v;
    }
  }
}

// Weight-gradient products C = A^T B over a long k (the mini-batch), both
// operands stored k-major: A(i, k) = A[k lda + i], B(k, j) = B[k ldb + j];
// with ones_row, row M of A is all ones and row M of the product (the column
// sums of B, the bias gradient) goes to ones_row.  Read one float per lane
// and k, as the k-split kernel must for such operands, the loads are bound
// by the compute unit's vector-memory issue rate; here each wave stages its
// k-range 32 k at a time into its own LDS slabs with 16-byte loads (8 lanes
// per k row, the next chunk's loads in flight meanwhile) and feeds the
// MFMAs from LDS in the k-split kernel's lane layout.  A workgroup of
// kWgWaves waves owns a 32 x 32 tile; the waves' partial tiles are added in
// LDS in wave order.
constexpr int kWgWaves = 16, kWgChunk = 32, kWgPad = 33;
struct WgradProblem {
  int M, N, K, kw, tiles_x;
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int ldc;
  float* ones_row;
};
// Up to three products in one launch (the backward's three weight gradients
// share K): problem q owns workgroups [start[q], start[q + 1]).
struct WgradSet {
  int n;
  int start[4];
  WgradProblem p[3];
};

__device__ __forceinline__ void wgrad_tile(const WgradProblem& P, int bx, int by) {
  __shared__ float stage[kWgWaves][2][kWgChunk][kWgPad];
  static_assert(sizeof(stage) >= sizeof(float) * kWgWaves * 16 * 64, "reduction area");
  float (*red)[16][64] = reinterpret_cast<float (*)[16][64]>(&stage[0][0][0][0]);
  const int M = P.M, N = P.N, K = P.K, kw = P.kw;
  const float* __restrict__ A = P.A;
  const float* __restrict__ B = P.B;
  const int64_t lda = P.lda, ldb = P.ldb;
  float* ones_row = P.ones_row;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 5;
  const int i0 = by * kWsTile, j0 = bx * kWsTile;
  const int kbeg = wave * kw;
  const int kend = (K - kbeg) < kw ? K : kbeg + kw;
  const int lr = lane >> 3, lc = 4 * (lane & 7);     // loader: rows lr + 8 q, columns lc .. lc + 3
  float ra[4][4], rb[4][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = k0 + 8 * q + lr;
      const bool krow = kk < kend;
      const int ia = i0 + lc, jb = j0 + lc;
      if (krow && ia + 3 < M) {
        f32x4 v;
        __builtin_memcpy(&v, A + (int64_t)kk * lda + ia, sizeof v);
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[q][e] = v[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ra[q][e] = !krow ? 0.0f : (ia + e < M ? A[(int64_t)kk * lda + ia + e] : (ones_row && ia + e == M ? 1.0f : 0.0f));
      }
      if (krow && jb + 3 < N) {
        f32x4 v;
        __builtin_memcpy(&v, B + (int64_t)kk * ldb + jb, sizeof v);
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[q][e] = v[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[q][e] = (krow && jb + e < N) ? B[(int64_t)kk * ldb + jb + e] : 0.0f;
      }
    }
  };
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  if (kbeg < kend) gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kWgChunk) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        stage[wave][0][8 * q + lr][lc + e] = ra[q][e];
        stage[wave][1][8 * q + lr][lc + e] = rb[q][e];
      }
    // The slabs are this wave's own: order its lanes' writes before their reads.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (k0 + kWgChunk < kend) gload(k0 + kWgChunk);
#pragma unroll
    for (int s = 0; s < kWgChunk / 8; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int kk = 8 * s + 4 * g + c;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(stage[wave][0][kk][lane & 31], stage[wave][1][kk][lane & 31],
                                                   acc, 0, 0, 0);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();                                   // every wave is done with the slabs
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
  __syncthreads();
  for (int e = tid; e < 16 * 64; e += kWgWaves * 64) {
    const int r = e >> 6, l = e & 63;
    float v = 0.0f;
#pragma unroll
    for (int w = 0; w < kWgWaves; ++w) v += red[w][r][l];
    const int i = i0 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    const int j = j0 + (l & 31);
    if (j >= N) continue;
    if (i < M) P.C[(int64_t)i * P.ldc + j] = v;
    else if (i == M && ones_row) ones_row[j] = v;
  }
}

__global__ __launch_bounds__(kWgWaves * 64) void k_gemm_wgrad(WgradSet s) {
  int q = 0;
  while (q + 1 < s.n && (int)blockIdx.x >= s.start[q + 1]) ++q;
  const int t = (int)blockIdx.x - s.start[q];
  wgrad_tile(s.p[q], t % s.p[q].tiles_x, t / s.p[q].tiles_x);
}

// Adds C = A^T B (+ ones row) to a set, both operands k-major.
static void wgrad_add(WgradSet& s, int M, int N, int K, const float* A, int64_t lda, const float* B, int64_t ldb,
                      float* C, int ldc, float* ones_row) {
  WgradProblem& P = s.p[s.n];
  const int MA = ones_row ? M + 1 : M;
  P.M = M; P.N = N; P.K = K;
  P.kw = ((K + kWgWaves - 1) / kWgWaves + kWgChunk - 1) / kWgChunk * kWgChunk;
  P.tiles_x = (N + kWsTile - 1) / kWsTile;
  P.A = A; P.lda = lda; P.B = B; P.ldb = ldb; P.C = C; P.ldc = ldc; P.ones_row = ones_row;
  if (s.n == 0) s.start[0] = 0;
  s.start[s.n + 1] = s.start[s.n] + P.tiles_x * ((MA + kWsTile - 1) / kWsTile);
  ++s.n;
}

static hipError_t wgrad_launch(const WgradSet& s, hipStream_t st) {
  if (s.n == 0 || s.start[s.n] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_wgrad, dim3(s.start[s.n]), dim3(kWgWaves * 64), 0, st, s);
  return hipGetLastError();
}

// The network's output layer, Y = H2 W3 + b3, one wave per row.  With T
// (training), also the loss gradient dY = 2 (Y - T) / (M * 6), the same
// expression k_mse_grad evaluates.
__global__ __launch_bounds__(256) void k_out_layer(int M, const float* __restrict__ H2, const float* __restrict__ W3,
                                                   const float* __restrict__ b3, float* __restrict__ Y,
                                                   const float* __restrict__ T, float* __restrict__ dY) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;                                    // whole waves
  float acc[kMlpOut];
  wave_row_dot<kMlpOut>(H2 + (int64_t)i * kMlpHid, W3, b3, kMlpHid, kMlpOut, acc);
  if ((threadIdx.x & 63) == 0) {
    const float count = (float)((int64_t)M * kMlpOut);
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
      const int64_t e = (int64_t)i * kMlpOut + o;
      Y[e] = acc[o];
      if (T) dY[e] = 2.0f * (acc[o] - T[e]) / count;
    }
  }
}

template <int EPI>
static hipError_t gemm(int M, int N, int K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
                       int64_t sbj, float* C, int ldc, const float* bias, const float* mask, int ldm, hipStream_t st,
                       float* ones_row = nullptr) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int MA = ones_row ? M + 1 : M;
  if (MA <= kWsMaxRows) {
    const dim3 g2((N + kWsTile - 1) / kWsTile, (MA + kWsTile - 1) / kWsTile);
    if (EPI == kEpiNone && sai == 1 && sbj == 1 && K >= 256) {   // weight gradients: both operands k-major
      WgradSet set{};
      wgrad_add(set, M, N, K, A, sak, B, sbk, C, ldc, ones_row);
      return wgrad_launch(set, st);
    }
    if (K >= 512) {            // long sums: 16 waves share k
      const int kw = ((K + 15) / 16 + 7) / 8 * 8;
      hipLaunchKernelGGL((k_gemm_wsplit<EPI, 16>), g2, dim3(16 * 64), 0, st, M, N, K, kw, A, sai, sak, B, sbk, sbj,
                         C, ldc, bias, mask, ldm, ones_row);
    } else {
      const int kw = ((K + 7) / 8 + 7) / 8 * 8;
      hipLaunchKernelGGL((k_gemm_wsplit<EPI, 8>), g2, dim3(8 * 64), 0, st, M, N, K, kw, A, sai, sak, B, sbk, sbj,
                         C, ldc, bias, mask, ldm, ones_row);
    }
    return hipGetLastError();
  }
  const dim3 grid((N + kGemmTile - 1) / kGemmTile, (MA + kGemmTile - 1) / kGemmTile);
  hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, st, M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, mask,
                     ldm, ones_row);
  return hipGetLastError();
}

// dY = 2 (Y - T) / count, elementwise over count values.
__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T,
                                                  int64_t count, float* __restrict__ dY) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) dY[i] = 2.0f * (Y[i] - T[i]) / (float)count;
}

// out[0] = mean of (Y - T)^2 over count values (one workgroup of 1024
// threads): thread t sums elements t, t + 1024, ... (eight loads in flight
// at a time), then the waves' sums, then the 16 wave totals in order.
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                              int64_t count, float* __restrict__ out) {
  __shared__ float red[16];
  constexpr int kU = 8;
  const int tid = threadIdx.x;
  float s = 0.0f;
  for (int64_t base = 0; base < count; base += 1024 * kU) {
    float d[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + (int64_t)u * 1024 + tid;
      d[u] = i < count ? Y[i] - T[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) s += d[u] * d[u];
  }
  s = wave_sum_f32(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    float t = 0.0f;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = t / (float)count;
  }
}

// The six tensors of one network as one index space for a single Adam launch.
struct AdamSet {
  float* p[6];
  const float* g[6];
  float* m[6];
  float* v[6];
  int64_t start[7];   // element e of the set is element e - start[t] of tensor t
};

// One Adam step over every parameter of the network, with bias-correction
// factors c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ __launch_bounds__(256) void k_adam(AdamSet a, float lr, float beta1, float beta2, float eps, float c1,
                                              float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.start[6]) return;
  int t = 0;
#pragma unroll
  for (int q = 1; q < 6; ++q) t += e >= a.start[q];
  const int64_t i = e - a.start[t];
  const float gi = a.g[t][i];
  const float mi = beta1 * a.m[t][i] + (1.0f - beta1) * gi;
  const float vi = beta2 * a.v[t][i] + (1.0f - beta2) * gi * gi;
  a.m[t][i] = mi;
  a.v[t][i] = vi;
  const float mh = mi * c1;
  const float vh = vi * c2;
  a.p[t][i] = a.p[t][i] - lr * mh / (__builtin_sqrtf(vh) + eps);
}

// The rows idx[r] of two tables at once (a mini-batch's inputs and targets):
// elements [0, n la) of the grid copy rows of a (row length la), the rest
// rows of b.
__global__ __launch_bounds__(256) void k_gather_rows2(const float* __restrict__ a, int la, float* __restrict__ da,
                                                      const float* __restrict__ b, int lb, float* __restrict__ db,
                                                      const int32_t* __restrict__ idx, int n) {
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t na = (int64_t)n * la;
  if (e < na) {
    const int r = (int)(e / la);
    da[e] = a[(int64_t)idx[r] * la + (e - (int64_t)r * la)];
    return;
  }
  e -= na;
  if (e >= (int64_t)n * lb) return;
  const int r = (int)(e / lb);
  db[e] = b[(int64_t)idx[r] * lb + (e - (int64_t)r * lb)];
}

// dst[r][:] = src[idx[r]][:] for r < n rows of row_len floats.
__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ src, int row_len,
                                                     const int32_t* __restrict__ idx, int n, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * row_len) return;
  const int r = (int)(e / row_len);
  const int c = (int)(e - (int64_t)r * row_len);
  dst[e] = src[(int64_t)idx[r] * row_len + c];
}

// ----------------------------------------------------------------------------- launchers

hipError_t mlp_hidden(const float* const* w, const float* X, int n, float* H1, float* H2, hipStream_t st) {
  // w = {w1, b1, w2, b2, w3, b3}
  hipError_t e = gemm<kEpiBiasRelu>(n, kMlpHid, kMlpIn, X, kMlpIn, 1, w[0], kMlpHid, 1, H1, kMlpHid, w[1], nullptr,
                                    0, st);
  if (e == hipSuccess)
    e = gemm<kEpiBiasRelu>(n, kMlpHid, kMlpHid, H1, kMlpHid, 1, w[2], kMlpHid, 1, H2, kMlpHid, w[3], nullptr, 0, st);
  return e;
}

hipError_t mlp_forward(const float* const* w, const float* X, int n, float* H1, float* H2, float* Y, hipStream_t st,
                       const float* T, float* dY) {
  hipError_t e = mlp_hidden(w, X, n, H1, H2, st);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(k_out_layer, dim3((n + 3) / 4), dim3(256), 0, st, n, H2, w[4], w[5], Y, T, dY);
  return hipGetLastError();
}

hipError_t mlp_backward(const float* const* w, const float* X, const float* H1, const float* H2, const float* Y,
                        const float* T, int n, float* const* g, float* dY, float* dZ1, float* dZ2, hipStream_t st,
                        bool dy_ready) {
  const int64_t cnt = (int64_t)n * kMlpOut;
  hipError_t e = hipSuccess;
  if (!dy_ready) {
    hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, Y, T, cnt, dY);
    e = hipGetLastError();
  }
  // dZ2 = (dY W3^T) * (H2 > 0), dZ1 = (dZ2 W2^T) * (H1 > 0)
  if (e == hipSuccess)
    e = gemm<kEpiMask>(n, kMlpHid, kMlpOut, dY, kMlpOut, 1, w[4], 1, kMlpOut, dZ2, kMlpHid, nullptr, H2, kMlpHid, st);
  if (e == hipSuccess)
    e = gemm<kEpiMask>(n, kMlpHid, kMlpHid, dZ2, kMlpHid, 1, w[2], 1, kMlpHid, dZ1, kMlpHid, nullptr, H1, kMlpHid, st);
  if (e != hipSuccess) return e;
  // dW1 = X^T dZ1, dW2 = H1^T dZ2, dW3 = H2^T dY, each with its bias gradient
  // (column sums of the second operand) as the ones row of the same product.
  if (n >= 256 && kMlpIn + 1 <= kWsMaxRows) {       // long sums: the three in one launch
    WgradSet set{};
    wgrad_add(set, kMlpIn, kMlpHid, n, X, kMlpIn, dZ1, kMlpHid, g[0], kMlpHid, g[1]);
    wgrad_add(set, kMlpHid, kMlpHid, n, H1, kMlpHid, dZ2, kMlpHid, g[2], kMlpHid, g[3]);
    wgrad_add(set, kMlpHid, kMlpOut, n, H2, kMlpHid, dY, kMlpOut, g[4], kMlpOut, g[5]);
    return wgrad_launch(set, st);
  }
  e = gemm<kEpiNone>(kMlpIn, kMlpHid, n, X, 1, kMlpIn, dZ1, kMlpHid, 1, g[0], kMlpHid, nullptr, nullptr, 0, st, g[1]);
  if (e == hipSuccess)
    e = gemm<kEpiNone>(kMlpHid, kMlpHid, n, H1, 1, kMlpHid, dZ2, kMlpHid, 1, g[2], kMlpHid, nullptr, nullptr, 0, st,
                       g[3]);
  if (e == hipSuccess)
    e = gemm<kEpiNone>(kMlpHid, kMlpOut, n, H2, 1, kMlpHid, dY, kMlpOut, 1, g[4], kMlpOut, nullptr, nullptr, 0, st,
                       g[5]);
  return e;
}

hipError_t mlp_adam(float* const* w, const float* const* g, float* const* m, float* const* v, int step, float lr,
                    float beta1, float beta2, float eps, hipStream_t st) {
  const int64_t sizes[6] = {(int64_t)kMlpIn * kMlpHid, kMlpHid, (int64_t)kMlpHid * kMlpHid, kMlpHid,
                            (int64_t)kMlpHid * kMlpOut, kMlpOut};
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
  AdamSet a;
  a.start[0] = 0;
  for (int t = 0; t < 6; ++t) {
    a.p[t] = w[t];
    a.g[t] = g[t];
    a.m[t] = m[t];
    a.v[t] = v[t];
    a.start[t + 1] = a.start[t] + sizes[t];
  }
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((a.start[6] + 255) / 256)), dim3(256), 0, st, a, lr, beta1, beta2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t mlp_mse(const float* Y, const float* T, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, st, Y, T, (int64_t)n * kMlpOut, out);
  return hipGetLastError();
}

hipError_t gather_rows2(const float* a, int la, float* da, const float* b, int lb, float* db, const int32_t* idx, int n,
                       hipStream_t st) {
  const int64_t total = (int64_t)n * (la + lb);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows2, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, la, da, b, lb, db,
                     idx, n);
  return hipGetLastError();
}

hipError_t gather_rows(const float* src, int row_len, const int32_t* idx, int n, float* dst, hipStream_t st) {
  const int64_t total = (int64_t)n * row_len;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, row_len, idx, n,
                     dst);
  return hipGetLastError();
}

}  // namespace rc
