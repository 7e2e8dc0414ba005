// gemm.hip -- the descriptor/query similarity GEMM on MFMA.
//
//   sim[row][col] = kappa(row, col) * max(0, <qn_row, dn_col>)
//
// qn (query vectors) and dn (object descriptors) are L2-normalised rows,
// zero-padded to a multiple of 32 elements, so the contraction is an "NT"
// GEMM with K contiguous in both operands.  The clamp at zero turns the
// cosine into the unary score in [0, 1]; on target rows (row < n_cls_rows) the
// soft class factor 0.3 multiplies objects whose known class differs from the
// query's parsed class (Appendix "Retrieval Details", composite-scoring step).
//
// FP32 path: v_mfma_f32_32x32x2f32.  A 256-thread block computes a 128x128
// tile; each of its four waves owns a 64x64 quadrant as 2x2 MFMA tiles of
// 32x32.  K advances 32 at a time through LDS (rows padded by 4 floats so the
// 16-byte fragment reads of 32 consecutive rows hit distinct banks); the next
// K tile is fetched into registers while the current one is consumed.  Within
// an 8-wide K slice, lane half h supplies elements 4h..4h+3 of the slice to
// four consecutive MFMAs, a fixed permutation of the K order shared by both
// operands (the sum is unchanged).
#include "farm_internal.h"

namespace farm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBN = 128, kBK = 32, kLda = kBK + 4;

__device__ inline float class_factor(int64_t row, int64_t col, const int32_t* row_cls, int64_t n_cls_rows,
                                     const int32_t* col_cls) {
  if (row >= n_cls_rows || col_cls == nullptr) return 1.0f;
  int rc = row_cls[row];
  int cc = col_cls[col];
  return (rc >= 0 && cc >= 0 && rc != cc) ? kClassFactor : 1.0f;
}

// Block index -> output tile, grouping consecutive launches of one XCD onto
// neighbouring tiles.  Workgroups are dispatched round-robin over the 8 XCDs,
// so block b runs on XCD b % 8; remapping makes each XCD sweep a contiguous
// band of tiles that share operand rows in its own L2.
__device__ inline void tile_of_block(int64_t& tm, int64_t& tn, int64_t tiles_m, int64_t tiles_n) {
  int64_t b = blockIdx.x;
  int64_t total = tiles_m * tiles_n;
  int64_t per_xcd = total / 8;
  int64_t lin = b;
  if (per_xcd > 0 && b < per_xcd * 8) lin = (b % 8) * per_xcd + b / 8;
  // column-major sweep in groups of 8 tile rows (an object block is reused by
  // the query blocks of a group while it is still in L2)
  const int64_t group = 8;
  int64_t gsize = group * tiles_n;
  int64_t g = lin / gsize;
  int64_t first_m = g * group;
  int64_t gm = tiles_m - first_m < group ? tiles_m - first_m : group;
  int64_t in = lin % gsize;
  tm = first_m + in % gm;
  tn = in / gm;
}

__global__ __launch_bounds__(256) void k_sim_gemm_f32(const float* __restrict__ A, const float* __restrict__ B,
                                                      int64_t M, int64_t N, int32_t ldk, float* __restrict__ C,
                                                      int64_t ldc, const int32_t* __restrict__ row_cls,
                                                      int64_t n_cls_rows, const int32_t* __restrict__ col_cls,
                                                      int64_t tiles_m, int64_t tiles_n) {
  __shared__ float As[kBM * kLda];
  __shared__ float Bs[kBN * kLda];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  tile_of_block(tm, tn, tiles_m, tiles_n);
  const int64_t m0 = tm * kBM, n0 = tn * kBN;

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float4 ra[4], rb[4];
  const int lr = tid >> 3, lc = (tid & 7) * 4;
  auto gload = [&](int kt) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int64_t gm = m0 + lr + 32 * p, gn = n0 + lr + 32 * p;
      ra[p] = gm < M ? *reinterpret_cast<const float4*>(A + gm * ldk + (int64_t)kt * kBK + lc)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
      rb[p] = gn < N ? *reinterpret_cast<const float4*>(B + gn * ldk + (int64_t)kt * kBK + lc)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      *reinterpret_cast<float4*>(&As[(lr + 32 * p) * kLda + lc]) = ra[p];
      *reinterpret_cast<float4*>(&Bs[(lr + 32 * p) * kLda + lc]) = rb[p];
    }
  };

  const int nk = ldk / kBK;
  gload(0);
  sstore();
  __syncthreads();
  const int h = lane >> 5, r = lane & 31;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 8) {
      float4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const float4*>(&As[(wm * 64 + i * 32 + r) * kLda + kk + 4 * h]);
        b[i] = *reinterpret_cast<const float4*>(&Bs[(wn * 64 + i * 32 + r) * kLda + kk + 4 * h]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].y, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].z, b[j].z, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, b[j].w, acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      sstore();
      __syncthreads();
    }
  }

  // 32x32 accumulator layout: register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4,
  // column l%32 of the MFMA tile.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int64_t row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        int64_t col = n0 + wn * 64 + j * 32 + r;
        if (row < M && col < N) {
          float val = fmaxf(acc[i][j][v], 0.f);
          C[row * ldc + col] = val * class_factor(row, col, row_cls, n_cls_rows, col_cls);
        }
      }
}

}  // namespace

hipError_t launch_sim_gemm_f32(const float* a, const float* b, int64_t m, int64_t n, int32_t ldk, float* c,
                               int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows, const int32_t* col_cls,
                               hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (ldk % kBK) return hipErrorInvalidValue;
  int64_t tiles_m = (m + kBM - 1) / kBM, tiles_n = (n + kBN - 1) / kBN;
  hipLaunchKernelGGL(k_sim_gemm_f32, dim3((unsigned)(tiles_m * tiles_n)), dim3(256), 0, s, a, b, m, n, ldk, c, ldc,
                     row_cls, n_cls_rows, col_cls, tiles_m, tiles_n);
  return hipGetLastError();
}

hipError_t launch_sim_gemm_bf16(const uint16_t*, const uint16_t*, int64_t, int64_t, int32_t, float*, int64_t,
                                const int32_t*, int64_t, const int32_t*, hipStream_t) {
  return hipErrorNotSupported;
}

hipError_t launch_sim_gemm_fp8(const uint8_t*, const float*, const uint8_t*, const float*, int64_t, int64_t,
                               int32_t, float*, int64_t, const int32_t*, int64_t, const int32_t*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace farm
