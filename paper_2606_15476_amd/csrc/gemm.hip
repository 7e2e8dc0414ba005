// gemm.hip -- the descriptor/query similarity GEMM on MFMA.
//
//   sim[row][col] = kappa(row, col) * max(0, sa[row] * sb[col] * <qn_row, dn_col>)
//
// qn (query vectors) and dn (object descriptors) are L2-normalised rows,
// zero-padded to a multiple of 128 elements, so the contraction is an "NT"
// GEMM with K contiguous in both operands.  The clamp at zero turns the cosine
// into the unary score in [0, 1]; on target rows (row < n_cls_rows) the soft
// class factor 0.3 multiplies objects whose known class differs from the
// query's parsed class (Appendix "Retrieval Details", composite-scoring step).
// FP8 rows carry per-row scales sa, sb (amax / 448); FP32 and BF16 have none.
//
// One kernel template serves the three operand types.  A 256-thread block
// computes a 128x128 tile; each of its four waves owns a 64x64 quadrant as 2x2
// MFMA tiles of 32x32.  K advances through LDS in slabs of 128 bytes per row
// (32 FP32, 64 BF16 or 128 FP8 elements); rows are padded by 16 bytes so the
// 16-byte fragment reads of 32 consecutive rows hit distinct banks, and the
// next slab is fetched into registers while the current one is consumed.
// Each 32-byte slice of a slab feeds the MFMA pipe from two lane halves of 16
// bytes: four v_mfma_f32_32x32x2f32 or one v_mfma_f32_32x32x16_bf16 per slice.
// Lane half h supplies bytes 16h..16h+15 of the slice to both operands, a fixed
// permutation of the K order shared by A and B (the sum is unchanged).  FP8
// takes 64-byte chunks instead, one gfx950 32x32x64 MFMA each (lane half h:
// bytes 32h..32h+31), twice the K per instruction of the 32x32x16 FP8 form.
#include "farm_internal.h"

namespace farm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

enum { kT32 = 0, kTBF16 = 1, kTFP8 = 2 };

constexpr int kBM = 128, kBN = 128;
constexpr int kSlab = 128;              // bytes of K per row per slab
constexpr int kRowU4 = kSlab / 16 + 1;  // padded LDS row length in 16-byte units

__device__ inline float class_factor(int64_t row, int64_t col, const int32_t* row_cls, int64_t n_cls_rows,
                                     const int32_t* col_cls) {
  if (row >= n_cls_rows || col_cls == nullptr) return 1.0f;
  int rc = row_cls[row];
  int cc = col_cls[col];
  return (rc >= 0 && cc >= 0 && rc != cc) ? kClassFactor : 1.0f;
}

// Block index -> output tile.  Workgroups are dispatched round-robin over the
// 8 XCDs (block b runs on XCD b % 8); the remap gives each XCD a contiguous
// band of tiles, swept column-major in groups of 8 tile rows so an object
// block is reused by the query blocks of a group while it sits in that XCD's L2.
__device__ inline void tile_of_block(int64_t& tm, int64_t& tn, int64_t tiles_m, int64_t tiles_n) {
  int64_t b = blockIdx.x;
  int64_t total = tiles_m * tiles_n;
  int64_t per_xcd = total / 8;
  int64_t lin = b;
  if (per_xcd > 0 && b < per_xcd * 8) lin = (b % 8) * per_xcd + b / 8;
  const int64_t group = 8;
  int64_t gsize = group * tiles_n;
  int64_t g = lin / gsize;
  int64_t first_m = g * group;
  int64_t gm = tiles_m - first_m < group ? tiles_m - first_m : group;
  int64_t in = lin % gsize;
  tm = first_m + in % gm;
  tn = in / gm;
}

// FP8 (OCP e4m3) 32x32x64 MFMA of gfx950 on 32 bytes of K per lane: the
// block-scaled form with unit scales (E8M0 127 = 2^0) -- the per-row scales are
// applied in the epilogue.  Twice the K of 32x32x16 per instruction.
__device__ inline void mfma_fp8_64(floatx16& acc, const uint4& a_lo, const uint4& a_hi, const uint4& b_lo,
                                   const uint4& b_hi) {
  const intx8 a = {(int)a_lo.x, (int)a_lo.y, (int)a_lo.z, (int)a_lo.w, (int)a_hi.x, (int)a_hi.y, (int)a_hi.z, (int)a_hi.w};
  const intx8 b = {(int)b_lo.x, (int)b_lo.y, (int)b_lo.z, (int)b_lo.w, (int)b_hi.x, (int)b_hi.y, (int)b_hi.z, (int)b_hi.w};
  acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
}

template <int T>
__device__ inline void mfma_slice(floatx16& acc, const uint4& a, const uint4& b) {
  if constexpr (T == kT32) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
  } else if constexpr (T == kTBF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc,
                                                  0, 0, 0);
  } else {
    long a0 = (long)((uint64_t)a.x | ((uint64_t)a.y << 32));
    long a1 = (long)((uint64_t)a.z | ((uint64_t)a.w << 32));
    long b0 = (long)((uint64_t)b.x | ((uint64_t)b.y << 32));
    long b1 = (long)((uint64_t)b.z | ((uint64_t)b.w << 32));
    acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a1, b1, acc, 0, 0, 0);
  }
}

// Epilogues: the similarity matrix (scales, clamp, class factor) or a plain
// layer output C = acc + bias[col] in FP32, or BF16 GELU(acc + bias[col]).
enum { kEpiSim = 0, kEpiBias = 1, kEpiGeluBf16 = 2 };

__device__ inline float gelu_erf(float v) { return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f)); }

__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int T, int EPI = kEpiSim>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T == kTFP8 ? 2 : 3))) void k_sim_gemm(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                  int64_t M, int64_t N, int64_t K_bytes, int64_t lda_bytes,
                                                  int64_t ldb_bytes, void* __restrict__ Cv, int64_t ldc,
                                                  const float* __restrict__ a_scale,
                                                  const float* __restrict__ b_scale,
                                                  const int32_t* __restrict__ row_cls, int64_t n_cls_rows,
                                                  const int32_t* __restrict__ col_cls, int64_t tiles_m,
                                                  int64_t tiles_n) {
  __shared__ uint4 As[kBM * kRowU4];
  __shared__ uint4 Bs[kBN * kRowU4];
  // epilogue inputs of the tile's rows (first kBM) and columns: class ids and
  // FP8 scales of the similarity epilogue, the bias of the layer epilogues.
  // They are read here, before any store of the block: a load issued after
  // the stores would wait for all of them (loads and stores share one
  // in-order counter).
  __shared__ int32_t e_cls[kBM + kBN];
  __shared__ float e_val[kBM + kBN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  tile_of_block(tm, tn, tiles_m, tiles_n);
  const int64_t m0 = tm * kBM, n0 = tn * kBN;
  {
    int32_t ec = -1;
    float ev = EPI == kEpiSim ? 1.0f : 0.0f;
    if (tid < kBM) {
      const int64_t row = m0 + tid;
      if (EPI == kEpiSim && row < M) {
        if (row < n_cls_rows && col_cls) ec = row_cls[row];
        if (T == kTFP8) ev = a_scale[row];
      }
    } else {
      const int64_t col = n0 + tid - kBM;
      if (col < N) {
        if (EPI == kEpiSim) {
          if (col_cls) ec = col_cls[col];
          if (T == kTFP8) ev = b_scale[col];
        } else if (b_scale) {
          ev = b_scale[col];
        }
      }
    }
    e_cls[tid] = ec;
    e_val[tid] = ev;
  }

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // Rows past the end of A or B are clamped to the last row: they only feed
  // accumulator rows/columns that are never stored, and the loads stay
  // unconditional so the next slab can be in flight under the MFMAs.
  const int lr = tid >> 3, lc = tid & 7;
  auto clamp_row = [](int64_t v, int64_t lim) { return v < lim ? v : lim - 1; };
  const uint4* a0p = reinterpret_cast<const uint4*>(A + clamp_row(m0 + lr, M) * lda_bytes + lc * 16);
  const uint4* a1p = reinterpret_cast<const uint4*>(A + clamp_row(m0 + lr + 32, M) * lda_bytes + lc * 16);
  const uint4* a2p = reinterpret_cast<const uint4*>(A + clamp_row(m0 + lr + 64, M) * lda_bytes + lc * 16);
  const uint4* a3p = reinterpret_cast<const uint4*>(A + clamp_row(m0 + lr + 96, M) * lda_bytes + lc * 16);
  const uint4* b0p = reinterpret_cast<const uint4*>(B + clamp_row(n0 + lr, N) * ldb_bytes + lc * 16);
  const uint4* b1p = reinterpret_cast<const uint4*>(B + clamp_row(n0 + lr + 32, N) * ldb_bytes + lc * 16);
  const uint4* b2p = reinterpret_cast<const uint4*>(B + clamp_row(n0 + lr + 64, N) * ldb_bytes + lc * 16);
  const uint4* b3p = reinterpret_cast<const uint4*>(B + clamp_row(n0 + lr + 96, N) * ldb_bytes + lc * 16);
  constexpr int kStepU4 = kSlab / 16;  // one slab in 16-byte units
  uint4 ra0 = a0p[0], ra1 = a1p[0], ra2 = a2p[0], ra3 = a3p[0];
  uint4 rb0 = b0p[0], rb1 = b1p[0], rb2 = b2p[0], rb3 = b3p[0];
  uint4* as = As + lr * kRowU4 + lc;
  uint4* bs = Bs + lr * kRowU4 + lc;
  as[0] = ra0; as[32 * kRowU4] = ra1; as[64 * kRowU4] = ra2; as[96 * kRowU4] = ra3;
  bs[0] = rb0; bs[32 * kRowU4] = rb1; bs[64 * kRowU4] = rb2; bs[96 * kRowU4] = rb3;
  __syncthreads();

  const int64_t nk = K_bytes / kSlab;
  const int h = lane >> 5, r = lane & 31;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int64_t kn = (kt + 1 < nk ? kt + 1 : kt) * kStepU4;
    ra0 = a0p[kn]; ra1 = a1p[kn]; ra2 = a2p[kn]; ra3 = a3p[kn];
    rb0 = b0p[kn]; rb1 = b1p[kn]; rb2 = b2p[kn]; rb3 = b3p[kn];
    // keep the next slab's loads in flight under this slab's MFMAs
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (T == kTFP8) {
      // two 64-byte K chunks per slab; lane half h takes bytes 32h..32h+31 of a chunk for both operands
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int u = 4 * c + 2 * h;
        const uint4 b0l = Bs[(wn * 64 + r) * kRowU4 + u], b0h = Bs[(wn * 64 + r) * kRowU4 + u + 1];
        const uint4 b1l = Bs[(wn * 64 + 32 + r) * kRowU4 + u], b1h = Bs[(wn * 64 + 32 + r) * kRowU4 + u + 1];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint4 al = As[(wm * 64 + 32 * i + r) * kRowU4 + u], ah = As[(wm * 64 + 32 * i + r) * kRowU4 + u + 1];
          mfma_fp8_64(acc[i][0], al, ah, b0l, b0h);
          mfma_fp8_64(acc[i][1], al, ah, b1l, b1h);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const uint4 a_0 = As[(wm * 64 + r) * kRowU4 + 2 * s + h];
        const uint4 a_1 = As[(wm * 64 + 32 + r) * kRowU4 + 2 * s + h];
        const uint4 b_0 = Bs[(wn * 64 + r) * kRowU4 + 2 * s + h];
        const uint4 b_1 = Bs[(wn * 64 + 32 + r) * kRowU4 + 2 * s + h];
        mfma_slice<T>(acc[0][0], a_0, b_0);
        mfma_slice<T>(acc[0][1], a_0, b_1);
        mfma_slice<T>(acc[1][0], a_1, b_0);
        mfma_slice<T>(acc[1][1], a_1, b_1);
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      as[0] = ra0; as[32 * kRowU4] = ra1; as[64 * kRowU4] = ra2; as[96 * kRowU4] = ra3;
      bs[0] = rb0; bs[32 * kRowU4] = rb1; bs[64 * kRowU4] = rb2; bs[96 * kRowU4] = rb3;
      __syncthreads();
    }
  }

  // 32x32 accumulator layout: register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4,
  // column l%32 of the MFMA tile.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int cl = wn * 64 + j * 32 + r;
      const int64_t col = n0 + cl;
      const int32_t cc = e_cls[kBM + cl];
      const float cv = e_val[kBM + cl];  // FP8 column scale, or the bias
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int64_t row = m0 + rl;
        if (row < M && col < N) {
          float val = acc[i][j][v];
          if constexpr (EPI == kEpiSim) {
            if (T == kTFP8) val = val * (e_val[rl] * cv);
            val = fmaxf(val, 0.f);
            const int32_t rc = e_cls[rl];
            static_cast<float*>(Cv)[row * ldc + col] =
                val * ((rc >= 0 && cc >= 0 && rc != cc) ? kClassFactor : 1.0f);
          } else if constexpr (EPI == kEpiBias) {
            static_cast<float*>(Cv)[row * ldc + col] = val + cv;
          } else {
            static_cast<uint16_t*>(Cv)[row * ldc + col] = to_bf16(gelu_erf(val + cv));
          }
        }
      }
    }
}

template <int T>
hipError_t launch_gemm(const void* a, const float* a_scale, const void* b, const float* b_scale, int64_t m, int64_t n,
                       int32_t ldk, int elem_bytes, float* c, int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows,
                       const int32_t* col_cls, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t ld_bytes = (int64_t)ldk * elem_bytes;
  if (ld_bytes % kSlab) return hipErrorInvalidValue;
  int64_t tiles_m = (m + kBM - 1) / kBM, tiles_n = (n + kBN - 1) / kBN;
  hipLaunchKernelGGL((k_sim_gemm<T, kEpiSim>), dim3((unsigned)(tiles_m * tiles_n)), dim3(256), 0, s,
                     static_cast<const uint8_t*>(a), static_cast<const uint8_t*>(b), m, n, ld_bytes, ld_bytes,
                     ld_bytes, static_cast<void*>(c), ldc, a_scale, b_scale, row_cls, n_cls_rows, col_cls, tiles_m,
                     tiles_n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sim_gemm_f32(const float* a, const float* b, int64_t m, int64_t n, int32_t ldk, float* c,
                               int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows, const int32_t* col_cls,
                               hipStream_t s) {
  return launch_gemm<kT32>(a, nullptr, b, nullptr, m, n, ldk, 4, c, ldc, row_cls, n_cls_rows, col_cls, s);
}

hipError_t launch_sim_gemm_bf16(const uint16_t* a, const uint16_t* b, int64_t m, int64_t n, int32_t ldk, float* c,
                                int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows, const int32_t* col_cls,
                                hipStream_t s) {
  return launch_gemm<kTBF16>(a, nullptr, b, nullptr, m, n, ldk, 2, c, ldc, row_cls, n_cls_rows, col_cls, s);
}

hipError_t launch_sim_gemm_fp8(const uint8_t* a, const float* a_scale, const uint8_t* b, const float* b_scale,
                               int64_t m, int64_t n, int32_t ldk, float* c, int64_t ldc, const int32_t* row_cls,
                               int64_t n_cls_rows, const int32_t* col_cls, hipStream_t s) {
  return launch_gemm<kTFP8>(a, a_scale, b, b_scale, m, n, ldk, 1, c, ldc, row_cls, n_cls_rows, col_cls, s);
}

hipError_t launch_gemm_nt_f32(const float* a, const float* b, int64_t m, int64_t n, int32_t ldk, float* c, int64_t ldc,
                              hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t ld_bytes = (int64_t)ldk * 4;
  if (ld_bytes % kSlab) return hipErrorInvalidValue;
  const int64_t tiles_m = (m + kBM - 1) / kBM, tiles_n = (n + kBN - 1) / kBN;
  hipLaunchKernelGGL((k_sim_gemm<kT32, kEpiBias>), dim3((unsigned)(tiles_m * tiles_n)), dim3(256), 0, s,
                     reinterpret_cast<const uint8_t*>(a), reinterpret_cast<const uint8_t*>(b), m, n, ld_bytes, ld_bytes,
                     ld_bytes, static_cast<void*>(c), ldc, nullptr, nullptr, nullptr, 0, nullptr, tiles_m, tiles_n);
  return hipGetLastError();
}

hipError_t launch_gemm_nt_bf16(const uint16_t* a, int64_t lda, const uint16_t* b, int64_t ldb, int64_t m, int64_t n,
                               int64_t k, void* c, int64_t ldc, const float* bias, bool gelu_bf16_out, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if ((k * 2) % kSlab || (lda * 2) % 16 || (ldb * 2) % 16) return hipErrorInvalidValue;
  int64_t tiles_m = (m + kBM - 1) / kBM, tiles_n = (n + kBN - 1) / kBN;
  if (gelu_bf16_out)
    hipLaunchKernelGGL((k_sim_gemm<kTBF16, kEpiGeluBf16>), dim3((unsigned)(tiles_m * tiles_n)), dim3(256), 0, s,
                       reinterpret_cast<const uint8_t*>(a), reinterpret_cast<const uint8_t*>(b), m, n, k * 2, lda * 2,
                       ldb * 2, c, ldc, nullptr, bias, nullptr, 0, nullptr, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((k_sim_gemm<kTBF16, kEpiBias>), dim3((unsigned)(tiles_m * tiles_n)), dim3(256), 0, s,
                       reinterpret_cast<const uint8_t*>(a), reinterpret_cast<const uint8_t*>(b), m, n, k * 2, lda * 2,
                       ldb * 2, c, ldc, nullptr, bias, nullptr, 0, nullptr, tiles_m, tiles_n);
  return hipGetLastError();
}

}  // namespace farm
