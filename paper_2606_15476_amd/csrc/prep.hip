// prep.hip -- building the device-resident memory and preparing query vectors.
//
// * Validation of a scene (finite descriptors and geometry, non-zero norms,
//   positive extents, unique ids) in one pass plus a hash probe for ids.
// * Row L2 normalisation into an FP32 master, with optional BF16 (round to
//   nearest even) and OCP FP8 e4m3 (per-row scale amax/448, round to nearest
//   even, saturating) copies; rows are zero-padded to a multiple of 128 so that
//   the similarity GEMM never needs a K tail.
// * Geometry in structure-of-arrays form, plus the lateral coordinate
//   h = c . r (viewer right vector) as an unevaluated sum hi + lo of two floats
//   computed with error-free transformations, so that lateral offsets
//   h_i - h_j stay accurate to a few ulps of the offset itself even 100 m from
//   the origin (LeftOf/RightOf evaluate a sigmoid of that offset divided by
//   0.1 m).
#include <math.h>

#include "farm_internal.h"

namespace farm {
namespace {

__device__ inline bool finitef(float v) { return isfinite(v); }

__global__ void k_validate(const float* __restrict__ desc, const float* __restrict__ center,
                           const float* __restrict__ extent, const uint32_t* __restrict__ id, int64_t n,
                           int32_t d, int* __restrict__ flags, uint32_t* __restrict__ table, int64_t table_mask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int bad = 0;
  for (int k = 0; k < 3; ++k) {
    float c = center[i * 3 + k];
    float e = extent[i * 3 + k];
    if (!finitef(c)) bad |= kBadCenter;
    if (!finitef(e) || !(e > 0.f)) bad |= kBadExtent;
  }
  uint32_t v = id[i];
  if (v == FARM_NO_ID) {
    bad |= kBadId;
  } else {
    // open addressing with linear probing; the table holds FARM_NO_ID when empty
    uint32_t h = v * 2654435761u;
    int64_t slot = (int64_t)(h & (uint32_t)table_mask);
    for (int64_t probe = 0; probe <= table_mask; ++probe) {
      uint32_t prev = atomicCAS(&table[slot], FARM_NO_ID, v);
      if (prev == FARM_NO_ID) break;
      if (prev == v) { bad |= kDupId; break; }
      slot = (slot + 1) & table_mask;
    }
  }
  if (bad) atomicOr(flags, bad);
  (void)desc;
  (void)d;
}

// Entity Gaussians and stored views: checks, structure-of-arrays layout and
// the log determinant of each covariance (FP64, cofactor expansion).
__global__ void k_entity_geometry(const float* __restrict__ cov_in, const float* __restrict__ view_in, int64_t n,
                                  float* __restrict__ cov, double* __restrict__ cov_ld, float* __restrict__ view,
                                  int* __restrict__ flags, int* __restrict__ first_bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int bad = 0;
  if (cov_in) {
    float c[6];
    bool fin = true;
    for (int k = 0; k < 6; ++k) {
      c[k] = cov_in[i * 6 + k];
      fin = fin && finitef(c[k]);
      cov[k * n + i] = c[k];
    }
    const double a = c[0], b = c[1], cc = c[2], d = c[3], e = c[4], f = c[5];
    const double m2 = a * d - b * b;                                    // leading 2x2 minor
    const double det = a * (d * f - e * e) - b * (b * f - e * cc) + cc * (b * e - d * cc);
    if (!fin || !(a > 0.0) || !(m2 > 0.0) || !(det > 0.0)) bad |= kBadCov;  // Sylvester's criterion
    cov_ld[i] = det > 0.0 ? log(det) : 0.0;
  }
  if (view_in) {
    float v[12];
    bool fin = true;
    for (int k = 0; k < 12; ++k) {
      v[k] = view_in[i * 12 + k];
      fin = fin && finitef(v[k]);
      view[k * n + i] = v[k];
    }
    // the rotation rows (right, down, forward) must be orthonormal
    bool ortho = true;
    for (int r = 0; r < 3; ++r)
      for (int t = r; t < 3; ++t) {
        const double g = (double)v[3 + 3 * r] * v[3 + 3 * t] + (double)v[4 + 3 * r] * v[4 + 3 * t] +
                         (double)v[5 + 3 * r] * v[5 + 3 * t];
        ortho = ortho && fabs(g - (r == t ? 1.0 : 0.0)) <= 1e-3;
      }
    if (!fin || !ortho) bad |= kBadView;
  }
  if (bad) {
    atomicOr(flags, bad);
    atomicMin(first_bad, (int)i);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP FP8 e4m3 ("e4m3fn": bias 7, no infinities, max 448), round to nearest
// even, saturating at +-448.
__device__ inline uint8_t fp8_e4m3_rne(float f) {
  uint8_t sign = (__float_as_uint(f) >> 31) ? 0x80 : 0x00;
  float a = fabsf(f);
  if (!(a < kFp8Max)) return sign | 0x7E;
  if (a < 0.015625f) {                      // below 2^-6: subnormal grid of 2^-9
    float m = rintf(a * 512.0f);            // exact scaling, RNE
    return sign | (uint8_t)m;               // m == 8 is the smallest normal (code 0x08)
  }
  int e;
  float fr = frexpf(a, &e);                 // a = fr * 2^e, fr in [0.5, 1)
  float m = rintf((fr * 2.0f - 1.0f) * 8.0f);  // mantissa of 1.mmm, RNE
  int ex = e - 1;
  if (m >= 8.0f) { m = 0.0f; ex += 1; }
  int code = ((ex + 7) << 3) | (int)m;
  if (code > 0x7E) code = 0x7E;
  return sign | (uint8_t)code;
}

__device__ inline float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float fp8_e4m3_to_float(uint8_t c) {
  float sgn = (c & 0x80) ? -1.0f : 1.0f;
  int e = (c >> 3) & 0xF, m = c & 7;
  if (e == 0) return sgn * (float)m * 0.001953125f;  // m * 2^-9
  return sgn * ldexpf(1.0f + (float)m * 0.125f, e - 7);
}

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// One wave per row (four rows per block, shuffle reductions): L2 norm, the
// FP32 copy, then the reduced-precision copies with the 2-norms of their
// values and of their rounding errors (accumulated in FP32 and rounded up by a
// relative 1e-3 margin; they feed an error bound, never a score).
constexpr int kNormRows = 4;
__global__ __launch_bounds__(64 * kNormRows) void k_normalize_rows(const float* __restrict__ src, int64_t rows,
                                                                   int32_t d, int32_t ldk, float* __restrict__ dst,
                                                                   LowPrecRows lp, int* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * kNormRows + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* s = src + row * (int64_t)d;
  float ss = 0.f;
  int bad = 0;
  for (int k = lane; k < d; k += 64) {
    const float v = s[k];
    if (!isfinite(v)) bad = 1;
    ss = fmaf(v, v, ss);
  }
  const bool anybad = __ballot(bad) != 0;
  const float nrm = sqrtf(wave_sum_f(ss));
  const bool zero = !(nrm > 0.f) || !isfinite(nrm);
  if (lane == 0 && (anybad || zero)) atomicOr(flags, anybad ? kBadDesc : kZeroNorm);
  const float inv = zero ? 0.f : 1.0f / nrm;
  float* o = dst + row * (int64_t)ldk;
  float amax = 0.f, eb = 0.f, nb = 0.f;
  for (int k = lane; k < ldk; k += 64) {
    const float v = (k < d && !zero) ? s[k] * inv : 0.f;
    o[k] = v;
    amax = fmaxf(amax, fabsf(v));
    if (lp.bf16) {
      const uint16_t b = bf16_rne(v);
      lp.bf16[row * (int64_t)ldk + k] = b;
      const float r = bf16_to_float(b);
      eb = fmaf(r - v, r - v, eb);
      nb = fmaf(r, r, nb);
    }
  }
  if (lp.bf16) {
    const float e2 = wave_sum_f(eb), n2 = wave_sum_f(nb);
    if (lane == 0) {
      if (lp.err_bf16) lp.err_bf16[row] = sqrtf(e2) * 1.001f + 1e-30f;
      if (lp.nrm_bf16) lp.nrm_bf16[row] = sqrtf(n2) * 1.001f;
    }
  }
  if (!lp.fp8) return;
  const float am = wave_max_f(amax);
  const float scale = am > 0.f ? am / kFp8Max : 1.0f;
  if (lane == 0) lp.fp8_scale[row] = scale;
  float ef = 0.f, nf = 0.f;
  for (int k = lane; k < ldk; k += 64) {
    const float v = (k < d && !zero) ? s[k] * inv : 0.f;
    const uint8_t c = fp8_e4m3_rne(v / scale);
    lp.fp8[row * (int64_t)ldk + k] = c;
    const float r = fp8_e4m3_to_float(c) * scale;
    ef = fmaf(r - v, r - v, ef);
    nf = fmaf(r, r, nf);
  }
  const float e2 = wave_sum_f(ef), n2 = wave_sum_f(nf);
  if (lane == 0) {
    if (lp.err_fp8) lp.err_fp8[row] = sqrtf(e2) * 1.001f + 1e-30f;
    if (lp.nrm_fp8) lp.nrm_fp8[row] = sqrtf(n2) * 1.001f;
  }
}

// Error-free transformations (Knuth two-sum, FMA two-product).  They rely on
// every product and sum being rounded on its own: no contraction into FMAs.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ void k_geometry(const float* __restrict__ center, const float* __restrict__ extent, int64_t n, float rx,
                           float ry, float* __restrict__ x, float* __restrict__ y, float* __restrict__ z,
                           float* __restrict__ hhi, float* __restrict__ hlo, float* __restrict__ ext,
                           float* __restrict__ vz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float cx = center[i * 3 + 0], cy = center[i * 3 + 1], cz = center[i * 3 + 2];
  x[i] = cx;
  y[i] = cy;
  z[i] = cz;
  // c . u as an unevaluated pair hi + lo (FMA two-products, two-sums), for the
  // right axis u = r (entries 0..n-1) and the viewing direction u = (-r_y, r_x)
  // (entries n..2n-1)
  auto dot2 = [&](float ux, float uy, float& hi, float& lo) {
#pragma clang fp contract(off)
    float p1 = cx * ux, e1 = fmaf(cx, ux, -p1);
    float p2 = cy * uy, e2 = fmaf(cy, uy, -p2);
    float s, e3;
    two_sum(p1, p2, s, e3);
    lo = e1 + e2 + e3;
    two_sum(s, lo, hi, lo);
  };
  dot2(rx, ry, hhi[i], hlo[i]);
  dot2(-ry, rx, hhi[n + i], hlo[n + i]);
  for (int k = 0; k < 3; ++k) ext[k * n + i] = extent[i * 3 + k];
  // bottom and top faces, scaled by 4 (exact): one rounding each, as z -+ e/2
  const float half = 0.5f * extent[i * 3 + 2];
  vz[i] = 4.0f * (cz - half);
  vz[n + i] = 4.0f * (cz + half);
}

}  // namespace

hipError_t launch_validate_memory(const float* desc, const float* center, const float* extent, const uint32_t* id,
                                  int64_t n, int32_t d, int* flags, uint32_t* table, int64_t table_size,
                                  hipStream_t s) {
  int64_t blocks = (table_size + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, table, table_size, FARM_NO_ID);
  blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, s, desc, center, extent, id, n, d, flags,
                     table, table_size - 1);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(const float* src, int64_t rows, int32_t d, int32_t ldk, float* dst_f32,
                                 const LowPrecRows& lp, int* flags, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize_rows, dim3((unsigned)((rows + kNormRows - 1) / kNormRows)), dim3(64 * kNormRows), 0, s,
                     src, rows, d, ldk, dst_f32, lp, flags);
  return hipGetLastError();
}

hipError_t launch_entity_geometry(const float* cov_in, const float* view_in, int64_t n, float* cov, double* cov_ld,
                                  float* view, int* flags, int* first_bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_entity_geometry, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cov_in, view_in, n, cov,
                     cov_ld, view, flags, first_bad);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p),
                     n, (uint32_t)v);
  return hipGetLastError();
}

hipError_t launch_geometry(const float* center, const float* extent, int64_t n, float rx, float ry, float* vz,
                           float* x, float* y, float* z, float* hr_hi, float* hr_lo, float* ext, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_geometry, dim3((unsigned)blocks), dim3(256), 0, s, center, extent, n, rx, ry, x, y, z, hr_hi,
                     hr_lo, ext, vz);
  return hipGetLastError();
}

}  // namespace farm
