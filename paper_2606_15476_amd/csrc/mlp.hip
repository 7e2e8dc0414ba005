// mlp.hip -- the anchor proposal network: BF16 training and inference kernels.
//
// Network (per (target o, anchor a) pair; nine logits, one per predicate with a list):
//   x  = [u_o (dp) | u_a (dp) | g(o, a) / 4 m (12) | 0 pad]   dp = d rounded up to 64
//   h1 = GELU(W1 x + b1),  h2 = GELU(W2 h1 + b2),  y = W3 h2 + b3
//   g  = [c_o - c_a, e_o, e_a, |c_o - c_a|, (c_o - c_a) . r, bottom_o - top_a]
// FP32 master weights and AdamW moments; the GEMMs run on BF16 copies of the
// weights and BF16 activations with FP32 accumulation (MFMA).  Loss: mean
// binary cross-entropy with logits on the labelled predicate of each pair.
//
// Batch layout: rows padded to a multiple of 64 (zero rows) so that the
// weight-gradient GEMMs, which contract over the batch, see whole K slabs.
// Backward: dY = (sigmoid(y_p) - label) / B on the labelled logit;
//   dW3 = dY^T h2, dh2 = dY W3, dZ2 = dh2 * GELU'(Z2), dW2 = dZ2^T h1,
//   dh1 = dZ2 W2, dZ1 = dh1 * GELU'(Z1), dW1 = dZ1^T x, db = column sums.
// The last step's batch tensors (Z1, A1, Z2, A2, Y, dZ2, dh1, dZ1) stay in
// their buffers until the next step (farm_mlp_get_batch copies them out).
#include <math.h>
#include <string.h>

#include <new>
#include <type_traits>
#include <vector>

#include "farm_internal.h"

namespace farm {
namespace {

constexpr int kNPred = FARM_NUM_PROP_PRED;  // one output per predicate
constexpr float kGeoScale = 0.25f;  // geometry features in units of 4 m

__device__ inline uint16_t bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float gelu(float v) { return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float v) {
  return 0.5f * (1.0f + erff(v * 0.70710678118654752f)) + v * 0.39894228040143268f * expf(-0.5f * v * v);
}

// 12 relative-geometry features of (o, a), scaled by 1/4 m.
__device__ inline float geo_feature(int f, int64_t o, int64_t a, const float* x, const float* y, const float* z,
                                    const float* ext, int64_t n, float rx, float ry) {
  const float dx = x[o] - x[a], dy = y[o] - y[a], dz = z[o] - z[a];
  float v;
  switch (f) {
    case 0: v = dx; break;
    case 1: v = dy; break;
    case 2: v = dz; break;
    case 3: case 4: case 5: v = ext[(f - 3) * n + o]; break;
    case 6: case 7: case 8: v = ext[(f - 6) * n + a]; break;
    case 9: v = sqrtf(dx * dx + dy * dy + dz * dz); break;
    case 10: v = dx * rx + dy * ry; break;
    default: v = (z[o] - 0.5f * ext[2 * n + o]) - (z[a] + 0.5f * ext[2 * n + a]); break;
  }
  return v * kGeoScale;
}

__global__ void k_mlp_inputs(const float* __restrict__ dn, int32_t ldk, int32_t d, int32_t dp, int32_t ldx,
                             const int32_t* __restrict__ o_idx, const int32_t* __restrict__ a_idx, int32_t nb,
                             const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
                             const float* __restrict__ ext, int64_t n, float rx, float ry,
                             uint16_t* __restrict__ X) {
  const int32_t b = blockIdx.x;
  const int64_t o = o_idx[b], a = a_idx[b];
  uint16_t* row = X + (int64_t)b * ldx;
  for (int k = threadIdx.x; k < ldx; k += blockDim.x) {
    float v = 0.f;
    if (k < d) v = dn[o * ldk + k];
    else if (k >= dp && k < dp + d) v = dn[a * ldk + (k - dp)];
    else if (k >= 2 * dp && k < 2 * dp + 12) v = geo_feature(k - 2 * dp, o, a, x, y, z, ext, n, rx, ry);
    row[k] = bf16(v);
  }
}

__global__ void k_zero_u16(uint16_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// 32x32 tiled transpose: dst[c][r] = src[r][c]
__global__ void k_transpose_u16(const uint16_t* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                                uint16_t* __restrict__ dst, int64_t ldd) {
  __shared__ uint16_t tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int i = threadIdx.y; i < 32; i += blockDim.y) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    tile[i][threadIdx.x] = (r < rows && c < cols) ? src[r * lds + c] : 0;
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += blockDim.y) {
    const int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (c < cols && r < rows) dst[c * ldd + r] = tile[threadIdx.x][i];
  }
}

__global__ void k_gelu_rows(const float* __restrict__ Z, uint16_t* __restrict__ A, int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) A[i] = bf16(gelu(Z[i]));
}

// y[b][c] = sum_k A2[b][k] W3r[c][k] + b3[c]
__global__ void k_head(const uint16_t* __restrict__ A2, const float* __restrict__ W3r, const float* __restrict__ b3,
                       int32_t nb, int32_t h, float* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * kNPred) return;
  const int64_t b = t / kNPred;
  const int c = (int)(t % kNPred);
  float acc = b3[c];
  for (int k = 0; k < h; ++k) acc = fmaf(from_bf16(A2[b * h + k]), W3r[c * h + k], acc);
  Y[t] = acc;
}

// per-row BCE loss on the labelled predicate and its gradient dY (mean over nb)
__global__ void k_bce(const float* __restrict__ Y, const int32_t* __restrict__ pred, const float* __restrict__ label,
                      int32_t nb, float* __restrict__ dY, float* __restrict__ loss_part) {
  __shared__ float red[256];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (b < nb) {
    const int p = pred[b];
    if (p >= 0 && p < kNPred) {  // a pair of a predicate without an output contributes nothing
      const float t = label[b], v = Y[b * kNPred + p];
      l = fmaxf(v, 0.f) - v * t + log1pf(expf(-fabsf(v)));
      for (int c = 0; c < kNPred; ++c) dY[b * kNPred + c] = c == p ? (1.0f / (1.0f + expf(-v)) - t) / (float)nb : 0.f;
    } else {
      for (int c = 0; c < kNPred; ++c) dY[b * kNPred + c] = 0.f;
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const float* __restrict__ part, int32_t nparts, int32_t nb, float* __restrict__ out) {
  if (threadIdx.x != 0) return;
  float s = 0.f;
  for (int i = 0; i < nparts; ++i) s += part[i];
  *out = s / (float)nb;
}

// Batch reductions run in two deterministic stages: chunks of kRedRows rows
// give partial sums (one thread per output column and chunk), then the
// partials are added in chunk order.
constexpr int kRedRows = 128;

// partial gW3[c][k] (k < h) and gb3[c] (k == h) over rows of chunk blockIdx.y
__global__ void k_head_grad_part(const float* __restrict__ dY, const uint16_t* __restrict__ A2, int32_t nb,
                                 int32_t h, float* __restrict__ part) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int cols = kNPred * (h + 1);
  if (t >= cols) return;
  const int c = t / (h + 1), k = t % (h + 1);
  const int64_t b0 = (int64_t)blockIdx.y * kRedRows, b1 = b0 + kRedRows < nb ? b0 + kRedRows : nb;
  float acc = 0.f;
  if (k < h)
    for (int64_t b = b0; b < b1; ++b) acc = fmaf(dY[b * kNPred + c], from_bf16(A2[b * h + k]), acc);
  else
    for (int64_t b = b0; b < b1; ++b) acc += dY[b * kNPred + c];
  part[(int64_t)blockIdx.y * cols + t] = acc;
}

// partial column sums of dZ over rows of chunk blockIdx.y
__global__ void k_colsum_part(const uint16_t* __restrict__ dZ, int32_t nb, int32_t h, float* __restrict__ part) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= h) return;
  const int64_t b0 = (int64_t)blockIdx.y * kRedRows, b1 = b0 + kRedRows < nb ? b0 + kRedRows : nb;
  float acc = 0.f;
  for (int64_t b = b0; b < b1; ++b) acc += from_bf16(dZ[b * h + k]);
  part[(int64_t)blockIdx.y * h + k] = acc;
}

// out[t] = sum over chunks of part[chunk][t], in chunk order; the head's
// columns are split into gW3 ([c][h]) and gb3 ([c]) when w3 is set
__global__ void k_sum_chunks(const float* __restrict__ part, int32_t chunks, int32_t cols, int32_t h, bool w3,
                             float* __restrict__ out, float* __restrict__ out_b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cols) return;
  float acc = 0.f;
  for (int i = 0; i < chunks; ++i) acc += part[(int64_t)i * cols + t];
  if (!w3) {
    out[t] = acc;
  } else {
    const int c = t / (h + 1), k = t % (h + 1);
    if (k < h) out[c * h + k] = acc;
    else out_b[c] = acc;
  }
}

// dZ2[b][k] = (sum_c dY[b][c] W3r[c][k]) * GELU'(Z2[b][k])
__global__ void k_head_back(const float* __restrict__ dY, const float* __restrict__ W3r, const float* __restrict__ Z2,
                            int32_t nb, int32_t h, uint16_t* __restrict__ dZ) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * h) return;
  const int64_t b = t / h;
  const int k = (int)(t % h);
  float acc = 0.f;
  for (int c = 0; c < kNPred; ++c) acc = fmaf(dY[b * kNPred + c], W3r[c * h + k], acc);
  dZ[t] = bf16(acc * gelu_grad(Z2[t]));
}

// dZ1 = dA1 * GELU'(Z1)
__global__ void k_gelu_back(const float* __restrict__ dA, const float* __restrict__ Z, int64_t total,
                            uint16_t* __restrict__ dZ) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) dZ[i] = bf16(dA[i] * gelu_grad(Z[i]));
}

__global__ void k_adamw(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float wd, float c1,
                        float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
}

__global__ void k_to_bf16(const float* __restrict__ src, int64_t n, uint16_t* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = bf16(src[i]);
}

__global__ void k_round_bf16(const float* __restrict__ src, int64_t n, float* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = from_bf16(bf16(src[i]));
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// host-side deterministic initialisation: splitmix64 -> uniform(-s, s)
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

// Refresh the BF16 weight copies from the FP32 masters.
static hipError_t refresh_copies(farm_mlp* m, hipStream_t s) {
  const int64_t h = m->h;
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(h * m->ldx)), dim3(256), 0, s, m->W1, h * m->ldx, m->W1b);
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(h * h)), dim3(256), 0, s, m->W2, h * h, m->W2b);
  hipLaunchKernelGGL(k_transpose_u16, dim3(blocks(h, 32), blocks(h, 32)), dim3(32, 8), 0, s, m->W2b, h, h, h, m->W2bT,
                     h);
  hipLaunchKernelGGL(k_round_bf16, dim3(blocks(kNPred * h)), dim3(256), 0, s, m->W3, (int64_t)kNPred * h, m->W3r);
  return hipGetLastError();
}

// Forward pass of nb pairs: inputs, Z1/A1, Z2/A2, logits Y.  With keep_pre the
// pre-activations are stored (training); otherwise GELU is fused into the GEMMs.
static hipError_t forward(farm_mlp* m, const farm_memory* mem, int32_t nb, const int32_t* o_idx, const int32_t* a_idx,
                          bool keep_pre, float* Y, hipStream_t s) {
  const int64_t h = m->h, ldx = m->ldx;
  hipLaunchKernelGGL(k_mlp_inputs, dim3((unsigned)nb), dim3(256), 0, s, mem->dn, mem->ldk, m->d, m->dp, m->ldx, o_idx,
                     a_idx, nb, mem->x, mem->y, mem->z, mem->ext, mem->n, mem->rx, mem->ry, m->X);
  hipError_t e;
  if (keep_pre) {
    if ((e = launch_gemm_nt_bf16(m->X, ldx, m->W1b, ldx, nb, h, ldx, m->Z1, h, m->b1, false, s))) return e;
    hipLaunchKernelGGL(k_gelu_rows, dim3(blocks((int64_t)nb * h)), dim3(256), 0, s, m->Z1, m->A1, (int64_t)nb * h);
    if ((e = launch_gemm_nt_bf16(m->A1, h, m->W2b, h, nb, h, h, m->Z2, h, m->b2, false, s))) return e;
    hipLaunchKernelGGL(k_gelu_rows, dim3(blocks((int64_t)nb * h)), dim3(256), 0, s, m->Z2, m->A2, (int64_t)nb * h);
  } else {
    if ((e = launch_gemm_nt_bf16(m->X, ldx, m->W1b, ldx, nb, h, ldx, m->A1, h, m->b1, true, s))) return e;
    if ((e = launch_gemm_nt_bf16(m->A1, h, m->W2b, h, nb, h, h, m->A2, h, m->b2, true, s))) return e;
  }
  hipLaunchKernelGGL(k_head, dim3(blocks((int64_t)nb * kNPred)), dim3(256), 0, s, m->A2, m->W3r, m->b3, nb, m->h, Y);
  return hipGetLastError();
}

}  // namespace farm

using namespace farm;

namespace {

farm_status alloc_mlp(farm_mlp* m) {
  auto take = [&](auto** p, size_t count) -> bool {
    void* v = nullptr;
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
    if (hipMalloc(&v, (count ? count : 1) * sizeof(T)) != hipSuccess) return false;
    m->allocs.push_back(v);
    m->bytes += count * sizeof(T);
    *p = static_cast<T*>(v);
    return true;
  };
  const size_t h = m->h, ldx = m->ldx, B = m->bpad;
  const size_t np = h * ldx + h + h * h + h + kNPred * h + kNPred;
  m->n_par = (int64_t)np;
  bool ok = take(&m->par, np) && take(&m->grad, np) && take(&m->m1, np) && take(&m->m2, np) &&
            take(&m->W1b, h * ldx) && take(&m->W2b, h * h) && take(&m->W2bT, h * h) && take(&m->W3r, kNPred * h) &&
            take(&m->X, B * ldx) && take(&m->XT, ldx * B) && take(&m->Z1, B * h) && take(&m->Z2, B * h) &&
            take(&m->A1, B * h) && take(&m->A1T, h * B) && take(&m->A2, B * h) && take(&m->Y, B * kNPred) &&
            take(&m->dY, B * kNPred) && take(&m->dA, B * h) && take(&m->dZ, B * h) && take(&m->dZ1, B * h) &&
            take(&m->dZT, h * B) &&
            take(&m->loss_part, B / 256 + 1) &&
            take(&m->red_part, (B / kRedRows + 1) * (kNPred * (h + 1)));
  if (!ok) {
    (void)hipGetLastError();
    return FARM_ERR_OOM;
  }
  float* p = m->par;
  m->W1 = p; p += h * ldx; m->b1 = p; p += h; m->W2 = p; p += h * h; m->b2 = p; p += h; m->W3 = p; p += kNPred * h;
  m->b3 = p;
  p = m->grad;
  m->gW1 = p; p += h * ldx; m->gb1 = p; p += h; m->gW2 = p; p += h * h; m->gb2 = p; p += h; m->gW3 = p;
  p += kNPred * h; m->gb3 = p;
  return FARM_OK;
}

void free_mlp(farm_mlp* m) {
  for (void* p : m->allocs) (void)hipFree(p);
  m->allocs.clear();
}

farm_status host_io(const farm_mlp* m, float* base, float* W1, float* b1, float* W2, float* b2, float* W3, float* b3,
                    bool to_host) {
  const size_t h = m->h, ldx = m->ldx;
  struct Part { float* host; size_t off, n; } parts[6] = {
      {W1, 0, h * ldx}, {b1, h * ldx, h}, {W2, h * ldx + h, h * h}, {b2, h * ldx + h + h * h, h},
      {W3, h * ldx + 2 * h + h * h, kNPred * h}, {b3, h * ldx + 2 * h + h * h + kNPred * h, kNPred}};
  if (hipDeviceSynchronize() != hipSuccess) { set_error("synchronize failed"); return FARM_ERR_HIP; }
  for (auto& pt : parts) {
    if (!pt.host) continue;
    hipError_t e = to_host ? hipMemcpy(pt.host, base + pt.off, pt.n * sizeof(float), hipMemcpyDeviceToHost)
                           : hipMemcpy(base + pt.off, pt.host, pt.n * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "weight copy");
  }
  return FARM_OK;
}

}  // namespace

extern "C" {

farm_status farm_mlp_create(int32_t d, int32_t max_batch, uint64_t seed, farm_mlp** out) {
  try {
    if (!out) { set_error("out is NULL"); return FARM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (d < 1 || d > 8192 || max_batch < 1 || max_batch > (1 << 22)) {
      set_error("invalid network shape (d %d, max_batch %d)", d, max_batch);
      return FARM_ERR_INVALID_ARG;
    }
    auto* m = new (std::nothrow) farm_mlp();
    if (!m) { set_error("host allocation failed"); return FARM_ERR_OOM; }
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; set_error("hipGetDevice failed"); return FARM_ERR_HIP; }
    m->d = d;
    m->dp = (int32_t)round_up(d, 64);
    m->ldx = 2 * m->dp + 64;
    m->h = FARM_MLP_HIDDEN;
    m->bmax = max_batch;
    m->bpad = (int32_t)round_up(max_batch, 256);
    farm_status st = alloc_mlp(m);
    if (st) { free_mlp(m); delete m; set_error("device allocation for the proposal network failed"); return st; }
    // initial weights: uniform(-sqrt(3/fan_in), +); biases 0; padding input columns 0
    const size_t h = m->h, ldx = m->ldx;
    std::vector<float> W1(h * ldx, 0.f), W2(h * h), W3(kNPred * h), z1(h, 0.f), z3(kNPred, 0.f);
    uint64_t state = seed;
    auto uni = [&](float s) { return s * (2.0f * (float)((splitmix(state) >> 11) * (1.0 / 9007199254740992.0)) - 1.0f); };
    const int in_used = 2 * d + 12;
    const float s1 = sqrtf(3.0f / (float)in_used), s2 = sqrtf(3.0f / (float)h);
    for (size_t j = 0; j < h; ++j)
      for (int k = 0; k < ldx; ++k) {
        const bool used = k < d || (k >= m->dp && k < m->dp + d) || (k >= 2 * m->dp && k < 2 * m->dp + 12);
        W1[j * ldx + k] = used ? uni(s1) : 0.f;
      }
    for (auto& v : W2) v = uni(s2);
    for (auto& v : W3) v = uni(s2);
    if ((st = host_io(m, m->par, W1.data(), z1.data(), W2.data(), z1.data(), W3.data(), z3.data(), false))) {
      free_mlp(m);
      delete m;
      return st;
    }
    const bool cleared = hipMemset(m->m1, 0, sizeof(float) * m->n_par) == hipSuccess &&
                         hipMemset(m->m2, 0, sizeof(float) * m->n_par) == hipSuccess &&
                         hipMemset(m->grad, 0, sizeof(float) * m->n_par) == hipSuccess &&
                         hipMemset(m->X, 0, sizeof(uint16_t) * (size_t)m->bpad * ldx) == hipSuccess &&
                         hipMemset(m->dZ, 0, sizeof(uint16_t) * (size_t)m->bpad * h) == hipSuccess &&
                         hipMemset(m->dZ1, 0, sizeof(uint16_t) * (size_t)m->bpad * h) == hipSuccess &&
                         hipMemset(m->A1, 0, sizeof(uint16_t) * (size_t)m->bpad * h) == hipSuccess;
    if (!cleared || refresh_copies(m, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      free_mlp(m);
      delete m;
      set_error("initialising the proposal network failed");
      return FARM_ERR_HIP;
    }
    *out = m;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_mlp_create");
    return FARM_ERR_OOM;
  }
}

farm_status farm_mlp_free(farm_mlp* m) {
  if (!m) return FARM_OK;
  (void)hipDeviceSynchronize();
  free_mlp(m);
  delete m;
  return FARM_OK;
}

farm_status farm_mlp_shape(const farm_mlp* m, int32_t* in_dim, int32_t* hidden) {
  if (!m) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  if (in_dim) *in_dim = m->ldx;
  if (hidden) *hidden = m->h;
  return FARM_OK;
}

farm_status farm_mlp_get_weights(const farm_mlp* m, float* W1, float* b1, float* W2, float* b2, float* W3, float* b3) {
  if (!m) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  return host_io(m, m->par, W1, b1, W2, b2, W3, b3, true);
}

farm_status farm_mlp_get_grads(const farm_mlp* m, float* W1, float* b1, float* W2, float* b2, float* W3, float* b3) {
  if (!m) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  return host_io(m, m->grad, W1, b1, W2, b2, W3, b3, true);
}

farm_status farm_mlp_get_batch(const farm_mlp* m, int32_t nb, float* Z1, uint16_t* A1, float* Z2, uint16_t* A2,
                              float* Y, uint16_t* dZ2, float* dA1, uint16_t* dZ1) {
  if (!m) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  if (nb < 1 || nb > m->bmax) { set_error("nb = %d outside [1, %d]", nb, m->bmax); return FARM_ERR_INVALID_ARG; }
  if (hipDeviceSynchronize() != hipSuccess) { set_error("synchronize failed"); return FARM_ERR_HIP; }
  const size_t hs = (size_t)nb * m->h;
  struct Part { void* host; const void* dev; size_t bytes; } parts[8] = {
      {Z1, m->Z1, hs * sizeof(float)},   {A1, m->A1, hs * sizeof(uint16_t)},
      {Z2, m->Z2, hs * sizeof(float)},   {A2, m->A2, hs * sizeof(uint16_t)},
      {Y, m->Y, (size_t)nb * kNPred * sizeof(float)},
      {dZ2, m->dZ, hs * sizeof(uint16_t)}, {dA1, m->dA, hs * sizeof(float)}, {dZ1, m->dZ1, hs * sizeof(uint16_t)}};
  for (auto& pt : parts) {
    if (!pt.host) continue;
    hipError_t e = hipMemcpy(pt.host, pt.dev, pt.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch copy");
  }
  return FARM_OK;
}

farm_status farm_mlp_set_weights(farm_mlp* m, const float* W1, const float* b1, const float* W2, const float* b2,
                                 const float* W3, const float* b3) {
  if (!m) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  farm_status st = host_io(m, m->par, const_cast<float*>(W1), const_cast<float*>(b1), const_cast<float*>(W2),
                           const_cast<float*>(b2), const_cast<float*>(W3), const_cast<float*>(b3), false);
  if (st) return st;
  if (refresh_copies(m, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("refreshing weight copies failed");
    return FARM_ERR_HIP;
  }
  return FARM_OK;
}

farm_status farm_mlp_inputs(farm_mlp* m, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                            const int32_t* a_idx, uint16_t* x_out, void* stream) {
  if (!m || !mem || !o_idx || !a_idx || !x_out) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
  if (mem->d != m->d || nb < 1 || nb > m->bmax) { set_error("shape mismatch"); return FARM_ERR_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mlp_inputs, dim3((unsigned)nb), dim3(256), 0, s, mem->dn, mem->ldk, m->d, m->dp, m->ldx, o_idx,
                     a_idx, nb, mem->x, mem->y, mem->z, mem->ext, mem->n, mem->rx, mem->ry, x_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FARM_OK : hip_fail(e, "inputs");
}

farm_status farm_mlp_logits(farm_mlp* m, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                            const int32_t* a_idx, float* logits, void* stream) {
  if (!m || !mem || !o_idx || !a_idx || !logits) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
  if (mem->d != m->d || nb < 1 || nb > m->bmax) { set_error("shape mismatch"); return FARM_ERR_INVALID_ARG; }
  hipError_t e = forward(m, mem, nb, o_idx, a_idx, false, logits, (hipStream_t)stream);
  return e == hipSuccess ? FARM_OK : hip_fail(e, "forward");
}

farm_status farm_mlp_step(farm_mlp* m, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                          const int32_t* a_idx, const int32_t* pred, const float* label, float lr, float weight_decay,
                          int32_t update, float* loss_out, void* stream) {
  try {
    if (!m || !mem || !o_idx || !a_idx || !pred || !label) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
    if (mem->d != m->d || nb < 1 || nb > m->bmax) { set_error("shape mismatch"); return FARM_ERR_INVALID_ARG; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t h = m->h, ldx = m->ldx;
    const int64_t nbp = round_up(nb, 64);
    hipError_t e;
    // zero the padding rows [nb, nbp) of the inputs and of dZ (they enter batch contractions)
    if (nbp > nb) {
      hipLaunchKernelGGL(k_zero_u16, dim3(blocks((nbp - nb) * ldx)), dim3(256), 0, s, m->X + nb * ldx,
                         (nbp - nb) * ldx);
      hipLaunchKernelGGL(k_zero_u16, dim3(blocks((nbp - nb) * h)), dim3(256), 0, s, m->A1 + nb * h, (nbp - nb) * h);
    }
    if ((e = forward(m, mem, nb, o_idx, a_idx, true, m->Y, s))) return hip_fail(e, "forward");
    const unsigned nparts = blocks(nb);
    hipLaunchKernelGGL(k_bce, dim3(nparts), dim3(256), 0, s, m->Y, pred, label, nb, m->dY, m->loss_part);
    if (loss_out) hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, m->loss_part, (int32_t)nparts, nb, loss_out);
    // head
    const unsigned chunks = (unsigned)((nb + kRedRows - 1) / kRedRows);
    const int32_t head_cols = kNPred * (int32_t)(h + 1);
    hipLaunchKernelGGL(k_head_grad_part, dim3(blocks(head_cols), chunks), dim3(256), 0, s, m->dY, m->A2, nb,
                       (int32_t)h, m->red_part);
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(head_cols)), dim3(256), 0, s, m->red_part, (int32_t)chunks,
                       head_cols, (int32_t)h, true, m->gW3, m->gb3);
    hipLaunchKernelGGL(k_head_back, dim3(blocks((int64_t)nb * h)), dim3(256), 0, s, m->dY, m->W3r, m->Z2, nb,
                       (int32_t)h, m->dZ);
    if (nbp > nb)
      hipLaunchKernelGGL(k_zero_u16, dim3(blocks((nbp - nb) * h)), dim3(256), 0, s, m->dZ + nb * h, (nbp - nb) * h);
    // layer 2
    hipLaunchKernelGGL(k_colsum_part, dim3(blocks(h), chunks), dim3(256), 0, s, m->dZ, nb, (int32_t)h, m->red_part);
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(h)), dim3(256), 0, s, m->red_part, (int32_t)chunks, (int32_t)h,
                       (int32_t)h, false, m->gb2, nullptr);
    hipLaunchKernelGGL(k_transpose_u16, dim3(blocks(h, 32), blocks(nbp, 32)), dim3(32, 8), 0, s, m->dZ, nbp, h, h,
                       m->dZT, nbp);
    hipLaunchKernelGGL(k_transpose_u16, dim3(blocks(h, 32), blocks(nbp, 32)), dim3(32, 8), 0, s, m->A1, nbp, h, h,
                       m->A1T, nbp);
    if ((e = launch_gemm_nt_bf16(m->dZT, nbp, m->A1T, nbp, h, h, nbp, m->gW2, h, nullptr, false, s)))
      return hip_fail(e, "dW2");
    if ((e = launch_gemm_nt_bf16(m->dZ, h, m->W2bT, h, nb, h, h, m->dA, h, nullptr, false, s)))
      return hip_fail(e, "dA1");
    // layer 1 (dZ1 in a buffer of its own, so that dZ2 stays readable after the step)
    hipLaunchKernelGGL(k_gelu_back, dim3(blocks((int64_t)nb * h)), dim3(256), 0, s, m->dA, m->Z1, (int64_t)nb * h,
                       m->dZ1);
    if (nbp > nb)
      hipLaunchKernelGGL(k_zero_u16, dim3(blocks((nbp - nb) * h)), dim3(256), 0, s, m->dZ1 + nb * h, (nbp - nb) * h);
    hipLaunchKernelGGL(k_colsum_part, dim3(blocks(h), chunks), dim3(256), 0, s, m->dZ1, nb, (int32_t)h, m->red_part);
    hipLaunchKernelGGL(k_sum_chunks, dim3(blocks(h)), dim3(256), 0, s, m->red_part, (int32_t)chunks, (int32_t)h,
                       (int32_t)h, false, m->gb1, nullptr);
    hipLaunchKernelGGL(k_transpose_u16, dim3(blocks(h, 32), blocks(nbp, 32)), dim3(32, 8), 0, s, m->dZ1, nbp, h, h,
                       m->dZT, nbp);
    hipLaunchKernelGGL(k_transpose_u16, dim3(blocks(ldx, 32), blocks(nbp, 32)), dim3(32, 8), 0, s, m->X, nbp, ldx,
                       ldx, m->XT, nbp);
    if ((e = launch_gemm_nt_bf16(m->dZT, nbp, m->XT, nbp, h, ldx, nbp, m->gW1, ldx, nullptr, false, s)))
      return hip_fail(e, "dW1");
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "backward");
    if (!update) return FARM_OK;
    m->step += 1;
    const float b1c = 0.9f, b2c = 0.999f;
    const float c1 = 1.0f - powf(b1c, (float)m->step), c2 = 1.0f - powf(b2c, (float)m->step);
    hipLaunchKernelGGL(k_adamw, dim3(blocks(m->n_par)), dim3(256), 0, s, m->par, m->grad, m->m1, m->m2, m->n_par, lr,
                       b1c, b2c, 1e-8f, weight_decay, c1, c2);
    if ((e = refresh_copies(m, s)) != hipSuccess) return hip_fail(e, "weight copies");
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_mlp_step");
    return FARM_ERR_HIP;
  }
}

}  // extern "C"
