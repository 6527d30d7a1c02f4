// Learned ICP initialiser: a small CNN trained and evaluated on the GPU.
//
// Input 5x60x80 (current depth; raycast depth and raycast normal of the
// previous frame in its camera frame; invalid pixels 0), four 3x3 stride-2
// padding-1 convolutions with ReLU (5->16->32->64->128), global average pool,
// 128->64 (ReLU) -> 6 = se(3) increment (phi, rho) of the previous camera.
// Convolutions (forward, input gradient, weight gradient) are implicit GEMMs
// on bf16 MFMA (v_mfma_f32_16x16x16_bf16) with FP32 accumulation; the small
// fully-connected layers, the loss and Adam run in FP32.  Master weights and
// Adam moments are FP32; the convolution weights are mirrored in bf16.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <mutex>
#include <string>
#include <vector>
#include "../../include/xslam.h"

namespace xsc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

constexpr int kCh[5] = {5, 16, 32, 64, 128};
constexpr int kH[5] = {60, 30, 15, 8, 4};
constexpr int kW[5] = {80, 40, 20, 10, 5};
constexpr int kFc0 = 128, kFc1 = 64, kFc2 = 6;
constexpr float kLossScale = 100.0f;   // 1 / 0.01 (rad, m)

__host__ __device__ constexpr int kdim(int l) { return kCh[l] * 9; }                 // Ci * 9 of conv l (0-based)
__host__ __device__ constexpr int kpad(int l) { return (kdim(l) + 15) / 16 * 16; }
// weight-gradient columns: k < Ci*9 weights, k == Ci*9 the bias (a column of ones)
__host__ __device__ constexpr int kpadb(int l) { return (kdim(l) + 1 + 15) / 16 * 16; }

// flat parameter offsets (same order as the oracle: w0 b0 w1 b1 ... fc1 W b fc2 W b)
struct Offs {
  int w[4], b[4], f1w, f1b, f2w, f2b, total;
};
__host__ __device__ inline Offs offsets() {
  Offs o;
  int p = 0;
  for (int l = 0; l < 4; ++l) {
    o.w[l] = p; p += kCh[l + 1] * kdim(l);
    o.b[l] = p; p += kCh[l + 1];
  }
  o.f1w = p; p += kFc1 * kFc0;
  o.f1b = p; p += kFc1;
  o.f2w = p; p += kFc2 * kFc1;
  o.f2b = p; p += kFc2;
  o.total = p;
  return o;
}

__device__ __forceinline__ bf16 f2bf(float f) {   // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return bf16(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(uint32_t(h) << 16); }

// ---------------------------------------------------------------------------
// implicit GEMMs on MFMA 16x16x16 bf16.  One wave computes one 16x16 tile of
// C = A B (A: M x K, B: K x N).  Lane l supplies A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16] (j = 0..3) and receives C[4(l/16)+j][l%16].
// ---------------------------------------------------------------------------

// forward: rows = output positions (n, oy, ox), cols = output channels,
// k = ci*9 + ky*3 + kx; out = relu(acc + bias) in bf16
template <int L>
__global__ __launch_bounds__(256) void k_conv_fwd(const bf16* __restrict__ x, const bf16* __restrict__ w,
                                                   const float* __restrict__ bias, bf16* __restrict__ y, int N) {
  constexpr int Ci = kCh[L], Co = kCh[L + 1], H = kH[L], W = kW[L], Ho = kH[L + 1], Wo = kW[L + 1];
  constexpr int K = kdim(L), KP = kpad(L);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int M = N * Ho * Wo;
  const int m0 = (blockIdx.x * 4 + wv) * 16, n0 = blockIdx.y * 16;
  const int row = m0 + (lane & 15), kq = 4 * (lane >> 4);
  const bool rok = row < M;
  const int n = rok ? row / (Ho * Wo) : 0, pr = rok ? row % (Ho * Wo) : 0;
  const int oy = pr / Wo, ox = pr % Wo;
  const int co = n0 + (lane & 15);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < KP; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      bf16 av = 0;
      if (rok && k < K) {
        const int ci = k / 9, r = k % 9, iy = 2 * oy - 1 + r / 3, ix = 2 * ox - 1 + r % 3;
        if (iy >= 0 && iy < H && ix >= 0 && ix < W) av = x[((size_t(n) * Ci + ci) * H + iy) * W + ix];
      }
      a[j] = short(av);
      b[j] = short(w[size_t(co) * KP + k]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r2 = m0 + kq + j;
    if (r2 < M) {
      const int nn = r2 / (Ho * Wo), p2 = r2 % (Ho * Wo);
      const float v = acc[j] + bias[co];
      y[(size_t(nn) * Co + co) * (Ho * Wo) + p2] = f2bf(v > 0.f ? v : 0.f);
    }
  }
}

// input gradient of conv L masked by relu'(its input).  Of the 9 taps of the
// stride-2 3x3 convolution only those of one parity class reach an input
// position: an even input row takes ky = 1 (output row iy/2), an odd one
// ky = 0 and 2 (output rows (iy+1)/2 and (iy-1)/2); columns likewise.  So the
// input positions are split into the four classes (iy mod 2, ix mod 2), and
// class (PY, PX) is an implicit GEMM of rows = its positions (n, iy, ix),
// cols = input channels, k = co * NT + t over its NT = (1 + PY)(1 + PX) taps:
// every MFMA operand is a tap that exists.
template <int L, int PY, int PX>
__global__ __launch_bounds__(256) void k_conv_bwd_x(const bf16* __restrict__ dz, const bf16* __restrict__ w,
                                                     const bf16* __restrict__ xin, bf16* __restrict__ dzin, int N) {
  constexpr int Ci = kCh[L], Co = kCh[L + 1], H = kH[L], W = kW[L], Ho = kH[L + 1], Wo = kW[L + 1];
  constexpr int NY = 1 + PY, NX = 1 + PX, NT = NY * NX;
  constexpr int Hc = (H - PY + 1) / 2, Wc = (W - PX + 1) / 2;   // positions of the class per image
  constexpr int K = Co * NT, KP = (K + 15) / 16 * 16, KPW = kpad(L);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int M = N * Hc * Wc;
  const int m0 = (blockIdx.x * 4 + wv) * 16, n0 = blockIdx.y * 16;
  const int row = m0 + (lane & 15), kq = 4 * (lane >> 4);
  const bool rok = row < M;
  const int n = rok ? row / (Hc * Wc) : 0, pr = rok ? row % (Hc * Wc) : 0;
  const int iy = 2 * (pr / Wc) + PY, ix = 2 * (pr % Wc) + PX;
  const int ci = n0 + (lane & 15);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < KP; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      bf16 av = 0, bv = 0;
      if (k < K) {
        const int co = k / NT, t = k % NT;
        const int ky = PY ? ((t / NX) ? 2 : 0) : 1, kx = PX ? ((t % NX) ? 2 : 0) : 1;
        const int oy = (iy + 1 - ky) >> 1, ox = (ix + 1 - kx) >> 1;
        if (rok && iy + 1 - ky >= 0 && ix + 1 - kx >= 0 && oy < Ho && ox < Wo)
          av = dz[((size_t(n) * Co + co) * Ho + oy) * Wo + ox];
        if (ci < Ci) bv = w[size_t(co) * KPW + ci * 9 + ky * 3 + kx];
      }
      a[j] = short(av);
      b[j] = short(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r2 = m0 + kq + j;
    if (r2 < M && ci < Ci) {
      const int nn = r2 / (Hc * Wc), p2 = r2 % (Hc * Wc);
      const int y2 = 2 * (p2 / Wc) + PY, x2 = 2 * (p2 % Wc) + PX;
      const size_t o = (size_t(nn) * Ci + ci) * (H * W) + size_t(y2) * W + x2;
      dzin[o] = f2bf(bf2f(xin[o]) > 0.f ? acc[j] : 0.f);
    }
  }
}

// weight gradient of conv L, split over position chunks: rows = output
// channels, cols = k (ci*9 + r), reduction over positions (n, oy, ox).
template <int L>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const bf16* __restrict__ dz, const bf16* __restrict__ x,
                                                     float* __restrict__ part, int N, int chunk) {
  constexpr int Ci = kCh[L], Co = kCh[L + 1], H = kH[L], W = kW[L], Ho = kH[L + 1], Wo = kW[L + 1];
  constexpr int K = kdim(L), KP = kpadb(L);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int P = N * Ho * Wo;
  // tile (co0, k0) of the Co x KP output, 4 waves = 4 tiles along k
  const int ntk = KP / 16;   // KP = kpadb here
  const int tile = blockIdx.x * 4 + wv;
  if (tile >= (Co / 16) * ntk) return;
  const int co0 = (tile / ntk) * 16, kk0 = (tile % ntk) * 16;
  const int p_begin = blockIdx.y * chunk, p_end = min(P, p_begin + chunk);
  const int co = co0 + (lane & 15), kcol = kk0 + (lane & 15), pq = 4 * (lane >> 4);
  int ci = 0, ky = 0, kx = 0;
  const bool kok = kcol < K;
  if (kok) { ci = kcol / 9; ky = (kcol % 9) / 3; kx = kcol % 3; }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int p0 = p_begin; p0 < p_end; p0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = p0 + pq + j;
      bf16 av = 0, bv = 0;
      if (p < p_end) {
        const int n = p / (Ho * Wo), pr = p % (Ho * Wo), oy = pr / Wo, ox = pr % Wo;
        av = dz[((size_t(n) * Co + co) * Ho + oy) * Wo + ox];
        const int iy = 2 * oy - 1 + ky, ix = 2 * ox - 1 + kx;
        if (kok && iy >= 0 && iy < H && ix >= 0 && ix < W) bv = x[((size_t(n) * Ci + ci) * H + iy) * W + ix];
        if (kcol == K) bv = 0x3f80;   // bf16 1.0: the bias column
      }
      a[j] = short(av);
      b[j] = short(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  float* out = part + size_t(blockIdx.y) * Co * KP;
#pragma unroll
  for (int j = 0; j < 4; ++j) out[size_t(co0 + pq + j) * KP + kcol] = acc[j];
}

// sum of the chunk partials (fixed order) into the flat FP32 gradient (the
// weights and, from the ones column, the bias)
template <int L>
__global__ void k_conv_grad_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ grad, Offs o) {
  constexpr int Co = kCh[L + 1], K = kdim(L), KP = kpadb(L);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Co * (K + 1)) return;
  const int co = t / (K + 1), k = t % (K + 1);
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t(c) * Co + co) * KP + k];
  if (k < K) grad[o.w[L] + co * K + k] = s;
  else grad[o.b[L] + co] = s;
}

// ---------------------------------------------------------------------------
// small FP32 kernels
// ---------------------------------------------------------------------------
__global__ void k_to_bf16(const float* __restrict__ in, bf16* __restrict__ out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

// bf16 padded copies of the four conv weight matrices [Co][KP]
__global__ void k_pack_weights(const float* __restrict__ master, bf16* __restrict__ wb, Offs o) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int base = 0;
  for (int l = 0; l < 4; ++l) {
    const int Co = kCh[l + 1], K = kdim(l), KP = kpad(l);
    if (t < Co * KP) {
      const int co = t / KP, k = t % KP;
      wb[base + t] = k < K ? f2bf(master[o.w[l] + co * K + k]) : bf16(0);
    }
    base += Co * KP;
  }
}

// global average pool + fc1 (relu) + fc2, one block per sample
__global__ __launch_bounds__(128) void k_head_fwd(const bf16* __restrict__ a4, const float* __restrict__ prm, Offs o,
                                                  float* __restrict__ g, float* __restrict__ h5,
                                                  float* __restrict__ xi) {
  const int n = blockIdx.x, t = threadIdx.x;
  __shared__ float gs[kFc0], hs[kFc1];
  {
    float s = 0.f;
    for (int p = 0; p < 20; ++p) s += bf2f(a4[(size_t(n) * kFc0 + t) * 20 + p]);
    gs[t] = s / 20.f;
    g[n * kFc0 + t] = gs[t];
  }
  __syncthreads();
  if (t < kFc1) {
    float s = prm[o.f1b + t];
    for (int c = 0; c < kFc0; ++c) s += prm[o.f1w + t * kFc0 + c] * gs[c];
    hs[t] = s > 0.f ? s : 0.f;
    h5[n * kFc1 + t] = hs[t];
  }
  __syncthreads();
  if (t < kFc2) {
    float s = prm[o.f2b + t];
    for (int c = 0; c < kFc1; ++c) s += prm[o.f2w + t * kFc1 + c] * hs[c];
    xi[n * kFc2 + t] = s;
  }
}

// loss and head gradients; d(pre-activation of conv 4) = relu' * dg / 20
__global__ __launch_bounds__(128) void k_head_bwd(const float* __restrict__ xi, const float* __restrict__ label,
                                                  const float* __restrict__ g, const float* __restrict__ h5,
                                                  const bf16* __restrict__ a4, const float* __restrict__ prm, Offs o,
                                                  int N, float* __restrict__ dxi_out, float* __restrict__ loss_part,
                                                  bf16* __restrict__ dz4) {
  const int n = blockIdx.x, t = threadIdx.x;
  __shared__ float dxs[kFc2], dh5[kFc1];
  if (t < kFc2) {
    const float d = (xi[n * kFc2 + t] - label[n * kFc2 + t]) * kLossScale;
    dxs[t] = 2.f * d * kLossScale / float(N);
    dxi_out[n * kFc2 + t] = dxs[t];
  }
  __syncthreads();
  if (t == 0) {
    float l = 0.f;
    for (int c = 0; c < kFc2; ++c) {
      const float d = (xi[n * kFc2 + c] - label[n * kFc2 + c]) * kLossScale;
      l += d * d;
    }
    loss_part[n] = l / float(N);
  }
  if (t < kFc1) {
    float s = 0.f;
    for (int c = 0; c < kFc2; ++c) s += dxs[c] * prm[o.f2w + c * kFc1 + t];
    dh5[t] = h5[n * kFc1 + t] > 0.f ? s : 0.f;       // relu'(z5) * dh5
  }
  __syncthreads();
  float dg = 0.f;
  for (int c = 0; c < kFc1; ++c) dg += dh5[c] * prm[o.f1w + c * kFc0 + t];
  for (int p = 0; p < 20; ++p) {
    const size_t q = (size_t(n) * kFc0 + t) * 20 + p;
    dz4[q] = f2bf(bf2f(a4[q]) > 0.f ? dg / 20.f : 0.f);
  }
  // per-sample head gradient contributions (summed over samples by k_head_grad)
}

// head parameter gradients summed over the batch (fixed order), FP32
__global__ void k_head_grad(const float* __restrict__ dxi, const float* __restrict__ g, const float* __restrict__ h5,
                            const float* __restrict__ prm, Offs o, int N, float* __restrict__ grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kFc2 * kFc1) {                       // fc2 W
    const int r = t / kFc1, c = t % kFc1;
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += dxi[n * kFc2 + r] * h5[n * kFc1 + c];
    grad[o.f2w + t] = s;
  } else if (t < kFc2 * kFc1 + kFc2) {         // fc2 b
    const int r = t - kFc2 * kFc1;
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += dxi[n * kFc2 + r];
    grad[o.f2b + r] = s;
  } else if (t < kFc2 * kFc1 + kFc2 + kFc1 * kFc0 + kFc1) {   // fc1 W and b
    const int u = t - kFc2 * kFc1 - kFc2;
    const int r = u < kFc1 * kFc0 ? u / kFc0 : u - kFc1 * kFc0;
    const int c = u < kFc1 * kFc0 ? u % kFc0 : -1;
    float s = 0.f;
    for (int n = 0; n < N; ++n) {
      float d5 = 0.f;
      for (int q = 0; q < kFc2; ++q) d5 += dxi[n * kFc2 + q] * prm[o.f2w + q * kFc1 + r];
      if (!(h5[n * kFc1 + r] > 0.f)) d5 = 0.f;
      s += d5 * (c >= 0 ? g[n * kFc0 + c] : 1.f);
    }
    if (c >= 0) grad[o.f1w + r * kFc0 + c] = s;
    else grad[o.f1b + r] = s;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mm = 0.9f * m[i] + 0.1f * g, vv = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mm;
  v[i] = vv;
  p[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

__global__ void k_sum(const float* __restrict__ a, int n, float* __restrict__ out) {
  __shared__ float s[256];
  float v = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) v += a[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

inline constexpr size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Buffers of one forward pass: the bf16 input and convolution outputs, the
// pooled features, the hidden layer and the se(3) output (FP32).
struct FwdBufs {
  bf16* act[5];
  float *g, *h5, *xi;
};
constexpr size_t fwd_bytes(int B) {
  size_t s = 0;
  for (int l = 0; l < 5; ++l) s += al(sizeof(bf16) * size_t(B) * kCh[l] * kH[l] * kW[l]);
  return s + al(sizeof(float) * size_t(B) * kFc0) + al(sizeof(float) * size_t(B) * kFc1) +
         al(sizeof(float) * size_t(B) * kFc2);
}
inline FwdBufs fwd_plan(int B, char* base) {
  FwdBufs b;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* q = base + off; off = al(off + bytes); return q; };
  for (int l = 0; l < 5; ++l) b.act[l] = (bf16*)take(sizeof(bf16) * size_t(B) * kCh[l] * kH[l] * kW[l]);
  b.g = (float*)take(sizeof(float) * size_t(B) * kFc0);
  b.h5 = (float*)take(sizeof(float) * size_t(B) * kFc1);
  b.xi = (float*)take(sizeof(float) * size_t(B) * kFc2);
  return b;
}

// Forward buffers of xslam_cnn_forward_noalloc: a fixed device array (about
// 3.9 MB for 32 samples), one copy per GPU, held until the process ends and
// shared by every call on that GPU.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, per device.
constexpr int kNoallocMaxBatch = 32;
constexpr size_t kScratchBytes = fwd_bytes(kNoallocMaxBatch);
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
inline int scratch_address(char** out, std::string& err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    err = "scratch: no current device";
    return XSLAM_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
      return XSLAM_ERR_HIP;
    }
    g_scratch_dev[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_dev[dev];
  return XSLAM_OK;
}

struct Cnn {
  int max_batch = 0;
  hipStream_t stream = nullptr;
  std::string err;
  Offs o;
  int nchunk = 64;
  int64_t step = 0;
  char* scratch_dev = nullptr;   // device address of the static forward scratch (this handle's GPU)
  // device buffers
  float *prm, *grad, *m, *v, *dxi, *lpart, *loss, *g, *h5, *xi, *part;
  bf16 *wb, *act[5], *dz[5];

  static size_t plan(int B, Cnn* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t q = off; off = al(off + bytes); return base ? base + q : nullptr; };
    Offs o = offsets();
    size_t wbn = 0;
    for (int l = 0; l < 4; ++l) wbn += size_t(kCh[l + 1]) * kpad(l);
    size_t maxpart = 0;
    for (int l = 0; l < 4; ++l) maxpart = std::max(maxpart, size_t(kCh[l + 1]) * kpadb(l));
    float* prm = (float*)take(sizeof(float) * o.total);
    float* grad = (float*)take(sizeof(float) * o.total);
    float* m = (float*)take(sizeof(float) * o.total);
    float* v = (float*)take(sizeof(float) * o.total);
    bf16* wb = (bf16*)take(sizeof(bf16) * wbn);
    bf16* act[5];
    bf16* dz[5];
    for (int l = 0; l < 5; ++l) act[l] = (bf16*)take(sizeof(bf16) * size_t(B) * kCh[l] * kH[l] * kW[l]);
    for (int l = 0; l < 5; ++l) dz[l] = (bf16*)take(sizeof(bf16) * size_t(B) * kCh[l] * kH[l] * kW[l]);
    float* g = (float*)take(sizeof(float) * B * kFc0);
    float* h5 = (float*)take(sizeof(float) * B * kFc1);
    float* xi = (float*)take(sizeof(float) * B * kFc2);
    float* dxi = (float*)take(sizeof(float) * B * kFc2);
    float* lpart = (float*)take(sizeof(float) * B);
    float* loss = (float*)take(sizeof(float));
    float* part = (float*)take(sizeof(float) * maxpart * 64);
    if (c) {
      c->o = o; c->prm = prm; c->grad = grad; c->m = m; c->v = v; c->wb = wb;
      for (int l = 0; l < 5; ++l) { c->act[l] = act[l]; c->dz[l] = dz[l]; }
      c->g = g; c->h5 = h5; c->xi = xi; c->dxi = dxi; c->lpart = lpart; c->loss = loss; c->part = part;
    }
    return off;
  }

  int check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { err = std::string(what) + ": " + hipGetErrorString(e); return XSLAM_ERR_HIP; }
    return XSLAM_OK;
  }

  bf16* wl(int l) {
    size_t off = 0;
    for (int q = 0; q < l; ++q) off += size_t(kCh[q + 1]) * kpad(q);
    return wb + off;
  }

  int pack() {
    int n = 0;
    for (int l = 0; l < 4; ++l) n = std::max(n, kCh[l + 1] * kpad(l));
    hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, stream, prm, wb, o);
    return check("pack");
  }

  template <int L> void conv_fwd(int N, bf16* const* a) {
    const int M = N * kH[L + 1] * kW[L + 1];
    hipLaunchKernelGGL(k_conv_fwd<L>, dim3((M + 63) / 64, kCh[L + 1] / 16), dim3(256), 0, stream, a[L], wl(L),
                       prm + o.b[L], a[L + 1], N);
  }
  FwdBufs own() {
    FwdBufs b;
    for (int l = 0; l < 5; ++l) b.act[l] = act[l];
    b.g = g; b.h5 = h5; b.xi = xi;
    return b;
  }
  int forward(const float* x, int N) { return forward(x, N, own()); }
  int forward(const float* x, int N, const FwdBufs& b) {
    const int64_t nin = int64_t(N) * 5 * 60 * 80;
    hipLaunchKernelGGL(k_to_bf16, dim3((nin + 255) / 256), dim3(256), 0, stream, x, b.act[0], nin);
    conv_fwd<0>(N, b.act);
    conv_fwd<1>(N, b.act);
    conv_fwd<2>(N, b.act);
    conv_fwd<3>(N, b.act);
    hipLaunchKernelGGL(k_head_fwd, dim3(N), dim3(128), 0, stream, b.act[4], prm, o, b.g, b.h5, b.xi);
    return check("cnn forward");
  }

  template <int L, int PY, int PX>
  void bwd_x_class(int N) {
    const int M = N * ((kH[L] - PY + 1) / 2) * ((kW[L] - PX + 1) / 2);
    hipLaunchKernelGGL((k_conv_bwd_x<L, PY, PX>), dim3((M + 63) / 64, (kCh[L] + 15) / 16), dim3(256), 0, stream,
                       dz[L + 1], wl(L), act[L], dz[L], N);
  }
  template <int L> void conv_bwd(int N) {
    // weight gradient over position chunks
    const int P = N * kH[L + 1] * kW[L + 1];
    int chunk = (P + nchunk - 1) / nchunk;
    chunk = (chunk + 15) / 16 * 16;
    const int nch = (P + chunk - 1) / chunk;
    const int tiles = (kCh[L + 1] / 16) * (kpadb(L) / 16);
    hipLaunchKernelGGL(k_conv_bwd_w<L>, dim3((tiles + 3) / 4, nch), dim3(256), 0, stream, dz[L + 1], act[L], part, N,
                       chunk);
    const int nt = kCh[L + 1] * (kdim(L) + 1);
    hipLaunchKernelGGL(k_conv_grad_reduce<L>, dim3((nt + 255) / 256), dim3(256), 0, stream, part, nch, grad, o);
    if constexpr (L > 0) {
      bwd_x_class<L, 0, 0>(N);
      bwd_x_class<L, 0, 1>(N);
      bwd_x_class<L, 1, 0>(N);
      bwd_x_class<L, 1, 1>(N);
    }
  }
  int train(const float* x, const float* label, int N, float lr, float* loss_host) {
    int rc = forward(x, N);
    if (rc) return rc;
    hipLaunchKernelGGL(k_head_bwd, dim3(N), dim3(128), 0, stream, xi, label, g, h5, act[4], prm, o, N, dxi, lpart,
                       dz[4]);
    const int nh = kFc2 * kFc1 + kFc2 + kFc1 * kFc0 + kFc1;
    hipLaunchKernelGGL(k_head_grad, dim3((nh + 255) / 256), dim3(256), 0, stream, dxi, g, h5, prm, o, N, grad);
    conv_bwd<3>(N);
    conv_bwd<2>(N);
    conv_bwd<1>(N);
    conv_bwd<0>(N);
    step += 1;
    const float c1 = 1.f - powf(0.9f, float(step)), c2 = 1.f - powf(0.999f, float(step));
    hipLaunchKernelGGL(k_adam, dim3((o.total + 255) / 256), dim3(256), 0, stream, prm, grad, m, v, o.total, lr, c1, c2);
    if ((rc = pack())) return rc;
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, stream, lpart, N, loss);
    if ((rc = check("cnn train"))) return rc;
    if (loss_host) {
      if (hipMemcpyAsync(loss_host, loss, sizeof(float), hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        return check("loss copy");
    }
    return XSLAM_OK;
  }
};

}  // namespace xsc

struct xslam_cnn_s {
  xsc::Cnn c;
};

namespace xsc {
// the stream a network handle launches on (a context may only use a network
// created on its own stream: the forward then joins the context's order and
// its graph capture)
void* cnn_stream(const xslam_cnn_s* h) { return h ? static_cast<void*>(h->c.stream) : nullptr; }
}  // namespace xsc

using namespace xsc;

extern "C" {

int32_t xslam_cnn_param_count(void) { return offsets().total; }

size_t xslam_cnn_workspace_bytes(int32_t max_batch) {
  if (max_batch < 1 || max_batch > 4096) return 0;
  return Cnn::plan(max_batch, nullptr, nullptr);
}

int xslam_cnn_create(void* ws, size_t bytes, void* stream, int32_t max_batch, xslam_cnn* out) {
  if (!out) return XSLAM_ERR_ARG;
  *out = nullptr;
  if (max_batch < 1 || max_batch > 4096) return XSLAM_ERR_ARG;
  if (!ws || bytes < Cnn::plan(max_batch, nullptr, nullptr) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return XSLAM_ERR_WORKSPACE;
  auto* h = new xslam_cnn_s();
  h->c.max_batch = max_batch;
  h->c.stream = static_cast<hipStream_t>(stream);
  Cnn::plan(max_batch, &h->c, static_cast<char*>(ws));
  if (scratch_address(&h->c.scratch_dev, h->c.err) != XSLAM_OK) {
    delete h;
    return XSLAM_ERR_HIP;
  }
  const size_t pb = sizeof(float) * h->c.o.total;
  if (hipMemsetAsync(h->c.m, 0, pb, h->c.stream) != hipSuccess || hipMemsetAsync(h->c.v, 0, pb, h->c.stream) != hipSuccess ||
      hipMemsetAsync(h->c.prm, 0, pb, h->c.stream) != hipSuccess || hipStreamSynchronize(h->c.stream) != hipSuccess) {
    delete h;
    return XSLAM_ERR_HIP;
  }
  *out = h;
  return XSLAM_OK;
}

int xslam_cnn_set_weights(xslam_cnn h, const float* host, size_t n) {
  if (!h || !host || n != size_t(h->c.o.total)) return XSLAM_ERR_ARG;
  if (hipMemcpyAsync(h->c.prm, host, n * sizeof(float), hipMemcpyHostToDevice, h->c.stream) != hipSuccess)
    return XSLAM_ERR_HIP;
  int rc = h->c.pack();
  if (rc) return rc;
  h->c.step = 0;
  const size_t pb = sizeof(float) * h->c.o.total;
  if (hipMemsetAsync(h->c.m, 0, pb, h->c.stream) != hipSuccess || hipMemsetAsync(h->c.v, 0, pb, h->c.stream) != hipSuccess)
    return XSLAM_ERR_HIP;
  return hipStreamSynchronize(h->c.stream) == hipSuccess ? XSLAM_OK : XSLAM_ERR_HIP;
}

int xslam_cnn_get_weights(xslam_cnn h, float* host, size_t n) {
  if (!h || !host || n != size_t(h->c.o.total)) return XSLAM_ERR_ARG;
  if (hipMemcpyAsync(host, h->c.prm, n * sizeof(float), hipMemcpyDeviceToHost, h->c.stream) != hipSuccess ||
      hipStreamSynchronize(h->c.stream) != hipSuccess)
    return XSLAM_ERR_HIP;
  return XSLAM_OK;
}

int xslam_cnn_get_grads(xslam_cnn h, float* host, size_t n) {
  if (!h || !host || n != size_t(h->c.o.total)) return XSLAM_ERR_ARG;
  if (hipMemcpyAsync(host, h->c.grad, n * sizeof(float), hipMemcpyDeviceToHost, h->c.stream) != hipSuccess ||
      hipStreamSynchronize(h->c.stream) != hipSuccess)
    return XSLAM_ERR_HIP;
  return XSLAM_OK;
}

int xslam_cnn_forward(xslam_cnn h, const float* x_dev, int32_t n, float* xi_dev) {
  if (!h || !x_dev || !xi_dev || n < 1 || n > h->c.max_batch) return XSLAM_ERR_ARG;
  int rc = h->c.forward(x_dev, n);
  if (rc) return rc;
  if (hipMemcpyAsync(xi_dev, h->c.xi, sizeof(float) * 6 * n, hipMemcpyDeviceToDevice, h->c.stream) != hipSuccess)
    return h->c.check("xi copy");
  return XSLAM_OK;
}

int xslam_cnn_forward_noalloc(xslam_cnn h, const float* x_dev, int32_t n, float* xi_dev) {
  if (!h || !x_dev || !xi_dev || n < 1) return XSLAM_ERR_ARG;
  if (n > kNoallocMaxBatch) {
    h->c.err = "forward_noalloc: batch of " + std::to_string(n) + " exceeds the static scratch's maximum of " +
               std::to_string(kNoallocMaxBatch);
    return XSLAM_ERR_WORKSPACE;
  }
  if (!h->c.scratch_dev) {
    h->c.err = "forward_noalloc: no scratch address";
    return XSLAM_ERR_STATE;
  }
  const FwdBufs b = fwd_plan(n, h->c.scratch_dev);
  int rc = h->c.forward(x_dev, n, b);
  if (rc) return rc;
  if (hipMemcpyAsync(xi_dev, b.xi, sizeof(float) * 6 * n, hipMemcpyDeviceToDevice, h->c.stream) != hipSuccess)
    return h->c.check("xi copy");
  return XSLAM_OK;
}

int xslam_cnn_train_step(xslam_cnn h, const float* x_dev, const float* label_dev, int32_t n, float lr,
                         float* loss_host) {
  if (!h || !x_dev || !label_dev || n < 1 || n > h->c.max_batch || !(lr > 0)) return XSLAM_ERR_ARG;
  return h->c.train(x_dev, label_dev, n, lr, loss_host);
}

const char* xslam_cnn_last_error(xslam_cnn h) { return h ? h->c.err.c_str() : "null"; }

int xslam_cnn_destroy(xslam_cnn h) {
  if (!h) return XSLAM_ERR_ARG;
  hipStreamSynchronize(h->c.stream);
  delete h;
  return XSLAM_OK;
}

}  // extern "C"
