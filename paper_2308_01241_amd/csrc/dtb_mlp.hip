// dtb_mlp.hip - the surrogate that screens assimilation proposals: a dense
// MLP (exact-erf GELU hidden layers, linear output) trained with MSE and
// Adam, plus top-k selection of the best-scored proposals.
//
// Every matrix product runs on MFMA (v_mfma_f32_16x16x32_bf16): operands in
// bfloat16, accumulation in FP32.  Master weights, Adam moments, biases,
// pre-activations and gradients are FP32.  Rounding points: layer inputs and
// weights (forward); the upstream gradient, saved activations and weights
// (backward).  A handle can instead keep every operand in FP32
// (v_mfma_f32_16x16x4_f32, same tiles and epilogues): the check of the
// kernels' index logic against an unrounded FP64 reference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dtb.h"

namespace dtb {
void set_error(const std::string& msg);
}

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
  u = __float_as_uint(f);
#else
  std::memcpy(&u, &f, 4);
#endif
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// an FP32 value as a matrix operand: bfloat16 bits (round to nearest even)
// or the float itself
__device__ inline uint16_t to_op(float x, uint16_t*) { return f2bf(x); }
__device__ inline float to_op(float x, float*) { return x; }

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum Epi { kHidden = 0, kOut = 1, kDGelu = 2, kStore = 3 };

// C(m, n) = sum_k A(m, k) B(k, n) over 64x64 output tiles, K in steps of 32.
//   A(m, k) = TA ? A[k lda + m] : A[m lda + k]      (Op: bfloat16 bits or float)
//   B(k, n) = TB ? B[n ldb + k] : B[k ldb + n]
// Four wavefronts per tile, each a 32x32 quarter = 2x2 MFMA 16x16 blocks.
// MFMA operand layout (16x16x32 bf16): lane l supplies A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16], e = 0..7; (16x16x4 f32): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; both return D[4 (l / 16) + r][l % 16].
template <bool TA, bool TB, int EPI, typename Op>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const Op* __restrict__ A, int lda,
                                              const Op* __restrict__ B, int ldb,
                                              const float* __restrict__ bias, float* __restrict__ Cf,
                                              Op* __restrict__ Cb, int ldc, const float* __restrict__ Zprev) {
  constexpr bool kF32 = sizeof(Op) == 4;
  constexpr int kRow = kF32 ? 33 : 40;  // LDS row pitch in elements (80 B for bf16)
  __shared__ __attribute__((aligned(16))) Op sA[64][kRow];  // [m][k]
  __shared__ __attribute__((aligned(16))) Op sB[64][kRow];  // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    for (int q = tid; q < 64 * 32; q += 256) {
      const int r = q >> 5, c = q & 31;
      const int m = m0 + r, k = k0 + c;
      Op v = Op(0);
      if (m < M && k < K) v = TA ? A[int64_t(k) * lda + m] : A[int64_t(m) * lda + k];
      sA[r][c] = v;
      const int nn = n0 + r;
      Op w = Op(0);
      if (nn < N && k < K) w = TB ? B[int64_t(nn) * ldb + k] : B[int64_t(k) * ldb + nn];
      sB[r][c] = w;
    }
    __syncthreads();
    if constexpr (kF32) {
#pragma unroll
      for (int kk = 0; kk < 32; kk += 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float a = sA[wm + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const float b = sB[wn + 16 * j + (lane & 15)][kk + (lane >> 4)];
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
          }
        }
      }
    } else {
      const int kk = 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sA[wm + 16 * i + (lane & 15)][kk]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sB[wn + 16 * j + (lane & 15)][kk]);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (row >= M || col >= N) continue;
        const int64_t o = int64_t(row) * ldc + col;
        const float x = acc[i][j][r];
        if (EPI == kHidden) {
          const float z = x + bias[col];
          Cf[o] = z;
          Cb[o] = to_op(gelu(z), Cb);
        } else if (EPI == kOut) {
          Cf[o] = x + bias[col];
        } else if (EPI == kDGelu) {
          const float dz = x * gelu_grad(Zprev[o]);
          Cf[o] = dz;
          Cb[o] = to_op(dz, Cb);
        } else {
          Cf[o] = x;
        }
      }
}

// FP32 values as matrix operands
template <typename Op>
__global__ void k_to_op(int64_t n, const float* __restrict__ x, Op* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_op(x[i], y);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// d(loss)/dY for loss = mean((Y - T)^2) and the loss itself (one block, fixed
// summation order: strided partial sums then a tree).
template <typename Op>
__global__ __launch_bounds__(1024) void k_mse(int64_t n, const float* __restrict__ Y, const float* __restrict__ T,
                                              float* __restrict__ dY, Op* __restrict__ dYb,
                                              double* __restrict__ loss) {
  __shared__ double s[1024];
  double acc = 0.0;
  const float scale = float(2.0 / double(n));
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float d = Y[i] - T[i];
    acc += double(d) * double(d);
    const float g = scale * d;
    dY[i] = g;
    dYb[i] = to_op(g, dYb);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s[0] / double(n);
}

// bias gradient: column sums of dZ [rows][cols], one thread per column, rows in order
__global__ void k_colsum(int rows, int cols, const float* __restrict__ dZ, float* __restrict__ g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += dZ[int64_t(r) * cols + c];
  g[c] = s;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m c1) / (sqrt(v c2) + eps), c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ wb, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = __fmaf_rn(b1, m[i], (1.f - b1) * gi);
  const float vi = __fmaf_rn(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

// top-k (ascending score, ties by index) of n <= 4096 scores: bitonic sort of
// (score, index) pairs in LDS by one 1024-thread block.
__global__ __launch_bounds__(1024) void k_topk(int n, int k, const float* __restrict__ score,
                                               int32_t* __restrict__ idx) {
  __shared__ float sk[4096];
  __shared__ int32_t si[4096];
  for (int q = threadIdx.x; q < 4096; q += 1024) {
    float x = q < n ? score[q] : INFINITY;
    if (!(x == x)) x = INFINITY;  // NaN ranks last
    sk[q] = x;
    si[q] = q < n ? q : 0x7FFFFFFF;
  }
  __syncthreads();
  for (int size = 2; size <= 4096; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = threadIdx.x; q < 4096; q += 1024) {
        const int p = q ^ stride;
        if (p > q) {
          const bool up = (q & size) == 0;
          const bool gt = sk[q] > sk[p] || (sk[q] == sk[p] && si[q] > si[p]);
          if (gt == up) {
            const float tk = sk[q];
            sk[q] = sk[p];
            sk[p] = tk;
            const int32_t ti = si[q];
            si[q] = si[p];
            si[p] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < k; q += 1024) idx[q] = si[q];
}

constexpr int kTopkMax = 4096;  // scores one selection sorts in LDS

// Staging area of dtb_topk_noalloc: the n scores of a call, then the k
// selected indices.  One copy per GPU the library runs on, held until the
// process ends.  Host code never uses this name as an address: it takes the
// device address from hipGetSymbolAddress (scratch_on) instead.
static __device__ __align__(256) uint32_t scratch[2 * kTopkMax];

}  // namespace

// =============================================================== host side
struct dtb_mlp {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<int> dims;            // in, hidden..., out
  std::vector<int64_t> woff, boff;  // per layer offsets in the flat parameter vector
  int64_t P = 0;
  int64_t step = 0;                 // Adam steps taken
  float* w = nullptr;               // [P] master parameters
  uint16_t* wb = nullptr;           // [P] bfloat16 copies
  float *m = nullptr, *v = nullptr, *g = nullptr;
  // activations for up to cap rows
  int cap = 0;
  bool f32_ops = false;              // operands in FP32 instead of bfloat16
  std::vector<float*> Z;            // pre-activations per layer (output layer: Y)
  std::vector<void*> Act;           // operand-typed layer inputs: Act[0] = X, Act[l] = gelu(Z[l-1])
  float *dZf[2] = {nullptr, nullptr};
  void* dZb[2] = {nullptr, nullptr}; // operand-typed copies of dZf
  float *Xf = nullptr, *Tf = nullptr;
  double* loss = nullptr;
  std::vector<void*> buf;           // activation allocations (freed on regrow)
};

namespace {

dtb_status mfail(dtb_status s, const std::string& msg) {
  dtb::set_error(msg);
  return s;
}

#define MLP_HIP(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return mfail(DTB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int layers_of(const dtb_mlp* h) { return int(h->dims.size()) - 1; }

dtb_status ensure_cap(dtb_mlp* h, int rows) {
  if (rows <= h->cap) return DTB_OK;
  MLP_HIP(hipStreamSynchronize(h->stream));
  for (void* p : h->buf) (void)hipFree(p);
  h->buf.clear();
  const int L = layers_of(h);
  int wmax = 0;
  for (int d : h->dims) wmax = std::max(wmax, d);
  auto al = [&](size_t bytes, void** p) -> hipError_t {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) h->buf.push_back(*p);
    return e;
  };
  h->Z.assign(L, nullptr);
  h->Act.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    MLP_HIP(al(size_t(rows) * h->dims[l + 1] * 4, reinterpret_cast<void**>(&h->Z[l])));
    MLP_HIP(al(size_t(rows) * h->dims[l] * 4, &h->Act[l]));  // 4 B: room for either operand type
  }
  for (int q = 0; q < 2; ++q) {
    MLP_HIP(al(size_t(rows) * wmax * 4, reinterpret_cast<void**>(&h->dZf[q])));
    MLP_HIP(al(size_t(rows) * wmax * 4, &h->dZb[q]));
  }
  MLP_HIP(al(size_t(rows) * h->dims[0] * 4, reinterpret_cast<void**>(&h->Xf)));
  MLP_HIP(al(size_t(rows) * h->dims[L] * 4, reinterpret_cast<void**>(&h->Tf)));
  h->cap = rows;
  return DTB_OK;
}

template <bool TA, bool TB, int EPI, typename Op>
hipError_t gemm(hipStream_t s, int M, int N, int K, const Op* A, int lda, const Op* B, int ldb, const float* bias,
                float* Cf, Op* Cb, int ldc, const float* Zprev) {
  dim3 grid(unsigned((N + 63) / 64), unsigned((M + 63) / 64));
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI, Op>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, bias, Cf, Cb, ldc,
                     Zprev);
  return hipGetLastError();
}

// the weights as operands: the bfloat16 copies, or the FP32 master weights
const uint16_t* op_weights(const dtb_mlp* h, uint16_t*) { return h->wb; }
const float* op_weights(const dtb_mlp* h, float*) { return h->w; }

// forward pass of `rows` rows whose FP32 inputs are in h->Xf; output in h->Z[L-1]
template <typename Op>
hipError_t forward_as(dtb_mlp* h, int rows) {
  const int L = layers_of(h);
  const int64_t nin = int64_t(rows) * h->dims[0];
  Op* const tag = nullptr;
  hipLaunchKernelGGL((k_to_op<Op>), dim3(unsigned((nin + 255) / 256)), dim3(256), 0, h->stream, nin, h->Xf,
                     static_cast<Op*>(h->Act[0]));
  hipError_t e = hipGetLastError();
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const int in = h->dims[l], out = h->dims[l + 1];
    const Op* W = op_weights(h, tag) + h->woff[l];
    const float* b = h->w + h->boff[l];
    const Op* a = static_cast<const Op*>(h->Act[l]);
    if (l < L - 1)
      e = gemm<false, true, kHidden, Op>(h->stream, rows, out, in, a, in, W, in, b, h->Z[l],
                                         static_cast<Op*>(h->Act[l + 1]), out, nullptr);
    else
      e = gemm<false, true, kOut, Op>(h->stream, rows, out, in, a, in, W, in, b, h->Z[l], nullptr, out, nullptr);
  }
  return e;
}

// gradient of mean((Y - T)^2) into h->g (T in h->Tf); needs forward() first
template <typename Op>
hipError_t backward_as(dtb_mlp* h, int rows) {
  const int L = layers_of(h);
  const int64_t nout = int64_t(rows) * h->dims[L];
  Op* const tag = nullptr;
  hipLaunchKernelGGL((k_mse<Op>), dim3(1), dim3(1024), 0, h->stream, nout, h->Z[L - 1], h->Tf, h->dZf[0],
                     static_cast<Op*>(h->dZb[0]), h->loss);
  hipError_t e = hipGetLastError();
  int cur = 0;
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    const int in = h->dims[l], out = h->dims[l + 1];
    // dW_l = dZ_l^T A_l    (out x in)
    e = gemm<true, false, kStore, Op>(h->stream, out, in, rows, static_cast<const Op*>(h->dZb[cur]), out,
                                      static_cast<const Op*>(h->Act[l]), in, nullptr, h->g + h->woff[l], nullptr,
                                      in, nullptr);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_colsum, dim3(unsigned((out + 255) / 256)), dim3(256), 0, h->stream, rows, out, h->dZf[cur],
                       h->g + h->boff[l]);
    e = hipGetLastError();
    if (e != hipSuccess || l == 0) break;
    // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})   (rows x in)
    e = gemm<false, false, kDGelu, Op>(h->stream, rows, in, out, static_cast<const Op*>(h->dZb[cur]), out,
                                       op_weights(h, tag) + h->woff[l], in, nullptr, h->dZf[1 - cur],
                                       static_cast<Op*>(h->dZb[1 - cur]), in, h->Z[l - 1]);
    cur = 1 - cur;
  }
  return e;
}

hipError_t forward(dtb_mlp* h, int rows) {
  return h->f32_ops ? forward_as<float>(h, rows) : forward_as<uint16_t>(h, rows);
}

hipError_t backward(dtb_mlp* h, int rows) {
  return h->f32_ops ? backward_as<float>(h, rows) : backward_as<uint16_t>(h, rows);
}

dtb_status copy_in(dtb_mlp* h, float* dst, const float* src, size_t bytes, int on_device) {
  MLP_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
  return DTB_OK;
}

uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

}  // namespace

extern "C" {

dtb_status dtb_mlp_create(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out, uint64_t seed,
                          void* hip_stream, dtb_mlp** out) {
  if (!out) return mfail(DTB_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_hidden < 0 || n_out < 1 || n_in > 65536 || hidden > 65536 || n_out > 65536 ||
      n_hidden > 64)
    return mfail(DTB_ERR_INVALID, "bad MLP dimensions");
  dtb_mlp* h = new (std::nothrow) dtb_mlp();
  if (!h) return mfail(DTB_ERR_OOM, "host allocation failed");
  h->dims.push_back(n_in);
  for (int q = 0; q < n_hidden; ++q) h->dims.push_back(hidden);
  h->dims.push_back(n_out);
  const int L = layers_of(h);
  for (int l = 0; l < L; ++l) {
    h->woff.push_back(h->P);
    h->P += int64_t(h->dims[l + 1]) * h->dims[l];
    h->boff.push_back(h->P);
    h->P += h->dims[l + 1];
  }
  h->stream = static_cast<hipStream_t>(hip_stream);
  auto bail = [&](dtb_status s) {
    dtb_mlp_destroy(h);
    return s;
  };
  if (!h->stream) {
    if (hipStreamCreate(&h->stream) != hipSuccess) return bail(mfail(DTB_ERR_HIP, "hipStreamCreate failed"));
    h->own_stream = true;
  }
  const size_t P = size_t(h->P);
  if (hipMalloc(&h->w, P * 4) != hipSuccess || hipMalloc(&h->wb, P * 2) != hipSuccess ||
      hipMalloc(&h->m, P * 4) != hipSuccess || hipMalloc(&h->v, P * 4) != hipSuccess ||
      hipMalloc(&h->g, P * 4) != hipSuccess || hipMalloc(&h->loss, 8) != hipSuccess)
    return bail(mfail(DTB_ERR_OOM, "hipMalloc of MLP parameters failed"));
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, from a counter hash of the seed
  std::vector<float> w(P, 0.f);
  for (int l = 0; l < L; ++l) {
    const double a = 1.0 / std::sqrt(double(h->dims[l]));
    const int64_t nw = int64_t(h->dims[l + 1]) * h->dims[l];
    for (int64_t q = 0; q < nw; ++q) {
      const double u = double(mix64(seed ^ mix64(uint64_t(h->woff[l] + q))) >> 11) * (1.0 / 9007199254740992.0);
      w[h->woff[l] + q] = float(a * (2.0 * u - 1.0));
    }
  }
  std::vector<uint16_t> wb(P);
  for (size_t q = 0; q < P; ++q) wb[q] = f2bf(w[q]);
  if (hipMemcpy(h->w, w.data(), P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->wb, wb.data(), P * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->m, 0, P * 4) != hipSuccess || hipMemset(h->v, 0, P * 4) != hipSuccess)
    return bail(mfail(DTB_ERR_HIP, "MLP parameter upload failed"));
  *out = h;
  return DTB_OK;
}

void dtb_mlp_destroy(dtb_mlp* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void* p : h->buf) (void)hipFree(p);
  for (void* p : {static_cast<void*>(h->w), static_cast<void*>(h->wb), static_cast<void*>(h->m),
                  static_cast<void*>(h->v), static_cast<void*>(h->g), static_cast<void*>(h->loss)})
    if (p) (void)hipFree(p);
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int64_t dtb_mlp_num_params(const dtb_mlp* h) { return h ? h->P : 0; }

dtb_status dtb_mlp_params(dtb_mlp* h, float* buf, int get, int on_device) {
  if (!h || !buf) return mfail(DTB_ERR_INVALID, "null handle or buffer");
  const size_t P = size_t(h->P);
  if (get) {
    MLP_HIP(hipMemcpyAsync(buf, h->w, P * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    MLP_HIP(hipStreamSynchronize(h->stream));
    return DTB_OK;
  }
  MLP_HIP(hipMemcpyAsync(h->w, buf, P * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
  hipLaunchKernelGGL(k_to_bf16, dim3(unsigned((P + 255) / 256)), dim3(256), 0, h->stream, int64_t(P), h->w, h->wb);
  MLP_HIP(hipGetLastError());
  MLP_HIP(hipMemsetAsync(h->m, 0, P * 4, h->stream));
  MLP_HIP(hipMemsetAsync(h->v, 0, P * 4, h->stream));
  MLP_HIP(hipStreamSynchronize(h->stream));
  h->step = 0;
  return DTB_OK;
}

dtb_status dtb_mlp_set_operands(dtb_mlp* h, int fp32) {
  if (!h || (fp32 != 0 && fp32 != 1)) return mfail(DTB_ERR_INVALID, "set_operands needs a handle and fp32 in {0, 1}");
  MLP_HIP(hipStreamSynchronize(h->stream));
  h->f32_ops = fp32 == 1;
  return DTB_OK;
}

dtb_status dtb_mlp_forward(dtb_mlp* h, const float* X, int32_t batch, float* Y, int on_device) {
  if (!h || !X || !Y || batch < 1) return mfail(DTB_ERR_INVALID, "bad forward arguments");
  dtb_status st = ensure_cap(h, batch);
  if (st) return st;
  const int L = layers_of(h);
  if ((st = copy_in(h, h->Xf, X, size_t(batch) * h->dims[0] * 4, on_device))) return st;
  MLP_HIP(forward(h, batch));
  MLP_HIP(hipMemcpyAsync(Y, h->Z[L - 1], size_t(batch) * h->dims[L] * 4,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  if (!on_device) MLP_HIP(hipStreamSynchronize(h->stream));
  return DTB_OK;
}

dtb_status dtb_mlp_grad(dtb_mlp* h, const float* X, const float* T, int32_t batch, float* loss, float* grads,
                        int on_device) {
  if (!h || !X || !T || batch < 1) return mfail(DTB_ERR_INVALID, "bad grad arguments");
  dtb_status st = ensure_cap(h, batch);
  if (st) return st;
  const int L = layers_of(h);
  if ((st = copy_in(h, h->Xf, X, size_t(batch) * h->dims[0] * 4, on_device)) ||
      (st = copy_in(h, h->Tf, T, size_t(batch) * h->dims[L] * 4, on_device)))
    return st;
  MLP_HIP(forward(h, batch));
  MLP_HIP(backward(h, batch));
  if (grads)
    MLP_HIP(hipMemcpyAsync(grads, h->g, size_t(h->P) * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           h->stream));
  double l = 0.0;
  MLP_HIP(hipMemcpyAsync(&l, h->loss, 8, hipMemcpyDeviceToHost, h->stream));
  MLP_HIP(hipStreamSynchronize(h->stream));
  if (loss) *loss = float(l);
  return DTB_OK;
}

dtb_status dtb_mlp_train_step(dtb_mlp* h, const float* X, const float* T, int32_t batch, float lr, float* loss,
                              int on_device) {
  if (!h || !X || !T || batch < 1 || !(lr > 0.f)) return mfail(DTB_ERR_INVALID, "bad train arguments");
  dtb_status st = ensure_cap(h, batch);
  if (st) return st;
  const int L = layers_of(h);
  if ((st = copy_in(h, h->Xf, X, size_t(batch) * h->dims[0] * 4, on_device)) ||
      (st = copy_in(h, h->Tf, T, size_t(batch) * h->dims[L] * 4, on_device)))
    return st;
  MLP_HIP(forward(h, batch));
  MLP_HIP(backward(h, batch));
  h->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = float(1.0 / (1.0 - std::pow(b1, double(h->step))));
  const float c2 = float(1.0 / (1.0 - std::pow(b2, double(h->step))));
  hipLaunchKernelGGL(k_adam, dim3(unsigned((h->P + 255) / 256)), dim3(256), 0, h->stream, h->P, h->w, h->m, h->v,
                     h->g, h->wb, lr, float(b1), float(b2), 1e-8f, c1, c2);
  MLP_HIP(hipGetLastError());
  if (loss) {
    double l = 0.0;
    MLP_HIP(hipMemcpyAsync(&l, h->loss, 8, hipMemcpyDeviceToHost, h->stream));
    MLP_HIP(hipStreamSynchronize(h->stream));
    *loss = float(l);
  }
  return DTB_OK;
}

dtb_status dtb_topk(const float* score, int32_t n, int32_t k, int32_t* idx, void* hip_stream, int on_device) {
  if (!score || !idx || n < 1 || n > kTopkMax || k < 1 || k > n)
    return mfail(DTB_ERR_INVALID, "top-k needs 1 <= k <= n <= 4096");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (on_device) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, n, k, score, idx);
    MLP_HIP(hipGetLastError());
    return DTB_OK;
  }
  float* ds = nullptr;
  int32_t* di = nullptr;
  hipError_t e = hipMalloc(&ds, size_t(n) * 4);
  if (e == hipSuccess) e = hipMalloc(&di, size_t(k) * 4);
  if (e == hipSuccess) e = hipMemcpyAsync(ds, score, size_t(n) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, n, k, ds, di);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(idx, di, size_t(k) * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (ds) (void)hipFree(ds);
  if (di) (void)hipFree(di);
  if (e != hipSuccess) return mfail(DTB_ERR_HIP, std::string("top-k: ") + hipGetErrorString(e));
  return DTB_OK;
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// The device address of `scratch` on `dev`, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
hipError_t scratch_on(int dev, uint32_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_at[dev] = p;
  }
  *out = static_cast<uint32_t*>(g_scratch_at[dev]);
  return hipSuccess;
}

}  // namespace

extern "C" {

dtb_status dtb_topk_noalloc(const float* score, int32_t n, int32_t k, int32_t* idx, void* hip_stream) {
  if (!score || !idx) return mfail(DTB_ERR_INVALID, "top-k (no allocation): score and idx must not be NULL");
  if (n < 1 || k < 1 || k > n) return mfail(DTB_ERR_INVALID, "top-k (no allocation) needs 1 <= k <= n");
  if (n > kTopkMax)
    return mfail(DTB_ERR_INVALID, "top-k (no allocation): n = " + std::to_string(n) +
                                      " exceeds the 4096 scores its static staging area holds");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int dev = -1;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  uint32_t* base = nullptr;
  if (e == hipSuccess) e = scratch_on(dev, &base);
  if (e != hipSuccess) return mfail(DTB_ERR_HIP, std::string("top-k (no allocation): ") + hipGetErrorString(e));
  float* ds = reinterpret_cast<float*>(base);            // [n] scores
  int32_t* di = reinterpret_cast<int32_t*>(base + kTopkMax);  // [k] indices
  e = hipMemcpyAsync(ds, score, size_t(n) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, n, k, ds, di);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(idx, di, size_t(k) * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return mfail(DTB_ERR_HIP, std::string("top-k (no allocation): ") + hipGetErrorString(e));
  return DTB_OK;
}

}  // extern "C"
