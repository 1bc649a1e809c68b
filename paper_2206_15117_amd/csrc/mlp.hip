// Kernel surrogate network on gfx950: a multilayer perceptron with BF16 weights and activations,
// FP32 accumulation on the matrix cores, FP32 master weights and Adam.
//
//   h_0 = x (features), h_l = SiLU(h_{l-1} W_l + b_l) for the hidden layers, y = h_L W_out + b_out.
//
// GEMM: C[M][N] (float) (+)= A[M][K] B[K][N] with bf16 operands given by arbitrary strides, so the
// forward product, the input gradient (B = W^T) and the weight gradient (A = h^T) share one
// kernel.  64x64 output tile per 256-thread workgroup, four waves of 32x32, K in steps of 32
// staged through LDS ([m][k] for A and [n][k] for B so each lane's four consecutive k values are
// one 8-byte read), v_mfma_f32_32x32x8_bf16, optional split-K with float atomics.
#include "common.hpp"
#include "mlp.hpp"

#include <cmath>

namespace pg {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

constexpr int TM = 64, TN = 64, TK = 32, KP = TK + 4;  // LDS row pitch in bf16 (8-byte aligned rows)

__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A,
                                                        int64_t sam, int64_t sak, const uint16_t* __restrict__ B,
                                                        int64_t sbk, int64_t sbn, float* __restrict__ C, int64_t ldc,
                                                        int ksplit, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t as[TM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t bs[TN][KP];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * ksplit, ke = min(K, kb + ksplit);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    for (int e = tid; e < TM * TK; e += 256) {
      const int mm = e / TK, kk = e % TK;
      const int gm = m0 + mm, gk = k0 + kk;
      as[mm][kk] = (gm < M && gk < ke) ? A[gm * sam + gk * sak] : uint16_t(0);
    }
    for (int e = tid; e < TN * TK; e += 256) {
      const int nn = e % TN, kk = e / TN;
      const int gn = n0 + nn, gk = k0 + kk;
      bs[nn][kk] = (gn < N && gk < ke) ? B[gk * sbk + gn * sbn] : uint16_t(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 8) {
      const int ko = kk + 4 * (lane >> 5);
      bf16x4 a, b;
      __builtin_memcpy(&a, &as[wm + (lane & 31)][ko], 8);
      __builtin_memcpy(&b, &bs[wn + (lane & 31)][ko], 8);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32 of the wave tile
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int j = n0 + wn + (lane & 31);
    if (i < M && j < N) {
      float* c = C + static_cast<int64_t>(i) * ldc + j;
      if (gridDim.z > 1) {
        unsafeAtomicAdd(c, acc[r]);
      } else if (accumulate) {
        *c += acc[r];
      } else {
        *c = acc[r];
      }
    }
  }
}

// y = x + b (row broadcast); a = SiLU(y) in bf16 when silu, else y stays float (output layer)
__global__ void bias_act_kernel(float* __restrict__ y, const float* __restrict__ b, int64_t rows, int64_t cols, int silu,
                                uint16_t* __restrict__ act) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float v = y[i] + b[i % cols];
    y[i] = v;
    if (silu) act[i] = f2bf(v / (1.0f + __expf(-v)));
  }
}

// grad of SiLU: g_pre = g_act * s (1 + z (1 - s)), s = sigmoid(z); output bf16 for the next GEMMs
__global__ void silu_back_kernel(const float* __restrict__ gact, const float* __restrict__ z, int64_t n,
                                 float* __restrict__ gpre, uint16_t* __restrict__ gpre_bf) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float s = 1.0f / (1.0f + __expf(-z[i]));
    const float g = gact[i] * s * (1.0f + z[i] * (1.0f - s));
    gpre[i] = g;
    gpre_bf[i] = f2bf(g);
  }
}

// Normalised squared error per sample: L = (1/B) sum_b |y_b - t_b|^2 / |t_b|^2.
// One workgroup per sample: loss partial and dL/dy = 2 (y - t) / (B |t_b|^2) (float and bf16).
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                   int64_t cols, int batch, float* __restrict__ grad,
                                                   uint16_t* __restrict__ grad_bf, float* __restrict__ loss) {
  __shared__ float red[2][256];
  const int b = blockIdx.x;
  const float* yb = y + b * cols;
  const float* tb = t + b * cols;
  float se = 0.0f, st = 0.0f;
  for (int64_t j = threadIdx.x; j < cols; j += 256) {
    const float d = yb[j] - tb[j];
    se += d * d;
    st += tb[j] * tb[j];
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = st;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  const float norm = fmaxf(red[1][0], 1e-30f);
  if (threadIdx.x == 0) unsafeAtomicAdd(loss, red[0][0] / norm / batch);
  const float sc = 2.0f / (batch * norm);
  for (int64_t j = threadIdx.x; j < cols; j += 256) {
    const float g = sc * (yb[j] - tb[j]);
    grad[b * cols + j] = g;
    grad_bf[b * cols + j] = f2bf(g);
  }
}

// bias gradient: column sums of g [rows][cols]
__global__ void colsum_kernel(const float* __restrict__ g, int64_t rows, int64_t cols, float* __restrict__ out) {
  const int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int64_t r = 0; r < rows; ++r) s += g[r * cols + j];
  out[j] = s;
}

__global__ void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ w_bf, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                            float omb1, float omb2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (w_bf) w_bf[i] = f2bf(wi);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = f2bf(x[i]);
}

// Counter-based uniform numbers (splitmix64 of seed + index), published generator; weights are
// U(-a, a) with a = sqrt(6 / fan_in) for SiLU layers and sqrt(3 / fan_in) for the output layer.
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void init_uniform_kernel(float* __restrict__ w, int64_t n, uint64_t seed, float a) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double u = static_cast<double>(splitmix64(seed + static_cast<uint64_t>(i)) >> 11) * (1.0 / 9007199254740992.0);
    w[i] = static_cast<float>((2.0 * u - 1.0) * a);
  }
}

__global__ void zero_rows_kernel(float* __restrict__ c, int64_t ldc, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) c[blockIdx.x * ldc + j] = 0.0f;
}

inline dim3 grid_1d(int64_t n) { return dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536))); }

}  // namespace

hipError_t mlp_gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                    int64_t sbn, float* C, int64_t ldc, bool accumulate, int split_k, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  int ksplit = K;
  if (split_k > 1) ksplit = ((K + split_k - 1) / split_k + TK - 1) / TK * TK;
  const int nz = (K + ksplit - 1) / ksplit;
  if (nz > 1 && !accumulate) {  // split-K partial tiles are added atomically onto zero
    hipLaunchKernelGGL(zero_rows_kernel, dim3(M), dim3(256), 0, s, C, ldc, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, nz);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, ksplit,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t mlp_bias_act(float* y, const float* b, int64_t rows, int64_t cols, bool silu, uint16_t* act, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, grid_1d(rows * cols), dim3(256), 0, s, y, b, rows, cols, silu ? 1 : 0, act);
  return hipGetLastError();
}

hipError_t mlp_silu_back(const float* gact, const float* z, int64_t n, float* gpre, uint16_t* gpre_bf, hipStream_t s) {
  hipLaunchKernelGGL(silu_back_kernel, grid_1d(n), dim3(256), 0, s, gact, z, n, gpre, gpre_bf);
  return hipGetLastError();
}

hipError_t mlp_loss(const float* y, const float* t, int64_t cols, int batch, float* grad, uint16_t* grad_bf,
                    float* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(batch), dim3(256), 0, s, y, t, cols, batch, grad, grad_bf, loss);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float* g, int64_t rows, int64_t cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(static_cast<unsigned>((cols + 255) / 256)), dim3(256), 0, s, g, rows, cols, out);
  return hipGetLastError();
}

// The decay rates, their complements and the bias corrections are formed in float64 on the host and
// rounded once: 1 - 0.999f in float32 is 1.3e-5 away from 0.001, which the second moment would carry.
hipError_t mlp_adam(float* w, uint16_t* w_bf, const float* g, float* m, float* v, int64_t n, float lr, double b1,
                    double b2, double eps, int64_t step, hipStream_t s) {
  const float c1 = static_cast<float>(1.0 / (1.0 - std::pow(b1, static_cast<double>(step))));
  const float c2 = static_cast<float>(1.0 / (1.0 - std::pow(b2, static_cast<double>(step))));
  hipLaunchKernelGGL(adam_kernel, grid_1d(n), dim3(256), 0, s, w, w_bf, g, m, v, n, lr, static_cast<float>(b1),
                     static_cast<float>(b2), static_cast<float>(1.0 - b1), static_cast<float>(1.0 - b2),
                     static_cast<float>(eps), c1, c2);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* x, int64_t n, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, grid_1d(n), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t mlp_init_uniform(float* w, int64_t n, uint64_t seed, float a, hipStream_t s) {
  hipLaunchKernelGGL(init_uniform_kernel, grid_1d(n), dim3(256), 0, s, w, n, seed, a);
  return hipGetLastError();
}

}  // namespace pg
