// Kernel surrogate network on gfx950: a multilayer perceptron with BF16 weights and activations,
// FP32 accumulation on the matrix cores, FP32 master weights and Adam.
//
//   h_0 = x (features), h_l = SiLU(h_{l-1} W_l + b_l) for the hidden layers, y = h_L W_out + b_out.
//
// GEMMs (C (+)= A B) run on the matrix cores with bf16 operands and float accumulation; the forward
// product, the input gradient (B = W^T) and the weight gradient (A = h^T) share one kernel that
// takes each operand either k-contiguous or row-contiguous.  Bias and SiLU are fused into the
// forward products' epilogue.
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

// GEMM C[M][N] (+)= A[M][K] B[K][N], bf16 operands, float accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16).  A is given k-contiguous ([M][K], row stride lda) or m-contiguous
// ([K][M]); B k-contiguous ([N][K], row stride ldb) or n-contiguous ([K][N]).  Each 256-thread
// workgroup computes a 128 x 128 tile, each wave 64 x 64 (2 x 2 MFMA tiles of 32 x 32).  Tiles of
// 128 rows x 32 k of both operands are staged in LDS as [row][k] (k-contiguous rows of 40 bf16,
// the four 8-element k chunks of a row XOR-swizzled by row / 8 so the 16-byte operand reads of 8
// lanes cover all 32 banks and the transposing stores spread over 16), double-buffered: the next
// k-step's global loads are in flight while the current one feeds the matrix cores, and one
// barrier per k-step separates the buffers.  Row-contiguous operands are transposed while being
// written into LDS.  The epilogue (store, accumulate, atomic add for a split contraction, or store
// with bias and optionally SiLU in bf16) is a template parameter.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32, LP = BK + 8;
enum GemmEpi { kEpiStore, kEpiAccumulate, kEpiAtomic, kEpiBias, kEpiBiasSilu };

// bf16 element offset of (row, k) in a staged tile: chunk k / 8 swizzled by (row / 8) mod 4
__device__ __forceinline__ int lds_at(int row, int k) { return row * LP + ((((k >> 3) ^ (row >> 3)) & 3) << 3) + (k & 7); }

// One operand tile (128 rows x BK) into registers: two 8-element chunks per thread.  k-contiguous
// sources: thread chunk c is row c / 4, k chunk c % 4.  Row-contiguous sources: c is k = c % 32,
// rows 8 (c / 32) .. + 7, so the lanes of a wave write 32 different k of one row into LDS.
template <bool KCONTIG, bool VEC>
struct TileLoader {
  u32x4 r[2];
  __device__ void load(const uint16_t* __restrict__ X, int64_t ld, int rows, int K, int row0, int k0, int tid) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + h * 256;
      const int row = KCONTIG ? c >> 2 : (c >> 5) * 8;
      const int k = KCONTIG ? (c & 3) * 8 : c & 31;
      const int gr = row0 + row, gk = k0 + k;
      const bool whole = VEC && (KCONTIG ? (gr < rows && gk + 8 <= K) : (gk < K && gr + 8 <= rows));
      if (whole) {
        const uint16_t* p = KCONTIG ? X + static_cast<int64_t>(gr) * ld + gk : X + static_cast<int64_t>(gk) * ld + gr;
        r[h] = *reinterpret_cast<const u32x4*>(p);
      } else {
        uint16_t e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int rr = KCONTIG ? gr : gr + i, kk = KCONTIG ? gk + i : gk;
          e[i] = (rr < rows && kk < K) ? X[KCONTIG ? static_cast<int64_t>(rr) * ld + kk : static_cast<int64_t>(kk) * ld + rr]
                                       : uint16_t(0);
        }
        __builtin_memcpy(&r[h], e, 16);
      }
    }
  }
  __device__ void store(uint16_t* S, int tid) const {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + h * 256;
      if constexpr (KCONTIG) {
        *reinterpret_cast<u32x4*>(S + lds_at(c >> 2, (c & 3) * 8)) = r[h];
      } else {
        uint16_t e[8];
        __builtin_memcpy(e, &r[h], 16);
        const int k = c & 31, row = (c >> 5) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) S[lds_at(row + i, k)] = e[i];
      }
    }
  }
};

template <bool A_K, bool B_K, bool VEC, int EPI>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K, const uint16_t* __restrict__ A,
                                                        int64_t lda, const uint16_t* __restrict__ B, int64_t ldb,
                                                        float* __restrict__ C, int64_t ldc, int ksplit,
                                                        const float* __restrict__ bias, uint16_t* __restrict__ act) {
  __shared__ __attribute__((aligned(16))) uint16_t as[2][BM * LP];
  __shared__ __attribute__((aligned(16))) uint16_t bs[2][BN * LP];
  // Workgroups are dealt to the 8 XCDs round-robin in launch order (x fastest), so with the plain
  // mapping the M tiles that share a B tile land on every XCD and each XCD's L2 fetches every B
  // tile.  When the tile count allows, XCD x takes the x-th contiguous eighth of the tiles (M tile
  // fastest): each B tile is then read into one L2 only.
  int mt = blockIdx.x, nt = blockIdx.y;
  {
    const int ntiles = gridDim.x * gridDim.y;
    if ((ntiles & 7) == 0 && ntiles >= 64) {
      const int lin = blockIdx.x + gridDim.x * blockIdx.y;
      const int logical = (lin & 7) * (ntiles >> 3) + (lin >> 3);
      mt = logical % gridDim.x;
      nt = logical / gridDim.x;
    }
  }
  const int m0 = mt * BM, n0 = nt * BN;
  const int kb = blockIdx.z * ksplit, ke = min(K, kb + ksplit);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  TileLoader<A_K, VEC> la;
  TileLoader<B_K, VEC> lb;
  la.load(A, lda, M, ke, m0, kb, tid);
  lb.load(B, ldb, N, ke, n0, kb, tid);
  la.store(as[0], tid);
  lb.store(bs[0], tid);
  __syncthreads();
  int cur = 0;
  for (int k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) {
      la.load(A, lda, M, ke, m0, k0 + BK, tid);
      lb.load(B, ldb, N, ke, n0, k0 + BK, tid);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int ko = ks + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        __builtin_memcpy(&a[i], &as[cur][lds_at(wm + i * 32 + (lane & 31), ko)], 16);
        __builtin_memcpy(&b[i], &bs[cur][lds_at(wn + i * 32 + (lane & 31), ko)], 16);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      la.store(as[cur ^ 1], tid);
      lb.store(bs[cur ^ 1], tid);
    }
    __syncthreads();
    cur ^= 1;
  }
  // accumulator r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32 of a 32 x 32 tile
  const bool inside = m0 + BM <= M && n0 + BN <= N;
  if constexpr (EPI == kEpiStore || EPI == kEpiBias) {
    // Whole tiles of a 16-byte aligned output: each wave stages one 32 x 32 block at a time in
    // its own 4 KiB of the (now idle) operand LDS and writes it back as rows of 16-byte streaming
    // stores, 8 lanes per 128-byte row: a quarter of the store instructions of the per-element
    // path below.  The final barrier of the k loop has retired every operand read.
    if (inside && (ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0) {
      float* stage = reinterpret_cast<float*>(&as[0][0]) + wave * 1024;  // [32][32]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int r = 0; r < 16; ++r) stage[(8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * 32 + (lane & 31)] = acc[i][j][r];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int c4 = (lane & 7) * 4;
          const int col = n0 + wn + j * 32 + c4;
          f32x4 bv = {0.0f, 0.0f, 0.0f, 0.0f};
          if constexpr (EPI == kEpiBias) bv = *reinterpret_cast<const f32x4*>(bias + col);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int rr = (lane >> 3) + 8 * k;
            const f32x4 v = *reinterpret_cast<const f32x4*>(stage + rr * 32 + c4) + bv;
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(C + static_cast<int64_t>(m0 + wm + i * 32 + rr) * ldc + col));
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      return;
    }
  }
  float bj[2] = {0.0f, 0.0f};
  if constexpr (EPI == kEpiBias || EPI == kEpiBiasSilu) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 32 + (lane & 31);
      bj[j] = col < N ? bias[col] : 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = n0 + wn + j * 32 + (lane & 31);
        if (inside || (row < M && col < N)) {
          float* c = C + static_cast<int64_t>(row) * ldc + col;
          float v = acc[i][j][r];
          if constexpr (EPI == kEpiAtomic) {
            unsafeAtomicAdd(c, v);
          } else {
            if constexpr (EPI == kEpiAccumulate) v += *c;
            if constexpr (EPI == kEpiBias || EPI == kEpiBiasSilu) v += bj[j];
            if constexpr (EPI == kEpiBias || EPI == kEpiStore)
              __builtin_nontemporal_store(v, c);  // streamed output: keep L2 for the weight tiles
            else
              *c = v;
            if constexpr (EPI == kEpiBiasSilu)
              act[static_cast<int64_t>(row) * ldc + col] = f2bf(__fdividef(v, 1.0f + __expf(-v)));
          }
        }
      }
}

// FP32 GEMM on the vector ALU for the surrogate's basis, projections and fold (float32 data,
// float32 accumulation): C = alpha op(A) op(B) (+ beta C), row-major, op = identity or transpose.
// 64 x 64 output tile per 256-thread workgroup, 4 x 4 per thread, k in steps of 16 staged in LDS as
// [k][row] (rows contiguous) so each thread reads its four rows and four columns as float4; a split
// contraction (gridDim.z > 1) adds alpha-scaled partial tiles atomically onto C.
constexpr int SG = 64, SK = 16, SP = SG + 4;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void sgemm_kernel(int64_t M, int64_t N, int64_t K, float alpha,
                                                    const float* __restrict__ A, int64_t lda,
                                                    const float* __restrict__ B, int64_t ldb, float beta,
                                                    float* __restrict__ C, int64_t ldc, int64_t ksplit) {
  __shared__ __attribute__((aligned(16))) float as[SK][SP];
  __shared__ __attribute__((aligned(16))) float bs[SK][SP];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * SG, n0 = static_cast<int64_t>(blockIdx.y) * SG;
  const int64_t kb = static_cast<int64_t>(blockIdx.z) * ksplit, ke = min(K, kb + ksplit);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  float acc[4][4] = {};
  for (int64_t k0 = kb; k0 < ke; k0 += SK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + i * 256;
      // A tile: element (m, k); k-contiguous (TA false) or m-contiguous (TA true) in memory
      const int am = TA ? e & 63 : e >> 4, ak = TA ? e >> 6 : e & 15;
      const int64_t gm = m0 + am, gk = k0 + ak;
      as[ak][am] = (gm < M && gk < ke) ? (TA ? A[gk * lda + gm] : A[gm * lda + gk]) : 0.0f;
      // B tile: element (k, n); n-contiguous (TB false) or k-contiguous (TB true)
      const int bn = TB ? e >> 4 : e & 63, bk = TB ? e & 15 : e >> 6;
      const int64_t gn = n0 + bn, gk2 = k0 + bk;
      bs[bk][bn] = (gn < N && gk2 < ke) ? (TB ? B[gn * ldb + gk2] : B[gk2 * ldb + gn]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SK; ++kk) {
      const float4 a = *reinterpret_cast<const float4*>(&as[kk][ty * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&bs[kk][tx * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = m0 + ty * 4 + i;
    if (row >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + tx * 4 + j;
      if (col >= N) continue;
      float* c = C + row * ldc + col;
      if (gridDim.z > 1) {
        unsafeAtomicAdd(c, alpha * acc[i][j]);
      } else {
        *c = beta == 0.0f ? alpha * acc[i][j] : fmaf(beta, *c, alpha * acc[i][j]);
      }
    }
  }
}

__global__ void scale_matrix_kernel(float* __restrict__ c, int64_t rows, int64_t cols, int64_t ldc, float beta) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float* p = c + (i / cols) * ldc + i % cols;
    *p = beta == 0.0f ? 0.0f : beta * *p;
  }
}

// x[r][c] *= scale[r]
__global__ void scale_rows_kernel(float* __restrict__ x, int64_t rows, int64_t cols, const float* __restrict__ scale) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] *= scale[i / cols];
}

// Transpose of a bf16 matrix: out[c][r] = in[r][c], in [rows][cols]; 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t* __restrict__ in, int64_t rows,
                                                             int64_t cols, uint16_t* __restrict__ out) {
  __shared__ uint16_t t[32][33];
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 32, c0 = static_cast<int64_t>(blockIdx.x) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8)
    if (r0 + y < rows && c0 + tx < cols) t[y][tx] = in[(r0 + y) * cols + c0 + tx];
  __syncthreads();
  for (int y = ty; y < 32; y += 8)
    if (c0 + y < cols && r0 + tx < rows) out[(c0 + y) * rows + r0 + tx] = t[tx][y];
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

template <bool A_K, bool B_K, int EPI>
hipError_t launch_gemm(int M, int N, int K, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, float* C,
                       int64_t ldc, int ksplit, int nz, const float* bias, uint16_t* act, bool vec, hipStream_t s) {
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, nz);
  if (vec)
    hipLaunchKernelGGL((gemm_mfma_kernel<A_K, B_K, true, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, ksplit, bias, act);
  else
    hipLaunchKernelGGL((gemm_mfma_kernel<A_K, B_K, false, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, ksplit, bias, act);
  return hipGetLastError();
}

template <bool A_K, bool B_K>
hipError_t launch_gemm_epi(int M, int N, int K, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb,
                           float* C, int64_t ldc, int ksplit, int nz, bool accumulate, const float* bias,
                           uint16_t* act, bool vec, hipStream_t s) {
  if (nz > 1)
    return launch_gemm<A_K, B_K, kEpiAtomic>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, bias, act, vec, s);
  if (accumulate)
    return launch_gemm<A_K, B_K, kEpiAccumulate>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, bias, act, vec, s);
  if (bias && act)
    return launch_gemm<A_K, B_K, kEpiBiasSilu>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, bias, act, vec, s);
  if (bias) return launch_gemm<A_K, B_K, kEpiBias>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, bias, act, vec, s);
  return launch_gemm<A_K, B_K, kEpiStore>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, bias, act, vec, s);
}

hipError_t mlp_gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                    int64_t sbn, float* C, int64_t ldc, bool accumulate, int split_k, hipStream_t s, const float* bias,
                    uint16_t* act) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  // each operand needs a unit stride along k or along its row index
  const bool a_k = sak == 1, b_k = sbk == 1;
  if (!(a_k || sam == 1) || !(b_k || sbn == 1)) return hipErrorInvalidValue;
  if (act && !bias) return hipErrorInvalidValue;
  const int64_t lda = a_k ? sam : sak, ldb = b_k ? sbn : sbk;
  int ksplit = K;
  if (split_k > 1) ksplit = ((K + split_k - 1) / split_k + BK - 1) / BK * BK;
  const int nz = (K + ksplit - 1) / ksplit;
  if (nz > 1 && bias) return hipErrorInvalidValue;  // the bias epilogue needs whole sums
  if (nz > 1 && !accumulate) {  // split-K partial tiles are added atomically onto zero (or onto C)
    hipLaunchKernelGGL(zero_rows_kernel, dim3(M), dim3(256), 0, s, C, ldc, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // 16-byte operand loads need 16-byte aligned rows (bf16 row stride a multiple of 8)
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0) &&
                   lda % 8 == 0 && ldb % 8 == 0;
  if (a_k && b_k)
    return launch_gemm_epi<true, true>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, accumulate, bias, act, vec, s);
  if (a_k)
    return launch_gemm_epi<true, false>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, accumulate, bias, act, vec, s);
  if (b_k)
    return launch_gemm_epi<false, true>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, accumulate, bias, act, vec, s);
  return launch_gemm_epi<false, false>(M, N, K, A, lda, B, ldb, C, ldc, ksplit, nz, accumulate, bias, act, vec, s);
}

hipError_t gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                    const float* B, int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tiles = ((M + SG - 1) / SG) * ((N + SG - 1) / SG);
  // split a deep contraction when the output tiles alone cannot fill the GPU (about 1024 workgroups)
  int64_t nz = 1;
  if (tiles < 1024 && K >= 2048) nz = std::min<int64_t>((1024 + tiles - 1) / tiles, K / 1024);
  nz = std::max<int64_t>(1, std::min<int64_t>(nz, 1024));
  const int64_t ksplit = ((K + nz - 1) / nz + SK - 1) / SK * SK;
  nz = K > 0 ? (K + ksplit - 1) / ksplit : 1;
  if (nz > 1 || K <= 0) {  // partial tiles go onto beta C
    hipLaunchKernelGGL(scale_matrix_kernel, grid_1d(M * N), dim3(256), 0, s, C, M, N, ldc, beta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || K <= 0) return e;
  }
  dim3 grid(static_cast<unsigned>((M + SG - 1) / SG), static_cast<unsigned>((N + SG - 1) / SG),
            static_cast<unsigned>(nz));
  if (ta && tb)
    hipLaunchKernelGGL((sgemm_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit);
  else if (ta)
    hipLaunchKernelGGL((sgemm_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit);
  else if (tb)
    hipLaunchKernelGGL((sgemm_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit);
  else
    hipLaunchKernelGGL((sgemm_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit);
  return hipGetLastError();
}

hipError_t scale_rows(float* x, int64_t rows, int64_t cols, const float* scale, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_rows_kernel, grid_1d(rows * cols), dim3(256), 0, s, x, rows, cols, scale);
  return hipGetLastError();
}

hipError_t mlp_transpose_bf16(const uint16_t* in, int64_t rows, int64_t cols, uint16_t* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>((cols + 31) / 32), static_cast<unsigned>((rows + 31) / 32));
  hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(256), 0, s, in, rows, cols, out);
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
