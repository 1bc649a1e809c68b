// Gridding, degridding and taper correction on gfx950.
//
// Gridding (Sec. 3.2, gridding stage) and degridding (Sec. 3.2, degridding
// stage) with 4x4 Mueller kernels.  One workgroup takes one work item: a chunk
// of visibilities that share a w-plane and a uv tile (binned by the plan,
// phase-sorted inside the tile so neighbouring visibilities reuse table lines
// in cache).  The tile's sub-grid of (T + S - 1)^2 points x npol lives in LDS,
// planar [q][re|im][y][x] so the 64 lanes of a wave, which walk consecutive
// taps of one visibility, hit consecutive banks.
//   grid:   each wave takes one visibility at a time; lane t owns tap t; the
//           npol x npol Mueller product is done in registers and added into
//           the LDS sub-grid with LDS float atomics (waves overlap); the
//           sub-grid is flushed with coalesced global float atomics.
//   degrid: the sub-grid is loaded once into LDS; each wave reduces one
//           visibility's taps with cross-lane shuffles.
#include "common.hpp"

namespace pg {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

__device__ inline int ceil_div_i(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

template <int NQC>
__device__ inline void load_taps(const float2* __restrict__ p, float2 (&t)[NQC]) {
  if constexpr (NQC % 2 == 0) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < NQC / 2; ++i) {
      const float4 v = q[i];
      t[2 * i] = make_float2(v.x, v.y);
      t[2 * i + 1] = make_float2(v.z, v.w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NQC; ++i) t[i] = p[i];
  }
}

template <int NQC>
__device__ inline void load_taps(const __half2* __restrict__ p, float2 (&t)[NQC]) {
  if constexpr (NQC % 4 == 0) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < NQC / 4; ++i) {
      const uint4 v = q[i];
      const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        __half2 h;
        __builtin_memcpy(&h, &w[j], 4);
        t[4 * i + j] = __half22float2(h);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NQC; ++i) t[i] = __half22float2(p[i]);
  }
}

template <int NP, typename TapT>
__global__ __launch_bounds__(kThreads) void grid_kernel(const Item* __restrict__ items, const int2* __restrict__ fine,
                                                        const int32_t* __restrict__ perm,
                                                        const float2* __restrict__ vis,
                                                        const TapT* __restrict__ table,
                                                        const PlaneInfo* __restrict__ planes, int os, int n,
                                                        float2* __restrict__ grid, int flags) {
  extern __shared__ float lds[];
  const Item it = items[blockIdx.x];
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, WW = W * W, SS = S * S, half = S * os / 2;
  const float inv_s = 1.0f / static_cast<float>(S);
  for (int i = threadIdx.x; i < 2 * NP * WW; i += kThreads) lds[i] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = it.start + wave; i < it.end; i += kWaves) {
    const int2 f = fine[i];
    const int k = perm[i];
    const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
    const int phx = x0 * os - f.x + half - 1, phy = y0 * os - f.y + half - 1;
    float2 v[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) v[c] = vis[static_cast<size_t>(k) * NP + c];
    const TapT* base = table + pl.offset + static_cast<size_t>(phy * os + phx) * SS * NP * NP;
    const int lx = x0 - it.ox, ly = y0 - it.oy;
    for (int t = lane; t < SS; t += 64) {
      const int ty = static_cast<int>((static_cast<float>(t) + 0.5f) * inv_s);
      const int tx = t - ty * S;
      float2 tap[NP * NP];
      load_taps<NP * NP>(base + static_cast<size_t>(t) * NP * NP, tap);
      const int off = (ly + ty) * W + lx + tx;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        float re = 0.0f, im = 0.0f;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const float2 a = tap[q * NP + c];
          re = fmaf(a.x, v[c].x, fmaf(-a.y, v[c].y, re));
          im = fmaf(a.x, v[c].y, fmaf(a.y, v[c].x, im));
        }
        atomicAdd(&lds[(2 * q) * WW + off], re);
        atomicAdd(&lds[(2 * q + 1) * WW + off], im);
      }
    }
  }
  __syncthreads();
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  for (int idx = threadIdx.x; idx < WW; idx += kThreads) {
    const int y = idx / W, x = idx - y * W;
    const int X = it.ox + x, Y = it.oy + y;
    if (X >= n || Y >= n) continue;
    const float sg = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const float re = lds[(2 * q) * WW + idx], im = lds[(2 * q + 1) * WW + idx];
      if (re != 0.0f || im != 0.0f) {
        float* g = reinterpret_cast<float*>(grid + q * pstride + static_cast<size_t>(Y) * n + X);
        unsafeAtomicAdd(g, sg * re);
        unsafeAtomicAdd(g + 1, sg * im);
      }
    }
  }
}

template <int NP, typename TapT>
__global__ __launch_bounds__(kThreads) void degrid_kernel(const Item* __restrict__ items,
                                                          const int2* __restrict__ fine,
                                                          const int32_t* __restrict__ perm,
                                                          const TapT* __restrict__ table,
                                                          const PlaneInfo* __restrict__ planes, int os, int n,
                                                          const float2* __restrict__ grid,
                                                          float2* __restrict__ vis_out, int flags) {
  extern __shared__ float lds[];
  const Item it = items[blockIdx.x];
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, WW = W * W, SS = S * S, half = S * os / 2;
  const float inv_s = 1.0f / static_cast<float>(S);
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  for (int idx = threadIdx.x; idx < WW; idx += kThreads) {
    const int y = idx / W, x = idx - y * W;
    const int X = it.ox + x, Y = it.oy + y;
    const bool in = X < n && Y < n;
    const float sg = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      float2 g = in ? grid[q * pstride + static_cast<size_t>(Y) * n + X] : make_float2(0.0f, 0.0f);
      lds[(2 * q) * WW + idx] = sg * g.x;
      lds[(2 * q + 1) * WW + idx] = sg * g.y;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = it.start + wave; i < it.end; i += kWaves) {
    const int2 f = fine[i];
    const int k = perm[i];
    const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
    const int phx = x0 * os - f.x + half - 1, phy = y0 * os - f.y + half - 1;
    const TapT* base = table + pl.offset + static_cast<size_t>(phy * os + phx) * SS * NP * NP;
    const int lx = x0 - it.ox, ly = y0 - it.oy;
    float acc[2 * NP];
#pragma unroll
    for (int c = 0; c < 2 * NP; ++c) acc[c] = 0.0f;
    for (int t = lane; t < SS; t += 64) {
      const int ty = static_cast<int>((static_cast<float>(t) + 0.5f) * inv_s);
      const int tx = t - ty * S;
      float2 tap[NP * NP];
      load_taps<NP * NP>(base + static_cast<size_t>(t) * NP * NP, tap);
      const int off = (ly + ty) * W + lx + tx;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const float gr = lds[(2 * q) * WW + off], gi = lds[(2 * q + 1) * WW + off];
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const float2 a = tap[q * NP + c];  // conj(a) * g
          acc[2 * c] = fmaf(a.x, gr, fmaf(a.y, gi, acc[2 * c]));
          acc[2 * c + 1] = fmaf(a.x, gi, fmaf(-a.y, gr, acc[2 * c + 1]));
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 2 * NP; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < NP; ++c) vis_out[static_cast<size_t>(k) * NP + c] = make_float2(acc[2 * c], acc[2 * c + 1]);
    }
  }
}

__global__ void zero_dropped(const int32_t* __restrict__ perm, int64_t n_kept, int64_t nvis, int np,
                             float2* __restrict__ vis_out) {
  const int64_t i = n_kept + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvis) return;
  const int64_t k = perm[i];
  for (int c = 0; c < np; ++c) vis_out[k * np + c] = make_float2(0.0f, 0.0f);
}

__global__ void fill_zero_kernel(uint64_t* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ void taper_image_kernel(const float2* __restrict__ in, float* __restrict__ out, int n,
                                   const double* __restrict__ inv_aa, double inv_w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const size_t idx = (static_cast<size_t>(blockIdx.z) * n + i) * n + j;
  const double sc = inv_aa[i] * inv_aa[j] * inv_w * (((i + j) & 1) ? -1.0 : 1.0);
  out[idx] = static_cast<float>(in[idx].x * sc);
}

__global__ void taper_predict_kernel(const float* __restrict__ in, float2* __restrict__ out, int n,
                                     const double* __restrict__ inv_aa) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const size_t idx = (static_cast<size_t>(blockIdx.z) * n + i) * n + j;
  const double sc = inv_aa[i] * inv_aa[j] * (((i + j) & 1) ? -1.0 : 1.0);
  out[idx] = make_float2(static_cast<float>(in[idx] * sc), 0.0f);
}

template <class F>
hipError_t allow_lds(F* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

template <int NP, typename TapT>
hipError_t run_grid(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                    hipStream_t s) {
  auto fn = grid_kernel<NP, TapT>;
  hipError_t e = allow_lds(fn, k->lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(p->n_items)), dim3(kThreads), k->lds_bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->os, k->n, grid, flags);
  return hipGetLastError();
}

template <int NP, typename TapT>
hipError_t run_degrid(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                      hipStream_t s) {
  auto fn = degrid_kernel<NP, TapT>;
  hipError_t e = allow_lds(fn, k->lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(p->n_items)), dim3(kThreads), k->lds_bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->os, k->n, grid, vis, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>(std::min<size_t>((n + 255) / 256, 16384));
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint64_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_grid(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                       hipStream_t s) {
  if (!(flags & PG_ACCUMULATE)) {
    hipError_t e = launch_fill_zero(grid, static_cast<size_t>(k->npol) * k->n * k->n * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  if (p->n_items == 0) return hipSuccess;
  const bool f16 = k->storage == PG_STORE_F16;
  if (k->npol == 4) return f16 ? run_grid<4, __half2>(p, k, vis, grid, flags, s) : run_grid<4, float2>(p, k, vis, grid, flags, s);
  return f16 ? run_grid<1, __half2>(p, k, vis, grid, flags, s) : run_grid<1, float2>(p, k, vis, grid, flags, s);
}

hipError_t launch_degrid(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                         hipStream_t s) {
  if (p->nvis > p->n_kept) {
    const int64_t nd = p->nvis - p->n_kept;
    hipLaunchKernelGGL(zero_dropped, dim3(static_cast<unsigned>((nd + 255) / 256)), dim3(256), 0, s,
                       p->perm.as<int32_t>(), p->n_kept, p->nvis, k->npol, vis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p->n_items == 0) return hipSuccess;
  const bool f16 = k->storage == PG_STORE_F16;
  if (k->npol == 4) return f16 ? run_degrid<4, __half2>(p, k, grid, vis, flags, s) : run_degrid<4, float2>(p, k, grid, vis, flags, s);
  return f16 ? run_degrid<1, __half2>(p, k, grid, vis, flags, s) : run_degrid<1, float2>(p, k, grid, vis, flags, s);
}

hipError_t launch_taper(const pg_kernels* k, const void* in, void* out, int direction, double weight_sum,
                        hipStream_t s) {
  dim3 grid((k->n + 255) / 256, k->n, k->npol);
  if (direction == PG_TAPER_IMAGE) {
    hipLaunchKernelGGL(taper_image_kernel, grid, dim3(256), 0, s, static_cast<const float2*>(in),
                       static_cast<float*>(out), k->n, k->inv_aa.as<double>(), 1.0 / weight_sum);
  } else {
    hipLaunchKernelGGL(taper_predict_kernel, grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<float2*>(out), k->n, k->inv_aa.as<double>());
  }
  return hipGetLastError();
}

}  // namespace pg
