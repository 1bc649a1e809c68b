// Hogbom minor cycle of Cotton-Schwab clean (Sec. 2.1), entirely on the device.
//
// One iteration is three launches that never return to the host:
//   peak:     max over the masked pixels of |I| packed with the inverted pixel index into one
//             64-bit key (largest |I| wins, ties go to the lowest index), one 64-bit atomicMax
//             per workgroup into this iteration's slot;
//   pick:     one thread decodes the key; below the threshold (or with no pixel) it raises the
//             done flag, otherwise it records the component gain x residual[q][peak] for every
//             Stokes plane and adds it to the model image;
//   subtract: residual[q][y][x] -= value[q] x psf[y - py + n/2][x - px + n/2] inside the patch.
// Every kernel returns at once once the done flag is up, so the remaining launches of the
// iteration budget are empty.  The subtraction is written without contraction (product rounded,
// then difference rounded) so that the float32 reference reproduces it bit for bit.
#include "common.hpp"

#include <mutex>
#include <vector>

namespace pg {
namespace {

struct CleanState {
  int done;
  int ncomp;
};

__device__ inline unsigned long long peak_key(float a, int64_t idx) {
  return (static_cast<unsigned long long>(__float_as_uint(a)) << 32) |
         static_cast<unsigned long long>(0xFFFFFFFFu - static_cast<uint32_t>(idx));
}

__global__ __launch_bounds__(256) void peak_kernel(const float* __restrict__ stokes_i, const uint8_t* __restrict__ mask,
                                                   int64_t npix, unsigned long long* __restrict__ slot,
                                                   const CleanState* __restrict__ st) {
  if (st->done) return;
  unsigned long long best = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < npix;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (mask && !mask[i]) continue;
    const unsigned long long key = peak_key(fabsf(stokes_i[i]), i);
    best = key > best ? key : best;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  __shared__ unsigned long long wbest[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wbest[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = wbest[0];
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) b = wbest[w] > b ? wbest[w] : b;
    if (b) atomicMax(slot, b);
  }
}

__global__ void pick_kernel(float* __restrict__ residual, int npol, int64_t npix,
                            const unsigned long long* __restrict__ slot, float gain, float threshold,
                            CleanState* __restrict__ st, int32_t* __restrict__ comp_pos,
                            float* __restrict__ comp_val, float* __restrict__ model) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
  const unsigned long long key = *slot;
  const float a = __uint_as_float(static_cast<uint32_t>(key >> 32));
  if (key == 0 || !(a >= threshold)) {
    st->done = 1;
    return;
  }
  const int64_t idx = static_cast<int64_t>(0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFFu));
  const int k = st->ncomp;
  comp_pos[k] = static_cast<int32_t>(idx);
  for (int q = 0; q < npol; ++q) {
    const float v = gain * residual[q * npix + idx];
    comp_val[static_cast<int64_t>(k) * npol + q] = v;
    if (model) model[q * npix + idx] += v;
  }
  st->ncomp = k + 1;
}

__global__ __launch_bounds__(256) void subtract_kernel(float* __restrict__ residual, const float* __restrict__ psf,
                                                       int n, int npol, int patch,
                                                       const CleanState* __restrict__ st,
                                                       const int32_t* __restrict__ comp_pos,
                                                       const float* __restrict__ comp_val) {
#pragma clang fp contract(off)
  if (st->done) return;
  const int k = st->ncomp - 1;
  const int idx = comp_pos[k];
  const int py = idx / n, px = idx - py * n;
  // rows and columns where the shifted psf (centre n/2) is inside both images and the patch
  const int y0 = max(max(0, py - n / 2), py - patch), y1 = min(min(n, py + n / 2), py + patch + 1);
  const int x0 = max(max(0, px - n / 2), px - patch), x1 = min(min(n, px + n / 2), px + patch + 1);
  const int w = x1 - x0, h = y1 - y0;
  if (w <= 0 || h <= 0) return;
  const int64_t npix = static_cast<int64_t>(n) * n;
  const int area = w * h;  // at most n^2 < 2^31
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < area; t += gridDim.x * blockDim.x) {
    const int y = y0 + t / w, x = x0 + t % w;
    const float p = psf[static_cast<int64_t>(y - py + n / 2) * n + (x - px + n / 2)];
    for (int q = 0; q < npol; ++q) {
      const float prod = comp_val[static_cast<int64_t>(k) * npol + q] * p;
      float* r = residual + q * npix + static_cast<int64_t>(y) * n + x;
      *r = *r - prod;
    }
  }
}

__global__ void clean_init_kernel(CleanState* st, unsigned long long* slots, int nslots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    st->done = 0;
    st->ncomp = 0;
  }
  if (i < nslots) slots[i] = 0;
}

__global__ void clean_count_kernel(const CleanState* st, int32_t* n_comp) { *n_comp = st->ncomp; }

// img[i] / ref for every pixel, ref = img[ref_index] read first into `held` (one thread), so the
// division never sees a pixel already divided.
__global__ void hold_value_kernel(const float* __restrict__ img, int64_t ref_index, float* __restrict__ held) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *held = img[ref_index];
}

__global__ void divide_by_held_kernel(float* __restrict__ img, int64_t count, const float* __restrict__ held) {
  const float r = *held;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    img[i] = img[i] / r;
}

// Scratch of the allocation-free entry point: the iteration state (256 B) and one 64-bit peak
// slot per iteration, for at most kStaticMaxIter iterations.  Each GPU holds its own copy; host
// code reaches it only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kStaticScratchBytes = 256 + 8 * static_cast<size_t>(PG_HOGBOM_STATIC_MAX_ITER);
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
std::vector<void*> g_static_ptr;  // per device, looked up once with that device current

}  // namespace

hipError_t hogbom_static_scratch(void** out, size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (static_cast<size_t>(dev) >= g_static_ptr.size()) g_static_ptr.resize(dev + 1, nullptr);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

hipError_t launch_masked_peak(const float* img, const uint8_t* mask, int64_t npix, void* scratch, hipStream_t s) {
  auto* st = static_cast<CleanState*>(scratch);
  auto* slot = reinterpret_cast<unsigned long long*>(static_cast<char*>(scratch) + 256);
  hipLaunchKernelGGL(clean_init_kernel, dim3(1), dim3(64), 0, s, st, slot, 1);
  const int blocks = static_cast<int>(std::min<int64_t>((npix + 255) / 256, 1024));
  hipLaunchKernelGGL(peak_kernel, dim3(blocks), dim3(256), 0, s, img, mask, npix, slot, st);
  return hipGetLastError();
}

hipError_t launch_normalise_at(float* img, int64_t count, int64_t ref_index, float* held, hipStream_t s) {
  hipLaunchKernelGGL(hold_value_kernel, dim3(1), dim3(64), 0, s, img, ref_index, held);
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((count + 255) / 256, 4096));
  hipLaunchKernelGGL(divide_by_held_kernel, dim3(blocks), dim3(256), 0, s, img, count, held);
  return hipGetLastError();
}

hipError_t launch_hogbom(float* residual, const float* psf, const uint8_t* mask, int n, int npol, float gain,
                         float threshold, int patch, int max_iter, int32_t* comp_pos, float* comp_val, float* model,
                         int32_t* n_comp, void* scratch, hipStream_t s) {
  auto* st = static_cast<CleanState*>(scratch);
  auto* slots = reinterpret_cast<unsigned long long*>(static_cast<char*>(scratch) + 256);
  hipLaunchKernelGGL(clean_init_kernel, dim3((max_iter + 255) / 256 + 1), dim3(256), 0, s, st, slots, max_iter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t npix = static_cast<int64_t>(n) * n;
  const int peak_blocks = static_cast<int>(std::min<int64_t>((npix + 255) / 256, 1024));
  const int64_t area = static_cast<int64_t>(std::min(n, 2 * patch + 1)) * std::min(n, 2 * patch + 1);
  const int sub_blocks = static_cast<int>(std::min<int64_t>((area + 255) / 256, 2048));
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(peak_kernel, dim3(peak_blocks), dim3(256), 0, s, residual, mask, npix, slots + it, st);
    hipLaunchKernelGGL(pick_kernel, dim3(1), dim3(64), 0, s, residual, npol, npix, slots + it, gain, threshold, st,
                       comp_pos, comp_val, model);
    hipLaunchKernelGGL(subtract_kernel, dim3(sub_blocks), dim3(256), 0, s, residual, psf, n, npol, patch, st,
                       comp_pos, comp_val);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(clean_count_kernel, dim3(1), dim3(1), 0, s, st, n_comp);
  return hipGetLastError();
}

}  // namespace pg
