// Visibility binning: float64 uv snapping, w-plane choice, (plane, tile, phase)
// keys, a stable LSD radix sort and the chunked work-item list.
//
// The snapping arithmetic is written with floating-point contraction off so the
// fine-grid integers are the ones plain float64 multiply/add produces.
#include <climits>

#include "common.hpp"

namespace pg {
namespace {

__device__ inline int64_t ceil_div_pos(int64_t a, int64_t b) {  // b > 0
  return a >= 0 ? (a + b - 1) / b : -((-a) / b);
}

__global__ void plan_keys_kernel(const double* __restrict__ uvw, int64_t nvis, int n, double ncell,
                                 double half_n, int os, int nplanes, const double* __restrict__ w_planes,
                                 const PlaneInfo* __restrict__ planes, int nt, uint64_t drop_key,
                                 uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                 int2* __restrict__ fine_all) {
#pragma clang fp contract(off)
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= nvis) return;
  const double u = uvw[3 * k], v = uvw[3 * k + 1], w = uvw[3 * k + 2];
  const double x = u * ncell + half_n;
  const double y = v * ncell + half_n;
  const double fxd = floor(x * static_cast<double>(os) + 0.5);
  const double fyd = floor(y * static_cast<double>(os) + 0.5);
  uint64_t key = drop_key;
  int2 f = make_int2(0, 0);
  if (isfinite(fxd) && isfinite(fyd) && isfinite(w) && fabs(fxd) < 1e9 && fabs(fyd) < 1e9) {
    const int64_t fx = static_cast<int64_t>(fxd), fy = static_cast<int64_t>(fyd);
    int p = 0;
    double best = fabs(w - w_planes[0]);
    for (int q = 1; q < nplanes; ++q) {
      double d = fabs(w - w_planes[q]);
      if (d < best) {
        best = d;
        p = q;
      }
    }
    const PlaneInfo pi = planes[p];
    const int64_t S = pi.support, half = S * os / 2;
    const int64_t x0 = ceil_div_pos(fx - half + 1, os), y0 = ceil_div_pos(fy - half + 1, os);
    const int64_t phx = x0 * os - fx + half - 1, phy = y0 * os - fy + half - 1;
    if (x0 >= 0 && y0 >= 0 && x0 + S <= n && y0 + S <= n) {
      const uint64_t ty = static_cast<uint64_t>(y0 / pi.tile), tx = static_cast<uint64_t>(x0 / pi.tile);
      key = (((static_cast<uint64_t>(p) * nt + ty) * nt + tx) * os + static_cast<uint64_t>(phy)) * os +
            static_cast<uint64_t>(phx);
      f = make_int2(static_cast<int>(fx), static_cast<int>(fy));
    }
  }
  keys[k] = key;
  vals[k] = static_cast<int32_t>(k);
  fine_all[k] = f;
}

// ---------------------------------------------------------------- scans (int32, exclusive or inclusive)
constexpr int SCAN_THREADS = 256, SCAN_ITEMS = 8, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

struct OpSum {
  __device__ static int32_t id() { return 0; }
  __device__ static int32_t op(int32_t a, int32_t b) { return a + b; }
};

template <class Op>
__device__ int32_t block_exclusive(int32_t v, int32_t* sh, int32_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    int32_t t = tid >= off ? sh[tid - off] : Op::id();
    __syncthreads();
    sh[tid] = Op::op(sh[tid], t);
    __syncthreads();
  }
  int32_t incl = sh[tid];
  *total = sh[SCAN_THREADS - 1];
  int32_t excl = tid ? sh[tid - 1] : Op::id();
  __syncthreads();
  (void)incl;
  return excl;
}

template <class Op>
__global__ void tile_reduce(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ part) {
  __shared__ int32_t sh[SCAN_THREADS];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t acc = Op::id();
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) acc = Op::op(acc, in[base + i]);
  int32_t total;
  block_exclusive<Op>(acc, sh, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

template <class Op>
__global__ void tile_scan(const int32_t* in, int32_t* out, int64_t n, const int32_t* part_excl,
                          bool inclusive) {  // in may equal out: each thread reads its items before writing
  __shared__ int32_t sh[SCAN_THREADS];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t acc = Op::id();
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : Op::id();
    acc = Op::op(acc, v[i]);
  }
  int32_t total;
  int32_t run = block_exclusive<Op>(acc, sh, &total);
  if (part_excl) run = Op::op(part_excl[blockIdx.x], run);
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int32_t nxt = Op::op(run, v[i]);
    if (base + i < n) out[base + i] = inclusive ? nxt : run;
    run = nxt;
  }
}

template <class Op>
hipError_t scan(const int32_t* in, int32_t* out, int64_t n, bool inclusive, int32_t* scratch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles == 1) {
    hipLaunchKernelGGL(tile_scan<Op>, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n, nullptr, inclusive);
    return hipGetLastError();
  }
  int32_t* part = scratch;
  hipLaunchKernelGGL(tile_reduce<Op>, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, n, part);
  hipError_t e = scan<Op>(part, part, tiles, false, scratch + tiles, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tile_scan<Op>, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, out, n, part, inclusive);
  return hipGetLastError();
}

int64_t scan_scratch(int64_t n) {
  int64_t total = 0;
  while (n > SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    total += n;
  }
  return total + 16;
}

// ---------------------------------------------------------------- stable LSD radix sort, 8-bit digits
constexpr int RS_THREADS = 256, RS_ROUNDS = 16, RS_TILE = RS_THREADS * RS_ROUNDS;

__global__ __launch_bounds__(RS_THREADS) void radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                         int32_t* __restrict__ hist, int nblocks) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
  for (int i = threadIdx.x; i < RS_TILE; i += RS_THREADS) {
    int64_t g = base + i;
    if (g < n) atomicAdd(&h[(keys[g] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[threadIdx.x * static_cast<int64_t>(nblocks) + blockIdx.x] = h[threadIdx.x];
}

// Each block writes its tile in index order: the rank of an element is the global offset of its
// digit for this block, plus the elements of the same digit earlier in the tile (earlier rounds,
// earlier waves of this round, lower lanes of this wave).
__global__ __launch_bounds__(RS_THREADS) void radix_scatter(const uint64_t* __restrict__ kin,
                                                            const int32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                            int64_t n, int shift, const int32_t* __restrict__ offs,
                                                            int nblocks) {
  __shared__ int32_t run[256];
  __shared__ int32_t wcnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  run[tid] = offs[tid * static_cast<int64_t>(nblocks) + blockIdx.x];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ROUNDS; ++r) {
    wcnt[0][tid] = 0;
    wcnt[1][tid] = 0;
    wcnt[2][tid] = 0;
    wcnt[3][tid] = 0;
    __syncthreads();
    const int64_t g = base + r * RS_THREADS + tid;
    const bool valid = g < n;
    const uint64_t key = valid ? kin[g] : 0;
    const int32_t val = valid ? vin[g] : 0;
    const int digit = valid ? static_cast<int>((key >> shift) & 255) : 256;
    uint64_t m = ~0ull;
    for (int b = 0; b < 9; ++b) {
      const int bit = (digit >> b) & 1;
      const uint64_t bal = __ballot(bit);
      m &= bit ? bal : ~bal;
    }
    const int rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[wave][digit] = __popcll(m);
    __syncthreads();
    if (valid) {
      int pos = run[digit] + rank;
      for (int w2 = 0; w2 < wave; ++w2) pos += wcnt[w2][digit];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
  }
}

// ---------------------------------------------------------------- work items
// Runs of one (plane, tile) bin are compacted with exclusive sum-scans only:
//   run flags -> run index -> run start positions -> chunks per run -> item offsets.
__global__ void count_kept(const uint64_t* __restrict__ keys, int64_t n, uint64_t drop_key, int32_t* counts) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (keys[i] != drop_key && (i + 1 == n || keys[i + 1] == drop_key)) counts[0] = static_cast<int32_t>(i + 1);
}

__global__ void run_flags(const uint64_t* __restrict__ keys, int64_t n, const int32_t* counts, int os,
                          int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int64_t nk = counts[0];
  const uint64_t oo = static_cast<uint64_t>(os) * os;
  flag[i] = (i < nk && (i == 0 || keys[i] / oo != keys[i - 1] / oo)) ? 1 : 0;
}

__global__ void run_scatter(const int32_t* __restrict__ flag, const int32_t* __restrict__ ridx, int64_t n,
                            int32_t* __restrict__ rstart, int32_t* counts) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) rstart[ridx[i]] = static_cast<int32_t>(i);
  if (i == n - 1) counts[2] = ridx[i] + flag[i];  // number of runs
}

__global__ void run_chunks(const int32_t* __restrict__ rstart, int64_t n, const int32_t* counts, int max_chunk,
                           int32_t* __restrict__ nchunk) {
  const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= n) return;
  const int64_t nruns = counts[2], nk = counts[0];
  int32_t c = 0;
  if (r < nruns) {
    const int64_t len = (r + 1 < nruns ? rstart[r + 1] : nk) - rstart[r];
    c = static_cast<int32_t>((len + max_chunk - 1) / max_chunk);
  }
  nchunk[r] = c;
}

__global__ void item_total(const int32_t* __restrict__ nchunk, const int32_t* __restrict__ cidx, int64_t n,
                           int32_t* counts) {
  counts[1] = cidx[n - 1] + nchunk[n - 1];
}

__global__ void fine_gather(const int32_t* __restrict__ perm, const int2* __restrict__ fine_all, int64_t n_kept,
                            int2* __restrict__ fine_sorted) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n_kept) fine_sorted[i] = fine_all[perm[i]];
}

__global__ void item_write(const uint64_t* __restrict__ keys, const int32_t* __restrict__ rstart,
                           const int32_t* __restrict__ nchunk, const int32_t* __restrict__ cidx, int64_t n_runs,
                           int64_t n_kept, int os, int nt, int max_chunk, const PlaneInfo* __restrict__ planes,
                           Item* __restrict__ items) {
  const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= n_runs) return;
  const int64_t s0 = rstart[r];
  const int64_t e0 = (r + 1 < n_runs) ? rstart[r + 1] : n_kept;
  const uint64_t bin = keys[s0] / (static_cast<uint64_t>(os) * os);
  const uint64_t nt2 = static_cast<uint64_t>(nt) * nt;
  const int plane = static_cast<int>(bin / nt2);
  const uint64_t rest = bin % nt2;
  const int tile = planes[plane].tile;
  Item it;
  it.plane = plane;
  it.oy = static_cast<int32_t>(rest / nt) * tile;
  it.ox = static_cast<int32_t>(rest % nt) * tile;
  it.pad[0] = it.pad[1] = it.pad[2] = 0;
  for (int32_t c = 0; c < nchunk[r]; ++c) {
    const int64_t a = s0 + static_cast<int64_t>(c) * max_chunk;
    it.start = static_cast<int32_t>(a);
    it.end = static_cast<int32_t>(a + max_chunk < e0 ? a + max_chunk : e0);
    items[cidx[r] + c] = it;
  }
}

inline dim3 blocks_for(int64_t n, int t = 256) { return dim3(static_cast<unsigned>((n + t - 1) / t)); }

}  // namespace

hipError_t launch_plan_keys(const double* uvw, int64_t nvis, int n, double cell, int os, int nplanes,
                            const double* w_planes, const PlaneInfo* planes, int nt, uint64_t drop_key,
                            uint64_t* keys, int32_t* vals, int2* fine_all, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const double ncell = static_cast<double>(n) * cell;
  hipLaunchKernelGGL(plan_keys_kernel, blocks_for(nvis), dim3(256), 0, s, uvw, nvis, n, ncell, n / 2.0, os,
                     nplanes, w_planes, planes, nt, drop_key, keys, vals, fine_all);
  return hipGetLastError();
}

int64_t plan_scratch_elems(int64_t nvis) { return 4 * nvis + scan_scratch(nvis) + 64; }

int64_t radix_scratch_elems(int64_t n) {
  const int64_t blocks = (n + RS_TILE - 1) / RS_TILE;
  return 256 * blocks + scan_scratch(256 * blocks) + 64;
}

hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp, int32_t* vals_tmp, int64_t n,
                            int bits, int32_t* scratch, int64_t scratch_elems, hipStream_t s,
                            bool* result_in_tmp) {
  *result_in_tmp = false;
  if (n <= 1) return hipSuccess;
  const int nblocks = static_cast<int>((n + RS_TILE - 1) / RS_TILE);
  if (scratch_elems < radix_scratch_elems(n)) return hipErrorInvalidValue;
  int32_t* hist = scratch;
  int32_t* sscr = scratch + 256 * static_cast<int64_t>(nblocks);
  uint64_t *ki = keys, *ko = keys_tmp;
  int32_t *vi = vals, *vo = vals_tmp;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(radix_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, ki, n, shift, hist, nblocks);
    hipError_t e = scan<OpSum>(hist, hist, 256 * static_cast<int64_t>(nblocks), false, sscr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n, shift, hist,
                       nblocks);
    std::swap(ki, ko);
    std::swap(vi, vo);
    *result_in_tmp = !*result_in_tmp;
  }
  return hipGetLastError();
}

// Stage A: counts[0] = n_kept, counts[1] = n_items, counts[2] = n_runs on the device; `scratch`
// keeps four int32 [nvis] arrays (run flags, run index / chunk offsets, run starts, chunks per run).
hipError_t launch_plan_stage_a(const uint64_t* keys_sorted, int64_t nvis, uint64_t drop_key, int os,
                               int max_chunk, int32_t* counts, int32_t* scratch, int64_t scratch_elems,
                               hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  if (scratch_elems < plan_scratch_elems(nvis)) return hipErrorInvalidValue;
  int32_t* flag = scratch;
  int32_t* idx = scratch + nvis;
  int32_t* rstart = scratch + 2 * nvis;
  int32_t* nchunk = scratch + 3 * nvis;
  int32_t* sscr = scratch + 4 * nvis;
  hipLaunchKernelGGL(count_kept, blocks_for(nvis), dim3(256), 0, s, keys_sorted, nvis, drop_key, counts);
  hipLaunchKernelGGL(run_flags, blocks_for(nvis), dim3(256), 0, s, keys_sorted, nvis, counts, os, flag);
  hipError_t e = scan<OpSum>(flag, idx, nvis, false, sscr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(run_scatter, blocks_for(nvis), dim3(256), 0, s, flag, idx, nvis, rstart, counts);
  hipLaunchKernelGGL(run_chunks, blocks_for(nvis), dim3(256), 0, s, rstart, nvis, counts, max_chunk, nchunk);
  e = scan<OpSum>(nchunk, idx, nvis, false, sscr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(item_total, dim3(1), dim3(1), 0, s, nchunk, idx, nvis, counts);
  return hipGetLastError();
}

hipError_t launch_plan_scatter(const uint64_t* keys_sorted, const int32_t* perm, const int2* fine_all,
                               int64_t n_kept, int64_t n_runs, int64_t nvis, int os, int nt, int max_chunk,
                               const PlaneInfo* planes, const int32_t* scratch, int2* fine_sorted, Item* items,
                               hipStream_t s) {
  if (n_kept == 0) return hipSuccess;
  const int32_t* cidx = scratch + nvis;
  const int32_t* rstart = scratch + 2 * nvis;
  const int32_t* nchunk = scratch + 3 * nvis;
  hipLaunchKernelGGL(fine_gather, blocks_for(n_kept), dim3(256), 0, s, perm, fine_all, n_kept, fine_sorted);
  hipLaunchKernelGGL(item_write, blocks_for(n_runs), dim3(256), 0, s, keys_sorted, rstart, nchunk, cidx, n_runs,
                     n_kept, os, nt, max_chunk, planes, items);
  return hipGetLastError();
}

}  // namespace pg
