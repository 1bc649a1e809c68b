// Gridding, degridding and taper correction on gfx950.
//
// Gridding (Sec. 3.2, gridding stage) and degridding (Sec. 3.2, degridding
// stage) with 4x4 Mueller kernels.  A work item is a chunk of visibilities that
// share a w-plane and a uv tile (binned by the plan, phase-sorted inside the
// tile so neighbouring visibilities reuse table lines in cache).  The tile's
// sub-grid of (T + S - 1)^2 points lives in LDS with a row pitch congruent to S
// modulo 32 complex elements, so the 64 lanes of a wave, which walk consecutive
// taps of one visibility across footprint rows, hit distinct banks.  Table taps
// are stored chunk-major per phase ([chunk][tap][e]), so each 16-byte load of 64
// consecutive taps is one contiguous 1 KiB block.
//   grid (row bands): the sub-grid rows are split into one band of equal load
//           per wave; each wave walks the item's visibilities and applies the
//           footprint rows inside its band with plain LDS read-modify-write
//           (bands are disjoint); one to four workgroups share an item, each
//           accumulating its share of the output correlations; the sub-grid is
//           flushed with coalesced global float atomics.
//   grid (LDS atomics): each wave takes whole visibilities and adds into the
//           sub-grid with LDS float atomics (narrow sub-grids only).
//   degrid: the sub-grid is loaded once into LDS; each wave takes a run of the
//           item's visibilities, degrids same-phase neighbours together and
//           reduces each visibility's taps across the wave; with float32 tables
//           two workgroups can share an item, one per pair of correlations.
#include "common.hpp"

namespace pg {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr size_t kBandScratch = (256 + 32) * sizeof(int);  // row loads and band bounds of the banded grid

__device__ inline int ceil_div_i(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

// Per-visibility metadata is the same for all lanes of a wave; keeping it in scalar registers lets
// the tap loads use a scalar base address plus one 32-bit lane offset.
__device__ inline int2 uniform(int2 v) {
  return make_int2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y));
}

template <typename TapT>
struct Chunk;
template <>
struct Chunk<float2> {
  static constexpr int E = 2;  // complex64 entries per 16-byte chunk
};
template <>
struct Chunk<__half2> {
  static constexpr int E = 4;  // float16 pairs per 16-byte chunk
};

// A wave-uniform global address made opaque to the optimiser: kept in scalar registers, so a load
// from it plus a 32-bit lane offset uses the scalar-base addressing form with no vector address
// arithmetic (left alone, the compiler folds several such bases into one and rebuilds each address
// with 64-bit vector adds).
typedef const __attribute__((address_space(1))) char GlobalBytes;
typedef float GlobalF2 __attribute__((ext_vector_type(2)));
typedef float GlobalF4 __attribute__((ext_vector_type(4)));
typedef unsigned GlobalU4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V load_global(GlobalBytes* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) V*>(p);
}
__device__ __forceinline__ GlobalBytes* uniform_base(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<GlobalBytes*>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <int NQC, typename TapT>
struct TapChunks {
  static constexpr int E = NQC < Chunk<TapT>::E ? NQC : Chunk<TapT>::E;
  static constexpr int NCH = NQC / E;
  static constexpr uint32_t kTapBytes = E * sizeof(TapT);  // bytes of one tap in one chunk
  GlobalBytes* base[NCH];  // wave-uniform: chunk j of one phase block [chunk][SS][E]
  __device__ TapChunks(const TapT* ph, int ss) {
    const uint32_t chunk_bytes = static_cast<uint32_t>(ss) * kTapBytes;
#pragma unroll
    for (int j = 0; j < NCH; ++j) base[j] = uniform_base(reinterpret_cast<const char*>(ph) + j * chunk_bytes);
  }
  // chunks first, first + stride, ... of the phase block ph
  __device__ TapChunks(const TapT* ph, int ss, int first, int stride) {
    const uint32_t chunk_bytes = static_cast<uint32_t>(ss) * kTapBytes;
#pragma unroll
    for (int j = 0; j < NCH; ++j)
      base[j] = uniform_base(reinterpret_cast<const char*>(ph) + static_cast<size_t>(first + j * stride) * chunk_bytes);
  }
  // All npol^2 taps of tap index t: per chunk, one scalar base plus a 32-bit lane offset.
  __device__ void load(uint32_t t, float2 (&out)[NQC]) const { load_at(t * kTapBytes, out); }
  __device__ void load_at(uint32_t boff, float2 (&out)[NQC]) const {
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      GlobalBytes* p = base[j] + boff;
      if constexpr (E == 2) {
        const GlobalF4 v = load_global<GlobalF4>(p);
        out[2 * j] = make_float2(v.x, v.y);
        out[2 * j + 1] = make_float2(v.z, v.w);
      } else if constexpr (E == 4) {
        const GlobalU4 v = load_global<GlobalU4>(p);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          __half2 h;
          __builtin_memcpy(&h, &w[e], 4);
          out[4 * j + e] = __half22float2(h);
        }
      } else if constexpr (sizeof(TapT) == 8) {
        const GlobalF2 v = load_global<GlobalF2>(p);
        out[j] = make_float2(v.x, v.y);
      } else {
        const unsigned w = load_global<unsigned>(p);
        __half2 h;
        __builtin_memcpy(&h, &w, 4);
        out[j] = __half22float2(h);
      }
    }
  }
};

// Lane position in a footprint walked 64 taps at a time: tap u sits at footprint row u / S, column
// u % S, i.e. sub-grid element off = (row0 + u / S) P + col0 + u % S.  The first position is
// computed once; every later step of 64 taps is a few adds and one compare (no division, no
// multiply: the compiler otherwise rebuilds off, and each Stokes plane's address, with quarter-
// rate integer multiplies).
struct FootStep {
  int S, dt, doff, wrap;  // dt = 64 mod S, doff = (64 / S) P + dt, wrap = P - S
  __device__ FootStep(int S_, int P) : S(S_) {
    const int dr = 64 / S_;
    dt = 64 - dr * S_;
    doff = dr * P + dt;
    wrap = P - S_;
  }
};
struct TapCursor {
  int tx, off;
  __device__ TapCursor(int u, int row0, int col0, float inv_s, int S, int P) {
    const int rr = static_cast<int>((static_cast<float>(u) + 0.5f) * inv_s);
    tx = u - rr * S;
    off = (row0 + rr) * P + col0 + tx;
  }
  __device__ __forceinline__ void advance(const FootStep& st) {
    tx += st.dt;
    off += st.doff;
    if (tx >= st.S) {
      tx -= st.S;
      off += st.wrap;
    }
  }
};

// Sum over the 64 lanes of a wave, left in lane 63, with DPP lane moves folded into the adds:
// pairs and quads (quad permutes), rows of 16 (rotations by 4 and 8), then the row broadcasts of
// lanes 15 and 31 into the rows above.  Vector ALU only; a shuffle through LDS would cost one LDS
// round trip per step.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_move<0xb1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4e>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x124>(v);       // row_ror 4
  v += dpp_move<0x128>(v);       // row_ror 8: every lane of a row holds the row's sum
  v += dpp_move<0x142, 0xa>(v);  // row_bcast 15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast 31 into rows 2 and 3
  return v;
}

// Workgroup -> work item map that keeps `group` consecutive items (one plane, neighbouring tiles,
// so the same kernel-table rows and overlapping sub-grid halos) on one XCD and its L2.  The
// hardware hands workgroups to the 8 XCDs round-robin (block b to XCD b mod 8), so block b =
// 8 j + x takes item (8 (j / group) + x) group + j mod group: a bijection of [0, 8 group m).
// group = 1 is the identity.  Launches pad the grid to a multiple of 8 group blocks.
__device__ __forceinline__ int xcd_item(int b, int group) {
  const int x = b & 7, j = b >> 3;
  return ((j / group) * 8 + x) * group + (j % group);
}

inline unsigned xcd_blocks(int64_t n_items, int group) {
  if (group <= 1) return static_cast<unsigned>(n_items);
  const int64_t span = 8LL * group;
  return static_cast<unsigned>((n_items + span - 1) / span * span);
}

template <int NP, typename TapT>
__global__ __launch_bounds__(kThreads) void grid_kernel(const Item* __restrict__ items, const int2* __restrict__ fine,
                                                        const int32_t* __restrict__ perm,
                                                        const float2* __restrict__ vis,
                                                        const TapT* __restrict__ table,
                                                        const PlaneInfo* __restrict__ planes, int os, int n,
                                                        float2* __restrict__ grid, int flags, int n_items,
                                                        int group) {
  extern __shared__ float lds[];  // [q][re|im][W][P]
  const int item = xcd_item(blockIdx.x, group);
  if (item >= n_items) return;
  const Item it = items[item];
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, P = pl.pitch, WP = W * P, SS = S * S, half = S * os / 2;
  const float inv_s = 1.0f / static_cast<float>(S);
  for (int i = threadIdx.x; i < 2 * NP * WP; i += kThreads) lds[i] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = it.start + wave; i < it.end; i += kWaves) {
    const int2 f = uniform(fine[i]);
    const int k = __builtin_amdgcn_readfirstlane(perm[i]);
    const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
    const int phx = x0 * os - f.x + half - 1, phy = y0 * os - f.y + half - 1;
    float2 v[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) v[c] = vis[static_cast<size_t>(k) * NP + c];
    const TapChunks<NP * NP, TapT> tc(table + pl.offset + static_cast<size_t>(phy * os + phx) * SS * NP * NP, SS);
    const int lx = x0 - it.ox, ly = y0 - it.oy;
    for (int t = lane; t < SS; t += 64) {
      const int ty = static_cast<int>((static_cast<float>(t) + 0.5f) * inv_s);
      const int tx = t - ty * S;
      float2 tap[NP * NP];
      tc.load(static_cast<uint32_t>(t), tap);
      const int off = (ly + ty) * P + lx + tx;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        float re = 0.0f, im = 0.0f;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const float2 a = tap[q * NP + c];
          re = fmaf(a.x, v[c].x, fmaf(-a.y, v[c].y, re));
          im = fmaf(a.x, v[c].y, fmaf(a.y, v[c].x, im));
        }
        atomicAdd(&lds[(2 * q) * WP + off], re);
        atomicAdd(&lds[(2 * q + 1) * WP + off], im);
      }
    }
  }
  __syncthreads();
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  for (int idx = threadIdx.x; idx < W * W; idx += kThreads) {
    const int y = idx / W, x = idx - y * W;
    const int X = it.ox + x, Y = it.oy + y;
    if (X >= n || Y >= n) continue;
    const int l = y * P + x;
    const float sg = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const float re = lds[(2 * q) * WP + l], im = lds[(2 * q + 1) * WP + l];
      if (re != 0.0f || im != 0.0f) {
        float* g = reinterpret_cast<float*>(grid + q * pstride + static_cast<size_t>(Y) * n + X);
        unsafeAtomicAdd(g, sg * re);
        unsafeAtomicAdd(g + 1, sg * im);
      }
    }
  }
}

// Target of the reproducible flush: 64-bit fixed-point accumulators [q][n][n][re, im] and the
// binary exponent that scales float sub-grid values into them.  Integer addition is associative,
// so the accumulated bits do not depend on the order in which workgroups flush.
struct FixedSink {
  unsigned long long* acc;
  const int* exp;
};

// One row (visibility) of a work item as one wave of the banded gridder sees it: the footprint rows
// inside the wave's band [r0, r1), flattened to cnt = (b - a) S taps starting at tap t0, with the
// row's visibility and kernel phase made wave-uniform (readlane of the lane that fetched them).
// j < 0 gives an empty row.
template <int NP, typename TapT, int NQ = NP>
struct BandRow {
  int cnt = 0, a = 0, lx = 0;
  uint32_t t0 = 0;
  float2 v[NP];
  TapChunks<NQ * NP, TapT> tc;
  // q0: first of the NQ output planes this workgroup accumulates (Mueller rows q0 .. q0 + NQ - 1,
  // which are chunks q0 NP / E .. of each phase block)
  __device__ BandRow(int j, int m_ly, int m_lx, int m_ph, int m_k, const float2* __restrict__ vis, int r0, int r1,
                     int S, int SS, const TapT* plane_table, int q0 = 0)
      : tc(plane_table, SS) {
    if (j < 0) {
#pragma unroll
      for (int c = 0; c < NP; ++c) v[c] = make_float2(0.0f, 0.0f);
      return;
    }
    const int ly = __builtin_amdgcn_readlane(m_ly, j);
    a = max(ly, r0);
    cnt = (min(ly + S, r1) - a) * S;
    t0 = static_cast<uint32_t>((a - ly) * S);
    lx = __builtin_amdgcn_readlane(m_lx, j);
    const int ph = __builtin_amdgcn_readlane(m_ph, j);
    tc = TapChunks<NQ * NP, TapT>(plane_table + (static_cast<size_t>(ph) * NP * NP + q0 * NP) * SS, SS);
    const int k = __builtin_amdgcn_readlane(m_k, j);  // uniform: the row's values come in by scalar loads
#pragma unroll
    for (int c = 0; c < NP; ++c) v[c] = vis[static_cast<size_t>(k) * NP + c];
  }
  // Adds the Mueller product of one tap into the LDS sub-grid at element off of each Stokes plane
  // (planes WP apart): all npol reads are issued before the arithmetic and all writes after it.
  __device__ __forceinline__ void apply(float2* lds, int off, const float2 (&tap)[NQ * NP], int WP) const {
    float2 g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = lds[q * WP + off];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        const float2 t2 = tap[q * NP + c];
        g[q].x = fmaf(t2.x, v[c].x, fmaf(-t2.y, v[c].y, g[q].x));
        g[q].y = fmaf(t2.x, v[c].y, fmaf(t2.y, v[c].x, g[q].y));
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q * WP + off] = g[q];
  }
};

// Banded variant: the sub-grid rows are split into NW contiguous bands of equal load (rows
// weighted by how many footprints of the item cover them); wave w owns band w and walks every
// visibility of the item, taking only the footprint rows inside its band.  Bands are disjoint, so
// the sub-grid (complex [q][W][P] in LDS) is updated with plain read-modify-write, no LDS atomics.
template <int NP, typename TapT, int NW, bool PAIR, int NQ = NP, bool FIXED = false>
__device__ __forceinline__ void grid_item_banded(const Item it, const int2* __restrict__ fine,
                                                 const int32_t* __restrict__ perm, const float2* __restrict__ vis,
                                                 const TapT* __restrict__ table, const PlaneInfo* __restrict__ planes,
                                                 int os, int n, float2* __restrict__ grid, int flags, int sub_bytes,
                                                 float* lds_f, int q0 = 0, FixedSink fx = FixedSink{nullptr, nullptr}) {
  float2* lds = reinterpret_cast<float2*>(lds_f);
  int* rowload = reinterpret_cast<int*>(reinterpret_cast<char*>(lds_f) + sub_bytes);  // [W + 1]
  int* band = rowload + 256;                                                             // [NW + 1]
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, P = pl.pitch, WP = W * P, SS = S * S, half = S * os / 2;
  const float inv_s = 1.0f / static_cast<float>(S);
  for (int i = threadIdx.x; i < NQ * WP; i += (NW * 64)) lds[i] = make_float2(0.0f, 0.0f);
  for (int i = threadIdx.x; i <= W; i += (NW * 64)) rowload[i] = 0;
  __syncthreads();
  // coverage count of every sub-grid row (difference array, then a prefix sum in one wave)
  for (int i = it.start + static_cast<int>(threadIdx.x); i < it.end; i += (NW * 64)) {
    const int ly = ceil_div_i(fine[i].y - half + 1, os) - it.oy;
    atomicAdd(&rowload[ly], 1);
    atomicAdd(&rowload[ly + S], -1);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave == 0) {
    int carry = 0;
    for (int r0 = 0; r0 < W; r0 += 64) {  // inclusive prefix sums: coverage, then cumulative load
      int c = (r0 + lane < W) ? rowload[r0 + lane] : 0;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(c, d, 64);
        if (lane >= d) c += o;
      }
      c += carry;
      carry = __shfl(c, 63, 64);
      if (r0 + lane < W) rowload[r0 + lane] = c;
    }
    __builtin_amdgcn_wave_barrier();
    carry = 0;
    for (int r0 = 0; r0 < W; r0 += 64) {
      int c = (r0 + lane < W) ? rowload[r0 + lane] : 0;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(c, d, 64);
        if (lane >= d) c += o;
      }
      c += carry;
      carry = __shfl(c, 63, 64);
      if (r0 + lane < W) rowload[r0 + lane] = c;
    }
    __builtin_amdgcn_wave_barrier();
    // band w starts at the first row whose cumulative load reaches w / NW of the total
    if (lane <= NW) {
      const long long total = rowload[W - 1];
      int r = 0;
      if (lane == NW) {
        r = W;
      } else if (lane > 0) {
        const long long thr = (total * lane + NW - 1) / NW;
        while (r < W && rowload[r] < thr) ++r;
        ++r;
        if (r > W) r = W;
      }
      band[lane] = r;
    }
  }
  __syncthreads();
  // band bounds are the same for the whole wave: scalar registers, so the row walk below (band
  // tests, row bounds) runs on the scalar unit instead of the vector ALU
  const int r0 = __builtin_amdgcn_readfirstlane(band[wave]), r1 = __builtin_amdgcn_readfirstlane(band[wave + 1]);
  const FootStep step(S, P);
  // Metadata of 64 rows is fetched lane-parallel in one coalesced load and broadcast per row with
  // readlane, so walking the item costs one memory latency per 64 rows, not two per row.
  for (int blk = it.start; blk < it.end && r0 < r1; blk += 64) {
    const int mine = blk + lane;
    int m_ly = -(1 << 20), m_lx = 0, m_ph = 0, m_k = 0;
    if (mine < it.end) {
      const int2 f = fine[mine];
      const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
      m_ly = y0 - it.oy;
      m_lx = x0 - it.ox;
      m_ph = (y0 * os - f.y + half - 1) * os + (x0 * os - f.x + half - 1);
      m_k = perm[mine];
    }
    // The rows of this block whose footprint meets the wave's band, as one 64-bit mask (each lane
    // tests its own row), walked in order with find-first-set on the scalar unit.
    // With PAIR, rows are taken two at a time: the first 64 taps of both are requested before either
    // is applied, so one memory latency covers two rows.  LDS updates stay in row order (a wave's LDS
    // operations execute in program order), so overlapping footprints need no synchronisation.
    uint64_t hits = __ballot(mine < it.end && max(m_ly, r0) < min(m_ly + S, r1));
    while (hits) {
      const int ja = __builtin_ctzll(hits);
      hits &= hits - 1;
      int jb = -1;
      if constexpr (PAIR) {
        if (hits) {
          jb = __builtin_ctzll(hits);
          hits &= hits - 1;
        }
      }
      const BandRow<NP, TapT, NQ> ra(ja, m_ly, m_lx, m_ph, m_k, vis, r0, r1, S, SS, table + pl.offset, q0);
      const BandRow<NP, TapT, NQ> rb(jb, m_ly, m_lx, m_ph, m_k, vis, r0, r1, S, SS, table + pl.offset, q0);
      constexpr uint32_t TB = TapChunks<NQ * NP, TapT>::kTapBytes;
      float2 ta[NQ * NP], tb[NQ * NP];
      const bool la = lane < ra.cnt, lb = lane < rb.cnt;
      uint32_t ba = (ra.t0 + static_cast<uint32_t>(lane)) * TB, bb = (rb.t0 + static_cast<uint32_t>(lane)) * TB;
      if (la) ra.tc.load_at(ba, ta);
      if (lb) rb.tc.load_at(bb, tb);
      TapCursor ca(lane, ra.a, ra.lx, inv_s, S, P);
      if (la) ra.apply(lds, ca.off, ta, WP);
#pragma unroll 1
      for (int u = lane + 64; u < ra.cnt; u += 64) {
        float2 t[NQ * NP];
        ba += 64 * TB;
        ra.tc.load_at(ba, t);
        ca.advance(step);
        ra.apply(lds, ca.off, t, WP);
      }
      TapCursor cb(lane, rb.a, rb.lx, inv_s, S, P);
      if (lb) rb.apply(lds, cb.off, tb, WP);
#pragma unroll 1
      for (int u = lane + 64; u < rb.cnt; u += 64) {
        float2 t[NQ * NP];
        bb += 64 * TB;
        rb.tc.load_at(bb, t);
        cb.advance(step);
        rb.apply(lds, cb.off, t, WP);
      }
    }
  }
  __syncthreads();
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  int fe = 0;
  if constexpr (FIXED) fe = __builtin_amdgcn_readfirstlane(*fx.exp);
  for (int idx = threadIdx.x; idx < W * W; idx += (NW * 64)) {
    const int y = idx / W, x = idx - y * W;
    const int X = it.ox + x, Y = it.oy + y;
    if (X >= n || Y >= n) continue;
    const int l = y * P + x;
    const float sg = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const float2 g = lds[q * WP + l];
      if (g.x != 0.0f || g.y != 0.0f) {
        const size_t o = (q0 + q) * pstride + static_cast<size_t>(Y) * n + X;
        if constexpr (FIXED) {
          // |value| 2^fe < 2^61 by the choice of fe, so the rounded value converts exactly
          atomicAdd(fx.acc + 2 * o, static_cast<unsigned long long>(static_cast<long long>(rintf(ldexpf(sg * g.x, fe)))));
          atomicAdd(fx.acc + 2 * o + 1,
                    static_cast<unsigned long long>(static_cast<long long>(rintf(ldexpf(sg * g.y, fe)))));
        } else {
          float* gp = reinterpret_cast<float*>(grid + o);
          unsafeAtomicAdd(gp, sg * g.x);
          unsafeAtomicAdd(gp + 1, sg * g.y);
        }
      }
    }
  }
}

template <int NP, typename TapT, int NW, int NQ = NP>
__global__ __launch_bounds__(NW * 64) void grid_banded_kernel(const Item* __restrict__ items,
                                                              const int2* __restrict__ fine,
                                                              const int32_t* __restrict__ perm,
                                                              const float2* __restrict__ vis,
                                                              const TapT* __restrict__ table,
                                                              const PlaneInfo* __restrict__ planes, int os, int n,
                                                              float2* __restrict__ grid, int flags, int sub_bytes,
                                                              int n_items, int group) {
  extern __shared__ float lds_f[];
  // NP / NQ workgroups per item, each accumulating NQ of the output planes
  const int w = xcd_item(blockIdx.x, group);
  const int item = w / (NP / NQ), part = w - item * (NP / NQ);
  if (item >= n_items) return;
  // two rows in flight costs registers: 1024-thread workgroups (capped at 128) take one at a time
  grid_item_banded<NP, TapT, NW, (NW <= 8), NQ>(items[item], fine, perm, vis, table, planes, os, n, grid, flags,
                                                sub_bytes, lds_f, part * NQ);
}

// Shared-tap gridder.  Rows of a work item are phase-sorted inside the tile, so runs of rows share
// one kernel phase: each wave takes a contiguous run of the item's rows and grids up to R rows of one
// phase per pass, loading every tap once and applying it to all R rows, whose sub-grid positions
// differ by wave-uniform offsets.  Waves overlap in the sub-grid, so it is accumulated with LDS
// integer atomics (on CDNA4 these run at about the rate of plain LDS read-modify-write; float LDS
// atomics are over an order of magnitude slower), exactly, in two-word fixed point:
//   * the item's scale 2^e puts B = max_q kbound[plane][q] x rows x the largest row sum
//     sum_c |Re V_c| + |Im V_c| (a bound on every value of the sub-grid and on the sum of the
//     magnitudes of its terms, independent of summation order) below 2^29; visibilities are
//     multiplied by 2^e as they are read, so every term y comes out already scaled;
//   * each term is split into h = floor(y) and l = trunc(fract(y) 2^f), f = min(20, 30 - log2 rows):
//     coarse words sum to less than 2^30 in magnitude, fine words lie in [0, 2^f) and sum to less
//     than 2^30, and the pair holds every float32 term to about one fine unit 2^-(e + f), far below
//     float32 rounding;
//   * real and imaginary words are packed into one 64-bit integer, im 2^32 + re, whose sums decode
//     exactly while |sum re| < 2^31: one 64-bit LDS atomic per word pair.  Coarse real words are
//     sign-extended into the upper half; fine words are never negative, so their pair is the two
//     32-bit registers side by side.
// The sub-grid of an item is therefore the same bits whatever the order of its additions.
constexpr int kSharedScratch = 64;  // bytes after the sub-grid words: the per-wave maxima

__device__ __forceinline__ unsigned long long pack_pair(int re, int im) {
  return static_cast<unsigned long long>((static_cast<long long>(im) << 32) + static_cast<long long>(re));
}
__device__ __forceinline__ unsigned long long pack_fine(unsigned re, unsigned im) {
  return (static_cast<unsigned long long>(im) << 32) | re;
}
// floor to int in one instruction (the compiler emits a floor and a truncating conversion)
__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ int2 unpack_pair(unsigned long long v) {
  const int re = static_cast<int>(static_cast<unsigned>(v));
  const int im = static_cast<int>(static_cast<long long>(v) >> 32) + (re < 0 ? 1 : 0);
  return make_int2(re, im);
}

// PF: two tap buffers (the next pass's taps in flight); off where the registers would not hold them
template <int NP, typename TapT, int R, int NQ, bool PF>
__device__ __forceinline__ void grid_rows_shared(unsigned long long* lds, int fine_off, const TapT* __restrict__ pt,
                                                 int j, int m_ly, int m_lx, int m_k, const float2* __restrict__ vis,
                                                 int S, int SS, int P, int WP, float inv_s, const FootStep& step,
                                                 int lane, int ex, float fscale) {
  const TapChunks<NQ * NP, TapT> tc(pt, SS);
  constexpr uint32_t TB = TapChunks<NQ * NP, TapT>::kTapBytes;
  const int ly0 = __builtin_amdgcn_readlane(m_ly, j), lx0 = __builtin_amdgcn_readlane(m_lx, j);
  int d[R];
  float2 v[R][NP];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    d[r] = (__builtin_amdgcn_readlane(m_ly, j + r) - ly0) * P + __builtin_amdgcn_readlane(m_lx, j + r) - lx0;
    const int k = __builtin_amdgcn_readlane(m_k, j + r);
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      const float2 a = vis[static_cast<size_t>(k) * NP + c];
      v[r][c] = make_float2(ldexpf(a.x, ex), ldexpf(a.y, ex));
    }
  }
  // one tap of the footprint for all R rows; off = the tap's sub-grid word for the run's first row
  auto tap_rows = [&](int off, const float2 (&tap)[NQ * NP]) {
    // an opaque copy of the cursor: the compiler would otherwise keep one strength-reduced address
    // per row and word, each stepped on every pass
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        float yr = 0.0f, yi = 0.0f;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const float2 a = tap[q * NP + c];
          yr = fmaf(a.x, v[r][c].x, fmaf(-a.y, v[r][c].y, yr));
          yi = fmaf(a.x, v[r][c].y, fmaf(a.y, v[r][c].x, yi));
        }
        unsigned long long* cell = lds + q * WP + off + d[r];
        atomicAdd(cell, pack_pair(floor_to_int(yr), floor_to_int(yi)));
        // fract(y) = y - floor(y) in [0, 1), truncated to f bits: the residual is below one fine unit
        atomicAdd(cell + fine_off, pack_fine(static_cast<unsigned>(__builtin_amdgcn_fractf(yr) * fscale),
                                             static_cast<unsigned>(__builtin_amdgcn_fractf(yi) * fscale)));
      }
    }
  };
  // Lane u takes taps u, u + 64, ... in passes of 64; after the full passes, a last pass takes the
  // SS mod 64 taps left (if any) on the lanes that have one.  The taps of the next pass are loaded
  // while this pass's rows are computed (two buffers, alternating; loads past the last tap read tap
  // SS - 1 and are not used), in a loop without branches so that each wait covers only the buffer
  // it needs.  When S divides 64 the footprint advances by whole rows and the cursor needs no wrap.
  TapCursor cur(lane, ly0, lx0, inv_s, S, P);
  const int full = SS >> 6;
  const bool tail_lane = lane < SS - (full << 6);
  const uint32_t b_last = static_cast<uint32_t>(SS - 1) * TB;
  const uint32_t b0 = static_cast<uint32_t>(lane) * TB;
  auto load_pass = [&](int p, float2 (&tap)[NQ * NP]) {
    tc.load_at(min(b0 + static_cast<uint32_t>(p) * (64 * TB), b_last), tap);
  };
  auto run = [&](auto advance) {
    if constexpr (PF) {
      float2 ta[NQ * NP], tb[NQ * NP];
      load_pass(0, ta);
      int p = 0;
      for (; p + 2 <= full; p += 2) {
        load_pass(p + 1, tb);
        tap_rows(cur.off, ta);
        advance();
        load_pass(p + 2, ta);
        tap_rows(cur.off, tb);
        advance();
      }
      if (p < full) {  // one full pass left, in ta; the tail pass (if any) goes to tb
        load_pass(p + 1, tb);
        tap_rows(cur.off, ta);
        advance();
        if (tail_lane) tap_rows(cur.off, tb);
      } else if (tail_lane) {  // ta holds the tail pass
        tap_rows(cur.off, ta);
      }
    } else {
      float2 ta[NQ * NP];
      for (int p = 0; p < full; ++p) {
        load_pass(p, ta);
        tap_rows(cur.off, ta);
        advance();
      }
      if (tail_lane) {
        load_pass(full, ta);
        tap_rows(cur.off, ta);
      }
    }
  };
  if (step.dt == 0) {
    run([&]() { cur.off += step.doff; });
  } else {
    run([&]() { cur.advance(step); });
  }
}

// FIXED: the reproducible mode's flush.  The item's values are exact integers at the scale
// 2^(e + f); they are moved to the launch-wide scale of the 64-bit accumulators by a shift (exact
// when it is a left shift, a floor when right) and added with integer atomics.
// TWO_BUFFERS: the single-plan launches take two tap buffers where the registers hold them; the
// batched launch keeps one (measured faster there)
template <int NP, typename TapT, int NW, int NQ = NP, bool FIXED = false, bool TWO_BUFFERS = true>
__device__ __forceinline__ void grid_item_shared(const Item it, const int2* __restrict__ fine,
                                                 const int32_t* __restrict__ perm, const float2* __restrict__ vis,
                                                 const TapT* __restrict__ table, const PlaneInfo* __restrict__ planes,
                                                 const float* __restrict__ kbound, int os, int n,
                                                 float2* __restrict__ grid, int flags, int sub_bytes, float* lds_f,
                                                 int q0 = 0, FixedSink fx = FixedSink{nullptr, nullptr}) {
  // [coarse | fine][q][W][P] packed (re, im) words; sub_bytes covers both
  unsigned long long* lds = reinterpret_cast<unsigned long long*>(lds_f);
  float* part = reinterpret_cast<float*>(reinterpret_cast<char*>(lds_f) + sub_bytes);  // [NW]
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, P = pl.pitch, WP = W * P, SS = S * S, half = S * os / 2;
  const int fine_off = NQ * WP;
  const float inv_s = 1.0f / static_cast<float>(S);
  for (int i = threadIdx.x; i < 2 * fine_off; i += NW * 64) lds[i] = 0ull;
  // largest row sum of |Re V_c| + |Im V_c| over the item (a maximum: the same in every thread and
  // for any partition of the rows)
  float m1 = 0.0f;
  constexpr int kRowsPerPass = 2;  // rows per thread whose loads are in flight together
  for (int i0 = it.start + static_cast<int>(threadIdx.x); i0 < it.end; i0 += kRowsPerPass * NW * 64) {
    int k[kRowsPerPass];
#pragma unroll
    for (int u = 0; u < kRowsPerPass; ++u) {
      const int i = i0 + u * NW * 64;
      k[u] = i < it.end ? perm[i] : -1;
    }
    float2 a[kRowsPerPass][NP];
#pragma unroll
    for (int u = 0; u < kRowsPerPass; ++u) {
      const size_t kk = static_cast<size_t>(k[u] < 0 ? 0 : k[u]);  // row 0 stands in, unused
#pragma unroll
      for (int c = 0; c < NP; ++c) a[u][c] = vis[kk * NP + c];
    }
#pragma unroll
    for (int u = 0; u < kRowsPerPass; ++u) {
      if (k[u] < 0) continue;
      float a1 = 0.0f;
#pragma unroll
      for (int c = 0; c < NP; ++c) a1 += fabsf(a[u][c].x) + fabsf(a[u][c].y);
      m1 = (a1 > m1 || a1 != a1) ? a1 : m1;  // a NaN row wins, so a non-finite item is recognised
    }
  }
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float other = __shfl_xor(m1, o, 64);
    m1 = (other > m1 || other != other) ? other : m1;
  }
  if (lane == 0) part[wave] = m1;
  __syncthreads();
  float kmax = 0.0f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) kmax = fmaxf(kmax, kbound[4 * it.plane + q0 + q]);
  float mrow = 0.0f;
  bool finite = true;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    finite = finite && part[w] == part[w] && part[w] <= 3.0e38f;
    mrow = fmaxf(mrow, part[w]);
  }
  const int rows = it.end - it.start;
  // in float64, so that only non-finite inputs (not a bound beyond the float range) stop the item
  const double b = static_cast<double>(kmax) * static_cast<double>(mrow) * static_cast<double>(rows);
  int ex = 0;
  if (!(b <= 1.0e300)) {
    finite = false;
  } else if (b > 0.0) {
    int e2 = 0;
    frexp(b, &e2);  // b < 2^e2
    ex = 29 - e2;
  }
  int lg = 0;  // ceil(log2(rows))
  while ((1 << lg) < rows && lg < 30) ++lg;
  const int fbits = min(20, 30 - lg);
  const float fscale = ldexpf(1.0f, fbits);
  const FootStep step(S, P);
  constexpr bool kPF = TWO_BUFFERS && NW * NQ <= 16;  // and room for them in the registers
  const int per = (rows + NW - 1) / NW;
  const int w0 = it.start + wave * per, w1 = min(it.end, w0 + per);
  for (int blk = w0; blk < w1 && finite; blk += 64) {
    const int mine = blk + lane;
    int m_ly = 0, m_lx = 0, m_ph = -1, m_k = 0;
    if (mine < w1) {
      const int2 f = fine[mine];
      const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
      m_ly = y0 - it.oy;
      m_lx = x0 - it.ox;
      m_ph = (y0 * os - f.y + half - 1) * os + (x0 * os - f.x + half - 1);
      m_k = perm[mine];
    }
    const int nrow = min(64, w1 - blk);
    for (int j = 0; j < nrow;) {
      const int ph = __builtin_amdgcn_readlane(m_ph, j);
      int run = 1;  // rows from j on with the same phase, up to 8
      while (run < 8 && j + run < nrow && __builtin_amdgcn_readlane(m_ph, j + run) == ph) ++run;
      run = __builtin_amdgcn_readfirstlane(run);
      const TapT* pt = table + pl.offset + (static_cast<size_t>(ph) * NP * NP + q0 * NP) * SS;
      if (run == 8) {
        grid_rows_shared<NP, TapT, 8, NQ, kPF>(lds, fine_off, pt, j, m_ly, m_lx, m_k, vis, S, SS, P, WP, inv_s, step, lane,
                                               ex, fscale);
      } else if (run >= 4) {
        grid_rows_shared<NP, TapT, 4, NQ, kPF>(lds, fine_off, pt, j, m_ly, m_lx, m_k, vis, S, SS, P, WP, inv_s, step, lane,
                                               ex, fscale);
        run = 4;
      } else if (run >= 2) {
        grid_rows_shared<NP, TapT, 2, NQ, kPF>(lds, fine_off, pt, j, m_ly, m_lx, m_k, vis, S, SS, P, WP, inv_s, step, lane,
                                               ex, fscale);
        run = 2;
      } else {
        grid_rows_shared<NP, TapT, 1, NQ, kPF>(lds, fine_off, pt, j, m_ly, m_lx, m_k, vis, S, SS, P, WP, inv_s, step, lane,
                                               ex, fscale);
      }
      j += run;
    }
  }
  __syncthreads();
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  if constexpr (FIXED) {
    if (!finite) return;  // the reproducible mode requires finite inputs
    const int sh = __builtin_amdgcn_readfirstlane(*fx.exp) - ex - fbits;
    for (int idx = threadIdx.x; idx < W * W; idx += NW * 64) {
      const int y = idx / W, x = idx - y * W;
      const int X = it.ox + x, Y = it.oy + y;
      if (X >= n || Y >= n) continue;
      const int l = y * P + x;
      const bool neg = shift && ((X + Y) & 1);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const unsigned long long cw = lds[q * WP + l], fw = lds[fine_off + q * WP + l];
        if ((cw | fw) == 0ull) continue;
        const int2 h = unpack_pair(cw), f = unpack_pair(fw);
        long long v[2] = {static_cast<long long>(static_cast<unsigned long long>(static_cast<long long>(h.x)) << fbits) + f.x,
                          static_cast<long long>(static_cast<unsigned long long>(static_cast<long long>(h.y)) << fbits) + f.y};
        const size_t o = (q0 + q) * pstride + static_cast<size_t>(Y) * n + X;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          long long a = neg ? -v[c] : v[c];
          if (sh >= 0) {
            a = static_cast<long long>(static_cast<unsigned long long>(a) << min(sh, 63));
          } else {
            a = sh > -63 ? (a >> -sh) : (a < 0 ? -1 : 0);
          }
          atomicAdd(fx.acc + 2 * o + c, static_cast<unsigned long long>(a));
        }
      }
    }
    return;
  }
  for (int idx = threadIdx.x; idx < W * W; idx += NW * 64) {
    const int y = idx / W, x = idx - y * W;
    const int X = it.ox + x, Y = it.oy + y;
    if (X >= n || Y >= n) continue;
    const int l = y * P + x;
    const float sg = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float* gp = reinterpret_cast<float*>(grid + (q0 + q) * pstride + static_cast<size_t>(Y) * n + X);
      if (!finite) {  // a non-finite visibility or table bound: the item's points become NaN
        unsafeAtomicAdd(gp, __int_as_float(0x7fc00000));
        unsafeAtomicAdd(gp + 1, __int_as_float(0x7fc00000));
        continue;
      }
      const unsigned long long cw = lds[q * WP + l], fw = lds[fine_off + q * WP + l];
      if ((cw | fw) != 0ull) {
        const int2 h = unpack_pair(cw), f = unpack_pair(fw);
        const double re = ldexp(static_cast<double>(h.x) + ldexp(static_cast<double>(f.x), -fbits), -ex);
        const double im = ldexp(static_cast<double>(h.y) + ldexp(static_cast<double>(f.y), -fbits), -ex);
        unsafeAtomicAdd(gp, sg * static_cast<float>(re));
        unsafeAtomicAdd(gp + 1, sg * static_cast<float>(im));
      }
    }
  }
}

template <int NP, typename TapT, int NW, int NQ = NP>
__global__ __launch_bounds__(NW * 64) void grid_shared_kernel(const Item* __restrict__ items,
                                                              const int2* __restrict__ fine,
                                                              const int32_t* __restrict__ perm,
                                                              const float2* __restrict__ vis,
                                                              const TapT* __restrict__ table,
                                                              const PlaneInfo* __restrict__ planes,
                                                              const float* __restrict__ kbound, int os, int n,
                                                              float2* __restrict__ grid, int flags, int sub_bytes,
                                                              int n_items, int group) {
  extern __shared__ float lds_f[];
  const int w = xcd_item(blockIdx.x, group);
  const int item = w / (NP / NQ), part = w - item * (NP / NQ);
  if (item >= n_items) return;
  grid_item_shared<NP, TapT, NW, NQ>(items[item], fine, perm, vis, table, planes, kbound, os, n, grid, flags,
                                     sub_bytes, lds_f, part * NQ);
}

// Reproducible gridding with the shared-tap kernel: 8 waves per workgroup and a number of output
// planes per workgroup that depends only on the kernel set, so every item's exact sub-grid, and the
// 64-bit sums of all items, are the same bits whatever the plan's launch settings.
template <int NP, typename TapT, int NQ>
__global__ __launch_bounds__(512) void grid_shared_fixed_kernel(const Item* __restrict__ items,
                                                                const int2* __restrict__ fine,
                                                                const int32_t* __restrict__ perm,
                                                                const float2* __restrict__ vis,
                                                                const TapT* __restrict__ table,
                                                                const PlaneInfo* __restrict__ planes,
                                                                const float* __restrict__ kbound, int os, int n,
                                                                int flags, int sub_bytes, FixedSink fx) {
  extern __shared__ float lds_f[];
  const int item = blockIdx.x / (NP / NQ), part = blockIdx.x - item * (NP / NQ);
  grid_item_shared<NP, TapT, 8, NQ, true>(items[item], fine, perm, vis, table, planes, kbound, os, n, nullptr, flags,
                                          sub_bytes, lds_f, part * NQ, fx);
}

// Reproducible gridding where the shared-tap kernel does not fit: one workgroup of 8 waves per
// work item, all planes, row bands (a fixed summation order inside the item whatever the plan's
// launch settings), flushed into the fixed-point accumulators.
template <int NP, typename TapT>
__global__ __launch_bounds__(512) void grid_fixed_kernel(const Item* __restrict__ items, const int2* __restrict__ fine,
                                                         const int32_t* __restrict__ perm,
                                                         const float2* __restrict__ vis,
                                                         const TapT* __restrict__ table,
                                                         const PlaneInfo* __restrict__ planes, int os, int n, int flags,
                                                         int sub_bytes, FixedSink fx) {
  extern __shared__ float lds_f[];
  grid_item_banded<NP, TapT, 8, true, NP, true>(items[blockIdx.x], fine, perm, vis, table, planes, os, n, nullptr,
                                                flags, sub_bytes, lds_f, 0, fx);
}

// Bounds for the fixed-point scale, as float bit patterns (non-negative floats order like their
// bits, so an integer atomic max is exact and order-independent):
//   bound[0] = max over kept rows of sum_c |re V_c| + |im V_c|
//   bound[1] = max over table entries of |re T| + |im T|
// |re (T V)| and |im (T V)| are at most (|re T| + |im T|)(|re V| + |im V|), so every grid value is
// at most n_kept bound[0] bound[1].
__device__ inline void wave_max_to(unsigned* out, float m) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

__global__ void vis_bound_kernel(const int32_t* __restrict__ perm, int64_t n_kept, int np,
                                 const float2* __restrict__ vis, unsigned* __restrict__ out) {
  float m = 0.0f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_kept;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t k = perm[i];
    float a = 0.0f;
    for (int c = 0; c < np; ++c) {
      const float2 v = vis[k * np + c];
      a += fabsf(v.x) + fabsf(v.y);
    }
    m = fmaxf(m, a);
  }
  wave_max_to(out, m);
}

// Largest |Re| + |Im| of any table entry: the maximum of the per-plane, per-row bounds kept with the
// tables (refreshed whenever a table is generated or written), without reading the table again.
__global__ void kbound_max_kernel(const float* __restrict__ kbound, int n, unsigned* __restrict__ out) {
  float m = 0.0f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, kbound[i]);
  wave_max_to(out, m);
}

// Binary exponent e with n_kept bound[0] bound[1] 2^e < 2^61: two bits of headroom below the int64
// range for the float rounding inside the sub-grid sums.  Zero when the bound is zero.
__global__ void fixed_exponent_kernel(const unsigned* __restrict__ bound, double n_kept, int* __restrict__ exp) {
  const double b = n_kept * static_cast<double>(__uint_as_float(bound[0])) * static_cast<double>(__uint_as_float(bound[1]));
  int e = 0;
  if (b > 0.0 && b <= 1.0e300) {
    int ex = 0;
    frexp(b, &ex);  // b < 2^ex
    e = 61 - ex;
  }
  *exp = e;
}

// grid (=, or += with accumulate) acc 2^-e, rounded once to float64 and once to float32.
__global__ void fixed_to_grid_kernel(const unsigned long long* __restrict__ acc, const int* __restrict__ exp,
                                     size_t count, float2* __restrict__ grid, int accumulate) {
  const int e = *exp;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float re = static_cast<float>(ldexp(static_cast<double>(static_cast<long long>(acc[2 * i])), -e));
    const float im = static_cast<float>(ldexp(static_cast<double>(static_cast<long long>(acc[2 * i + 1])), -e));
    if (accumulate) {
      const float2 g = grid[i];
      grid[i] = make_float2(g.x + re, g.y + im);
    } else {
      grid[i] = make_float2(re, im);
    }
  }
}

// The batch field table is read through the constant address space: the compiler then takes the
// pointers it holds to address global memory.  Read through a plain pointer, their address space
// is unknown and every access through them compiles to flat instructions (slower, with 64-bit
// addresses in vector registers: 166 instead of 117 VGPRs in the float16 4-pol gridder).
typedef const __attribute__((address_space(4))) FieldArgs ConstFieldArgs;

// Many fields in one launch: workgroup b takes the (field, item) pair work[b] (field -1: nothing to
// do).  The host lays the list out field by field, largest field first, each in plan order (plane
// by plane, tile by tile) and cut into groups of consecutive items that each run on one XCD (block
// b runs on XCD b mod 8).  The hardware hands out workgroups in index order, so one or two fields'
// kernel tables and grids are live in the caches at a time and the smallest field fills the tail.
// On the 16-field float16 workload this beats one launch per field (grid 48.0 ms against 51.7,
// degrid 22.5 against 23.2).  A list ordered by item cost across all fields was slower (53 ms and
// 26 ms: sixteen tables compete for the caches), and a persistent form that pulled pairs from a
// device counter slower still (every item then ends in workgroup-wide barriers around the queue
// access with no other workgroup to overlap them).
template <int NP, typename TapT, int NW>
__global__ __launch_bounds__(NW * 64) void grid_banded_batch(const FieldArgs* __restrict__ fields,
                                                             const int2* __restrict__ work, int flags,
                                                             int sub_bytes) {
  extern __shared__ float lds_f[];
  const int2 wr = work[blockIdx.x];
  if (wr.x < 0) return;
  ConstFieldArgs& fa = ((ConstFieldArgs*)fields)[wr.x];
  grid_item_banded<NP, TapT, NW, (NW <= 8)>(fa.items[wr.y], fa.fine, fa.perm, fa.vis,
                                            static_cast<const TapT*>(fa.table), fa.planes, fa.os, fa.n, fa.grid,
                                            flags, sub_bytes, lds_f);
}

// The shared-tap gridder over a batch: workgroup b takes part b mod (NP / NQ) (its NQ output
// planes) of the (field, item) pair work[b / (NP / NQ)].
template <int NP, typename TapT, int NW, int NQ>
__global__ __launch_bounds__(NW * 64) void grid_shared_batch(const FieldArgs* __restrict__ fields,
                                                             const int2* __restrict__ work, int flags,
                                                             int sub_bytes) {
  extern __shared__ float lds_f[];
  const int2 wr = work[blockIdx.x / (NP / NQ)];
  if (wr.x < 0) return;
  const int part = blockIdx.x % (NP / NQ);
  ConstFieldArgs& fa = ((ConstFieldArgs*)fields)[wr.x];
  grid_item_shared<NP, TapT, NW, NQ, false, false>(fa.items[wr.y], fa.fine, fa.perm, fa.vis,
                                                   static_cast<const TapT*>(fa.table), fa.planes, fa.kbound, fa.os,
                                                   fa.n, fa.grid, flags, sub_bytes, lds_f, part * NQ);
}

// Degrid sub-grid layout in LDS: full-pol planes in pairs, [q / 2][W][P][q % 2], so that a row
// reads planes (0, 1) and (2, 3) as two 16-byte values from consecutive cells (16-byte stride:
// no bank conflicts along a footprint row); one plane: [W][P].
template <int NP>
__device__ __forceinline__ int degrid_lds_index(int q, int cell, int WP) {
  if constexpr (NP == 1) {
    return cell;
  } else {
    return ((q >> 1) * WP + cell) * 2 + (q & 1);
  }
}

// The NP grid values of one sub-grid cell: one plane, or the two plane pairs as aligned 16-byte
// reads (ds_read_b128; two 8-byte halves would each meet a two-way bank conflict at this stride)
template <int NP>
__device__ __forceinline__ void degrid_cell(const float2* lds, const float2* lds_hi, int cell, float2 (&g)[NP]) {
  if constexpr (NP == 1) {
    g[0] = lds[cell];
  } else {
    static_assert(NP == 4, "full-pol sub-grids hold two plane pairs");
    const float4 a = reinterpret_cast<const float4*>(lds)[cell];
    const float4 b = reinterpret_cast<const float4*>(lds_hi)[cell];
    g[0] = make_float2(a.x, a.y);
    g[1] = make_float2(a.z, a.w);
    g[2] = make_float2(b.x, b.y);
    g[3] = make_float2(b.z, b.w);
  }
}

// Sums over the 64 lanes of the 2 NC R accumulators of a degrid pass (row r, value e = 2 c + re/im
// at flat index v = 2 NC r + e), NC >= 2, by halving: a 32-lane swap pairs values v and v + 1 (lanes
// 0-31 then carry v, lanes 32-63 v + 1, each summed over the two halves), a 16-lane swap pairs those
// registers (rows 0-3 of register h then carry v = 4 h, 4 h + 2, 4 h + 1, 4 h + 3), and four DPP adds
// finish each 16-lane row.  About 2.5 instructions per value instead of ten for a separate reduction
// of each, and the first lane of each row stores its value (one store per register).
template <int NP, int NC, int R>
__device__ __forceinline__ void degrid_sum_rows(float (&acc)[R][2 * NC], int j, int m_k,
                                                float2* __restrict__ vis_out, int flags, int lane, int c0) {
  constexpr int E = 2 * NC, M = R * E;  // E is a multiple of 4
  float half[M / 2];
#pragma unroll
  for (int i = 0; i < M / 2; ++i) {
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[(2 * i) / E][(2 * i) % E]),
                                                     __float_as_uint(acc[(2 * i + 1) / E][(2 * i + 1) % E]),
                                                     false, false);
    half[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  const int rho = lane >> 4;
  const int e_row = (rho & 1) * 2 + (rho >> 1);  // value offset carried by 16-lane row rho
  float* out = reinterpret_cast<float*>(vis_out);
#pragma unroll
  for (int h = 0; h < M / 4; ++h) {
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(half[2 * h]), __float_as_uint(half[2 * h + 1]),
                                                     false, false);
    float v = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    v += dpp_move<0x128>(v);  // row_ror 8
    v += dpp_move<0x124>(v);  // row_ror 4
    v += dpp_move<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0xb1>(v);   // quad_perm [1, 0, 3, 2]: every lane of the row holds its sum
    const int r = (4 * h) / E;               // the same row for the four values of register h
    const int e = (4 * h) % E + e_row;
    const int k = __builtin_amdgcn_readlane(m_k, j + r);
    if ((lane & 15) == 0) {
      float* o = out + (static_cast<size_t>(k) * NP + c0 + (e >> 1)) * 2 + (e & 1);
      *o = (flags & PG_ACCUMULATE) ? *o + v : v;
    }
  }
}

// R consecutive rows of a work item that share one kernel phase (rows are phase-sorted inside a
// tile), degridded together: every tap is loaded once and applied to all R rows, whose sub-grid
// positions differ by a wave-uniform offset.  One 64-lane sum per row and output value; lane 63
// writes the rows' visibilities.
constexpr int kDegridRun = 8;  // longest run of same-phase rows whose tap loads one degrid pass shares

template <int NP, typename TapT, int R, int NC = NP>
__device__ __forceinline__ void degrid_rows(const float2* lds, const TapT* phase_table, int j, int m_ly, int m_lx,
                                            int m_k, int S, int SS, int P, int WP, float inv_s,
                                            const FootStep& step, float2* __restrict__ vis_out, int flags,
                                            int lane, int c0 = 0) {
  // NC < NP: this workgroup computes correlations c0 .. c0 + NC - 1, from Mueller entries (q, c0 ..)
  // which sit in every (NP / NC)-th 16-byte chunk of the phase block
  const TapChunks<NP * NC, TapT> tc = NC == NP ? TapChunks<NP * NC, TapT>(phase_table, SS)
                                               : TapChunks<NP * NC, TapT>(phase_table, SS, c0 / NC, NP / NC);
  const float2* lds_hi = lds + 2 * WP;  // planes (2, 3) of the plane-pair layout
  const int ly0 = __builtin_amdgcn_readlane(m_ly, j), lx0 = __builtin_amdgcn_readlane(m_lx, j);
  int d[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    d[r] = (__builtin_amdgcn_readlane(m_ly, j + r) - ly0) * P + (__builtin_amdgcn_readlane(m_lx, j + r) - lx0);
  float acc[R][2 * NC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 2 * NC; ++c) acc[r][c] = 0.0f;
  constexpr uint32_t TB = TapChunks<NP * NC, TapT>::kTapBytes;
  TapCursor cur(lane, ly0, lx0, inv_s, S, P);
  uint32_t boff = static_cast<uint32_t>(lane) * TB;
#pragma unroll(R == 1 ? 2 : 1)
  for (int t = lane; t < SS; t += 64) {
    float2 tap[NP * NC];
    tc.load_at(boff, tap);
    const int off = cur.off;
    boff += 64 * TB;
    cur.advance(step);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float2 gq[NP];
      degrid_cell<NP>(lds, lds_hi, off + d[r], gq);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const float2 g = gq[q];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 a = tap[q * NC + c];  // conj(a) * g
          acc[r][2 * c] = fmaf(a.x, g.x, fmaf(a.y, g.y, acc[r][2 * c]));
          acc[r][2 * c + 1] = fmaf(a.x, g.y, fmaf(-a.y, g.x, acc[r][2 * c + 1]));
        }
      }
    }
  }
  if constexpr (NC >= 2) {
    degrid_sum_rows<NP, NC, R>(acc, j, m_k, vis_out, flags, lane, c0);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < 2 * NC; ++c) acc[r][c] = wave_sum_to_lane63(acc[r][c]);
      const int k = __builtin_amdgcn_readlane(m_k, j + r);
      if (lane == 63) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (flags & PG_ACCUMULATE) {
            float2& o = vis_out[static_cast<size_t>(k) * NP + c0 + c];
            o = make_float2(o.x + acc[r][2 * c], o.y + acc[r][2 * c + 1]);
          } else {
            vis_out[static_cast<size_t>(k) * NP + c0 + c] = make_float2(acc[r][2 * c], acc[r][2 * c + 1]);
          }
      }
    }
  }
}

template <int NP, typename TapT, int NW, int NC = NP>
__device__ __forceinline__ void degrid_item(const Item it, const int2* __restrict__ fine,
                                            const int32_t* __restrict__ perm, const TapT* __restrict__ table,
                                            const PlaneInfo* __restrict__ planes, int os, int n,
                                            const float2* __restrict__ grid, float2* __restrict__ vis_out,
                                            int flags, float* lds_f, int c0 = 0) {
  float2* lds = reinterpret_cast<float2*>(lds_f);  // plane pairs: [q / 2][W][P][q % 2]
  const PlaneInfo pl = planes[it.plane];
  const int S = pl.support, W = pl.width, P = pl.pitch, WP = W * P, SS = S * S, half = S * os / 2;
  const float inv_s = 1.0f / static_cast<float>(S);
  const bool shift = (flags & PG_FFTSHIFT) != 0;
  const size_t pstride = static_cast<size_t>(n) * n;
  // sub-grid fill: kFill cells per thread per pass, all their loads issued before the first LDS
  // write, so that a pass costs one memory round trip (one workgroup per CU leaves nothing else to
  // run meanwhile)
  constexpr int kFill = 4;
  const int cells = W * W;
  for (int base = threadIdx.x; base < cells; base += kFill * NW * 64) {
    float2 g[kFill][NP];
    int dst[kFill];
    float sg[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int idx = base + u * NW * 64;
      const int y = idx / W, x = idx - y * W;
      const int X = it.ox + x, Y = it.oy + y;
      const bool in = idx < cells && X < n && Y < n;
      dst[u] = idx < cells ? y * P + x : -1;
      sg[u] = (shift && ((X + Y) & 1)) ? -1.0f : 1.0f;
#pragma unroll
      for (int q = 0; q < NP; ++q)
        g[u][q] = in ? grid[q * pstride + static_cast<size_t>(Y) * n + X] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      if (dst[u] < 0) continue;
#pragma unroll
      for (int q = 0; q < NP; ++q)
        lds[degrid_lds_index<NP>(q, dst[u], WP)] = make_float2(sg[u] * g[u][q].x, sg[u] * g[u][q].y);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const FootStep step(S, P);
  // wave w takes a contiguous run of the item's rows, so rows of one phase stay together; their
  // metadata comes in 64 at a time by one coalesced load and is broadcast per row with readlane
  const int per = (it.end - it.start + NW - 1) / NW;
  const int w0 = it.start + wave * per, w1 = min(it.end, w0 + per);
  for (int blk = w0; blk < w1; blk += 64) {
    const int mine = blk + lane;
    int m_ly = 0, m_lx = 0, m_ph = -1, m_k = 0;
    if (mine < w1) {
      const int2 f = fine[mine];
      const int x0 = ceil_div_i(f.x - half + 1, os), y0 = ceil_div_i(f.y - half + 1, os);
      m_ly = y0 - it.oy;
      m_lx = x0 - it.ox;
      m_ph = (y0 * os - f.y + half - 1) * os + (x0 * os - f.x + half - 1);
      m_k = perm[mine];
    }
    const int nrow = min(64, w1 - blk);
    for (int j = 0; j < nrow;) {
      const int ph = __builtin_amdgcn_readlane(m_ph, j);
      int run = 1;  // rows from j on with the same phase, up to kDegridRun
      while (run < kDegridRun && j + run < nrow && __builtin_amdgcn_readlane(m_ph, j + run) == ph) ++run;
      run = __builtin_amdgcn_readfirstlane(run);
      const TapT* pt = table + pl.offset + static_cast<size_t>(ph) * SS * NP * NP;
      if (kDegridRun >= 8 && run == 8) {
        degrid_rows<NP, TapT, 8, NC>(lds, pt, j, m_ly, m_lx, m_k, S, SS, P, WP, inv_s, step, vis_out, flags, lane,
                                    c0);
      } else if (run >= 4) {
        run = 4;
        degrid_rows<NP, TapT, 4, NC>(lds, pt, j, m_ly, m_lx, m_k, S, SS, P, WP, inv_s, step, vis_out, flags, lane,
                                    c0);
      } else if (run >= 2) {
        degrid_rows<NP, TapT, 2, NC>(lds, pt, j, m_ly, m_lx, m_k, S, SS, P, WP, inv_s, step, vis_out, flags, lane,
                                    c0);
        run = 2;
      } else {
        degrid_rows<NP, TapT, 1, NC>(lds, pt, j, m_ly, m_lx, m_k, S, SS, P, WP, inv_s, step, vis_out, flags, lane,
                                    c0);
      }
      j += run;
    }
  }
}

template <int NP, typename TapT, int NW, int NC = NP>
__global__ __launch_bounds__(NW * 64) void degrid_kernel(const Item* __restrict__ items,
                                                         const int2* __restrict__ fine,
                                                         const int32_t* __restrict__ perm,
                                                         const TapT* __restrict__ table,
                                                         const PlaneInfo* __restrict__ planes, int os, int n,
                                                         const float2* __restrict__ grid,
                                                         float2* __restrict__ vis_out, int flags, int n_items,
                                                         int group) {
  extern __shared__ float lds_f[];
  // NP / NC workgroups per item, each computing NC of the correlations
  const int w = xcd_item(blockIdx.x, group);
  const int item = w / (NP / NC), part = w - item * (NP / NC);
  if (item >= n_items) return;
  degrid_item<NP, TapT, NW, NC>(items[item], fine, perm, table, planes, os, n, grid, vis_out, flags, lds_f,
                                part * NC);
}

template <int NP, typename TapT, int NW>
__global__ __launch_bounds__(NW * 64) void degrid_batch(const FieldArgs* __restrict__ fields,
                                                        const int2* __restrict__ work, int flags) {
  extern __shared__ float lds_f[];
  const int2 wr = work[blockIdx.x];
  if (wr.x < 0) return;
  ConstFieldArgs& fa = ((ConstFieldArgs*)fields)[wr.x];
  degrid_item<NP, TapT, NW>(fa.items[wr.y], fa.fine, fa.perm, static_cast<const TapT*>(fa.table), fa.planes, fa.os,
                            fa.n, fa.grid, fa.vis, flags, lds_f);
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
                                     const double* __restrict__ inv_aa, double scale) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const size_t idx = (static_cast<size_t>(blockIdx.z) * n + i) * n + j;
  const double sc = scale * inv_aa[i] * inv_aa[j] * (((i + j) & 1) ? -1.0 : 1.0);
  out[idx] = make_float2(static_cast<float>(in[idx] * sc), 0.0f);
}

template <class F>
hipError_t allow_lds(F* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

template <int NP, typename TapT, int NW, int NQ = NP>
hipError_t run_grid_banded(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                           hipStream_t s) {
  auto fn = grid_banded_kernel<NP, TapT, NW, NQ>;
  const size_t sub = k->lds_bytes / NP * NQ;
  const size_t bytes = sub + kBandScratch;
  hipError_t e = allow_lds(fn, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(xcd_blocks(p->n_items * (NP / NQ), p->xcd_group)), dim3(NW * 64), bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->os, k->n, grid, flags, static_cast<int>(sub),
                     static_cast<int>(p->n_items), p->xcd_group);
  return hipGetLastError();
}

template <int NP, typename TapT, int NW, int NQ = NP>
hipError_t run_grid_shared(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                           hipStream_t s) {
  auto fn = grid_shared_kernel<NP, TapT, NW, NQ>;
  const size_t sub = 2 * (k->lds_bytes / NP * NQ);  // coarse and fine words
  const size_t bytes = sub + kSharedScratch;
  hipError_t e = allow_lds(fn, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(xcd_blocks(p->n_items * (NP / NQ), p->xcd_group)), dim3(NW * 64), bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->kbound.as<float>(), k->os, k->n, grid, flags,
                     static_cast<int>(sub), static_cast<int>(p->n_items), p->xcd_group);
  return hipGetLastError();
}

// Output planes per workgroup: the plan's grid_planes (0: all), halved while the two-word sub-grid
// would not fit the LDS.
template <int NP, typename TapT, int NW>
hipError_t run_grid_shared_planes(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                                  hipStream_t s) {
  if constexpr (NP == 4) {
    int nq = (p->grid_planes == 1 || p->grid_planes == 2) ? p->grid_planes : 4;
    while (nq > 1 && 2 * (k->lds_bytes / 4 * nq) + kSharedScratch > 163840) nq /= 2;
    if (nq == 2) return run_grid_shared<NP, TapT, NW, 2>(p, k, vis, grid, flags, s);
    if (nq == 1) return run_grid_shared<NP, TapT, NW, 1>(p, k, vis, grid, flags, s);
  }
  return run_grid_shared<NP, TapT, NW>(p, k, vis, grid, flags, s);
}

// Output planes per workgroup (the plan's grid_planes; 0 or npol: all).  With fewer, NP / NQ
// workgroups share each work item, each accumulating NQ planes from its NQ rows of the Mueller
// kernels: the sub-grid in LDS shrinks by NP / NQ, so more workgroups fit on a CU.
template <int NP, typename TapT, int NW>
hipError_t run_grid_banded_planes(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                                  hipStream_t s) {
  if constexpr (NP == 4) {
    if (p->grid_planes == 2) return run_grid_banded<NP, TapT, NW, 2>(p, k, vis, grid, flags, s);
    if (p->grid_planes == 1) return run_grid_banded<NP, TapT, NW, 1>(p, k, vis, grid, flags, s);
  }
  return run_grid_banded<NP, TapT, NW>(p, k, vis, grid, flags, s);
}

template <int NP, typename TapT>
hipError_t run_grid(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                    hipStream_t s) {
  // Banded ownership needs enough sub-grid rows to give every wave a band; the LDS-atomic
  // variant serves narrow sub-grids.  The plan's launch setting or a call flag can force either.
  bool banded = k->max_width >= 2 * p->grid_waves;
  bool shared = p->grid_variant == 3;
  if (p->grid_variant == 1) banded = false;
  if (p->grid_variant == 2) banded = true;
  if (flags & (PG_VARIANT_ATOMIC | PG_VARIANT_BANDED)) shared = false;
  if (flags & PG_VARIANT_ATOMIC) banded = false;
  if (flags & PG_VARIANT_BANDED) banded = true;
  if (flags & PG_VARIANT_SHARED) shared = true;
  // the shared-tap kernel holds two words per value: one output plane of the widest sub-grid must
  // fit twice, else the row-band kernel serves the launch
  if (2 * (k->lds_bytes / NP) + kSharedScratch > 163840) shared = false;
  if (shared) {
    switch (p->grid_waves) {
      case 4: return run_grid_shared_planes<NP, TapT, 4>(p, k, vis, grid, flags, s);
      case 6: return run_grid_shared_planes<NP, TapT, 6>(p, k, vis, grid, flags, s);
      case 8: return run_grid_shared_planes<NP, TapT, 8>(p, k, vis, grid, flags, s);
      default: return run_grid_shared_planes<NP, TapT, 16>(p, k, vis, grid, flags, s);
    }
  }
  if (banded) {
    switch (p->grid_waves) {
      case 4: return run_grid_banded_planes<NP, TapT, 4>(p, k, vis, grid, flags, s);
      case 6: return run_grid_banded_planes<NP, TapT, 6>(p, k, vis, grid, flags, s);
      case 8: return run_grid_banded_planes<NP, TapT, 8>(p, k, vis, grid, flags, s);
      default: return run_grid_banded_planes<NP, TapT, 16>(p, k, vis, grid, flags, s);
    }
  }
  auto fn = grid_kernel<NP, TapT>;
  hipError_t e = allow_lds(fn, k->lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(xcd_blocks(p->n_items, p->xcd_group)), dim3(kThreads), k->lds_bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->os, k->n, grid, flags, static_cast<int>(p->n_items), p->xcd_group);
  return hipGetLastError();
}

template <int NP, typename TapT, int NW>
hipError_t run_degrid_nw(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                         hipStream_t s) {
  // Two workgroups per item, each computing two of the four correlations from every second
  // 16-byte chunk of the float32 table (Mueller entries (q, c) with c in its pair).  Blocks 2i and
  // 2i + 1 take item i, so with the hardware's round-robin over the 8 XCDs every even XCD holds
  // the first half of the tables in its L2 and every odd XCD the second (the plan's XCD grouping
  // is not applied here).
  if constexpr (NP == 4 && sizeof(TapT) == 8) {
    if (p->degrid_corrs == 2) {
      auto fn = degrid_kernel<NP, TapT, NW, 2>;
      hipError_t e = allow_lds(fn, k->lds_bytes);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(p->n_items * 2)), dim3(NW * 64), k->lds_bytes, s,
                         p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), k->table.as<TapT>(),
                         k->planes.as<PlaneInfo>(), k->os, k->n, grid, vis, flags, static_cast<int>(p->n_items), 1);
      return hipGetLastError();
    }
  }
  auto fn = degrid_kernel<NP, TapT, NW>;
  hipError_t e = allow_lds(fn, k->lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(xcd_blocks(p->n_items, p->xcd_group)), dim3(NW * 64), k->lds_bytes, s,
                     p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), k->table.as<TapT>(),
                     k->planes.as<PlaneInfo>(), k->os, k->n, grid, vis, flags, static_cast<int>(p->n_items),
                     p->xcd_group);
  return hipGetLastError();
}

template <int NP, typename TapT>
hipError_t run_degrid(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                      hipStream_t s) {
  switch (p->degrid_waves) {
    case 4: return run_degrid_nw<NP, TapT, 4>(p, k, grid, vis, flags, s);
    case 6: return run_degrid_nw<NP, TapT, 6>(p, k, grid, vis, flags, s);
    case 8: return run_degrid_nw<NP, TapT, 8>(p, k, grid, vis, flags, s);
    default: return run_degrid_nw<NP, TapT, 16>(p, k, grid, vis, flags, s);
  }
}

template <int NP, typename TapT, int NW, int NQ>
hipError_t run_batch_grid_shared(const pg_batch* b, int flags, hipStream_t s) {
  auto fn = grid_shared_batch<NP, TapT, NW, NQ>;
  const size_t sub = 2 * (b->lds_bytes / NP * NQ);
  const size_t bytes = sub + kSharedScratch;
  hipError_t e = allow_lds(fn, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(b->n_blocks * (NP / NQ))), dim3(NW * 64), bytes, s,
                     b->fields.as<FieldArgs>(), b->work.as<int2>(), flags, static_cast<int>(sub));
  return hipGetLastError();
}

template <int NP, typename TapT, int NW>
hipError_t run_batch_grid(const pg_batch* b, int flags, hipStream_t s) {
  if (b->grid_variant == 3 && 2 * (b->lds_bytes / NP) + kSharedScratch <= 163840) {
    // the first field's output planes per workgroup, halved while they do not fit twice in the LDS
    if constexpr (NP == 4) {
      int nq = (b->grid_planes == 1 || b->grid_planes == 2) ? b->grid_planes : 4;
      while (nq > 1 && 2 * (b->lds_bytes / 4 * nq) + kSharedScratch > 163840) nq /= 2;
      if (nq == 4) return run_batch_grid_shared<NP, TapT, NW, 4>(b, flags, s);
      if (nq == 2) return run_batch_grid_shared<NP, TapT, NW, 2>(b, flags, s);
      return run_batch_grid_shared<NP, TapT, NW, 1>(b, flags, s);
    } else {
      return run_batch_grid_shared<NP, TapT, NW, NP>(b, flags, s);
    }
  }
  auto fn = grid_banded_batch<NP, TapT, NW>;
  const size_t bytes = b->lds_bytes + kBandScratch;
  hipError_t e = allow_lds(fn, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(b->n_blocks)), dim3(NW * 64), bytes, s, b->fields.as<FieldArgs>(),
                     b->work.as<int2>(), flags, static_cast<int>(b->lds_bytes));
  return hipGetLastError();
}

template <int NP, typename TapT, int NW>
hipError_t run_batch_degrid(const pg_batch* b, int flags, hipStream_t s) {
  auto fn = degrid_batch<NP, TapT, NW>;
  hipError_t e = allow_lds(fn, b->lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(b->n_blocks)), dim3(NW * 64), b->lds_bytes, s,
                     b->fields.as<FieldArgs>(), b->work.as<int2>(), flags);
  return hipGetLastError();
}

template <int NP, typename TapT>
hipError_t dispatch_batch(const pg_batch* b, int flags, hipStream_t s, bool grid) {
  const int nw = grid ? b->grid_waves : b->degrid_waves;
  if (grid) {
    if (nw == 4) return run_batch_grid<NP, TapT, 4>(b, flags, s);
    if (nw == 6) return run_batch_grid<NP, TapT, 6>(b, flags, s);
    if (nw == 8) return run_batch_grid<NP, TapT, 8>(b, flags, s);
    return run_batch_grid<NP, TapT, 16>(b, flags, s);
  }
  if (nw == 4) return run_batch_degrid<NP, TapT, 4>(b, flags, s);
  if (nw == 6) return run_batch_degrid<NP, TapT, 6>(b, flags, s);
  if (nw == 8) return run_batch_degrid<NP, TapT, 8>(b, flags, s);
  return run_batch_degrid<NP, TapT, 16>(b, flags, s);
}

hipError_t batch_body(const pg_batch* b, int flags, hipStream_t s, bool grid) {
  const bool f16 = b->storage == PG_STORE_F16;
  if (b->npol == 4) return f16 ? dispatch_batch<4, __half2>(b, flags, s, grid) : dispatch_batch<4, float2>(b, flags, s, grid);
  return f16 ? dispatch_batch<1, __half2>(b, flags, s, grid) : dispatch_batch<1, float2>(b, flags, s, grid);
}

}  // namespace

hipError_t launch_batch_grid(const pg_batch* b, int flags, hipStream_t s) {
  for (int f = 0; f < b->nfields; ++f) {
    if (!(flags & PG_ACCUMULATE)) {
      const pg_kernels* k = b->kernels[f];
      hipError_t e = launch_fill_zero(b->grids[f], static_cast<size_t>(k->npol) * k->n * k->n * sizeof(float2), s);
      if (e != hipSuccess) return e;
    }
  }
  if (b->n_work == 0) return hipSuccess;
  return batch_body(b, flags, s, true);
}

hipError_t launch_batch_degrid(const pg_batch* b, int flags, hipStream_t s) {
  for (int f = 0; f < b->nfields; ++f) {
    const pg_plan* p = b->plans[f];
    if (p->nvis > p->n_kept) {
      const int64_t nd = p->nvis - p->n_kept;
      hipLaunchKernelGGL(zero_dropped, dim3(static_cast<unsigned>((nd + 255) / 256)), dim3(256), 0, s,
                         p->perm.as<int32_t>(), p->n_kept, p->nvis, b->npol, static_cast<float2*>(b->vis[f]));
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (b->n_work == 0) return hipSuccess;
  return batch_body(b, flags, s, false);
}

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

size_t grid_fixed_scratch_bytes(const pg_kernels* k) {
  return 256 + static_cast<size_t>(k->npol) * k->n * k->n * 2 * sizeof(unsigned long long);
}

namespace {
template <int NP, typename TapT>
hipError_t run_grid_fixed(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                          void* scratch, hipStream_t s) {
  unsigned* bound = static_cast<unsigned*>(scratch);
  int* exp = reinterpret_cast<int*>(static_cast<char*>(scratch) + 8);
  auto* acc = reinterpret_cast<unsigned long long*>(static_cast<char*>(scratch) + 256);
  const size_t count = static_cast<size_t>(k->npol) * k->n * k->n;
  hipError_t e = launch_fill_zero(scratch, grid_fixed_scratch_bytes(k), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(vis_bound_kernel, dim3(static_cast<unsigned>(std::min<int64_t>((p->n_kept + 255) / 256, 4096))),
                     dim3(256), 0, s, p->perm.as<int32_t>(), p->n_kept, NP, vis, bound);
  hipLaunchKernelGGL(kbound_max_kernel, dim3(1), dim3(64), 0, s, k->kbound.as<float>(), 4 * k->nplanes, bound + 1);
  hipLaunchKernelGGL(fixed_exponent_kernel, dim3(1), dim3(1), 0, s, bound, static_cast<double>(p->n_kept), exp);
  // one output plane per workgroup: the fastest shape of the shared-tap kernel on the full-pol
  // workload, and one that fits wherever the kernel fits at all
  const int nq = 1;
  const size_t sub = 2 * (k->lds_bytes / NP * nq);
  if (sub + kSharedScratch <= 163840) {
    auto launch = [&](auto fn) -> hipError_t {
      hipError_t e2 = allow_lds(fn, sub + kSharedScratch);
      if (e2 != hipSuccess) return e2;
      hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(p->n_items * (NP / nq))), dim3(512), sub + kSharedScratch, s,
                         p->items.as<Item>(), p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(),
                         k->planes.as<PlaneInfo>(), k->kbound.as<float>(), k->os, k->n, flags, static_cast<int>(sub),
                         FixedSink{acc, exp});
      return hipSuccess;
    };
    e = launch(grid_shared_fixed_kernel<NP, TapT, 1>);
  } else {
    auto fn = grid_fixed_kernel<NP, TapT>;
    const size_t bytes = k->lds_bytes + kBandScratch;
    e = allow_lds(fn, bytes);
    if (e == hipSuccess)
      hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(p->n_items)), dim3(512), bytes, s, p->items.as<Item>(),
                         p->fine.as<int2>(), p->perm.as<int32_t>(), vis, k->table.as<TapT>(), k->planes.as<PlaneInfo>(),
                         k->os, k->n, flags, static_cast<int>(k->lds_bytes), FixedSink{acc, exp});
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fixed_to_grid_kernel, dim3(static_cast<unsigned>(std::min<size_t>((count + 255) / 256, 16384))),
                     dim3(256), 0, s, acc, exp, count, grid, (flags & PG_ACCUMULATE) ? 1 : 0);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_grid_fixed(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                             void* scratch, hipStream_t s) {
  if (p->n_items == 0) {
    if (flags & PG_ACCUMULATE) return hipSuccess;
    return launch_fill_zero(grid, static_cast<size_t>(k->npol) * k->n * k->n * sizeof(float2), s);
  }
  const bool f16 = k->storage == PG_STORE_F16;
  if (k->npol == 4)
    return f16 ? run_grid_fixed<4, __half2>(p, k, vis, grid, flags, scratch, s)
               : run_grid_fixed<4, float2>(p, k, vis, grid, flags, scratch, s);
  return f16 ? run_grid_fixed<1, __half2>(p, k, vis, grid, flags, scratch, s)
             : run_grid_fixed<1, float2>(p, k, vis, grid, flags, scratch, s);
}

hipError_t launch_degrid(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                         hipStream_t s) {
  if (p->nvis > p->n_kept && !(flags & PG_ACCUMULATE)) {  // accumulating leaves dropped rows as they are
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
                       static_cast<float2*>(out), k->n, k->inv_aa.as<double>(), weight_sum);
  }
  return hipGetLastError();
}

}  // namespace pg
