// Internal definitions shared by the host orchestration and the HIP kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "polgrid.h"

namespace pg {

// Work item of the gridder: one chunk of visibilities sharing a (plane, uv tile).
struct Item {
  int32_t plane;
  int32_t oy, ox;      // grid origin of the tile's sub-grid
  int32_t start, end;  // range in binned order
  int32_t pad[3];
};
static_assert(sizeof(Item) == 32, "Item layout is part of pg_plan_desc");

// Per-plane constants the device kernels read.
struct PlaneInfo {
  int64_t offset;   // first table entry of the plane
  int32_t support;  // S
  int32_t tile;     // T
  int32_t width;    // sub-grid side T + S - 1
  int32_t pitch;    // LDS row pitch in complex elements, >= width, == S (mod 32)
};

// LDS row pitch of a sub-grid row: the footprint rows a wave touches are S apart in tap order,
// so a pitch congruent to S modulo 32 complex elements keeps 64 consecutive taps on distinct banks.
inline int lds_pitch(int width, int support) { return width + (((support - width) % 32) + 32) % 32; }

// Table entries per load chunk: two complex64 (16 B) or four float16 pairs (16 B), capped by npol^2.
inline int chunk_entries(int storage, int nqc) {
  const int e = storage == PG_STORE_F16 ? 4 : 2;
  return nqc < e ? nqc : e;
}

// One field (channel or mosaic pointing) of a batched launch, as the device sees it.
struct FieldArgs {
  const Item* items;
  const int2* fine;
  const int32_t* perm;
  float2* vis;        // grid: input, degrid: output
  const void* table;  // float2 or __half2 entries
  const PlaneInfo* planes;
  float2* grid;       // grid: output, degrid: input
  const float* kbound;  // per-plane Mueller-row table bounds (shared-tap gridder)
  int32_t os, n;
};

void set_error(const std::string& msg);

// Registered device allocator (hipMalloc/hipFree when both hooks are NULL).
struct Allocator {
  void* (*alloc_fn)(size_t, void*, void*) = nullptr;
  void (*free_fn)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
Allocator current_allocator();

// RAII device buffer; frees through the allocator it came from.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  Allocator a;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), s(o.s), a(o.a) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      s = o.s;
      a = o.a;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  bool alloc(size_t b, hipStream_t st) {
    reset();
    s = st;
    a = current_allocator();
    if (b == 0) return true;
    if (a.alloc_fn) {
      p = a.alloc_fn(b, st, a.ctx);
    } else if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
    }
    if (p) bytes = b;
    return p != nullptr;
  }
  void reset() {
    if (p) {
      if (a.alloc_fn && a.free_fn) {
        a.free_fn(p, s, a.ctx);
      } else if (!a.alloc_fn) {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace pg

struct pg_kernels {
  int32_t npol = 1, kind = 0, storage = 0, os = 2, n = 0, nplanes = 0, mk = 0, aa_support = 7;
  double cell = 0;
  std::vector<double> w_planes;
  std::vector<int32_t> support, tile;
  std::vector<int64_t> plane_offset;  // [nplanes + 1]
  std::vector<double> aa_pixels;      // [n]
  int32_t max_width = 0;              // max sub-grid side over planes
  size_t lds_bytes = 0;               // sub-grid bytes of the widest plane
  pg::DevBuf table;                   // float2 or __half2 entries
  pg::DevBuf planes;                  // PlaneInfo [nplanes]
  pg::DevBuf w_dev;                   // double [nplanes]
  pg::DevBuf inv_aa;                  // double [n], 1 / AA(pixel)
  pg::DevBuf kbound;                  // float [nplanes][4]: max over a plane's entries of Mueller row q of |re| + |im|
};

struct pg_plan {
  int64_t nvis = 0, n_kept = 0, n_dropped = 0, n_items = 0;
  int32_t max_chunk = 0;
  int32_t n = 0, os = 0;                // geometry the plan was binned for
  int32_t grid_variant = 0;             // 0 auto, 1 LDS atomics, 2 row bands
  int32_t grid_waves = 16, degrid_waves = 16;  // waves per workgroup
  int32_t xcd_group = 1;                // consecutive work items kept on one XCD
  int32_t grid_planes = 0;              // output planes per banded-gridder workgroup (0: all)
  int32_t degrid_corrs = 0;             // correlations per degrid workgroup (0: all; 2 for float32 full-pol)
  std::vector<int32_t> support, tile;
  pg::DevBuf perm;    // int32 [nvis]
  pg::DevBuf fine;    // int2 [n_kept]
  pg::DevBuf items;   // Item [n_items]
};

struct pg_batch {
  int32_t nfields = 0, npol = 1, storage = 0;
  int64_t n_work = 0;    // (field, item) pairs
  int64_t n_blocks = 0;  // launch size: n_work plus no-op entries that even out the XCD queues
  size_t lds_bytes = 0;          // largest sub-grid over the fields
  int32_t grid_waves = 16, degrid_waves = 16;
  int32_t grid_variant = 0;  // 3: shared-tap gridder (from the first field's plan), else row bands
  int32_t grid_planes = 0;   // output planes per shared-tap workgroup (from the first field's plan)
  std::vector<const pg_plan*> plans;
  std::vector<const pg_kernels*> kernels;
  std::vector<void*> vis, grids;
  pg::DevBuf fields;   // FieldArgs [nfields]
  pg::DevBuf work;     // int2 (field, item) [n_blocks] in launch order; (-1, -1) = no-op
};

// ---- launchers implemented in the .hip files (all enqueue on `s`)
namespace pg {

// Kernel generation (kernels_gen.hip)
hipError_t launch_screen(const double2* phi, const double* aa_lat, double w, double fov, int mk, int nqc,
                         double2* out, hipStream_t s);
hipError_t launch_twiddles(int support, int os, int mk, double2* e, hipStream_t s);
hipError_t launch_zgemm_nt(int batch, int m, int n, int k, const double2* a, int64_t stride_a,
                           const double2* b, int64_t stride_b, double2* c, int64_t stride_c, hipStream_t s);
hipError_t launch_zgemm_nn(int batch, int m, int n, int k, const double2* a, int64_t stride_a,
                           const double2* b, int64_t stride_b, double2* c, int64_t stride_c, hipStream_t s);
hipError_t launch_pack(const double2* t, int support, int os, int nqc, int storage, void* table, hipStream_t s);

// Plan (plan.hip)
hipError_t launch_plan_keys(const double* uvw, int64_t nvis, int n, double cell, int os, int nplanes,
                            const double* w_planes, const PlaneInfo* planes, int nt, uint64_t drop_key,
                            uint64_t* keys, int32_t* vals, int2* fine_all, hipStream_t s);
hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp, int32_t* vals_tmp,
                            int64_t n, int bits, int32_t* scratch, int64_t scratch_elems, hipStream_t s,
                            bool* result_in_tmp);
int64_t radix_scratch_elems(int64_t n);
int64_t plan_scratch_elems(int64_t nvis);
hipError_t launch_plan_stage_a(const uint64_t* keys_sorted, int64_t nvis, uint64_t drop_key, int os,
                               int max_chunk, int32_t* counts, int32_t* scratch, int64_t scratch_elems,
                               hipStream_t s);
hipError_t launch_plan_scatter(const uint64_t* keys_sorted, const int32_t* perm, const int2* fine_all,
                               int64_t n_kept, int64_t n_runs, int64_t nvis, int os, int nt, int max_chunk,
                               const PlaneInfo* planes, const int32_t* scratch, int2* fine_sorted, Item* items,
                               hipStream_t s);

// Gridding (grid.hip)
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_grid(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                       hipStream_t s);
hipError_t launch_degrid(const pg_plan* p, const pg_kernels* k, const float2* grid, float2* vis, int flags,
                         hipStream_t s);
// Recompute kbound for planes [plane0, plane0 + nplanes) from the table (after any table write).
hipError_t refresh_kernel_bound(pg_kernels* k, int plane0, int nplanes, hipStream_t s);
// Reproducible gridding (PG_DETERMINISTIC) with caller-provided scratch of grid_fixed_scratch_bytes(k).
size_t grid_fixed_scratch_bytes(const pg_kernels* k);
hipError_t launch_grid_fixed(const pg_plan* p, const pg_kernels* k, const float2* vis, float2* grid, int flags,
                             void* scratch, hipStream_t s);
hipError_t launch_taper(const pg_kernels* k, const void* in, void* out, int direction, double weight_sum,
                        hipStream_t s);
hipError_t launch_hogbom(float* residual, const float* psf, const uint8_t* mask, int n, int npol, float gain,
                         float threshold, int patch, int max_iter, int32_t* comp_pos, float* comp_val, float* model,
                         int32_t* n_comp, void* scratch, hipStream_t s);
// Masked |I| peak into the 64-bit key at scratch + 256 (scratch: 264 bytes); pixel normalisation.
hipError_t launch_masked_peak(const float* img, const uint8_t* mask, int64_t npix, void* scratch, hipStream_t s);
hipError_t launch_normalise_at(float* img, int64_t count, int64_t ref_index, float* held, hipStream_t s);
// Device address (on the current device) and size of the fixed scratch array of pg_hogbom_noalloc.
hipError_t hogbom_static_scratch(void** out, size_t* bytes);
hipError_t launch_batch_grid(const pg_batch* b, int flags, hipStream_t s);
hipError_t launch_batch_degrid(const pg_batch* b, int flags, hipStream_t s);

// Host numerics (pswf.cpp, mueller.cpp)
std::vector<double> pswf0(double c, const std::vector<double>& x);
// Screens Phi[q][c][mk][mk] (complex, interleaved) for the given kind.
bool build_screens(int npol, int kind, const double* jones, const double* jones_b, int mk, double eps, int convention,
                   std::vector<double>& phi, std::string& err);

}  // namespace pg
