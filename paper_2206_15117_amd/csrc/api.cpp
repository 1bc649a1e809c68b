// C-ABI entry points: host-side validation, kernel generation orchestration,
// plan construction and launch dispatch.  No C++ exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "mosaic.hpp"

namespace pg {

namespace {
thread_local std::string g_error;
std::mutex g_alloc_mu;
Allocator g_alloc;
constexpr size_t kLdsBudget = 160 * 1024 - 1280;  // sub-grid share of the 160 KiB; the rest is gridder scratch

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PG_HIP(call, what)                   \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_finite(double v) { return std::isfinite(v); }

int check_geometry(const pg_geometry& g, int npol) {
  if (g.n < 8 || g.n > 16384 || (g.n & 1)) return fail(PG_EINVAL, "n must be even and in [8, 16384]");
  if (!(g.cell > 0.0) || !is_finite(g.cell)) return fail(PG_EINVAL, "cell must be positive and finite");
  if (g.n * g.cell >= 2.0) return fail(PG_EINVAL, "field of view n*cell must be below 2 (direction cosines)");
  if (g.os < 2 || g.os > 16 || (g.os & 1)) return fail(PG_EINVAL, "os must be even and in [2, 16]");
  if (g.nplanes < 1 || g.nplanes > 1024) return fail(PG_EINVAL, "nplanes must be in [1, 1024]");
  if (!g.w_planes || !g.support || !g.tile) return fail(PG_EINVAL, "w_planes, support and tile must be non-NULL");
  for (int p = 0; p < g.nplanes; ++p) {
    if (!is_finite(g.w_planes[p])) return fail(PG_EINVAL, "w_planes must be finite");
    if (p && !(g.w_planes[p] > g.w_planes[p - 1])) return fail(PG_EINVAL, "w_planes must be strictly ascending");
    if (g.support[p] < 1 || g.support[p] > 64) return fail(PG_EINVAL, "support must be in [1, 64]");
    if (g.support[p] > g.n) return fail(PG_EINVAL, "support must not exceed n");
    if (g.tile[p] < 1 || g.tile[p] > g.n) return fail(PG_EINVAL, "tile must be in [1, n]");
    const int w = g.tile[p] + g.support[p] - 1;
    if (static_cast<size_t>(w) * lds_pitch(w, g.support[p]) * npol * 8 > kLdsBudget)
      return fail(PG_EUNSUPPORTED, "plane " + std::to_string(p) +
                                       ": sub-grid (tile + support - 1) rows x padded pitch x npol x 8 B exceeds 162560 B of LDS");
  }
  if (g.aa_support < 1 || g.aa_support > 64) return fail(PG_EINVAL, "aa_support must be in [1, 64]");
  if (g.mk < 2 || g.mk > 4096 || (g.mk & 1)) return fail(PG_EINVAL, "mk must be even and in [2, 4096]");
  return PG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

namespace {

int make_kernels_impl(const pg_kernel_spec* spec, hipStream_t s, pg_kernels** out, bool generate) {
  if (!spec || !out) return fail(PG_EINVAL, "spec and out must be non-NULL");
  *out = nullptr;
  if (spec->npol != 1 && spec->npol != 4) return fail(PG_EINVAL, "npol must be 1 or 4");
  if (spec->kind != PG_KIND_GRID && spec->kind != PG_KIND_DEGRID) return fail(PG_EINVAL, "kind must be PG_KIND_GRID or PG_KIND_DEGRID");
  if (spec->storage != PG_STORE_F32 && spec->storage != PG_STORE_F16) return fail(PG_EINVAL, "storage must be PG_STORE_F32 or PG_STORE_F16");
  if (spec->stokes_convention != PG_STOKES_IAU && spec->stokes_convention != PG_STOKES_PAPER)
    return fail(PG_EINVAL, "stokes_convention must be PG_STOKES_IAU or PG_STOKES_PAPER");
  if (!(spec->eps_null >= 0.0) || !is_finite(spec->eps_null)) return fail(PG_EINVAL, "eps_null must be finite and >= 0");
  int rc = check_geometry(spec->g, spec->npol);
  if (rc != PG_OK) return rc;
  if (spec->npol == 1 && (spec->jones || spec->jones_b))
    return fail(PG_EUNSUPPORTED, "npol = 1 (Stokes I only) takes no Jones field");

  const pg_geometry& g = spec->g;
  const int mk = g.mk, np = spec->npol, nqc = np * np;
  std::vector<double> phi;
  std::string err;
  if (generate &&
      !build_screens(np, spec->kind, spec->jones, spec->jones_b, mk, spec->eps_null, spec->stokes_convention, phi, err))
    return fail(PG_EINVAL, err);

  auto* k = new (std::nothrow) pg_kernels();
  if (!k) return fail(PG_ENOMEM, "host allocation failed");
  std::unique_ptr<pg_kernels> guard(k);
  k->npol = np;
  k->kind = spec->kind;
  k->storage = spec->storage;
  k->os = g.os;
  k->n = g.n;
  k->nplanes = g.nplanes;
  k->mk = mk;
  k->aa_support = g.aa_support;
  k->cell = g.cell;
  k->w_planes.assign(g.w_planes, g.w_planes + g.nplanes);
  k->support.assign(g.support, g.support + g.nplanes);
  k->tile.assign(g.tile, g.tile + g.nplanes);
  k->plane_offset.assign(g.nplanes + 1, 0);
  std::vector<PlaneInfo> pinfo(g.nplanes);
  int smax = 0;
  for (int p = 0; p < g.nplanes; ++p) {
    const int64_t S = g.support[p];
    k->plane_offset[p + 1] = k->plane_offset[p] + static_cast<int64_t>(g.os) * g.os * S * S * nqc;
    pinfo[p].offset = k->plane_offset[p];
    pinfo[p].support = g.support[p];
    pinfo[p].tile = g.tile[p];
    pinfo[p].width = g.tile[p] + g.support[p] - 1;
    pinfo[p].pitch = lds_pitch(pinfo[p].width, g.support[p]);
    k->max_width = std::max(k->max_width, pinfo[p].width);
    k->lds_bytes = std::max(k->lds_bytes, static_cast<size_t>(pinfo[p].width) * pinfo[p].pitch * np * 8);
    smax = std::max(smax, g.support[p]);
  }

  // Anti-aliasing function on the kernel lattice and at the image pixels.
  const double c = M_PI * g.aa_support / 2.0;
  std::vector<double> xl(mk), xp(g.n);
  for (int a = 0; a < mk; ++a) xl[a] = 2.0 * (a - mk / 2) / mk;
  for (int j = 0; j < g.n; ++j) xp[j] = 2.0 * (j - g.n / 2) / g.n;
  std::vector<double> aa_lat = pswf0(c, xl);
  k->aa_pixels = pswf0(c, xp);
  std::vector<double> inv_aa(g.n);
  for (int j = 0; j < g.n; ++j) inv_aa[j] = 1.0 / k->aa_pixels[j];

  const size_t entry = spec->storage == PG_STORE_F16 ? 4 : 8;
  if (!k->table.alloc(k->plane_offset.back() * entry, s) || !k->planes.alloc(sizeof(PlaneInfo) * g.nplanes, s) ||
      !k->w_dev.alloc(sizeof(double) * g.nplanes, s) || !k->inv_aa.alloc(sizeof(double) * g.n, s) ||
      !k->kbound.alloc(sizeof(float) * 4 * g.nplanes, s))
    return fail(PG_ENOMEM, "device allocation failed in make_kernels");
  PG_HIP(hipMemcpyAsync(k->planes.p, pinfo.data(), pinfo.size() * sizeof(PlaneInfo), hipMemcpyHostToDevice, s), "upload planes");
  PG_HIP(hipMemcpyAsync(k->w_dev.p, k->w_planes.data(), g.nplanes * sizeof(double), hipMemcpyHostToDevice, s), "upload w");
  PG_HIP(hipMemcpyAsync(k->inv_aa.p, inv_aa.data(), g.n * sizeof(double), hipMemcpyHostToDevice, s), "upload taper");
  if (!generate) {
    PG_HIP(hipMemsetAsync(k->table.p, 0, k->table.bytes, s), "clear table");
    PG_HIP(launch_fill_zero(k->kbound.p, k->kbound.bytes, s), "clear bound");
    PG_HIP(hipStreamSynchronize(s), "kernels_alloc sync");
    *out = guard.release();
    return PG_OK;
  }

  const size_t npix = static_cast<size_t>(mk) * mk;
  const size_t lmax = static_cast<size_t>(smax) * g.os;
  DevBuf phi_d, aa_d, f_d, e_d, a_d, t_d;
  if (!phi_d.alloc(sizeof(double2) * nqc * npix, s) || !aa_d.alloc(sizeof(double) * mk, s) ||
      !f_d.alloc(sizeof(double2) * nqc * npix, s) || !e_d.alloc(sizeof(double2) * lmax * mk, s) ||
      !a_d.alloc(sizeof(double2) * nqc * mk * lmax, s) || !t_d.alloc(sizeof(double2) * nqc * lmax * lmax, s))
    return fail(PG_ENOMEM, "device allocation failed in make_kernels");
  PG_HIP(hipMemcpyAsync(phi_d.p, phi.data(), phi.size() * sizeof(double), hipMemcpyHostToDevice, s), "upload screens");
  PG_HIP(hipMemcpyAsync(aa_d.p, aa_lat.data(), mk * sizeof(double), hipMemcpyHostToDevice, s), "upload AA");
  const double fov = g.n * g.cell;
  for (int p = 0; p < g.nplanes; ++p) {
    const int S = g.support[p];
    const int len = S * g.os;
    PG_HIP(launch_screen(phi_d.as<double2>(), aa_d.as<double>(), g.w_planes[p], fov, mk, nqc, f_d.as<double2>(), s), "screen");
    PG_HIP(launch_twiddles(S, g.os, mk, e_d.as<double2>(), s), "twiddles");
    // A[qc][b][dx] = sum_a F[qc][b][a] E[dx][a]
    PG_HIP(launch_zgemm_nt(nqc, mk, len, mk, f_d.as<double2>(), npix, e_d.as<double2>(), 0, a_d.as<double2>(),
                           static_cast<int64_t>(mk) * len, s), "dft stage 1");
    // T[qc][dy][dx] = sum_b E[dy][b] A[qc][b][dx]
    PG_HIP(launch_zgemm_nn(nqc, len, len, mk, e_d.as<double2>(), 0, a_d.as<double2>(), static_cast<int64_t>(mk) * len,
                           t_d.as<double2>(), static_cast<int64_t>(len) * len, s), "dft stage 2");
    void* dst = static_cast<char*>(k->table.p) + k->plane_offset[p] * entry;
    PG_HIP(launch_pack(t_d.as<double2>(), S, g.os, nqc, spec->storage, dst, s), "pack");
  }
  PG_HIP(refresh_kernel_bound(k, 0, g.nplanes, s), "kernel bound");
  PG_HIP(hipStreamSynchronize(s), "make_kernels sync");
  *out = guard.release();
  return PG_OK;
}

bool same_geometry(const pg_plan* p, const pg_kernels* k) {
  return p->n == k->n && p->os == k->os && p->support == k->support && p->tile == k->tile;
}

int plan_impl(const pg_kernels* k, const double* uvw, int64_t nvis, int32_t max_chunk, hipStream_t s, pg_plan** out,
              int64_t* n_dropped) {
  if (!k || !out) return fail(PG_EINVAL, "kernels and out must be non-NULL");
  *out = nullptr;
  if (nvis < 0 || nvis > 0x7ffffff0LL) return fail(PG_EINVAL, "nvis must be in [0, 2^31 - 16]");
  if (nvis > 0 && !uvw) return fail(PG_EINVAL, "uvw must be non-NULL when nvis > 0");
  if (max_chunk < 1 || max_chunk > (1 << 30)) return fail(PG_EINVAL, "max_chunk must be in [1, 2^30]");
  auto* p = new (std::nothrow) pg_plan();
  if (!p) return fail(PG_ENOMEM, "host allocation failed");
  std::unique_ptr<pg_plan> guard(p);
  p->nvis = nvis;
  p->max_chunk = max_chunk;
  p->n = k->n;
  p->os = k->os;
  p->support = k->support;
  p->tile = k->tile;
  const int min_tile = *std::min_element(k->tile.begin(), k->tile.end());
  const int nt = (k->n + min_tile - 1) / min_tile;
  const unsigned __int128 nbins = static_cast<unsigned __int128>(k->nplanes) * nt * nt * k->os * k->os;
  int bits = 1;
  while (bits < 64 && (static_cast<unsigned __int128>(1) << bits) <= nbins) ++bits;  // 2^bits > max key + 1
  if ((static_cast<unsigned __int128>(1) << bits) <= nbins) return fail(PG_EUNSUPPORTED, "binning key exceeds 64 bits");
  const uint64_t drop_key = bits == 64 ? ~0ull : ((1ull << bits) - 1);
  if (nvis == 0) {
    if (n_dropped) *n_dropped = 0;
    *out = guard.release();
    return PG_OK;
  }
  // the binning temporaries share one allocation (each allocation may call back into a caller's
  // allocator): keys and sort buffers, fine positions, scratch and counts, 256-byte aligned parts
  const int64_t sc = std::max(radix_scratch_elems(nvis), plan_scratch_elems(nvis));
  const size_t part_bytes[7] = {static_cast<size_t>(8 * nvis), static_cast<size_t>(8 * nvis),
                                static_cast<size_t>(4 * nvis), static_cast<size_t>(4 * nvis),
                                static_cast<size_t>(8 * nvis), static_cast<size_t>(4 * sc), 16};
  size_t part_off[7], tmp_bytes = 0;
  for (int i = 0; i < 7; ++i) {
    part_off[i] = tmp_bytes;
    tmp_bytes += (part_bytes[i] + 255) / 256 * 256;
  }
  DevBuf tmp;
  if (!tmp.alloc(tmp_bytes, s) || !p->perm.alloc(4 * nvis, s)) return fail(PG_ENOMEM, "device allocation failed in plan");
  char* base = static_cast<char*>(tmp.p);
  auto* keys = reinterpret_cast<uint64_t*>(base + part_off[0]);
  auto* keys_t = reinterpret_cast<uint64_t*>(base + part_off[1]);
  auto* vals = reinterpret_cast<int32_t*>(base + part_off[2]);
  auto* vals_t = reinterpret_cast<int32_t*>(base + part_off[3]);
  auto* fine_all = reinterpret_cast<int2*>(base + part_off[4]);
  auto* scratch = reinterpret_cast<int32_t*>(base + part_off[5]);
  auto* counts = reinterpret_cast<int32_t*>(base + part_off[6]);
  PG_HIP(launch_fill_zero(counts, 16, s), "zero counts");
  PG_HIP(launch_plan_keys(uvw, nvis, k->n, k->cell, k->os, k->nplanes, k->w_dev.as<double>(), k->planes.as<PlaneInfo>(),
                          nt, drop_key, keys, vals, fine_all, s), "plan keys");
  bool in_tmp = false;
  PG_HIP(radix_sort_pairs(keys, vals, keys_t, vals_t, nvis, bits, scratch, sc, s, &in_tmp), "radix sort");
  const uint64_t* ks = in_tmp ? keys_t : keys;
  const int32_t* vs = in_tmp ? vals_t : vals;
  PG_HIP(launch_plan_stage_a(ks, nvis, drop_key, k->os, max_chunk, counts, scratch, sc, s), "plan items");
  int32_t hc[4] = {0, 0, 0, 0};
  PG_HIP(hipMemcpyAsync(hc, counts, 16, hipMemcpyDeviceToHost, s), "read counts");
  PG_HIP(hipStreamSynchronize(s), "plan sync");
  p->n_kept = hc[0];
  p->n_items = hc[1];
  const int64_t n_runs = hc[2];
  p->n_dropped = nvis - p->n_kept;
  if (!p->fine.alloc(8 * std::max<int64_t>(p->n_kept, 1), s) || !p->items.alloc(sizeof(Item) * std::max<int64_t>(p->n_items, 1), s))
    return fail(PG_ENOMEM, "device allocation failed in plan");
  PG_HIP(hipMemcpyAsync(p->perm.p, vs, 4 * nvis, hipMemcpyDeviceToDevice, s), "copy perm");
  PG_HIP(launch_plan_scatter(ks, vs, fine_all, p->n_kept, n_runs, nvis, k->os, nt, max_chunk,
                             k->planes.as<PlaneInfo>(), scratch, p->fine.as<int2>(), p->items.as<Item>(), s),
         "plan scatter");
  PG_HIP(hipStreamSynchronize(s), "plan sync");
  if (n_dropped) *n_dropped = p->n_dropped;
  *out = guard.release();
  return PG_OK;
}

int check_run(const pg_plan* p, const pg_kernels* k, const void* a, const void* b, int32_t flags, int allowed) {
  if (!p || !k) return fail(PG_EINVAL, "plan and kernels must be non-NULL");
  if (!b) return fail(PG_EINVAL, "output buffer must be non-NULL");
  if (!a && p->nvis > 0) return fail(PG_EINVAL, "input buffer must be non-NULL");
  if (flags & ~allowed) return fail(PG_EINVAL, "unknown flag bits");
  if (!same_geometry(p, k)) return fail(PG_EINVAL, "plan was built for a different geometry than these kernels");
  return PG_OK;
}

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" {

int pg_version(void) { return (1 << 16) | 0; }

const char* pg_last_error(void) { return g_error.c_str(); }

void pg_set_allocator(void* (*alloc_fn)(size_t, void*, void*), void (*free_fn)(void*, void*, void*), void* ctx) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (!alloc_fn || !free_fn) {
    g_alloc = Allocator();
  } else {
    g_alloc.alloc_fn = alloc_fn;
    g_alloc.free_fn = free_fn;
    g_alloc.ctx = ctx;
  }
}

int pg_make_kernels(const pg_kernel_spec* spec, void* stream, pg_kernels** out) {
  g_error.clear();
  try {
    return make_kernels_impl(spec, static_cast<hipStream_t>(stream), out, true);
  } catch (...) {
    return fail(PG_ENOMEM, "exception in make_kernels");
  }
}

int pg_kernels_alloc(const pg_kernel_spec* spec, void* stream, pg_kernels** out) {
  g_error.clear();
  try {
    return make_kernels_impl(spec, static_cast<hipStream_t>(stream), out, false);
  } catch (...) {
    return fail(PG_ENOMEM, "exception in kernels_alloc");
  }
}

int pg_kernels_info(const pg_kernels* k, pg_kernels_desc* out) {
  g_error.clear();
  if (!k || !out) return fail(PG_EINVAL, "kernels and out must be non-NULL");
  out->npol = k->npol;
  out->kind = k->kind;
  out->storage = k->storage;
  out->os = k->os;
  out->n = k->n;
  out->nplanes = k->nplanes;
  out->table = k->table.p;
  out->plane_offset = k->plane_offset.data();
  out->aa_pixels = k->aa_pixels.data();
  return PG_OK;
}

int pg_kernels_copy_table(const pg_kernels* k, void* dst, void* stream) {
  g_error.clear();
  if (!k || !dst) return fail(PG_EINVAL, "kernels and dst must be non-NULL");
  PG_HIP(hipMemcpyAsync(dst, k->table.p, k->table.bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
         "copy table");
  return PG_OK;
}

int pg_kernels_load_table(pg_kernels* k, const void* src, void* stream) {
  g_error.clear();
  if (!k || !src) return fail(PG_EINVAL, "kernels and src must be non-NULL");
  PG_HIP(hipMemcpyAsync(k->table.p, src, k->table.bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
         "load table");
  PG_HIP(refresh_kernel_bound(k, 0, k->nplanes, static_cast<hipStream_t>(stream)), "kernel bound");
  return PG_OK;
}

void pg_kernels_destroy(pg_kernels* k) { delete k; }

int pg_plan_create(const pg_kernels* k, const double* uvw, int64_t nvis, int32_t max_chunk, void* stream,
                   pg_plan** out, int64_t* n_dropped) {
  g_error.clear();
  try {
    return plan_impl(k, uvw, nvis, max_chunk, static_cast<hipStream_t>(stream), out, n_dropped);
  } catch (...) {
    return fail(PG_ENOMEM, "exception in plan_create");
  }
}

int pg_plan_info(const pg_plan* p, pg_plan_desc* out) {
  g_error.clear();
  if (!p || !out) return fail(PG_EINVAL, "plan and out must be non-NULL");
  out->nvis = p->nvis;
  out->n_kept = p->n_kept;
  out->n_dropped = p->n_dropped;
  out->n_items = p->n_items;
  out->perm = p->perm.as<int32_t>();
  out->fine = p->fine.as<int32_t>();
  out->items = p->items.as<int32_t>();
  return PG_OK;
}

int pg_plan_copy(const pg_plan* p, int32_t* perm, int32_t* fine, int32_t* items, void* stream) {
  g_error.clear();
  if (!p) return fail(PG_EINVAL, "plan must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (perm && p->nvis) PG_HIP(hipMemcpyAsync(perm, p->perm.p, 4 * p->nvis, hipMemcpyDeviceToDevice, s), "copy perm");
  if (fine && p->n_kept) PG_HIP(hipMemcpyAsync(fine, p->fine.p, 8 * p->n_kept, hipMemcpyDeviceToDevice, s), "copy fine");
  if (items && p->n_items)
    PG_HIP(hipMemcpyAsync(items, p->items.p, sizeof(Item) * p->n_items, hipMemcpyDeviceToDevice, s), "copy items");
  return PG_OK;
}

void pg_plan_destroy(pg_plan* p) { delete p; }

int pg_plan_set_launch(pg_plan* p, int32_t grid_variant, int32_t grid_waves, int32_t degrid_waves,
                       int32_t xcd_group, int32_t grid_planes, int32_t degrid_corrs) {
  g_error.clear();
  if (!p) return fail(PG_EINVAL, "plan must be non-NULL");
  if (grid_variant < 0 || grid_variant > 3) return fail(PG_EINVAL, "grid_variant must be 0, 1, 2 or 3");
  auto ok = [](int w) { return w == 4 || w == 6 || w == 8 || w == 16; };
  if (!ok(grid_waves) || !ok(degrid_waves)) return fail(PG_EINVAL, "waves per workgroup must be 4, 6, 8 or 16");
  if (xcd_group < 1 || xcd_group > 4096) return fail(PG_EINVAL, "xcd_group must be in [1, 4096]");
  if (grid_planes != 0 && grid_planes != 1 && grid_planes != 2 && grid_planes != 4)
    return fail(PG_EINVAL, "grid_planes must be 0, 1, 2 or 4");
  if (degrid_corrs != 0 && degrid_corrs != 2 && degrid_corrs != 4)
    return fail(PG_EINVAL, "degrid_corrs must be 0, 2 or 4");
  p->xcd_group = xcd_group;
  p->grid_planes = grid_planes;
  p->degrid_corrs = degrid_corrs;
  p->grid_variant = grid_variant;
  p->grid_waves = grid_waves;
  p->degrid_waves = degrid_waves;
  return PG_OK;
}

int pg_grid(const pg_plan* p, const pg_kernels* k, const void* vis, void* grid, int32_t flags, void* stream) {
  g_error.clear();
  int rc = check_run(p, k, vis, grid, flags,
                     PG_ACCUMULATE | PG_FFTSHIFT | PG_VARIANT_ATOMIC | PG_VARIANT_BANDED | PG_VARIANT_SHARED |
                         PG_DETERMINISTIC);
  if (rc != PG_OK) return rc;
  const int variants = ((flags & PG_VARIANT_ATOMIC) != 0) + ((flags & PG_VARIANT_BANDED) != 0) +
                       ((flags & PG_VARIANT_SHARED) != 0);
  if (variants > 1) return fail(PG_EINVAL, "choose one grid variant");
  if ((flags & PG_DETERMINISTIC) && (flags & (PG_VARIANT_ATOMIC | PG_VARIANT_SHARED)))
    return fail(PG_EINVAL, "PG_DETERMINISTIC uses the row-band kernel, not PG_VARIANT_ATOMIC or PG_VARIANT_SHARED");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (flags & PG_DETERMINISTIC) {
    try {
      DevBuf scratch;
      if (!scratch.alloc(grid_fixed_scratch_bytes(k), s)) return fail(PG_ENOMEM, "device allocation failed in grid");
      PG_HIP(launch_grid_fixed(p, k, static_cast<const float2*>(vis), static_cast<float2*>(grid), flags, scratch.p, s),
             "deterministic grid");
    } catch (...) {
      return fail(PG_ENOMEM, "exception in grid");
    }
    return PG_OK;
  }
  PG_HIP(launch_grid(p, k, static_cast<const float2*>(vis), static_cast<float2*>(grid), flags, s), "grid");
  return PG_OK;
}

int pg_degrid(const pg_plan* p, const pg_kernels* k, const void* grid, void* vis_out, int32_t flags, void* stream) {
  g_error.clear();
  int rc = check_run(p, k, grid, vis_out, flags, PG_ACCUMULATE | PG_FFTSHIFT);
  if (rc != PG_OK) return rc;
  if (!grid) return fail(PG_EINVAL, "grid must be non-NULL");
  PG_HIP(launch_degrid(p, k, static_cast<const float2*>(grid), static_cast<float2*>(vis_out), flags,
                       static_cast<hipStream_t>(stream)), "degrid");
  return PG_OK;
}

int pg_batch_create(const pg_field* fields, int32_t nfields, void* stream, pg_batch** out) {
  g_error.clear();
  try {
    if (!fields || !out || nfields < 1 || nfields > 65536)
      return fail(PG_EINVAL, "fields and out must be non-NULL and nfields in [1, 65536]");
    *out = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* b = new (std::nothrow) pg_batch();
    if (!b) return fail(PG_ENOMEM, "host allocation failed");
    std::unique_ptr<pg_batch> guard(b);
    b->nfields = nfields;
    std::vector<FieldArgs> fa(nfields);
    struct Cost {
      int64_t cost;
      int32_t field, item;
    };
    std::vector<Cost> costs;
    for (int f = 0; f < nfields; ++f) {
      const pg_field& fd = fields[f];
      if (!fd.plan || !fd.kernels || !fd.grid) return fail(PG_EINVAL, "field " + std::to_string(f) + ": NULL plan, kernels or grid");
      if (!fd.vis && fd.plan->nvis > 0) return fail(PG_EINVAL, "field " + std::to_string(f) + ": NULL visibilities");
      if (!same_geometry(fd.plan, fd.kernels)) return fail(PG_EINVAL, "field " + std::to_string(f) + ": plan and kernels differ in geometry");
      if (f == 0) {
        b->npol = fd.kernels->npol;
        b->storage = fd.kernels->storage;
        b->grid_waves = fd.plan->grid_waves;
        b->degrid_waves = fd.plan->degrid_waves;
        b->grid_variant = fd.plan->grid_variant;
        b->grid_planes = fd.plan->grid_planes;
      } else if (fd.kernels->npol != b->npol || fd.kernels->storage != b->storage) {
        return fail(PG_EINVAL, "all fields of a batch must share npol and table storage");
      }
      b->plans.push_back(fd.plan);
      b->kernels.push_back(fd.kernels);
      b->vis.push_back(fd.vis);
      b->grids.push_back(fd.grid);
      b->lds_bytes = std::max(b->lds_bytes, fd.kernels->lds_bytes);
      fa[f] = FieldArgs{fd.plan->items.as<Item>(), fd.plan->fine.as<int2>(), fd.plan->perm.as<int32_t>(),
                        static_cast<float2*>(fd.vis), fd.kernels->table.p, fd.kernels->planes.as<PlaneInfo>(),
                        static_cast<float2*>(fd.grid), fd.kernels->kbound.as<float>(), fd.kernels->os,
                        fd.kernels->n};
      std::vector<Item> items(fd.plan->n_items);
      if (fd.plan->n_items) {
        PG_HIP(hipMemcpyAsync(items.data(), fd.plan->items.p, sizeof(Item) * items.size(), hipMemcpyDeviceToHost, s),
               "read items");
        PG_HIP(hipStreamSynchronize(s), "batch sync");
      }
      for (int64_t i = 0; i < fd.plan->n_items; ++i) {
        const int S = fd.kernels->support[items[i].plane];
        const int W = fd.kernels->tile[items[i].plane] + S - 1;
        costs.push_back({static_cast<int64_t>(items[i].end - items[i].start) * S * S + static_cast<int64_t>(W) * W,
                         f, static_cast<int32_t>(i)});
      }
    }
    // Fields largest first (total estimated cost), each in plan order (plane by plane, tile by
    // tile), cut into groups of up to `group` consecutive items (the first field's XCD grouping).
    // Group k goes to XCD k mod 8, behind that XCD's earlier groups; XCD x's j-th entry is block
    // 8 j + x.  Shorter XCD queues are padded with no-op entries.  Field-major order keeps one or
    // two fields' kernel tables and grids in the caches at a time; the first large field starts
    // first and the smallest field fills the tail.
    const int group = std::max(1, fields[0].plan->xcd_group);
    std::vector<int64_t> field_cost(nfields, 0);
    for (const auto& c : costs) field_cost[c.field] += c.cost;
    std::vector<int> rank(nfields), by_cost(nfields);
    for (int f = 0; f < nfields; ++f) by_cost[f] = f;
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) { return field_cost[x] > field_cost[y]; });
    for (int r = 0; r < nfields; ++r) rank[by_cost[r]] = r;
    std::stable_sort(costs.begin(), costs.end(), [&](const Cost& x, const Cost& y) { return rank[x.field] < rank[y.field]; });
    struct Group {
      size_t first, count;
    };
    std::vector<Group> groups;
    for (size_t i = 0; i < costs.size();) {
      size_t e = i;
      while (e < costs.size() && e - i < static_cast<size_t>(group) && costs[e].field == costs[i].field) ++e;
      groups.push_back({i, e - i});
      i = e;
    }
    std::vector<int2> queue[8];
    for (size_t k = 0; k < groups.size(); ++k)
      for (size_t i = 0; i < groups[k].count; ++i) {
        const Cost& c = costs[groups[k].first + i];
        queue[k % 8].push_back(make_int2(c.field, c.item));
      }
    size_t depth = 0;
    for (const auto& q : queue) depth = std::max(depth, q.size());
    std::vector<int2> work(depth * 8, make_int2(-1, -1));
    for (int x = 0; x < 8; ++x)
      for (size_t j = 0; j < queue[x].size(); ++j) work[8 * j + x] = queue[x][j];
    b->n_work = static_cast<int64_t>(costs.size());
    b->n_blocks = static_cast<int64_t>(work.size());
    if (!b->fields.alloc(sizeof(FieldArgs) * nfields, s) || !b->work.alloc(sizeof(int2) * std::max<size_t>(work.size(), 1), s))
      return fail(PG_ENOMEM, "device allocation failed in batch_create");
    PG_HIP(hipMemcpyAsync(b->fields.p, fa.data(), sizeof(FieldArgs) * nfields, hipMemcpyHostToDevice, s), "upload fields");
    if (!work.empty())
      PG_HIP(hipMemcpyAsync(b->work.p, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, s), "upload work");
    PG_HIP(hipStreamSynchronize(s), "batch sync");
    *out = guard.release();
    return PG_OK;
  } catch (...) {
    return fail(PG_ENOMEM, "exception in batch_create");
  }
}

int pg_batch_grid(const pg_batch* b, int32_t flags, void* stream) {
  g_error.clear();
  if (!b) return fail(PG_EINVAL, "batch must be non-NULL");
  if (flags & ~(PG_ACCUMULATE | PG_FFTSHIFT)) return fail(PG_EINVAL, "unknown flag bits");
  PG_HIP(launch_batch_grid(b, flags, static_cast<hipStream_t>(stream)), "batch grid");
  return PG_OK;
}

int pg_batch_degrid(const pg_batch* b, int32_t flags, void* stream) {
  g_error.clear();
  if (!b) return fail(PG_EINVAL, "batch must be non-NULL");
  if (flags & ~PG_FFTSHIFT) return fail(PG_EINVAL, "unknown flag bits");
  PG_HIP(launch_batch_degrid(b, flags, static_cast<hipStream_t>(stream)), "batch degrid");
  return PG_OK;
}

int64_t pg_batch_work_items(const pg_batch* b) { return b ? b->n_work : -1; }

void pg_batch_destroy(pg_batch* b) { delete b; }

int pg_taper(const pg_kernels* k, const void* in, void* out, int32_t direction, double weight_sum, void* stream) {
  g_error.clear();
  if (!k || !in || !out) return fail(PG_EINVAL, "kernels, in and out must be non-NULL");
  if (direction != PG_TAPER_IMAGE && direction != PG_TAPER_PREDICT) return fail(PG_EINVAL, "unknown taper direction");
  if (direction == PG_TAPER_IMAGE && (!(weight_sum > 0.0) || !is_finite(weight_sum)))
    return fail(PG_EINVAL, "weight_sum must be positive and finite");
  if (direction == PG_TAPER_PREDICT && !is_finite(weight_sum)) return fail(PG_EINVAL, "scale must be finite");
  PG_HIP(launch_taper(k, in, out, direction, weight_sum, static_cast<hipStream_t>(stream)), "taper");
  return PG_OK;
}

namespace {
int check_frame(const pg_sky_frame* f, const char* what) {
  if (!f) return fail(PG_EINVAL, std::string(what) + " frame must be non-NULL");
  if (f->n < 2 || f->n > 65536) return fail(PG_EINVAL, std::string(what) + " frame: n must be in [2, 65536]");
  if (!(f->cell > 0.0) || !is_finite(f->cell)) return fail(PG_EINVAL, std::string(what) + " frame: cell must be positive and finite");
  if (!is_finite(f->ra)) return fail(PG_EINVAL, std::string(what) + " frame: ra must be finite");
  if (!(std::fabs(f->dec) <= 1.5707963267948966)) return fail(PG_EINVAL, std::string(what) + " frame: |dec| must be <= pi/2");
  return PG_OK;
}
}  // namespace

int pg_reproject(const float* src, const float* src_weight, const pg_sky_frame* src_frame, float* dst,
                 float* dst_weight, const pg_sky_frame* dst_frame, int32_t npol, int32_t flags, void* stream) {
  g_error.clear();
  if (!src || !dst) return fail(PG_EINVAL, "src and dst must be non-NULL");
  int rc = check_frame(src_frame, "source");
  if (rc != PG_OK) return rc;
  rc = check_frame(dst_frame, "destination");
  if (rc != PG_OK) return rc;
  if (npol < 1 || npol > 4) return fail(PG_EINVAL, "npol must be in [1, 4]");
  if (flags & ~PG_ACCUMULATE) return fail(PG_EINVAL, "unknown flag bits");
  PG_HIP(launch_reproject(src, src_weight, *src_frame, dst, dst_weight, *dst_frame, npol, (flags & PG_ACCUMULATE) != 0,
                          static_cast<hipStream_t>(stream)),
         "reproject");
  return PG_OK;
}

int pg_phase_rotate(const double* uvw_in, const void* vis_in, int64_t nvis, int32_t npol, double ra_from,
                    double dec_from, double ra_to, double dec_to, double* uvw_out, void* vis_out, void* stream) {
  g_error.clear();
  if (nvis < 0 || nvis > (int64_t(1) << 40)) return fail(PG_EINVAL, "nvis must be in [0, 2^40]");
  if (nvis > 0 && (!uvw_in || !vis_in || !vis_out)) return fail(PG_EINVAL, "uvw_in, vis_in and vis_out must be non-NULL");
  if (npol < 1 || npol > 4) return fail(PG_EINVAL, "npol must be in [1, 4]");
  if (!is_finite(ra_from) || !is_finite(ra_to)) return fail(PG_EINVAL, "ra must be finite");
  if (!(std::fabs(dec_from) <= 1.5707963267948966) || !(std::fabs(dec_to) <= 1.5707963267948966))
    return fail(PG_EINVAL, "|dec| must be <= pi/2");
  if (nvis == 0) return PG_OK;
  PG_HIP(launch_phase_rotate(uvw_in, vis_in, nvis, npol, ra_from, dec_from, ra_to, dec_to, uvw_out, vis_out,
                             static_cast<hipStream_t>(stream)),
         "phase rotate");
  return PG_OK;
}

int pg_weight_normalise(float* img, const float* weight, int32_t n, int32_t npol, float min_weight, void* stream) {
  g_error.clear();
  if (!img || !weight) return fail(PG_EINVAL, "img and weight must be non-NULL");
  if (n < 1 || n > 65536) return fail(PG_EINVAL, "n must be in [1, 65536]");
  if (npol < 1 || npol > 4) return fail(PG_EINVAL, "npol must be in [1, 4]");
  if (!(min_weight > 0.0f) || !std::isfinite(min_weight)) return fail(PG_EINVAL, "min_weight must be positive and finite");
  PG_HIP(launch_weight_normalise(img, weight, n, npol, min_weight, static_cast<hipStream_t>(stream)), "normalise");
  return PG_OK;
}

int pg_mosaic_gamma(const float* beams, int32_t nfields, int32_t n, double floor_frac, double scale, float* weight_sum,
                    float* img, int32_t npol, void* stream) {
  g_error.clear();
  if (!beams || !weight_sum || !img) return fail(PG_EINVAL, "beams, weight_sum and img must be non-NULL");
  if (nfields < 1 || nfields > 65536) return fail(PG_EINVAL, "nfields must be in [1, 65536]");
  if (n < 1 || n > 65536) return fail(PG_EINVAL, "n must be in [1, 65536]");
  if (static_cast<int64_t>(nfields) * n * n > (int64_t(1) << 40)) return fail(PG_EINVAL, "beam cube too large");
  if (npol < 1 || npol > 4) return fail(PG_EINVAL, "npol must be in [1, 4]");
  if (!(floor_frac >= 0.0 && floor_frac <= 1.0)) return fail(PG_EINVAL, "floor_frac must be in [0, 1]");
  if (!is_finite(scale)) return fail(PG_EINVAL, "scale must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DevBuf scratch;
    if (!scratch.alloc(256, s)) return fail(PG_ENOMEM, "device allocation failed in mosaic_gamma");
    PG_HIP(launch_mosaic_gamma(beams, nfields, n, floor_frac, scale, weight_sum, img, npol, scratch.as<unsigned>(), s),
           "mosaic gamma");
  } catch (...) {
    return fail(PG_ENOMEM, "exception in mosaic_gamma");
  }
  return PG_OK;
}

static int check_hogbom(const float* residual, const float* psf, const int32_t* comp_pos, const float* comp_val,
                 const int32_t* n_comp, int32_t n, int32_t npol, float gain, float threshold, int32_t max_iter) {
  if (!residual || !psf || !comp_pos || !comp_val || !n_comp)
    return fail(PG_EINVAL, "residual, psf, comp_pos, comp_val and n_comp must be non-NULL");
  if (n < 2 || n > 16384 || (n & 1)) return fail(PG_EINVAL, "n must be even and in [2, 16384]");
  if (npol < 1 || npol > 4) return fail(PG_EINVAL, "npol must be in [1, 4]");
  if (!(gain > 0.0f && gain <= 1.0f)) return fail(PG_EINVAL, "gain must be in (0, 1]");
  if (!(threshold >= 0.0f) || !std::isfinite(threshold)) return fail(PG_EINVAL, "threshold must be finite and >= 0");
  if (max_iter < 0 || max_iter > (1 << 20)) return fail(PG_EINVAL, "max_iter must be in [0, 2^20]");
  return PG_OK;
}

int pg_hogbom(float* residual, const float* psf, const uint8_t* mask, int32_t n, int32_t npol, float gain,
              float threshold, int32_t psf_patch, int32_t max_iter, int32_t* comp_pos, float* comp_val, float* model,
              int32_t* n_comp, void* stream) {
  g_error.clear();
  const int rc = check_hogbom(residual, psf, comp_pos, comp_val, n_comp, n, npol, gain, threshold, max_iter);
  if (rc != PG_OK) return rc;
  const int patch = (psf_patch <= 0 || psf_patch > n) ? n : psf_patch;
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DevBuf scratch;
    if (!scratch.alloc(256 + 8 * static_cast<size_t>(std::max(max_iter, 1)), s))
      return fail(PG_ENOMEM, "device allocation failed in hogbom");
    PG_HIP(launch_hogbom(residual, psf, mask, n, npol, gain, threshold, patch, max_iter, comp_pos, comp_val, model,
                         n_comp, scratch.p, s),
           "hogbom");
  } catch (...) {
    return fail(PG_ENOMEM, "exception in hogbom");
  }
  return PG_OK;
}

int pg_masked_peak(const float* img, const uint8_t* mask, int64_t npix, float* peak, int64_t* index, void* stream) {
  g_error.clear();
  if (!img || !peak || !index) return fail(PG_EINVAL, "img, peak and index must be non-NULL");
  if (npix < 1 || npix > (int64_t(1) << 32) - 1) return fail(PG_EINVAL, "npix must be in [1, 2^32 - 1]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DevBuf scratch;
    if (!scratch.alloc(256 + 8, s)) return fail(PG_ENOMEM, "device allocation failed in masked_peak");
    PG_HIP(launch_masked_peak(img, mask, npix, scratch.p, s), "masked peak");
    unsigned long long key = 0;
    PG_HIP(hipMemcpyAsync(&key, static_cast<char*>(scratch.p) + 256, 8, hipMemcpyDeviceToHost, s), "peak readback");
    PG_HIP(hipStreamSynchronize(s), "peak sync");
    if (key == 0) {
      *peak = 0.0f;
      *index = -1;
    } else {
      const uint32_t bits = static_cast<uint32_t>(key >> 32);
      std::memcpy(peak, &bits, 4);
      *index = static_cast<int64_t>(0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFFu));
    }
  } catch (...) {
    return fail(PG_ENOMEM, "exception in masked_peak");
  }
  return PG_OK;
}

int pg_normalise_at(float* img, int64_t count, int64_t ref_index, void* stream) {
  g_error.clear();
  if (!img) return fail(PG_EINVAL, "img must be non-NULL");
  if (count < 1 || ref_index < 0 || ref_index >= count) return fail(PG_EINVAL, "need 0 <= ref_index < count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    DevBuf held;
    if (!held.alloc(4, s)) return fail(PG_ENOMEM, "device allocation failed in normalise_at");
    PG_HIP(launch_normalise_at(img, count, ref_index, held.as<float>(), s), "normalise");
  } catch (...) {
    return fail(PG_ENOMEM, "exception in normalise_at");
  }
  return PG_OK;
}

int pg_hogbom_noalloc(float* residual, const float* psf, const uint8_t* mask, int32_t n, int32_t npol, float gain,
                      float threshold, int32_t psf_patch, int32_t max_iter, int32_t* comp_pos, float* comp_val,
                      float* model, int32_t* n_comp, void* stream) {
  g_error.clear();
  const int rc = check_hogbom(residual, psf, comp_pos, comp_val, n_comp, n, npol, gain, threshold, max_iter);
  if (rc != PG_OK) return rc;
  if (max_iter > PG_HOGBOM_STATIC_MAX_ITER)
    return fail(PG_EINVAL, "max_iter exceeds PG_HOGBOM_STATIC_MAX_ITER (" +
                               std::to_string(PG_HOGBOM_STATIC_MAX_ITER) + ") for pg_hogbom_noalloc");
  const int patch = (psf_patch <= 0 || psf_patch > n) ? n : psf_patch;
  void* scratch = nullptr;
  size_t bytes = 0;
  PG_HIP(hogbom_static_scratch(&scratch, &bytes), "hogbom_noalloc scratch address");
  if (256 + 8 * static_cast<size_t>(std::max(max_iter, 1)) > bytes) return fail(PG_EINVAL, "scratch too small");
  PG_HIP(launch_hogbom(residual, psf, mask, n, npol, gain, threshold, patch, max_iter, comp_pos, comp_val, model,
                       n_comp, scratch, static_cast<hipStream_t>(stream)),
         "hogbom_noalloc");
  return PG_OK;
}

}  // extern "C"
