// Host-side driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host
// code (argument validation, geometry checks, the Mueller screens of Sec. 3.2-3.3 with the Eq. 6
// regularisation, the prolate spheroidal anti-aliasing function, error reporting).
//
// Runs without a GPU: a registered allocator that always fails stops every creating call at its
// first device allocation, after all host work for it is done, so each call must return PG_ENOMEM
// (valid arguments) or PG_EINVAL / PG_EUNSUPPORTED (invalid ones).  Exits non-zero on any
// unexpected return code; the sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "polgrid.h"

namespace {

int g_failures = 0;
int g_calls = 0;

void* fail_alloc(size_t, void*, void*) { return nullptr; }
void no_free(void*, void*, void*) {}

void expect(int got, int want, const char* what) {
  ++g_calls;
  const char* msg = pg_last_error();
  if (got != want) {
    std::fprintf(stderr, "FAIL %s: got %d want %d (%s)\n", what, got, want, msg ? msg : "");
    ++g_failures;
  }
  if (got != PG_OK && (!msg || std::strlen(msg) == 0)) {
    std::fprintf(stderr, "FAIL %s: error %d without a message\n", what, got);
    ++g_failures;
  }
}

struct Geometry {
  std::vector<double> w;
  std::vector<int32_t> support, tile;
  pg_geometry g{};
  Geometry(int n, int os, int nplanes, int s0, int tile0, int mk) {
    for (int p = 0; p < nplanes; ++p) {
      w.push_back(-100.0 + 200.0 * p / std::max(1, nplanes - 1));
      support.push_back(s0 + 2 * (p % 3));
      tile.push_back(tile0);
    }
    g.n = n;
    g.cell = 1e-4;
    g.os = os;
    g.nplanes = nplanes;
    g.w_planes = w.data();
    g.support = support.data();
    g.tile = tile.data();
    g.aa_support = 7;
    g.mk = mk;
  }
};

std::vector<double> random_jones(int mk, std::mt19937_64& rng, double leak) {
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> j(2 * 4 * static_cast<size_t>(mk) * mk);
  const size_t npix = static_cast<size_t>(mk) * mk;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (size_t px = 0; px < npix; ++px) {
        const size_t o = 2 * ((static_cast<size_t>(a) * 2 + b) * npix + px);
        const double base = (a == b) ? 1.0 : 0.0;
        j[o] = base + leak * nd(rng);
        j[o + 1] = leak * nd(rng);
      }
  return j;
}

pg_kernel_spec spec_of(const Geometry& geo, int npol, int kind, const double* jones, const double* jones_b, double eps,
                       int conv, int storage) {
  pg_kernel_spec s{};
  s.g = geo.g;
  s.npol = npol;
  s.kind = kind;
  s.jones = jones;
  s.eps_null = eps;
  s.stokes_convention = conv;
  s.storage = storage;
  s.jones_b = jones_b;
  return s;
}

void kernels_cases() {
  std::mt19937_64 rng(2206);
  for (int mk : {16, 32, 34}) {
    Geometry geo(64, 4, 3, 7, 8, mk);
    const std::vector<double> ja = random_jones(mk, rng, 0.1), jb = random_jones(mk, rng, 0.2);
    for (int kind : {PG_KIND_GRID, PG_KIND_DEGRID})
      for (int conv : {PG_STOKES_IAU, PG_STOKES_PAPER})
        for (int storage : {PG_STORE_F32, PG_STORE_F16}) {
          pg_kernels* k = reinterpret_cast<pg_kernels*>(0x1);
          pg_kernel_spec s = spec_of(geo, 4, kind, ja.data(), nullptr, 0.2, conv, storage);
          expect(pg_make_kernels(&s, nullptr, &k), PG_ENOMEM, "make_kernels full-pol");
          if (k) ++g_failures;
          s.jones_b = jb.data();
          expect(pg_make_kernels(&s, nullptr, &k), PG_ENOMEM, "make_kernels two antenna types");
          s.jones = nullptr;
          s.jones_b = nullptr;
          expect(pg_make_kernels(&s, nullptr, &k), PG_ENOMEM, "make_kernels no A-term");
          s.eps_null = 0.0;
          expect(pg_make_kernels(&s, nullptr, &k), PG_ENOMEM, "make_kernels eps 0");
          s = spec_of(geo, 1, kind, nullptr, nullptr, 0.2, conv, storage);
          expect(pg_make_kernels(&s, nullptr, &k), PG_ENOMEM, "make_kernels Stokes I");
          expect(pg_kernels_alloc(&s, nullptr, &k), PG_ENOMEM, "kernels_alloc");
        }
    // J = [[1, 0], [0, 0]] (only the X receptor): the Stokes Mueller matrix is rank one, and with
    // eps = 0 the Eq. 6 regularisation leaves it singular
    std::vector<double> xonly(ja.size(), 0.0);
    for (size_t px = 0; px < static_cast<size_t>(mk) * mk; ++px) xonly[2 * px] = 1.0;
    pg_kernels* k = nullptr;
    pg_kernel_spec s = spec_of(geo, 4, PG_KIND_GRID, xonly.data(), nullptr, 0.0, PG_STOKES_IAU, PG_STORE_F32);
    expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "make_kernels singular screens");
    s = spec_of(geo, 1, PG_KIND_GRID, ja.data(), nullptr, 0.2, PG_STOKES_IAU, PG_STORE_F32);
    expect(pg_make_kernels(&s, nullptr, &k), PG_EUNSUPPORTED, "make_kernels Stokes I with Jones");
  }
  // invalid specs
  Geometry geo(64, 4, 3, 7, 8, 16);
  pg_kernels* k = nullptr;
  pg_kernel_spec s = spec_of(geo, 4, PG_KIND_GRID, nullptr, nullptr, 0.2, PG_STOKES_IAU, PG_STORE_F32);
  expect(pg_make_kernels(nullptr, nullptr, &k), PG_EINVAL, "null spec");
  expect(pg_make_kernels(&s, nullptr, nullptr), PG_EINVAL, "null out");
  s.npol = 2;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "npol 2");
  s.npol = 4;
  s.kind = 7;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "bad kind");
  s.kind = PG_KIND_GRID;
  s.eps_null = std::nan("");
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "NaN eps");
  s.eps_null = -1.0;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "negative eps");
  s.eps_null = 0.2;
  s.storage = 5;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "bad storage");
  s.storage = PG_STORE_F32;
  s.stokes_convention = 9;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "bad convention");
  s.stokes_convention = PG_STOKES_IAU;
  const pg_geometry good = s.g;
  s.g.n = 63;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "odd n");
  s.g = good;
  s.g.os = 3;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "odd os");
  s.g = good;
  s.g.nplanes = 0;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "no planes");
  s.g = good;
  s.g.w_planes = nullptr;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "null w_planes");
  s.g = good;
  s.g.mk = 15;
  expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "odd mk");
  {
    Geometry bad(64, 4, 3, 7, 8, 16);
    bad.w = {10.0, 5.0, 20.0};
    bad.g.w_planes = bad.w.data();
    s.g = bad.g;
    expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "w not ascending");
    Geometry s0(64, 4, 3, 0, 8, 16);
    s.g = s0.g;
    expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "support 0");
    Geometry t0(64, 4, 3, 7, 0, 16);
    s.g = t0.g;
    expect(pg_make_kernels(&s, nullptr, &k), PG_EINVAL, "tile 0");
    Geometry wide(1024, 4, 2, 48, 200, 16);  // sub-grid beyond the LDS budget
    s.g = wide.g;
    expect(pg_make_kernels(&s, nullptr, &k), PG_EUNSUPPORTED, "tile too wide");
  }
}

void other_cases() {
  pg_plan* p = nullptr;
  expect(pg_plan_create(nullptr, nullptr, 0, 64, nullptr, &p, nullptr), PG_EINVAL, "plan without kernels");
  expect(pg_grid(nullptr, nullptr, nullptr, nullptr, 0, nullptr), PG_EINVAL, "grid nulls");
  expect(pg_degrid(nullptr, nullptr, nullptr, nullptr, 0, nullptr), PG_EINVAL, "degrid nulls");
  expect(pg_batch_create(nullptr, 0, nullptr, nullptr), PG_EINVAL, "batch nulls");
  pg_mlp* m = nullptr;
  expect(pg_mlp_create(8, 64, 2, 300, 256, 1, nullptr, &m), PG_ENOMEM, "mlp_create");
  expect(pg_mlp_create(0, 64, 2, 300, 256, 1, nullptr, &m), PG_EINVAL, "mlp_create n_in 0");
  expect(pg_mlp_create(8, 64, 2, 300, 0, 1, nullptr, &m), PG_EINVAL, "mlp_create batch 0");
  float* fake = reinterpret_cast<float*>(256);
  int32_t* ifake = reinterpret_cast<int32_t*>(256);
  expect(pg_hogbom(fake, fake, nullptr, 64, 1, 0.1f, 0.0f, 0, 10, ifake, fake, nullptr, ifake, nullptr), PG_ENOMEM,
         "hogbom");
  expect(pg_hogbom(fake, fake, nullptr, 63, 1, 0.1f, 0.0f, 0, 10, ifake, fake, nullptr, ifake, nullptr), PG_EINVAL,
         "hogbom odd n");
  expect(pg_hogbom(fake, fake, nullptr, 64, 1, 0.0f, 0.0f, 0, 10, ifake, fake, nullptr, ifake, nullptr), PG_EINVAL,
         "hogbom gain 0");
  expect(pg_hogbom_noalloc(fake, fake, nullptr, 64, 1, 0.1f, 0.0f, 0, PG_HOGBOM_STATIC_MAX_ITER + 1, ifake, fake,
                           nullptr, ifake, nullptr),
         PG_EINVAL, "hogbom_noalloc beyond its scratch");
  expect(pg_mosaic_gamma(fake, 2, 64, 1e-3, 0.5, fake, fake, 1, nullptr), PG_ENOMEM, "mosaic_gamma");
  expect(pg_mosaic_gamma(fake, 2, 64, 2.0, 0.5, fake, fake, 1, nullptr), PG_EINVAL, "mosaic_gamma floor");
  expect(pg_gemm_f32(0, 0, 4, 4, 4, 1.0f, nullptr, 4, fake, 4, 0.0f, fake, 4, nullptr), PG_EINVAL, "gemm null a");
  expect(pg_gemm_f32(0, 0, 4, 4, 4, 1.0f, fake, 2, fake, 4, 0.0f, fake, 4, nullptr), PG_EINVAL, "gemm lda");
  expect(pg_scale_rows(nullptr, 4, 4, fake, nullptr), PG_EINVAL, "scale_rows null");
  expect(pg_weight_normalise(fake, fake, 0, 1, 0.1f, nullptr), PG_EINVAL, "weight_normalise n 0");
  expect(pg_phase_rotate(nullptr, nullptr, 5, 4, 0.0, 0.0, 0.1, 0.1, nullptr, nullptr, nullptr), PG_EINVAL,
         "phase_rotate nulls");
}

}  // namespace

int main() {
  if (pg_version() <= 0) return 2;
  pg_set_allocator(fail_alloc, no_free, nullptr);
  kernels_cases();
  other_cases();
  pg_set_allocator(nullptr, nullptr, nullptr);
  std::printf("host sanitize driver: %d calls, %d failures\n", g_calls, g_failures);
  return g_failures == 0 ? 0 : 1;
}
