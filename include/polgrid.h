/*
 * polgrid: full-polarisation A x W-projection convolutional gridding and
 * degridding for AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2206.15117, "A GPU-based Imager with Polarised Primary-beam
 * Correction".  Visibilities are spread onto (or read back from) the uv grid
 * through oversampled kernels, each the Fourier transform of an anti-aliasing
 * function times a w-correction screen times one cell of a 4x4 Mueller matrix
 * (Sec. 3.2); gridding kernels come from the null-regularised inverse of the
 * Stokes Mueller matrix (Sec. 3.3, Eq. 6).
 *
 * Conventions used by every call
 *   - Grid side n (even).  Image pixel (i, j) is at l = (j - n/2) cell,
 *     m = (i - n/2) cell; visibility (u, v) sits at grid position
 *     x = u n cell + n/2, y = v n cell + n/2, snapped in float64 onto the
 *     1/os fine grid with round-half-up.
 *   - Kernel footprint: the S x S box of grid points starting at
 *     X0 = ceil((fine - S os/2 + 1) / os); visibilities whose box leaves
 *     [0, n) are dropped (not gridded; degridded to 0).
 *   - W-plane: nearest plane centre, ties to the lower plane.
 *   - npol = 1: Stokes I only (one correlation in, one grid out).
 *     npol = 4: correlations XX, XY, YX, YY in; Stokes I, Q, U, V grids out
 *     (Eq. 3, Eq. 4 with U = (XY + YX)/2).
 *   - Visibilities: complex64 [nvis][npol] (interleaved re, im), device memory.
 *   - Grids: complex64 planar [npol][n][n] (row = v, column = u), device memory.
 *   - Images: float32 [npol][n][n], device memory.
 *   - uvw: float64 [nvis][3] in wavelengths, device memory.
 *   - Weights are not part of the interface: callers pre-multiply visibilities,
 *     which keeps pg_grid and pg_degrid an exact adjoint pair.
 *
 * Ownership: the caller owns every buffer passed in; the library owns
 * pg_kernels and pg_plan objects, which are immutable after creation and may
 * be shared between streams and threads.  Their device memory comes from the
 * allocator registered with pg_set_allocator (hipMalloc/hipFree by default).
 *
 * Errors: every int-returning call returns PG_OK (0) or a negative PG_E* code;
 * arguments are validated on the host before anything is enqueued, and the
 * reason is available from pg_last_error().  No C++ exception crosses the ABI.
 *
 * Asynchrony: pg_grid, pg_degrid and pg_taper only enqueue work on `stream`
 * (a hipStream_t, NULL for the default stream).  pg_make_kernels and
 * pg_plan_create synchronise `stream` once before returning.
 */
#ifndef POLGRID_H
#define POLGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PG_OK 0
#define PG_EINVAL (-1)       /* bad argument; nothing was enqueued */
#define PG_ENOMEM (-2)       /* the allocator returned NULL */
#define PG_EHIP (-3)         /* a HIP runtime call failed */
#define PG_EUNSUPPORTED (-4) /* valid request this build does not handle */

#define PG_KIND_GRID 0   /* screens (M'^S)^-1 S: correlations -> Stokes (Sec. 3.2-3.3) */
#define PG_KIND_DEGRID 1 /* screens (S^-1 M^S)^H: conjugate maps Stokes sky -> correlations (Eq. 2) */

#define PG_STORE_F32 0 /* table entries complex64 */
#define PG_STORE_F16 1 /* table entries two float16 (re, im); arithmetic stays float32 */

#define PG_STOKES_IAU 0   /* U = (XY + YX)/2 */
#define PG_STOKES_PAPER 1 /* U = i (XY + YX)/2 as printed in Eq. 4 */

/* pg_grid / pg_degrid flags */
#define PG_ACCUMULATE 1 /* pg_grid: add onto the existing grid instead of overwriting it;
                           pg_degrid: add onto vis_out (dropped rows keep their values) */
#define PG_FFTSHIFT 2   /* the grid in memory is G(X,Y) (-1)^(X+Y): the centring modulation
                           the FFT needs is folded into the grid flush / degrid gather */
#define PG_VARIANT_ATOMIC 4 /* pg_grid: force the LDS-atomic accumulation kernel */
#define PG_VARIANT_BANDED 8 /* pg_grid: force the row-band ownership kernel (no LDS atomics);
                               without either flag the library picks by sub-grid width.
                               Both give the same result up to float32 summation order. */
#define PG_VARIANT_SHARED 32 /* pg_grid: force the shared-tap kernel: rows of one kernel phase share
                                each tap load, and the sub-grid is summed exactly in two-word fixed
                                point with LDS integer atomics (per item and plane, scaled from a
                                bound on its values); an item with a non-finite visibility turns
                                its grid points into NaN.  Needs twice one output plane's sub-grid
                                in LDS; where that does not fit the row-band kernel runs instead */
#define PG_DETERMINISTIC 16 /* pg_grid: bit-for-bit reproducible result.  Each work item's sub-grid
                               is summed exactly (the shared-tap kernel's fixed point, 8 waves and
                               one output plane per workgroup whatever the plan's launch settings;
                               where that does not fit the LDS, row bands in a fixed order), and
                               the sub-grids are added
                               into 64-bit fixed-point accumulators with integer atomics, which do
                               not depend on the order of the additions.  The fixed-point
                               scale is a power of two chosen per call from a bound on every grid
                               value (rows kept x largest row |vis|_1 x largest |re|+|im| of a
                               table entry), so that no sum can overflow; inputs must be finite.
                               Allocates npol * n * n * 16 bytes of device scratch per call
                               (through the registered allocator).  Not with PG_VARIANT_ATOMIC. */

/* pg_taper directions */
#define PG_TAPER_IMAGE 0   /* complex FFT output -> real image / (AA(l) AA(m)) / weight_sum */
#define PG_TAPER_PREDICT 1 /* real model image -> complex (model / (AA(l) AA(m))) for the inverse FFT */

typedef struct pg_geometry {
  int32_t n;               /* grid side, even, 8 .. 16384 */
  double cell;             /* image pixel size, radians */
  int32_t os;              /* oversampling factor, even, 2 .. 16 */
  int32_t nplanes;         /* number of w-planes, 1 .. 1024 */
  const double* w_planes;  /* host [nplanes], ascending, wavelengths */
  const int32_t* support;  /* host [nplanes], taps per axis, 1 .. 64 */
  const int32_t* tile;     /* host [nplanes], uv tile side used to bin visibilities, >= 1; the
                              sub-grid (tile + support - 1) rows x pitch x npol x 8 B must fit
                              162560 B of LDS, pitch = the width rounded up to == support mod 32 */
  int32_t aa_support;      /* support of the prolate spheroidal anti-aliasing function (7) */
  int32_t mk;              /* samples per side of the image lattice kernels are built on (even) */
} pg_geometry;

typedef struct pg_kernel_spec {
  pg_geometry g;
  int32_t npol;              /* 1 or 4 */
  int32_t kind;              /* PG_KIND_GRID or PG_KIND_DEGRID */
  const double* jones;       /* host complex128 [2][2][mk][mk] (row = m, column = l) on the lattice
                                l_a = (a - mk/2) n cell / mk; NULL = no A-term (identity) */
  double eps_null;           /* Eq. 6 mask fraction epsilon (0.2 typical); used by PG_KIND_GRID */
  int32_t stokes_convention; /* PG_STOKES_IAU or PG_STOKES_PAPER */
  int32_t storage;           /* PG_STORE_F32 or PG_STORE_F16 */
  const double* jones_b;     /* host complex128 [2][2][mk][mk] or NULL: the second antenna's Jones field
                                of a baseline between two antenna types; the Mueller matrix is then
                                J_a (x) conj(J_b) with J_a from `jones` (Sec. 3.2), so kernels are
                                unique to the baseline class.  NULL: identical antennas */
} pg_kernel_spec;

typedef struct pg_kernels pg_kernels;
typedef struct pg_plan pg_plan;

/* Read-only view of a kernel set, for inspection and tests. */
typedef struct pg_kernels_desc {
  int32_t npol, kind, storage, os, n, nplanes;
  const void* table;            /* device; per plane [os][os][npol^2/E][S][S][E] entries
                                   (phase_y, phase_x, chunk, tap_y, tap_x, e) with Mueller cell
                                   q * npol + c = chunk * E + e, E = min(npol^2, 2) for F32 and
                                   min(npol^2, 4) for F16 (one 16-byte chunk per tap); tap t of
                                   phase ph has fine-grid offset ph - S os/2 + 1 + t os */
  const int64_t* plane_offset;  /* host [nplanes + 1], offsets into table in entries */
  const double* aa_pixels;      /* host [n], anti-aliasing function at the image pixels */
} pg_kernels_desc;

/* Read-only view of a plan, for inspection and tests. */
typedef struct pg_plan_desc {
  int64_t nvis, n_kept, n_dropped, n_items;
  const int32_t* perm;   /* device [nvis]: visibility index in binned order, kept first */
  const int32_t* fine;   /* device [n_kept][2]: (fine_x, fine_y) in binned order */
  const int32_t* items;  /* device [n_items][8]: plane, origin_y, origin_x, start, end, 0, 0, 0 */
} pg_plan_desc;

/* Library version, (major << 16) | minor. */
int pg_version(void);

/* Message for the last failing call on this thread; valid until the next pg_* call. */
const char* pg_last_error(void);

/* Device memory hooks.  alloc(bytes, stream, ctx) returns device memory or NULL;
 * free(ptr, stream, ctx) releases it.  Passing NULL restores hipMalloc/hipFree.
 * Applies to objects created afterwards; every object frees through the hooks it was created
 * with, so the hook functions and ctx must stay valid until those objects are destroyed. */
void pg_set_allocator(void* (*alloc_fn)(size_t, void*, void*),
                      void (*free_fn)(void*, void*, void*), void* ctx);

/* Kernel generation (Sec. 3.2: image-domain anti-aliasing x w-correction x Mueller
 * cell, Fourier transformed into the uv domain; Sec. 3.3, Eq. 6 for gridding).
 * For plane p, output q and input c the table holds the zero-padded (x os)
 * inverse DFT of f = AA(l) AA(m) exp(-2 pi i w_p (n-1)) Phi_qc(l, m) sampled on
 * the mk x mk lattice, restricted to offsets |d| < S_p os / 2.  Host float64
 * Mueller algebra, device float64 transforms, stored in spec->storage.
 * Synchronises `stream`.  Errors: PG_EINVAL (bad spec), PG_EUNSUPPORTED (sub-grid
 * of some plane larger than the 162560-byte LDS budget), PG_ENOMEM, PG_EHIP. */
int pg_make_kernels(const pg_kernel_spec* spec, void* stream, pg_kernels** out);
int pg_kernels_info(const pg_kernels* k, pg_kernels_desc* out);
/* Copy the whole table (plane_offset[nplanes] entries of 8 bytes (F32) or 4 bytes (F16)) into
 * caller device memory `dst`; enqueue only. */
int pg_kernels_copy_table(const pg_kernels* k, void* dst, void* stream);
/* The inverse of pg_kernels_copy_table, for restoring a saved kernel set into one made by
 * pg_kernels_alloc with the same spec: overwrite the whole table from caller device memory `src`
 * (the same byte count and layout).  Call before the kernel set is shared.  Enqueue only.
 * Errors: PG_EINVAL. */
int pg_kernels_load_table(pg_kernels* k, const void* src, void* stream);
void pg_kernels_destroy(pg_kernels* k);

/* Visibility binning: float64 uvw -> fine positions, w-plane, anchor tile and
 * oversampling phase; stable sort by (plane, tile_y, tile_x, phase_y, phase_x);
 * work items are runs of one (plane, tile) cut into chunks of at most max_chunk, in [1, 2^30]
 * (the fixed-point bounds of the shared-tap gridder hold for items of up to 2^30 rows).
 * Synchronises `stream` (to size the outputs, and once more before returning, so the plan is
 * complete for any stream) and returns the drop count in *n_dropped (host, may be NULL).
 * nvis may be 0.  Errors: PG_EINVAL, PG_ENOMEM, PG_EHIP. */
int pg_plan_create(const pg_kernels* k, const double* uvw, int64_t nvis, int32_t max_chunk,
                   void* stream, pg_plan** out, int64_t* n_dropped);
int pg_plan_info(const pg_plan* p, pg_plan_desc* out);
/* Copy the plan's perm [nvis], fine [n_kept][2] and items [n_items][8] int32 arrays into caller
 * device memory (any destination may be NULL); enqueue only. */
int pg_plan_copy(const pg_plan* p, int32_t* perm, int32_t* fine, int32_t* items, void* stream);
void pg_plan_destroy(pg_plan* p);

/* Launch tuning of the kernels that run over this plan (results are unchanged up to float32
 * summation order): grid_variant 0 = choose by sub-grid width, 1 = LDS-atomic accumulation,
 * 2 = row-band ownership, 3 = shared taps with fixed-point LDS accumulation (PG_VARIANT_SHARED);
 * grid_waves and degrid_waves = waves per workgroup, 4, 6, 8 or 16;
 * xcd_group = how many consecutive work items (in plan order) run on one XCD, so that they share
 * its L2 (1 = plain order, up to 4096); grid_planes = output correlation planes per row-band
 * workgroup, 0 (all), 1, 2 or 4: with 1 or 2, npol / grid_planes workgroups share each work item,
 * each holding only its planes' sub-grid in LDS and reading only its rows of the 4x4 Mueller
 * kernels (ignored where it does not divide npol); degrid_corrs = output correlations per degrid
 * workgroup, 0 (all), 2 or 4: with 2 (float32 full-pol tables only, ignored otherwise) two
 * workgroups share each work item, each reading the half of the Mueller kernels its two
 * correlations need, placed on alternate XCDs (the XCD grouping is then not applied to the
 * degrid).  Set before the plan is shared between threads.  Errors: PG_EINVAL. */
int pg_plan_set_launch(pg_plan* p, int32_t grid_variant, int32_t grid_waves, int32_t degrid_waves,
                       int32_t xcd_group, int32_t grid_planes, int32_t degrid_corrs);

/* Gridding (Sec. 3.2, Sec. 4):
 *   G_q(X,Y) (+)= sum_k sum_c T_{p_k,q,c}(X os - fine_x,k, Y os - fine_y,k) V_{k,c}.
 * vis: complex64 [nvis][npol] (the plan's nvis); grid: complex64 [npol][n][n].
 * Without PG_ACCUMULATE the grid is overwritten.  Enqueue only, except with PG_DETERMINISTIC,
 * whose scratch is freed (stream-ordered through the registered allocator, else by hipFree, which
 * waits for the device) before the call returns.  Errors: PG_EINVAL, PG_ENOMEM (deterministic
 * scratch), PG_EHIP. */
int pg_grid(const pg_plan* p, const pg_kernels* k, const void* vis, void* grid, int32_t flags,
            void* stream);

/* Degridding, the exact adjoint of pg_grid (Sec. 3.2, degridding stage):
 *   V_{k,c} = sum_q sum_{X,Y} conj(T_{p_k,q,c}(...)) G_q(X, Y); dropped visibilities get 0
 *   (with PG_ACCUMULATE: V_{k,c} is added to vis_out and dropped rows are left alone).
 * grid: complex64 [npol][n][n]; vis_out: complex64 [nvis][npol].  Enqueue only. */
int pg_degrid(const pg_plan* p, const pg_kernels* k, const void* grid, void* vis_out, int32_t flags,
              void* stream);

/* Overwrite one Mueller cell (q, c) of one plane of a kernel set with caller data: src is device
 * float [os][os][S][S][2] (phase_y, phase_x, tap_y, tap_x, re/im), converted to the table's
 * storage.  Used to run the gridder on generated (e.g. learned) kernels; call before the kernel
 * set is shared.  Enqueue only.  Errors: PG_EINVAL. */
int pg_kernels_write_cell(pg_kernels* k, int32_t plane, int32_t q, int32_t c, const float* src, void* stream);

/* A kernel set with the geometry, storage, anti-aliasing taper and plane layout that
 * pg_make_kernels would give for `spec`, whose table is all zeros instead of generated (Jones
 * field, eps_null and stokes_convention are not used).  It is filled by pg_kernels_import, e.g.
 * with learned kernels, and then grids and degrids like any other kernel set.  Synchronises
 * `stream`.  Errors: as pg_make_kernels. */
int pg_kernels_alloc(const pg_kernel_spec* spec, void* stream, pg_kernels** out);

/* Every Mueller cell of planes plane0 .. plane0 + nplanes - 1 as plain float32 device data:
 * dst is [nplanes][npol (q)][npol (c)][os (phase_y)][os (phase_x)][S][S][re, im], the same
 * (phase, tap) convention as the table definition above (Sec. 3.2 kernels).  The planes must share
 * one support S.  Enqueue only.  Errors: PG_EINVAL (range, mixed supports, NULL). */
int pg_kernels_export(const pg_kernels* k, int32_t plane0, int32_t nplanes, float* dst, void* stream);

/* The inverse of pg_kernels_export: overwrite every cell of planes plane0 .. plane0 + nplanes - 1
 * with cell_scale[q npol + c] x src (src device float32, layout as above; cell_scale host,
 * npol^2 values, or NULL for 1), rounded to the table's storage.  Call before the kernel set is
 * shared.  Enqueue only.  Errors: PG_EINVAL. */
int pg_kernels_import(pg_kernels* k, int32_t plane0, int32_t nplanes, const float* src, const float* cell_scale,
                      void* stream);

/* ------------------------------------------------------------------ kernel surrogate network
 * A multilayer perceptron that emits one oversampled kernel cell from a feature vector: hidden
 * layers of `width` SiLU units, a linear output layer of n_out values.  Weights are float32
 * masters with bfloat16 copies; every product runs on the matrix cores with bfloat16 operands
 * and float32 accumulation; training minimises (1/B) sum_b |y_b - t_b|^2 / |t_b|^2 with Adam
 * (beta 0.9, 0.999, eps 1e-8).  Weights start U(-a, a), a = sqrt(6 / fan_in) (sqrt(3 / fan_in)
 * for the output layer), from a counter-based generator (splitmix64 of seed + index).
 * Not in the paper: a learned replacement for on-the-fly kernel generation. */
typedef struct pg_mlp pg_mlp;
#define PG_MLP_W 0      /* float [d_in][d_out] master weights of a layer */
#define PG_MLP_W_BF16 1 /* bfloat16 copy */
#define PG_MLP_B 2      /* float [d_out] bias */
#define PG_MLP_GW 3     /* float [d_in][d_out] weight gradient of the last train step */
#define PG_MLP_GB 4     /* float [d_out] bias gradient */
#define PG_MLP_ACT 5    /* bfloat16 [batch][d_in] input activation of the layer (layer 0: features) */
#define PG_MLP_PRE 6    /* float [batch][d_out] pre-activation (output layer: the network output) */
#define PG_MLP_GY 7     /* float [batch][n_out] loss gradient at the output (last train step) */
#define PG_MLP_GY_BF16 8 /* its bfloat16 copy, the operand of the output layer's gradient products */
#define PG_MLP_GZ 9     /* float [batch][d_1] gradient at the first layer's pre-activation */
#define PG_MLP_GZ_BF16 10 /* its bfloat16 copy */
#define PG_MLP_MW 11     /* float [d_in][d_out] Adam first moment of the layer's weights */
#define PG_MLP_VW 12     /* float [d_in][d_out] Adam second moment of the layer's weights */
#define PG_MLP_MB 13     /* float [d_out] Adam first moment of the layer's bias */
#define PG_MLP_VB 14     /* float [d_out] Adam second moment of the layer's bias */

int pg_mlp_create(int32_t n_in, int32_t width, int32_t hidden_layers, int64_t n_out, int32_t max_batch,
                  uint64_t seed, void* stream, pg_mlp** out);
/* x: device float [batch][n_in]; y: device float [batch][n_out], written directly by the output
 * layer's product, or NULL to leave the output in the network's own buffer (PG_MLP_PRE of the
 * output layer; with y given that buffer is not updated).  Enqueue only. */
int pg_mlp_forward(pg_mlp* m, const float* x, int32_t batch, float* y, void* stream);
/* Forward, loss, backward and (if update) one Adam step; loss_out: device float or NULL. */
int pg_mlp_train_step(pg_mlp* m, const float* x, const float* target, int32_t batch, float lr, int32_t update,
                      float* loss_out, void* stream);
/* Copy a parameter, gradient or activation of `layer` (0 = first) into device memory. */
int pg_mlp_copy(const pg_mlp* m, int32_t what, int32_t layer, void* dst, void* stream);
/* Set a layer's float weights [d_in][d_out] and bias [d_out] from device memory. */
int pg_mlp_load(pg_mlp* m, int32_t layer, const float* w, const float* b, void* stream);
/* Restore one piece of a layer's training state from device memory, for resuming from a saved
 * checkpoint: what = PG_MLP_W (the bfloat16 copies are refreshed), PG_MLP_B, PG_MLP_MW, PG_MLP_VW,
 * PG_MLP_MB or PG_MLP_VB, sizes as listed above.  Enqueue only.  Errors: PG_EINVAL. */
int pg_mlp_set(pg_mlp* m, int32_t what, int32_t layer, const void* src, void* stream);
/* Adam's step counter (the number of updates taken; bias corrections use it): read, or set when
 * resuming (step >= 0).  Host calls.  Errors: PG_EINVAL. */
int pg_mlp_get_step(const pg_mlp* m, int64_t* step);
int pg_mlp_set_step(pg_mlp* m, int64_t step);
void pg_mlp_destroy(pg_mlp* m);

/* Float32 matrix product for the surrogate's training (its kernel basis, the projections of teacher
 * kernels onto it and the fold of the output layer with it): C = alpha op(A) op(B) + beta C with
 * row-major storage, op(X) = X (transX = 0) or X^T (transX != 0); op(A) is m x k, op(B) k x n, C
 * m x n, leading dimensions lda, ldb, ldc (elements).  Float32 accumulation; deep contractions are
 * split across workgroups and summed with float atomics (order of the partial sums varies).  All
 * pointers device memory; enqueue only.  Errors: PG_EINVAL (sizes, leading dimensions, NULLs). */
int pg_gemm_f32(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, float alpha, const float* a,
                int64_t lda, const float* b, int64_t ldb, float beta, float* c, int64_t ldc, void* stream);
/* x[r][c] *= scale[r] for a device float32 [rows][cols] matrix and device scale [rows]; enqueue only. */
int pg_scale_rows(float* x, int64_t rows, int64_t cols, const float* scale, void* stream);

/* ------------------------------------------------------------------ Hogbom minor cycle
 * The minor cycle of Cotton-Schwab clean (Sec. 2.1; Hogbom's algorithm), run on the device with no
 * host round trip.  Each iteration takes the masked pixel of largest |I| (plane 0 of residual;
 * ties go to the lowest pixel index); if that value is below `threshold` (or no pixel is masked
 * in) the cycle stops; otherwise it records the component v_q = gain x residual[q][peak] for
 * every plane q, adds it to model[q][peak] (model may be NULL), and subtracts
 * v_q x psf[y - py + n/2][x - px + n/2] from residual[q] wherever the shifted point-spread function
 * overlaps the image within `psf_patch` pixels of the peak (psf_patch <= 0: no limit).  Products
 * and differences are each rounded to float32 (no fused multiply-add), so a float32 reference
 * reproduces the cycle exactly.
 *   residual  float32 [npol][n][n], in/out;  psf float32 [n][n], peak at (n/2, n/2);
 *   mask      uint8 [n][n] (non-zero = cleanable; the paper masks where the beam is below a
 *             fraction eps of its peak, Sec. 3.3) or NULL for every pixel;
 *   comp_pos  int32 [max_iter] flat pixel indices, comp_val float32 [max_iter][npol];
 *   n_comp    int32 [1] (device): the number of components found.
 * All pointers are device memory.  Enqueue only (3 launches per iteration of the budget; the
 * launches after the stop return at once).  Errors: PG_EINVAL, PG_ENOMEM, PG_EHIP. */
int pg_hogbom(float* residual, const float* psf, const uint8_t* mask, int32_t n, int32_t npol, float gain,
              float threshold, int32_t psf_patch, int32_t max_iter, int32_t* comp_pos, float* comp_val, float* model,
              int32_t* n_comp, void* stream);

/* Peak search of a major cycle (Sec. 2.1): the largest |img[i]| over the pixels i < npix with
 * mask[i] != 0 (mask NULL: all), and its index (the lowest on ties).  img float32 and mask uint8,
 * device memory; peak and index host pointers, written before return (peak 0 and index -1 when no
 * pixel is masked in).  Allocates 264 bytes of scratch per call; synchronises `stream`.
 * Errors: PG_EINVAL, PG_ENOMEM, PG_EHIP. */
int pg_masked_peak(const float* img, const uint8_t* mask, int64_t npix, float* peak, int64_t* index, void* stream);
/* img[i] = img[i] / img[ref_index] for i < count, in place (e.g. a point-spread function scaled to
 * one at the phase centre); the reference value is read before any pixel is divided.  Device
 * memory; allocates 4 bytes of scratch per call; enqueue only.  Errors: PG_EINVAL, PG_ENOMEM. */
int pg_normalise_at(float* img, int64_t count, int64_t ref_index, void* stream);

/* pg_hogbom without any device allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * kernels as pg_hogbom; the scratch pg_hogbom allocates per call (iteration state and one 64-bit
 * peak slot per iteration) is instead a fixed device array of the library, 256 + 8 x
 * PG_HOGBOM_STATIC_MAX_ITER bytes (about 512 KiB) on each GPU it runs on, held until the process
 * ends.  Every call on one GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams or threads) race; each call clears the part it uses before its first iteration.  Only
 * kernel launches are enqueued (no hipMalloc, hipFree, memset or copy).  Errors: as pg_hogbom, and
 * PG_EINVAL when max_iter exceeds PG_HOGBOM_STATIC_MAX_ITER. */
#define PG_HOGBOM_STATIC_MAX_ITER 65536
int pg_hogbom_noalloc(float* residual, const float* psf, const uint8_t* mask, int32_t n, int32_t npol, float gain,
                      float threshold, int32_t psf_patch, int32_t max_iter, int32_t* comp_pos, float* comp_val,
                      float* model, int32_t* n_comp, void* stream);

/* ------------------------------------------------------------------ batched launch
 * Many fields (channels or mosaic pointings, each with its own plan, kernels, visibilities and
 * grid; uneven visibility counts) gridded or degridded by ONE launch over every (field, work
 * item) pair: fields largest first, each in plan order, in groups of consecutive items (the first
 * plan's XCD grouping) that each run on one XCD, so uneven fields balance across the GPU with
 * one or two fields' tables in the caches at a time (multi-field mosaics and channel-dependent
 * beams, Sec. 2.2, Sec. 3.2).
 * All fields share npol and table storage; geometries may differ.  The launch shape (waves per
 * workgroup, XCD grouping) is taken from the first field's plan (pg_plan_set_launch). */
typedef struct pg_field {
  const pg_plan* plan;
  const pg_kernels* kernels;
  void* vis;   /* complex64 [nvis][npol] device: input of pg_batch_grid, output of pg_batch_degrid */
  void* grid;  /* complex64 [npol][n][n] device: output of pg_batch_grid, input of pg_batch_degrid */
} pg_field;
typedef struct pg_batch pg_batch;

/* Builds the device field table and the ordered work list; the plans, kernels and buffers must
 * outlive the batch.  Synchronises `stream`.  Errors: PG_EINVAL (NULLs, npol or storage mismatch,
 * plan/kernel geometry mismatch), PG_ENOMEM, PG_EHIP. */
int pg_batch_create(const pg_field* fields, int32_t nfields, void* stream, pg_batch** out);
/* Enqueue: zero every grid (unless PG_ACCUMULATE), one grid launch over all work items.
 * Allocates nothing and calls only kernel launches, so it may be captured in a HIP graph. */
int pg_batch_grid(const pg_batch* b, int32_t flags, void* stream);
/* Enqueue: zero dropped visibilities, one degrid launch over all work items.  Capturable. */
int pg_batch_degrid(const pg_batch* b, int32_t flags, void* stream);
/* Number of (field, work item) pairs in the batch; -1 for NULL. */
int64_t pg_batch_work_items(const pg_batch* b);
void pg_batch_destroy(pg_batch* b);

/* Image-domain taper correction around the FFT (Sec. 2.2, Sec. 3.2).
 * PG_TAPER_IMAGE:   in complex64 [npol][n][n] = FFT of a PG_FFTSHIFT grid;
 *                   out float32 [npol][n][n] = Re((-1)^(i+j) in) / (AA(l_j) AA(m_i)) / weight_sum.
 * PG_TAPER_PREDICT: in float32 [npol][n][n] model; out complex64 [npol][n][n] =
 *                   weight_sum x (-1)^(i+j) model / (AA AA), ready for an unnormalised inverse
 *                   FFT whose result is a PG_FFTSHIFT grid (weight_sum is a scale here: 1 for a
 *                   plain prediction, -1 to subtract the model with PG_ACCUMULATE degridding).
 * Enqueue only.  Errors: PG_EINVAL. */
int pg_taper(const pg_kernels* k, const void* in, void* out, int32_t direction, double weight_sum,
             void* stream);

/* ------------------------------------------------------------------ image-domain mosaics
 * Sec. 2.2: each mosaic field is imaged at its own phase centre and image-plane reprojection
 * builds the mosaic at a common phase centre; before degridding, the model is reprojected back
 * to each field's phase centre.  A sky frame is an n x n orthographic (SIN) projection about
 * (ra, dec) (radians) with pixel (row i, column j) at direction cosines l = (j - n/2) cell,
 * m = (i - n/2) cell, where l = cos d sin(a - ra), m = sin d cos(dec) - cos d sin(dec) cos(a - ra). */
typedef struct pg_sky_frame {
  int32_t n;   /* pixels per side, 2 .. 65536 */
  double cell; /* radians per pixel, > 0 */
  double ra;   /* phase centre, radians (finite) */
  double dec;  /* phase centre, radians, |dec| <= pi/2 */
} pg_sky_frame;

/* Reprojection: for every destination pixel, its direction is mapped into the source frame at
 * pixel position (x, y) (x = column), computed in float64.  The pixel is covered when the
 * direction is in front of both phase centres and -1e-6 <= x, y <= n_src - 1 + 1e-6 (positions
 * then clamped to [0, n_src - 1]); s_q = bilinear sample of src plane q at (x, y) and
 * w = bilinear sample of src_weight (1 if src_weight is NULL); uncovered: s_q = 0, w = 0.
 *   flags 0:             dst[q] = s_q,        dst_weight = w   (if dst_weight is non-NULL)
 *   flags PG_ACCUMULATE: dst[q] += w s_q,     dst_weight += w
 * src float32 [npol][n_src][n_src], src_weight float32 [n_src][n_src] or NULL, dst float32
 * [npol][n_dst][n_dst], dst_weight float32 [n_dst][n_dst] or NULL; all device memory, the
 * caller's; src and dst must not overlap.  npol 1..4.  Enqueue only.  Errors: PG_EINVAL. */
int pg_reproject(const float* src, const float* src_weight, const pg_sky_frame* src_frame, float* dst,
                 float* dst_weight, const pg_sky_frame* dst_frame, int32_t npol, int32_t flags, void* stream);

/* Phase rotation (Sec. 4 lists it with reprojection among the GPU-suited steps): visibilities
 * stored about phase centre (ra_from, dec_from) are moved to (ra_to, dec_to) (radians), so that a
 * field can be imaged about its own pointing centre (Sec. 2.2).  Per row, with b = u e + v n + w c
 * on the old centre's east/north/centre axes: uvw_out = (b.e', b.n', b.c') on the new centre's
 * axes (float64), and every correlation is multiplied by exp(2 pi i (w - w')) (float64 phase,
 * float32 complex product; the predict convention V = sum I exp(+2 pi i (u l + v m + w (n-1)))).
 * uvw_in float64 [nvis][3], vis_in complex64 [nvis][npol], device memory; uvw_out (may be NULL)
 * and vis_out likewise, the caller's; in place (out == in) is allowed.  npol 1..4.  Enqueue only.
 * Errors: PG_EINVAL. */
int pg_phase_rotate(const double* uvw_in, const void* vis_in, int64_t nvis, int32_t npol, double ra_from,
                    double dec_from, double ra_to, double dec_to, double* uvw_out, void* vis_out, void* stream);

/* Mosaic normalisation: img[q][p] = img[q][p] / weight[p] where weight[p] >= min_weight, else 0
 * (the weighted mean of the fields accumulated by pg_reproject).  img float32 [npol][n][n],
 * weight float32 [n][n], device memory.  min_weight > 0.  Enqueue only.  Errors: PG_EINVAL. */
int pg_weight_normalise(float* img, const float* weight, int32_t n, int32_t npol, float min_weight, void* stream);

/* ------------------------------------------------------------------ UV-domain mosaics
 * Sec. 2.2, Eq. 1: every mosaic field is gridded onto one common grid about the mosaic phase
 * centre through its own primary beam (pg_grid with the field's PG_KIND_DEGRID kernels, whose Jones
 * field is the beam centred on the field's pointing, and PG_ACCUMULATE), and after the FFT and the
 * taper the image is multiplied by
 *   gamma(l, m) = [sqrt(S) / max sqrt(S)] [1 / S],  S(l, m) = sum_i B_i(l, m)^2,
 * the primary-beam pattern normalised to 1 over the image times the weighting correction.
 * beams: float32 [nfields][n][n] device, B_i (power beam) at the image pixels; weight_sum: float32
 * [n][n] device, receives S; img: float32 [npol][n][n] device, multiplied in place by
 * scale x gamma where S >= floor_frac x max S and set to 0 elsewhere (no data there; Eq. 1 would
 * divide by a vanishing S).  scale folds in the caller's normalisation: 1/2 for the Stokes
 * convention of this library, whose (S^-1)^H S^-1 = 2 I makes an unpolarised sky enter the common
 * image as 2 S I.  Allocates 256 bytes of scratch per call; enqueue only.  Errors: PG_EINVAL,
 * PG_ENOMEM, PG_EHIP. */
int pg_mosaic_gamma(const float* beams, int32_t nfields, int32_t n, double floor_frac, double scale, float* weight_sum,
                    float* img, int32_t npol, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* POLGRID_H */
