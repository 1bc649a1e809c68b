// Image-plane reprojection for image-domain mosaics (Sec. 2.2): field images made at their own
// phase centres are resampled onto a common mosaic frame, and the model image is resampled back
// onto each field before its FFT and degridding.
//
// A frame is an n x n orthographic (SIN) projection about (ra0, dec0) with pixel (row i, column j)
// at direction cosines l = (j - n/2) cell, m = (i - n/2) cell: the components of the unit
// direction vector along the frame's east, north and centre axes.  Going from one frame to the
// other is therefore a fixed rotation of (l, m, n): R[a][b] = (axis a of the source frame) .
// (axis b of the destination frame), computed once on the host in float64.  One thread per
// destination pixel: (l0, m0, sqrt(1 - l0^2 - m0^2)) -> R -> source (l, m, n) -> source pixel
// (x, y) -> bilinear sample of every Stokes plane and of the optional weight image.  Coordinates
// and bilinear weights are float64 (at 8192^2 the offsets need more than float32's 24 bits); the
// output is float32.  HBM-bound: npol x (4 B read + 4 or 8 B written or read-modify-written) per
// destination pixel, plus the weight image.
#include <algorithm>
#include <cmath>

#include "mosaic.hpp"

namespace pg {
namespace {

constexpr double kEdge = 1e-6;  // pixels: border tolerance of the covered test

struct Axes {
  double e[3], nth[3], c[3];  // east, north, centre unit vectors of a frame
};

Axes axes_of(const pg_sky_frame& f) {
  const double sa = std::sin(f.ra), ca = std::cos(f.ra), sd = std::sin(f.dec), cd = std::cos(f.dec);
  return Axes{{-sa, ca, 0.0}, {-sd * ca, -sd * sa, cd}, {cd * ca, cd * sa, sd}};
}

struct Rotation {
  double r[3][3];  // source (l, m, n) = r . destination (l, m, n)
};

Rotation rotation(const pg_sky_frame& src, const pg_sky_frame& dst) {
  const Axes s = axes_of(src), d = axes_of(dst);
  const double* sa[3] = {s.e, s.nth, s.c};
  const double* da[3] = {d.e, d.nth, d.c};
  Rotation r;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) r.r[a][b] = sa[a][0] * da[b][0] + sa[a][1] * da[b][1] + sa[a][2] * da[b][2];
  return r;
}

struct FrameD {
  int n;
  double cell;
};

__global__ __launch_bounds__(256) void reproject_kernel(const float* __restrict__ src,
                                                        const float* __restrict__ src_w, FrameD sf,
                                                        float* __restrict__ dst, float* __restrict__ dst_w,
                                                        FrameD df, Rotation rot, int npol, int accumulate) {
  const int64_t npix_d = static_cast<int64_t>(df.n) * df.n;
  const int64_t npix_s = static_cast<int64_t>(sf.n) * sf.n;
  for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < npix_d;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(p / df.n), j = static_cast<int>(p - static_cast<int64_t>(i) * df.n);
    const double l0 = (j - df.n / 2) * df.cell, m0 = (i - df.n / 2) * df.cell;
    const double r2 = l0 * l0 + m0 * m0;
    double val[4] = {0.0, 0.0, 0.0, 0.0};
    double w = 0.0;
    if (r2 < 1.0) {
      const double n0 = sqrt(1.0 - r2);
      const double l = rot.r[0][0] * l0 + rot.r[0][1] * m0 + rot.r[0][2] * n0;
      const double m = rot.r[1][0] * l0 + rot.r[1][1] * m0 + rot.r[1][2] * n0;
      const double nn = rot.r[2][0] * l0 + rot.r[2][1] * m0 + rot.r[2][2] * n0;
      const double x = l / sf.cell + sf.n / 2, y = m / sf.cell + sf.n / 2;
      const double hi = sf.n - 1;
      if (nn > 0.0 && x >= -kEdge && y >= -kEdge && x <= hi + kEdge && y <= hi + kEdge) {
        const double xc = fmin(fmax(x, 0.0), hi), yc = fmin(fmax(y, 0.0), hi);
        const int x0 = min(static_cast<int>(floor(xc)), sf.n - 2), y0 = min(static_cast<int>(floor(yc)), sf.n - 2);
        const double fx = xc - x0, fy = yc - y0;
        const double w00 = (1.0 - fy) * (1.0 - fx), w01 = (1.0 - fy) * fx, w10 = fy * (1.0 - fx), w11 = fy * fx;
        const int64_t b = static_cast<int64_t>(y0) * sf.n + x0;
        for (int q = 0; q < npol; ++q) {
          const float* s = src + q * npix_s + b;
          val[q] = w00 * s[0] + w01 * s[1] + w10 * s[sf.n] + w11 * s[sf.n + 1];
        }
        w = src_w ? w00 * src_w[b] + w01 * src_w[b + 1] + w10 * src_w[b + sf.n] + w11 * src_w[b + sf.n + 1] : 1.0;
      }
    }
    if (accumulate) {
      for (int q = 0; q < npol; ++q) dst[q * npix_d + p] += static_cast<float>(w * val[q]);
      if (dst_w) dst_w[p] += static_cast<float>(w);
    } else {
      for (int q = 0; q < npol; ++q) dst[q * npix_d + p] = static_cast<float>(val[q]);
      if (dst_w) dst_w[p] = static_cast<float>(w);
    }
  }
}

__global__ __launch_bounds__(256) void weight_normalise_kernel(float* __restrict__ img,
                                                               const float* __restrict__ weight, int64_t npix,
                                                               int npol, float min_weight) {
  for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float w = weight[p];
    for (int q = 0; q < npol; ++q) {
      float* v = img + q * npix + p;
      *v = w >= min_weight ? *v / w : 0.0f;
    }
  }
}

// Phase rotation: one thread per visibility row.  uvw about the new centre = q . uvw (q[a][b] =
// axis a of the new frame . axis b of the old), and every correlation is multiplied by
// exp(2 pi i (w_old - w_new)); float64 phase, float32 products.  In place is allowed (each
// thread reads its row before writing it).  HBM-bound: 24 + 8 npol bytes in and out per row.
__global__ __launch_bounds__(256) void phase_rotate_kernel(const double* uvw_in, const float2* vis_in, int64_t nvis,
                                                           int npol, Rotation q, double* uvw_out, float2* vis_out) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < nvis;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double u = uvw_in[3 * k], v = uvw_in[3 * k + 1], w = uvw_in[3 * k + 2];
    const double u2 = q.r[0][0] * u + q.r[0][1] * v + q.r[0][2] * w;
    const double v2 = q.r[1][0] * u + q.r[1][1] * v + q.r[1][2] * w;
    const double w2 = q.r[2][0] * u + q.r[2][1] * v + q.r[2][2] * w;
    double s, c;
    sincospi(2.0 * (w - w2), &s, &c);
    const float cs = static_cast<float>(c), sn = static_cast<float>(s);
    for (int p = 0; p < npol; ++p) {
      const float2 a = vis_in[k * npol + p];
      vis_out[k * npol + p] = make_float2(a.x * cs - a.y * sn, a.x * sn + a.y * cs);
    }
    if (uvw_out) {
      uvw_out[3 * k] = u2;
      uvw_out[3 * k + 1] = v2;
      uvw_out[3 * k + 2] = w2;
    }
  }
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536)); }

// UV-domain mosaic correction (Sec. 2.2, Eq. 1).  Pass 1: S = sum_i B_i^2 per pixel (written out as
// the mosaic weight map) and its maximum (float bits of a non-negative value order like unsigned
// integers, so one atomicMax per workgroup).  Pass 2: img *= scale sqrt(S / S_max) / S where S
// clears floor * S_max, else 0.  HBM-bound: (nfields + 1) x 4 B, then (npol x 8 + 4) B per pixel.
__global__ __launch_bounds__(256) void beam_sumsq_kernel(const float* __restrict__ beams, int nfields, int64_t npix,
                                                         float* __restrict__ sumsq, unsigned* __restrict__ max_bits) {
  float best = 0.0f;
  for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float s = 0.0f;
    for (int f = 0; f < nfields; ++f) {
      const float b = beams[f * npix + p];
      s = fmaf(b, b, s);
    }
    sumsq[p] = s;
    best = fmaxf(best, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = fmaxf(best, __shfl_xor(best, o, 64));
  __shared__ float wb[4];
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float b = fmaxf(fmaxf(wb[0], wb[1]), fmaxf(wb[2], wb[3]));
    atomicMax(max_bits, __float_as_uint(b));
  }
}

__global__ __launch_bounds__(256) void mosaic_gamma_kernel(const float* __restrict__ sumsq,
                                                           const unsigned* __restrict__ max_bits, float floor_frac,
                                                           float scale, int npol, int64_t npix, float* __restrict__ img) {
  const float smax = __uint_as_float(*max_bits);
  const float inv_root_max = smax > 0.0f ? 1.0f / sqrtf(smax) : 0.0f;
  for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float s = sumsq[p];
    const float g = (s > 0.0f && s >= floor_frac * smax) ? scale * (sqrtf(s) * inv_root_max) / s : 0.0f;
    for (int q = 0; q < npol; ++q) img[q * npix + p] *= g;
  }
}

__global__ void zero_u32_kernel(unsigned* p) { *p = 0u; }

}  // namespace

hipError_t launch_reproject(const float* src, const float* src_w, const pg_sky_frame& sf, float* dst, float* dst_w,
                            const pg_sky_frame& df, int npol, int accumulate, hipStream_t s) {
  const int64_t npix = static_cast<int64_t>(df.n) * df.n;
  hipLaunchKernelGGL(reproject_kernel, dim3(blocks_for(npix)), dim3(256), 0, s, src, src_w, FrameD{sf.n, sf.cell}, dst,
                     dst_w, FrameD{df.n, df.cell}, rotation(sf, df), npol, accumulate);
  return hipGetLastError();
}

hipError_t launch_weight_normalise(float* img, const float* weight, int n, int npol, float min_weight, hipStream_t s) {
  const int64_t npix = static_cast<int64_t>(n) * n;
  hipLaunchKernelGGL(weight_normalise_kernel, dim3(blocks_for(npix)), dim3(256), 0, s, img, weight, npix, npol,
                     min_weight);
  return hipGetLastError();
}

hipError_t launch_phase_rotate(const double* uvw_in, const void* vis_in, int64_t nvis, int npol, double ra_from,
                               double dec_from, double ra_to, double dec_to, double* uvw_out, void* vis_out,
                               hipStream_t s) {
  const pg_sky_frame from{2, 1.0, ra_from, dec_from}, to{2, 1.0, ra_to, dec_to};
  hipLaunchKernelGGL(phase_rotate_kernel, dim3(blocks_for(nvis)), dim3(256), 0, s, uvw_in,
                     static_cast<const float2*>(vis_in), nvis, npol, rotation(to, from), uvw_out,
                     static_cast<float2*>(vis_out));
  return hipGetLastError();
}

hipError_t launch_mosaic_gamma(const float* beams, int nfields, int n, double floor_frac, double scale,
                               float* weight_sum, float* img, int npol, unsigned* max_bits, hipStream_t s) {
  const int64_t npix = static_cast<int64_t>(n) * n;
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((npix + 255) / 256, 8192));
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, max_bits);
  hipLaunchKernelGGL(beam_sumsq_kernel, dim3(blocks), dim3(256), 0, s, beams, nfields, npix, weight_sum, max_bits);
  hipLaunchKernelGGL(mosaic_gamma_kernel, dim3(blocks), dim3(256), 0, s, weight_sum, max_bits,
                     static_cast<float>(floor_frac), static_cast<float>(scale), npol, npix, img);
  return hipGetLastError();
}

}  // namespace pg
