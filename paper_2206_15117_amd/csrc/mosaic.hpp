// Launchers of the image-domain mosaic and phase-rotation kernels (mosaic.hip).
#pragma once
#include "common.hpp"

namespace pg {
hipError_t launch_reproject(const float* src, const float* src_w, const pg_sky_frame& sf, float* dst, float* dst_w,
                            const pg_sky_frame& df, int npol, int accumulate, hipStream_t s);
hipError_t launch_weight_normalise(float* img, const float* weight, int n, int npol, float min_weight, hipStream_t s);
hipError_t launch_phase_rotate(const double* uvw_in, const void* vis_in, int64_t nvis, int npol, double ra_from,
                               double dec_from, double ra_to, double dec_to, double* uvw_out, void* vis_out,
                               hipStream_t s);
hipError_t launch_mosaic_gamma(const float* beams, int nfields, int n, double floor_frac, double scale,
                               float* weight_sum, float* img, int npol, unsigned* max_bits, hipStream_t s);
}  // namespace pg
