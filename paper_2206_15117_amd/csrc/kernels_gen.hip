// Device side of kernel generation (Sec. 3.2): image-domain screens
// AA(l) AA(m) exp(-2 pi i w (n-1)) Phi_qc(l, m), their separable zero-padded DFT
// into the oversampled uv domain (two complex float64 matrix products per
// Mueller cell), and packing into the [phase_y][phase_x][tap_y][tap_x][q][c]
// table the gridder reads.
#include "common.hpp"
#include "mlp.hpp"

namespace pg {
namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void screen_kernel(const double2* __restrict__ phi, const double* __restrict__ aa, double w,
                              double fov, int mk, int nqc, double2* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= mk) return;
  const double step = fov / mk;
  const double l = (a - mk / 2) * step, m = (b - mk / 2) * step;
  const double r2 = l * l + m * m;
  const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
  double s, c;
  sincospi(2.0 * w * nm1, &s, &c);
  const double g = aa[a] * aa[b];
  const double2 scr = make_double2(g * c, -g * s);  // AA AA exp(-2 pi i w (n-1))
  const size_t px = static_cast<size_t>(b) * mk + a;
  const size_t npix = static_cast<size_t>(mk) * mk;
  for (int qc = 0; qc < nqc; ++qc) out[qc * npix + px] = cmul(scr, phi[qc * npix + px]);
}

// e[di][a] = exp(+2 pi i d (a - mk/2) / (os mk)) / mk with d = di - (S os/2 - 1); the last row
// (d = S os / 2, outside the open footprint) is zero.
__global__ void twiddle_kernel(int support, int os, int mk, double2* __restrict__ e) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int di = blockIdx.y;
  if (a >= mk) return;
  const int len = support * os;
  double2 v = make_double2(0.0, 0.0);
  if (di < len - 1) {
    const long long d = di - (len / 2 - 1);
    const long long period = 2LL * os * mk;  // exp(i pi x) has period 2 in x = num / (os mk)
    long long num = (2LL * d * (a - mk / 2)) % period;
    if (num < 0) num += period;
    double s, c;
    sincospi(static_cast<double>(num) / (static_cast<double>(os) * mk), &s, &c);
    v = make_double2(c / mk, s / mk);
  }
  e[static_cast<size_t>(di) * mk + a] = v;
}

// Batched complex float64 GEMM, C[m][n] = A[m][k] op(B); op(B) = B[k][n] (NN) or B[n][k]^T (NT).
constexpr int BM = 32, BN = 32, BK = 16;

template <bool BT>
__global__ __launch_bounds__(256) void zgemm_kernel(int m, int n, int k, const double2* __restrict__ A,
                                                    int64_t sa, const double2* __restrict__ B, int64_t sb,
                                                    double2* __restrict__ C, int64_t sc) {
  __shared__ double2 as[BK][BM + 1];
  __shared__ double2 bs[BK][BN + 1];
  const int z = blockIdx.z;
  A += z * sa;
  B += z * sb;
  C += z * sc;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  double2 acc[2][2] = {};
  for (int k0 = 0; k0 < k; k0 += BK) {
    for (int idx = threadIdx.x; idx < BM * BK; idx += 256) {
      int mm = idx / BK, kk = idx % BK;
      int gm = m0 + mm, gk = k0 + kk;
      as[kk][mm] = (gm < m && gk < k) ? A[static_cast<size_t>(gm) * k + gk] : make_double2(0.0, 0.0);
    }
    for (int idx = threadIdx.x; idx < BN * BK; idx += 256) {
      int nn, kk;
      if (BT) {
        nn = idx / BK;
        kk = idx % BK;
      } else {
        kk = idx / BN;
        nn = idx % BN;
      }
      int gn = n0 + nn, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gn < n && gk < k) v = BT ? B[static_cast<size_t>(gn) * k + gk] : B[static_cast<size_t>(gk) * n + gn];
      bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      double2 a0 = as[kk][ty], a1 = as[kk][ty + 16];
      double2 b0 = bs[kk][tx], b1 = bs[kk][tx + 16];
      double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j].x = fma(av[i].x, bv[j].x, fma(-av[i].y, bv[j].y, acc[i][j].x));
          acc[i][j].y = fma(av[i].x, bv[j].y, fma(av[i].y, bv[j].x, acc[i][j].y));
        }
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < m && gn < n) C[static_cast<size_t>(gm) * n + gn] = acc[i][j];
    }
}

// Table layout per plane: [phase_y][phase_x][chunk][tap_y][tap_x][e], entry (q, c) = chunk * E + e,
// so that one 16-byte chunk of 64 consecutive taps is 1 KiB of contiguous memory.
//   table entry = T[qc][ph_y + t_y os][ph_x + t_x os]
__global__ void pack_kernel(const double2* __restrict__ t, int support, int os, int nqc, int storage, int ce,
                            void* __restrict__ table) {
  const size_t len = static_cast<size_t>(support) * os;
  const size_t ss = static_cast<size_t>(support) * support;
  const size_t nch = nqc / ce;
  const size_t total = ss * os * os * nqc;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t e = i % ce;
    size_t r = i / ce;
    const size_t tap = r % ss;
    r /= ss;
    const size_t ch = r % nch;
    const size_t phase = r / nch;
    const size_t qc = ch * ce + e;
    const size_t ty = tap / support, tx = tap % support;
    const size_t py = phase / os, px = phase % os;
    const double2 v = t[(qc * len + py + ty * os) * len + px + tx * os];
    if (storage == PG_STORE_F16) {
      // direct float64 -> float16 rounding (no intermediate float32 rounding)
      const _Float16 re = static_cast<_Float16>(v.x), im = static_cast<_Float16>(v.y);
      __half hr, hi;
      __builtin_memcpy(&hr, &re, 2);
      __builtin_memcpy(&hi, &im, 2);
      static_cast<__half2*>(table)[i] = __halves2half2(hr, hi);
    } else {
      static_cast<float2*>(table)[i] = make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
    }
  }
}

// One Mueller cell of one plane from a dense [phase_y][phase_x][tap_y][tap_x][re, im] float array
// into the chunk-major table.
// Moves Mueller cells between a chunk-major table and a plain float buffer laid out
// [plane][cell][phase_y][phase_x][tap_y][tap_x][re, im].  Planes plane0 .. plane0+nplanes-1 share
// one support, so plane i starts os^2 S^2 nqc entries after plane i-1; cells are qc0 .. qc0+ncell-1.
// to_table: table <- scale[qc] * buf (rounded to the storage type); else buf <- table.
__global__ void cell_io_kernel(void* __restrict__ table, int storage, int nqc, int ce, int os, int support,
                               int64_t offset0, int nplanes, int qc0, int ncell, float* __restrict__ buf,
                               int to_table, CellScale scale) {
  const size_t ss = static_cast<size_t>(support) * support;
  const size_t per_cell = ss * os * os;
  const size_t total = per_cell * ncell * nplanes;
  const size_t nch = nqc / ce;
  const size_t plane_stride = per_cell * nqc;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t r = i % per_cell, pc = i / per_cell;
    const int qc = qc0 + static_cast<int>(pc % ncell);
    const size_t plane = pc / ncell;
    const size_t phase = r / ss, tap = r % ss;
    const size_t ch = qc / ce, e = qc % ce;
    const size_t dst = offset0 + plane * plane_stride + ((phase * nch + ch) * ss + tap) * ce + e;
    if (to_table) {
      const float re = buf[2 * i] * scale.v[qc], im = buf[2 * i + 1] * scale.v[qc];
      if (storage == PG_STORE_F16) {
        static_cast<__half2*>(table)[dst] = __floats2half2_rn(re, im);
      } else {
        static_cast<float2*>(table)[dst] = make_float2(re, im);
      }
    } else {
      float2 v;
      if (storage == PG_STORE_F16) {
        v = __half22float2(static_cast<const __half2*>(table)[dst]);
      } else {
        v = static_cast<const float2*>(table)[dst];
      }
      buf[2 * i] = v.x;
      buf[2 * i + 1] = v.y;
    }
  }
}

// kbound[4 p + q] = max over the entries of Mueller row q in plane p's table of |re| + |im|, the
// bound the shared-tap gridder scales its fixed point from.  Block b takes phase b / nch, chunk
// b mod nch of the plane: entries [b ss E, (b + 1) ss E), entry i of it is tap i / E, Mueller cell
// chunk E + i mod E.  Per-thread maxima per row q, then a wave maximum and one integer atomic max
// on the float bits per wave (non-negative floats order like their bits).
__device__ inline float2 entry_value(float2 t) { return t; }
__device__ inline float2 entry_value(__half2 t) { return __half22float2(t); }

template <typename TapT>
__global__ __launch_bounds__(256) void kernel_bound_kernel(const TapT* __restrict__ plane_table, int ss, int e_per_chunk,
                                                           int nch, int npol, unsigned* __restrict__ out) {
  const int chunk = static_cast<int>(blockIdx.x % static_cast<unsigned>(nch));
  const TapT* blk = plane_table + static_cast<size_t>(blockIdx.x) * ss * e_per_chunk;
  float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = threadIdx.x; i < ss * e_per_chunk; i += 256) {
    const int q = (chunk * e_per_chunk + (i & (e_per_chunk - 1))) / npol;
    const float2 t = entry_value(blk[i]);
    const float a = fabsf(t.x) + fabsf(t.y);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
      if (qq == q) m[qq] = fmaxf(m[qq], a);
  }
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    float v = m[qq];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    if ((threadIdx.x & 63) == 0 && v > 0.0f) atomicMax(out + qq, __float_as_uint(v));
  }
}

}  // namespace

hipError_t cell_io(void* table, int storage, int nqc, int ce, int os, int support, int64_t offset0, int nplanes,
                   int qc0, int ncell, float* buf, bool to_table, const CellScale& scale, hipStream_t s) {
  const size_t total = static_cast<size_t>(support) * support * os * os * ncell * nplanes;
  if (total == 0) return hipSuccess;
  const int blocks = static_cast<int>(std::min<size_t>((total + 255) / 256, 65535));
  hipLaunchKernelGGL(cell_io_kernel, dim3(blocks), dim3(256), 0, s, table, storage, nqc, ce, os, support, offset0,
                     nplanes, qc0, ncell, buf, to_table ? 1 : 0, scale);
  return hipGetLastError();
}

hipError_t launch_screen(const double2* phi, const double* aa_lat, double w, double fov, int mk, int nqc,
                         double2* out, hipStream_t s) {
  dim3 grid((mk + 127) / 128, mk);
  hipLaunchKernelGGL(screen_kernel, grid, dim3(128), 0, s, phi, aa_lat, w, fov, mk, nqc, out);
  return hipGetLastError();
}

hipError_t launch_twiddles(int support, int os, int mk, double2* e, hipStream_t s) {
  dim3 grid((mk + 127) / 128, support * os);
  hipLaunchKernelGGL(twiddle_kernel, grid, dim3(128), 0, s, support, os, mk, e);
  return hipGetLastError();
}

hipError_t launch_zgemm_nt(int batch, int m, int n, int k, const double2* a, int64_t stride_a,
                           const double2* b, int64_t stride_b, double2* c, int64_t stride_c, hipStream_t s) {
  dim3 grid((n + BN - 1) / BN, (m + BM - 1) / BM, batch);
  hipLaunchKernelGGL(zgemm_kernel<true>, grid, dim3(256), 0, s, m, n, k, a, stride_a, b, stride_b, c, stride_c);
  return hipGetLastError();
}

hipError_t launch_zgemm_nn(int batch, int m, int n, int k, const double2* a, int64_t stride_a,
                           const double2* b, int64_t stride_b, double2* c, int64_t stride_c, hipStream_t s) {
  dim3 grid((n + BN - 1) / BN, (m + BM - 1) / BM, batch);
  hipLaunchKernelGGL(zgemm_kernel<false>, grid, dim3(256), 0, s, m, n, k, a, stride_a, b, stride_b, c, stride_c);
  return hipGetLastError();
}

hipError_t refresh_kernel_bound(pg_kernels* k, int plane0, int nplanes, hipStream_t s) {
  if (nplanes <= 0) return hipSuccess;
  hipError_t e = launch_fill_zero(k->kbound.as<float>() + 4 * plane0, sizeof(float) * 4 * nplanes, s);
  if (e != hipSuccess) return e;
  const int nqc = k->npol * k->npol;
  const int ec = chunk_entries(k->storage, nqc), nch = nqc / ec;
  for (int p = plane0; p < plane0 + nplanes; ++p) {
    const unsigned blocks = static_cast<unsigned>(k->os * k->os * nch);
    unsigned* out = reinterpret_cast<unsigned*>(k->kbound.as<float>() + 4 * p);
    const int ss = k->support[p] * k->support[p];
    if (k->storage == PG_STORE_F16)
      hipLaunchKernelGGL(kernel_bound_kernel<__half2>, dim3(blocks), dim3(256), 0, s,
                         k->table.as<__half2>() + k->plane_offset[p], ss, ec, nch, k->npol, out);
    else
      hipLaunchKernelGGL(kernel_bound_kernel<float2>, dim3(blocks), dim3(256), 0, s,
                         k->table.as<float2>() + k->plane_offset[p], ss, ec, nch, k->npol, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pack(const double2* t, int support, int os, int nqc, int storage, void* table, hipStream_t s) {
  size_t total = static_cast<size_t>(support) * os * support * os * nqc;
  int blocks = static_cast<int>(std::min<size_t>((total + 255) / 256, 65535));
  hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, s, t, support, os, nqc, storage,
                     chunk_entries(storage, nqc), table);
  return hipGetLastError();
}

}  // namespace pg
