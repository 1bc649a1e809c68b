// C-ABI of the kernel-surrogate network: creation, forward, one training step (forward, loss,
// backward, Adam), parameter and activation access, and writing a generated kernel into a table.
#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "mlp.hpp"

struct pg_mlp {
  int32_t n_in = 0, width = 0, hidden = 0, max_batch = 0;
  int64_t n_out = 0;
  int64_t step = 0;
  std::vector<int64_t> dims;  // d_0 = n_in, d_1..d_hidden = width, d_{hidden+1} = n_out
  struct Layer {
    pg::DevBuf w, w_bf, b, gw, gb, mw, vw, mb, vb;
    pg::DevBuf w_bft;  // bf16 [d_out][d_in]: the forward product's k-contiguous operand
  };
  std::vector<Layer> layers;          // layers[l] maps d_l -> d_{l+1}
  pg::DevBuf x_bf;                    // [B][n_in] bf16
  std::vector<pg::DevBuf> pre, act;   // pre[l] float [B][d_{l+1}], act[l] bf16 [B][d_{l+1}] (hidden only)
  pg::DevBuf gy, gy_bf, ga, gz, gz_bf, loss;
  int32_t last_batch = 0;
};

namespace pg {
void set_error(const std::string& msg);
}

namespace {
int fail(int code, const std::string& m) {
  pg::set_error(m);
  return code;
}
#define PGM_HIP(call, what)                                                                    \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(PG_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Contraction split for a product whose 128 x 128 output tiles alone cannot fill the GPU: enough
// slices for about 512 workgroups, each slice at least 256 deep.
int split_for(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
  if (tiles >= 512) return 1;
  const int64_t split = std::min<int64_t>((512 + tiles - 1) / tiles, K / 256);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(split, 256)));
}

// y: where the output layer writes (NULL: the network's own pre-activation buffer, which the
// training step reads).
int forward_impl(pg_mlp* m, const float* x, int batch, hipStream_t s, float* y = nullptr) {
  const int L = static_cast<int>(m->layers.size());
  PGM_HIP(pg::mlp_to_bf16(x, static_cast<int64_t>(batch) * m->n_in, m->x_bf.as<uint16_t>(), s), "features");
  const uint16_t* a = m->x_bf.as<uint16_t>();
  for (int l = 0; l < L; ++l) {
    const int64_t din = m->dims[l], dout = m->dims[l + 1];
    const bool hidden = l + 1 < L;
    float* z = (!hidden && y) ? y : m->pre[l].as<float>();
    // z = a W + b, and for hidden layers SiLU(z) in bf16, in the product's epilogue
    PGM_HIP(pg::mlp_gemm(batch, static_cast<int>(dout), static_cast<int>(din), a, din, 1, m->layers[l].w_bft.as<uint16_t>(),
                         1, din, z, dout, false, 1, s, m->layers[l].b.as<float>(),
                         hidden ? m->act[l].as<uint16_t>() : nullptr),
            "forward gemm");
    if (hidden) a = m->act[l].as<uint16_t>();
  }
  m->last_batch = batch;
  return PG_OK;
}
}  // namespace

extern "C" {

int pg_mlp_create(int32_t n_in, int32_t width, int32_t hidden_layers, int64_t n_out, int32_t max_batch, uint64_t seed,
                  void* stream, pg_mlp** out) {
  pg::set_error("");
  if (!out) return fail(PG_EINVAL, "out must be non-NULL");
  *out = nullptr;
  if (n_in < 1 || n_in > 4096 || width < 1 || width > 8192 || hidden_layers < 1 || hidden_layers > 16 || n_out < 1 ||
      n_out > (int64_t(1) << 30) || max_batch < 1 || max_batch > 65536)
    return fail(PG_EINVAL, "bad network shape");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* m = new (std::nothrow) pg_mlp();
  if (!m) return fail(PG_ENOMEM, "host allocation failed");
  std::unique_ptr<pg_mlp> guard(m);
  m->n_in = n_in;
  m->width = width;
  m->hidden = hidden_layers;
  m->n_out = n_out;
  m->max_batch = max_batch;
  m->dims.push_back(n_in);
  for (int i = 0; i < hidden_layers; ++i) m->dims.push_back(width);
  m->dims.push_back(n_out);
  const int L = hidden_layers + 1;
  m->layers.resize(L);
  m->pre.resize(L);
  m->act.resize(L);
  const int64_t B = max_batch;
  for (int l = 0; l < L; ++l) {
    const int64_t din = m->dims[l], dout = m->dims[l + 1], nw = din * dout;
    auto& ly = m->layers[l];
    if (!ly.w.alloc(4 * nw, s) || !ly.w_bf.alloc(2 * nw, s) || !ly.w_bft.alloc(2 * nw, s) || !ly.b.alloc(4 * dout, s) ||
        !ly.gw.alloc(4 * nw, s) ||
        !ly.gb.alloc(4 * dout, s) || !ly.mw.alloc(4 * nw, s) || !ly.vw.alloc(4 * nw, s) || !ly.mb.alloc(4 * dout, s) ||
        !ly.vb.alloc(4 * dout, s) || !m->pre[l].alloc(4 * B * dout, s))
      return fail(PG_ENOMEM, "device allocation failed in mlp_create");
    if (l + 1 < L && !m->act[l].alloc(2 * B * dout, s)) return fail(PG_ENOMEM, "device allocation failed in mlp_create");
    const float a = static_cast<float>(std::sqrt((l + 1 < L ? 6.0 : 3.0) / static_cast<double>(din)));
    PGM_HIP(pg::mlp_init_uniform(ly.w.as<float>(), nw, seed + (static_cast<uint64_t>(l) << 40), a, s), "init");
    PGM_HIP(pg::mlp_to_bf16(ly.w.as<float>(), nw, ly.w_bf.as<uint16_t>(), s), "init bf16");
    PGM_HIP(pg::mlp_transpose_bf16(ly.w_bf.as<uint16_t>(), din, dout, ly.w_bft.as<uint16_t>(), s), "init transpose");
    for (pg::DevBuf* z : {&ly.b, &ly.mw, &ly.vw, &ly.mb, &ly.vb, &ly.gb})
      PGM_HIP(pg::launch_fill_zero(z->p, z->bytes, s), "zero");
  }
  const int64_t wmax = *std::max_element(m->dims.begin() + 1, m->dims.end() - 1);
  if (!m->x_bf.alloc(2 * B * n_in + 16, s) || !m->gy.alloc(4 * B * n_out, s) || !m->gy_bf.alloc(2 * B * n_out + 16, s) ||
      !m->ga.alloc(4 * B * wmax, s) || !m->gz.alloc(4 * B * wmax, s) || !m->gz_bf.alloc(2 * B * wmax + 16, s) ||
      !m->loss.alloc(8, s))
    return fail(PG_ENOMEM, "device allocation failed in mlp_create");
  PGM_HIP(hipStreamSynchronize(s), "mlp sync");
  *out = guard.release();
  return PG_OK;
}

int pg_mlp_forward(pg_mlp* m, const float* x, int32_t batch, float* y, void* stream) {
  pg::set_error("");
  if (!m || !x) return fail(PG_EINVAL, "network and features must be non-NULL");
  if (batch < 1 || batch > m->max_batch) return fail(PG_EINVAL, "batch must be in [1, max_batch]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return forward_impl(m, x, batch, s, y);
}

int pg_mlp_train_step(pg_mlp* m, const float* x, const float* target, int32_t batch, float lr, int32_t update,
                      float* loss_out, void* stream) {
  pg::set_error("");
  if (!m || !x || !target) return fail(PG_EINVAL, "network, features and targets must be non-NULL");
  if (batch < 1 || batch > m->max_batch) return fail(PG_EINVAL, "batch must be in [1, max_batch]");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(PG_EINVAL, "learning rate must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = forward_impl(m, x, batch, s);
  if (rc != PG_OK) return rc;
  const int L = static_cast<int>(m->layers.size());
  PGM_HIP(pg::launch_fill_zero(m->loss.p, 8, s), "zero loss");
  PGM_HIP(pg::mlp_loss(m->pre.back().as<float>(), target, m->n_out, batch, m->gy.as<float>(), m->gy_bf.as<uint16_t>(),
                       m->loss.as<float>(), s), "loss");
  // backward: g_z of layer l in (gz_f, gz_b); the output layer's is the loss gradient
  const float* gz_f = m->gy.as<float>();
  const uint16_t* gz_b = m->gy_bf.as<uint16_t>();
  for (int l = L - 1; l >= 0; --l) {
    const int64_t din = m->dims[l], dout = m->dims[l + 1];
    const uint16_t* a_in = l == 0 ? m->x_bf.as<uint16_t>() : m->act[l - 1].as<uint16_t>();
    // gW[din][dout] = a_in^T g_z ; contraction over the batch
    PGM_HIP(pg::mlp_gemm(static_cast<int>(din), static_cast<int>(dout), batch, a_in, 1, din, gz_b, dout, 1,
                         m->layers[l].gw.as<float>(), dout, false, split_for(din, dout, batch), s),
            "weight gradient");
    PGM_HIP(pg::mlp_colsum(gz_f, batch, dout, m->layers[l].gb.as<float>(), s), "bias gradient");
    if (l > 0) {
      // g_a[B][din] = g_z W^T ; contraction over dout (split when the output is narrow)
      PGM_HIP(pg::mlp_gemm(batch, static_cast<int>(din), static_cast<int>(dout), gz_b, dout, 1,
                           m->layers[l].w_bf.as<uint16_t>(), 1, dout, m->ga.as<float>(), din, false,
                           split_for(batch, din, dout), s),
              "input gradient");
      PGM_HIP(pg::mlp_silu_back(m->ga.as<float>(), m->pre[l - 1].as<float>(), static_cast<int64_t>(batch) * din,
                                m->gz.as<float>(), m->gz_bf.as<uint16_t>(), s), "silu backward");
      gz_f = m->gz.as<float>();
      gz_b = m->gz_bf.as<uint16_t>();
    }
  }
  if (update) {
    m->step += 1;
    for (int l = 0; l < L; ++l) {
      auto& ly = m->layers[l];
      const int64_t nw = m->dims[l] * m->dims[l + 1];
      PGM_HIP(pg::mlp_adam(ly.w.as<float>(), ly.w_bf.as<uint16_t>(), ly.gw.as<float>(), ly.mw.as<float>(),
                           ly.vw.as<float>(), nw, lr, 0.9, 0.999, 1e-8, m->step, s), "adam");
      PGM_HIP(pg::mlp_transpose_bf16(ly.w_bf.as<uint16_t>(), m->dims[l], m->dims[l + 1], ly.w_bft.as<uint16_t>(), s),
              "adam transpose");
      PGM_HIP(pg::mlp_adam(ly.b.as<float>(), nullptr, ly.gb.as<float>(), ly.mb.as<float>(), ly.vb.as<float>(),
                           m->dims[l + 1], lr, 0.9, 0.999, 1e-8, m->step, s), "adam");
    }
  }
  if (loss_out) PGM_HIP(hipMemcpyAsync(loss_out, m->loss.p, 4, hipMemcpyDeviceToDevice, s), "copy loss");
  return PG_OK;
}

int pg_mlp_copy(const pg_mlp* m, int32_t what, int32_t layer, void* dst, void* stream) {
  pg::set_error("");
  if (!m || !dst) return fail(PG_EINVAL, "network and dst must be non-NULL");
  const int L = static_cast<int>(m->layers.size());
  if (layer < 0 || layer >= L) return fail(PG_EINVAL, "layer out of range");
  const auto& ly = m->layers[layer];
  const int64_t din = m->dims[layer], dout = m->dims[layer + 1], B = m->last_batch;
  const void* src = nullptr;
  int64_t bytes = 0;
  switch (what) {
    case PG_MLP_W: src = ly.w.p; bytes = 4 * din * dout; break;
    case PG_MLP_W_BF16: src = ly.w_bf.p; bytes = 2 * din * dout; break;
    case PG_MLP_B: src = ly.b.p; bytes = 4 * dout; break;
    case PG_MLP_GW: src = ly.gw.p; bytes = 4 * din * dout; break;
    case PG_MLP_GB: src = ly.gb.p; bytes = 4 * dout; break;
    case PG_MLP_ACT: src = layer == 0 ? m->x_bf.p : m->act[layer - 1].p; bytes = 2 * B * din; break;
    case PG_MLP_PRE: src = m->pre[layer].p; bytes = 4 * B * dout; break;
    case PG_MLP_GY: src = m->gy.p; bytes = 4 * B * m->n_out; break;
    case PG_MLP_GY_BF16: src = m->gy_bf.p; bytes = 2 * B * m->n_out; break;
    case PG_MLP_GZ: src = m->gz.p; bytes = 4 * B * m->dims[1]; break;
    case PG_MLP_GZ_BF16: src = m->gz_bf.p; bytes = 2 * B * m->dims[1]; break;
    case PG_MLP_MW: src = ly.mw.p; bytes = 4 * din * dout; break;
    case PG_MLP_VW: src = ly.vw.p; bytes = 4 * din * dout; break;
    case PG_MLP_MB: src = ly.mb.p; bytes = 4 * dout; break;
    case PG_MLP_VB: src = ly.vb.p; bytes = 4 * dout; break;
    default: return fail(PG_EINVAL, "unknown quantity");
  }
  PGM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)), "copy");
  return PG_OK;
}

int pg_mlp_load(pg_mlp* m, int32_t layer, const float* w, const float* b, void* stream) {
  pg::set_error("");
  if (!m || !w || !b) return fail(PG_EINVAL, "network, w and b must be non-NULL");
  if (layer < 0 || layer >= static_cast<int>(m->layers.size())) return fail(PG_EINVAL, "layer out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto& ly = m->layers[layer];
  const int64_t nw = m->dims[layer] * m->dims[layer + 1];
  PGM_HIP(hipMemcpyAsync(ly.w.p, w, 4 * nw, hipMemcpyDeviceToDevice, s), "load w");
  PGM_HIP(hipMemcpyAsync(ly.b.p, b, 4 * m->dims[layer + 1], hipMemcpyDeviceToDevice, s), "load b");
  PGM_HIP(pg::mlp_to_bf16(ly.w.as<float>(), nw, ly.w_bf.as<uint16_t>(), s), "load bf16");
  PGM_HIP(pg::mlp_transpose_bf16(ly.w_bf.as<uint16_t>(), m->dims[layer], m->dims[layer + 1], ly.w_bft.as<uint16_t>(), s),
          "load transpose");
  return PG_OK;
}

int pg_mlp_set(pg_mlp* m, int32_t what, int32_t layer, const void* src, void* stream) {
  pg::set_error("");
  if (!m || !src) return fail(PG_EINVAL, "network and src must be non-NULL");
  if (layer < 0 || layer >= static_cast<int>(m->layers.size())) return fail(PG_EINVAL, "layer out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto& ly = m->layers[layer];
  const int64_t din = m->dims[layer], dout = m->dims[layer + 1];
  pg::DevBuf* dst = nullptr;
  int64_t bytes = 0;
  switch (what) {
    case PG_MLP_W: dst = &ly.w; bytes = 4 * din * dout; break;
    case PG_MLP_B: dst = &ly.b; bytes = 4 * dout; break;
    case PG_MLP_MW: dst = &ly.mw; bytes = 4 * din * dout; break;
    case PG_MLP_VW: dst = &ly.vw; bytes = 4 * din * dout; break;
    case PG_MLP_MB: dst = &ly.mb; bytes = 4 * dout; break;
    case PG_MLP_VB: dst = &ly.vb; bytes = 4 * dout; break;
    default: return fail(PG_EINVAL, "settable: PG_MLP_W, PG_MLP_B and the Adam moments");
  }
  PGM_HIP(hipMemcpyAsync(dst->p, src, bytes, hipMemcpyDeviceToDevice, s), "set");
  if (what == PG_MLP_W) {
    PGM_HIP(pg::mlp_to_bf16(ly.w.as<float>(), din * dout, ly.w_bf.as<uint16_t>(), s), "set bf16");
    PGM_HIP(pg::mlp_transpose_bf16(ly.w_bf.as<uint16_t>(), din, dout, ly.w_bft.as<uint16_t>(), s), "set transpose");
  }
  return PG_OK;
}

int pg_mlp_get_step(const pg_mlp* m, int64_t* step) {
  pg::set_error("");
  if (!m || !step) return fail(PG_EINVAL, "network and step must be non-NULL");
  *step = m->step;
  return PG_OK;
}

int pg_mlp_set_step(pg_mlp* m, int64_t step) {
  pg::set_error("");
  if (!m) return fail(PG_EINVAL, "network must be non-NULL");
  if (step < 0) return fail(PG_EINVAL, "step must be >= 0");
  m->step = step;
  return PG_OK;
}

void pg_mlp_destroy(pg_mlp* m) { delete m; }

int pg_gemm_f32(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, float alpha, const float* a,
                int64_t lda, const float* b, int64_t ldb, float beta, float* c, int64_t ldc, void* stream) {
  pg::set_error("");
  if (m < 0 || n < 0 || k < 0) return fail(PG_EINVAL, "m, n and k must be >= 0");
  if ((m > 0 && n > 0) && !c) return fail(PG_EINVAL, "c must be non-NULL");
  if (m > 0 && n > 0 && k > 0 && (!a || !b)) return fail(PG_EINVAL, "a and b must be non-NULL");
  if (lda < (transa ? m : k) || ldb < (transb ? k : n) || ldc < n)
    return fail(PG_EINVAL, "leading dimensions must cover a row of the stored matrix");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(PG_EINVAL, "alpha and beta must be finite");
  PGM_HIP(pg::gemm_f32(transa != 0, transb != 0, m, n, k, alpha, a, lda, b, ldb, beta, c, ldc,
                       static_cast<hipStream_t>(stream)),
          "gemm_f32");
  return PG_OK;
}

int pg_scale_rows(float* x, int64_t rows, int64_t cols, const float* scale, void* stream) {
  pg::set_error("");
  if (rows < 0 || cols < 0) return fail(PG_EINVAL, "rows and cols must be >= 0");
  if (rows > 0 && cols > 0 && (!x || !scale)) return fail(PG_EINVAL, "x and scale must be non-NULL");
  PGM_HIP(pg::scale_rows(x, rows, cols, scale, static_cast<hipStream_t>(stream)), "scale_rows");
  return PG_OK;
}

int pg_kernels_write_cell(pg_kernels* k, int32_t plane, int32_t q, int32_t c, const float* src, void* stream) {
  pg::set_error("");
  if (!k || !src) return fail(PG_EINVAL, "kernels and src must be non-NULL");
  if (plane < 0 || plane >= k->nplanes || q < 0 || q >= k->npol || c < 0 || c >= k->npol)
    return fail(PG_EINVAL, "plane or Mueller cell out of range");
  const int nqc = k->npol * k->npol;
  pg::CellScale one;
  for (float& v : one.v) v = 1.0f;
  PGM_HIP(pg::cell_io(k->table.p, k->storage, nqc, pg::chunk_entries(k->storage, nqc), k->os, k->support[plane],
                      k->plane_offset[plane], 1, q * k->npol + c, 1, const_cast<float*>(src), true, one,
                      static_cast<hipStream_t>(stream)),
          "write cell");
  PGM_HIP(pg::refresh_kernel_bound(k, plane, 1, static_cast<hipStream_t>(stream)), "kernel bound");
  return PG_OK;
}

namespace {
int check_plane_range(const pg_kernels* k, int32_t plane0, int32_t nplanes) {
  if (plane0 < 0 || nplanes < 0 || plane0 > k->nplanes - nplanes) return fail(PG_EINVAL, "plane range out of bounds");
  for (int p = plane0 + 1; p < plane0 + nplanes; ++p)
    if (k->support[p] != k->support[plane0]) return fail(PG_EINVAL, "planes of one transfer must share their support");
  return PG_OK;
}
}  // namespace

int pg_kernels_export(const pg_kernels* k, int32_t plane0, int32_t nplanes, float* dst, void* stream) {
  pg::set_error("");
  if (!k || (!dst && nplanes > 0)) return fail(PG_EINVAL, "kernels and dst must be non-NULL");
  const int rc = check_plane_range(k, plane0, nplanes);
  if (rc != PG_OK || nplanes == 0) return rc;
  const int nqc = k->npol * k->npol;
  pg::CellScale one;
  for (float& v : one.v) v = 1.0f;
  PGM_HIP(pg::cell_io(k->table.p, k->storage, nqc, pg::chunk_entries(k->storage, nqc), k->os, k->support[plane0],
                      k->plane_offset[plane0], nplanes, 0, nqc, dst, false, one, static_cast<hipStream_t>(stream)),
          "export cells");
  return PG_OK;
}

int pg_kernels_import(pg_kernels* k, int32_t plane0, int32_t nplanes, const float* src, const float* cell_scale,
                      void* stream) {
  pg::set_error("");
  if (!k || (!src && nplanes > 0)) return fail(PG_EINVAL, "kernels and src must be non-NULL");
  const int rc = check_plane_range(k, plane0, nplanes);
  if (rc != PG_OK || nplanes == 0) return rc;
  const int nqc = k->npol * k->npol;
  pg::CellScale sc;
  for (int i = 0; i < 16; ++i) sc.v[i] = (cell_scale && i < nqc) ? cell_scale[i] : 1.0f;
  for (int i = 0; i < nqc; ++i)
    if (!std::isfinite(sc.v[i])) return fail(PG_EINVAL, "cell_scale must be finite");
  PGM_HIP(pg::cell_io(k->table.p, k->storage, nqc, pg::chunk_entries(k->storage, nqc), k->os, k->support[plane0],
                      k->plane_offset[plane0], nplanes, 0, nqc, const_cast<float*>(src), true, sc,
                      static_cast<hipStream_t>(stream)),
          "import cells");
  PGM_HIP(pg::refresh_kernel_bound(k, plane0, nplanes, static_cast<hipStream_t>(stream)), "kernel bound");
  return PG_OK;
}

}  // extern "C"
