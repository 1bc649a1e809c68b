// Device launchers of the kernel-surrogate network (mlp.hip).  bf16 values are uint16_t bit patterns.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pg {
// C (+)= A B; bias (optional, not with a split contraction) adds a row vector, act (optional)
// receives SiLU(C) in bf16 with C's row stride.
hipError_t mlp_gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                    int64_t sbn, float* C, int64_t ldc, bool accumulate, int split_k, hipStream_t s,
                    const float* bias = nullptr, uint16_t* act = nullptr);
hipError_t gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                    const float* B, int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s);
hipError_t scale_rows(float* x, int64_t rows, int64_t cols, const float* scale, hipStream_t s);
hipError_t mlp_transpose_bf16(const uint16_t* in, int64_t rows, int64_t cols, uint16_t* out, hipStream_t s);
hipError_t mlp_silu_back(const float* gact, const float* z, int64_t n, float* gpre, uint16_t* gpre_bf, hipStream_t s);
hipError_t mlp_loss(const float* y, const float* t, int64_t cols, int batch, float* grad, uint16_t* grad_bf,
                    float* loss, hipStream_t s);
hipError_t mlp_colsum(const float* g, int64_t rows, int64_t cols, float* out, hipStream_t s);
hipError_t mlp_adam(float* w, uint16_t* w_bf, const float* g, float* m, float* v, int64_t n, float lr, double b1,
                    double b2, double eps, int64_t step, hipStream_t s);
hipError_t mlp_to_bf16(const float* x, int64_t n, uint16_t* out, hipStream_t s);
hipError_t mlp_init_uniform(float* w, int64_t n, uint64_t seed, float a, hipStream_t s);
struct CellScale {
  float v[16];
};
hipError_t cell_io(void* table, int storage, int nqc, int ce, int os, int support, int64_t offset0, int nplanes,
                   int qc0, int ncell, float* buf, bool to_table, const CellScale& scale, hipStream_t s);
}  // namespace pg
