// mlp_host.h -- launchers of the warm-start network kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdlb {
hipError_t mlp_gemm(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                    long sbk, long sbn, int ldc, int accumulate, hipStream_t s);
// split-K GEMM for products with few output tiles and a long depth (the weight
// gradients, whose depth is the batch): up to MLP_SPLITK_MAX slices of the
// depth write partial products into `partial` (slices x M x N floats), which a
// second kernel adds in slice order into C
constexpr int MLP_SPLITK_MAX = 16;
// blocks of the loss kernel, one FP64 partial each
constexpr int MLP_LOSS_PARTS = 1024;
int mlp_splitk_slices(int M, int N, int K);
hipError_t mlp_gemm_splitk(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                           long sbk, long sbn, int ldc, int accumulate, float *partial, hipStream_t s);
hipError_t mlp_bias_act(float *Z, const float *b, uint16_t *H, int M, int N, int act, hipStream_t s);
// dZ = dH * GELU'(Z) (BF16) and db = column sums of dZ (FP32, row slices added
// in slice order; partial holds at least min(64, max_slices) x N floats)
hipError_t mlp_gelu_bwd_colsum(const float *dH, const float *Z, uint16_t *dZb, float *db, int M, int N, float *partial,
                               int max_slices, hipStream_t s);
hipError_t mlp_mse(const float *Y, const float *T, uint16_t *dYb, float *dYf, double *part, long n, float *loss,
                   hipStream_t s);
// db[n] = sum_m dZ[m][n], in row slices through `partial` (at least MLP_SPLITK_MAX x N floats)
hipError_t mlp_colsum(const float *dZ, float *db, int M, int N, float *partial, hipStream_t s);
hipError_t mlp_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s);
hipError_t mlp_adamw(float *p, float *m, float *v, const float *g, long n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, const long *wmap, uint16_t *wb, const long *wmapT,
                     uint16_t *wbT, hipStream_t s);
}  // namespace fdlb
