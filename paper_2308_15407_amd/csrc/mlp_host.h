// mlp_host.h -- launchers of the warm-start network kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdlb {
hipError_t mlp_gemm(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                    long sbk, long sbn, int ldc, int accumulate, hipStream_t s);
hipError_t mlp_bias_act(float *Z, const float *b, uint16_t *H, int M, int N, int act, hipStream_t s);
hipError_t mlp_gelu_bwd(const float *dH, const float *Z, uint16_t *dZb, float *dZf, long n, hipStream_t s);
hipError_t mlp_mse(const float *Y, const float *T, uint16_t *dYb, float *dYf, double *part, long n, float *loss,
                   hipStream_t s);
hipError_t mlp_colsum(const float *dZ, float *db, int M, int N, hipStream_t s);
hipError_t mlp_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s);
hipError_t mlp_adamw(float *p, float *m, float *v, const float *g, long n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, const long *wmap, uint16_t *wb, hipStream_t s);
}  // namespace fdlb
