// mlp_kernels.hip -- gfx950 kernels of the warm-start network: a multilayer
// perceptron with GELU hidden layers, BF16 weights and activations, FP32
// accumulation, FP32 master weights and AdamW.
//
// GEMM: C[M,N] (fp32) = A[M,K] * B[K,N] (+ C if accumulate), A and B in BF16
// with arbitrary element strides, on v_mfma_f32_16x16x16_bf16 tiles: a 256-thread
// block owns a 64x64 tile of C (each wave a 32x32 quarter as 2x2 MFMA tiles);
// A and B tiles of depth 16 are staged in LDS with k contiguous.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_host.h"

namespace fdlb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GT = 64;   // C tile edge
constexpr int GK = 16;   // depth per MFMA step

__global__ void __launch_bounds__(256) k_gemm_bf16(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                                   float *__restrict__ C, int M, int N, int K, long sam, long sak,
                                                   long sbk, long sbn, int ldc, int accumulate, int kchunk,
                                                   long cslice) {
  __shared__ uint16_t sA[GT][GK + 4];   // [m][k]
  __shared__ uint16_t sB[GT][GK + 4];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  // split K: block z takes depths [kb, ke) and writes its own slice of C
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  C += blockIdx.z * cslice;
  const int wr = wv >> 1, wc = wv & 1;
  v4f acc[2][2];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GK) {
    // stage: 64x16 elements of A and of B, 4 per thread each
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, kk = e % GK;
      const int gm = m0 + r, gn = n0 + r, gk = k0 + kk;
      sA[r][kk] = (gm < M && gk < ke) ? A[(long)gm * sam + (long)gk * sak] : (uint16_t)0;
      sB[r][kk] = (gn < N && gk < ke) ? B[(long)gk * sbk + (long)gn * sbn] : (uint16_t)0;
    }
    __syncthreads();
    const int row = lane & 15, kq = (lane >> 4) * 4;
    v4s a[2], b[2];
    for (int i = 0; i < 2; i++) {
      const uint16_t *pa = &sA[wr * 32 + i * 16 + row][kq];
      a[i] = (v4s){(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
      const uint16_t *pb = &sB[wc * 32 + i * 16 + row][kq];
      b[i] = (v4s){(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
    }
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // D layout: lane l holds column l%16, rows 4*(l/16)+t
  const int col = lane & 15, rq = (lane >> 4) * 4;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++)
      for (int t = 0; t < 4; t++) {
        const int gm = m0 + wr * 32 + i * 16 + rq + t, gn = n0 + wc * 32 + j * 16 + col;
        if (gm < M && gn < N) {
          float *p = &C[(long)gm * ldc + gn];
          *p = accumulate ? *p + acc[i][j][t] : acc[i][j][t];
        }
      }
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z += b (per column); H = GELU(Z) in BF16 (act != 0) or Y = Z (output layer)
__global__ void k_bias_act(float *__restrict__ Z, const float *__restrict__ b, uint16_t *__restrict__ H, int M,
                           int N, int act) {
  const long n = (long)M * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float z = Z[i] + b[i % N];
    Z[i] = z;
    if (act) H[i] = f2bf(gelu(z));
  }
}

// dZ = dH * GELU'(Z) in BF16 (and fp32 copy for the bias gradient)
__global__ void k_gelu_bwd(const float *__restrict__ dH, const float *__restrict__ Z, uint16_t *__restrict__ dZb,
                           float *__restrict__ dZf, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = dH[i] * gelu_d(Z[i]);
    dZf[i] = d;
    dZb[i] = f2bf(d);
  }
}

// MSE: loss partial per block, dY = 2 (Y - T) / (M N)
__global__ void __launch_bounds__(256) k_mse(const float *__restrict__ Y, const float *__restrict__ T,
                                             uint16_t *__restrict__ dYb, float *__restrict__ dYf,
                                             double *__restrict__ part, long n) {
  __shared__ double red[256];
  double s = 0;
  const float sc = 2.0f / (float)n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    s += (double)d * d;
    dYf[i] = sc * d;
    dYb[i] = f2bf(sc * d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *__restrict__ part, int nparts, long n, float *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < nparts; i++) s += part[i];
    *out = (float)(s / (double)n);
  }
}

// db[n] = sum_m dZ[m][n]: a 1024-thread block per 64 columns; wave w sums rows
// w, w + 16, ... of its lane's column in four interleaved partial sums (loads
// coalesced along the row), then the 16 wave sums are added in wave order
// (a fixed order: the result does not depend on timing)
__global__ void __launch_bounds__(1024) k_colsum(const float *__restrict__ dZ, float *__restrict__ db, int M, int N) {
  __shared__ float red[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (n < N) {
    int m = wv;
    for (; m + 48 < M; m += 64) {
      s0 += dZ[(long)m * N + n];
      s1 += dZ[(long)(m + 16) * N + n];
      s2 += dZ[(long)(m + 32) * N + n];
      s3 += dZ[(long)(m + 48) * N + n];
    }
    for (; m < M; m += 16) s0 += dZ[(long)m * N + n];
  }
  red[wv][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wv == 0 && n < N) {
    float s = 0.f;
    for (int w = 0; w < 16; w++) s += red[w][lane];
    db[n] = s;
  }
}

// C[m][n] (ldc) (+)= sum over z of P[z][m][n] (slices of M x N), in z order
__global__ void k_splitk_sum(const float *__restrict__ P, float *__restrict__ C, int M, int N, int S, int ldc,
                             int accumulate) {
  const long mn = (long)M * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < mn; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < S; z++) s += P[z * mn + i];
    const long o = (i / N) * ldc + i % N;
    C[o] = accumulate ? C[o] + s : s;
  }
}

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

// AdamW on the fp32 master parameters; refresh the BF16 weight copies
__global__ void k_adamw(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ g, long n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2, const long *__restrict__ wmap, uint16_t *__restrict__ wb) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float pi = p[i];
    pi -= lr * (mi / c1 / (sqrtf(vi / c2) + eps) + wd * pi);
    p[i] = pi;
    const long w = wmap[i];
    if (w >= 0) wb[w] = f2bf(pi);
  }
}

// --------------------------------------------------------------------------
hipError_t mlp_gemm(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                    long sbk, long sbn, int ldc, int accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  dim3 g((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm_bf16, g, dim3(256), 0, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, K, 0L);
  return hipGetLastError();
}

static int blocks_for(long n);

int mlp_splitk_slices(int M, int N, int K) {
  const int tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  if (tiles >= 64 || K < 512) return 1;
  int S = 128 / tiles;
  if (S > K / 256) S = K / 256;
  if (S > MLP_SPLITK_MAX) S = MLP_SPLITK_MAX;
  return S < 1 ? 1 : S;
}

hipError_t mlp_gemm_splitk(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                           long sbk, long sbn, int ldc, int accumulate, float *partial, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  const int S = mlp_splitk_slices(M, N, K);
  if (S <= 1 || !partial) return mlp_gemm(A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, s);
  // depth per slice, a multiple of the MFMA depth; every slice is non-empty
  const int kc = ((K + S - 1) / S + GK - 1) / GK * GK;
  const int Sr = (K + kc - 1) / kc;
  dim3 g((N + GT - 1) / GT, (M + GT - 1) / GT, Sr);
  hipLaunchKernelGGL(k_gemm_bf16, g, dim3(256), 0, s, A, B, partial, M, N, K, sam, sak, sbk, sbn, N, 0, kc,
                     (long)M * N);
  hipLaunchKernelGGL(k_splitk_sum, dim3(blocks_for((long)M * N)), dim3(256), 0, s, partial, C, M, N, Sr, ldc,
                     accumulate);
  return hipGetLastError();
}

static int blocks_for(long n) { long b = (n + 255) / 256; return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048); }

hipError_t mlp_bias_act(float *Z, const float *b, uint16_t *H, int M, int N, int act, hipStream_t s) {
  hipLaunchKernelGGL(k_bias_act, dim3(blocks_for((long)M * N)), dim3(256), 0, s, Z, b, H, M, N, act);
  return hipGetLastError();
}

hipError_t mlp_gelu_bwd(const float *dH, const float *Z, uint16_t *dZb, float *dZf, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for(n)), dim3(256), 0, s, dH, Z, dZb, dZf, n);
  return hipGetLastError();
}

hipError_t mlp_mse(const float *Y, const float *T, uint16_t *dYb, float *dYf, double *part, long n, float *loss,
                   hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, Y, T, dYb, dYf, part, n);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, nb, n, loss);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float *dZ, float *db, int M, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(1024), 0, s, dZ, db, M, N);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t mlp_adamw(float *p, float *m, float *v, const float *g, long n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, const long *wmap, uint16_t *wb, hipStream_t s) {
  hipLaunchKernelGGL(k_adamw, dim3(blocks_for(n)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, wd, c1, c2, wmap, wb);
  return hipGetLastError();
}

}  // namespace fdlb
