// mlp_kernels.hip -- gfx950 kernels of the warm-start network: a multilayer
// perceptron with GELU hidden layers, BF16 weights and activations, FP32
// accumulation, FP32 master weights and AdamW.
//
// GEMM: C[M,N] (fp32) = A[M,K] * B[K,N] (+ C if accumulate), A and B in BF16
// with arbitrary element strides.  A 256-thread block owns a 64x64 tile of C
// (each wave a 32x32 quarter as 2x2 tiles of v_mfma_f32_16x16x16_bf16), or a
// 128x128 tile for large products (each wave 64x64 as 2x2 tiles of
// v_mfma_f32_32x32x16_bf16).  A and B tiles of depth 32 are staged in two LDS
// buffers with k contiguous, read from global memory with 16-byte loads along
// whichever index is contiguous.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_host.h"

namespace fdlb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GT = 64;   // C tile edge
constexpr int GK = 32;   // depth per staged step (two MFMA depths of 16)
constexpr int GP = GK + 8;   // LDS row pitch in elements (80 B: 16-byte aligned rows)

// How one operand tile (64 rows of the outer index o = m or n, GK of depth k)
// is read from global memory: KVEC, eight consecutive k per 16-byte load (k
// contiguous, row stride a multiple of 8); OVEC, eight consecutive o per
// 16-byte load (o contiguous); SCALAR, one element per load (any strides).
enum { LD_KVEC = 0, LD_OVEC = 1, LD_SCALAR = 2 };

// element (o, k) of an operand with strides (so, sk); zero outside [0, no) x [kb, ke)
__device__ __forceinline__ uint16_t ld1(const uint16_t *X, long so, long sk, int o, int k, int no, int ke) {
  return (o < no && k < ke) ? X[(long)o * so + (long)k * sk] : (uint16_t)0;
}

__device__ __forceinline__ uint4 pack8(const uint16_t (&e)[8]) {
  uint4 v;
  v.x = e[0] | ((uint32_t)e[1] << 16); v.y = e[2] | ((uint32_t)e[3] << 16);
  v.z = e[4] | ((uint32_t)e[5] << 16); v.w = e[6] | ((uint32_t)e[7] << 16);
  return v;
}

// A thread's share of a TM x GK operand tile (TM = 64 or 128 rows of the outer
// index o = m or n): NU units of eight elements.  Unit u = tid + 256 q is,
// for KVEC, row u / 4 and depths (u % 4) * 8 .. +7; for OVEC, depth u % GK
// and rows (u / GK) * 8 .. +7 (depth fastest across lanes: the transposing
// 2-byte LDS stores of 32 lanes then fall in consecutive words instead of two
// banks); for SCALAR, the elements tid + 256 (8 q + j), j < 8, of the
// row-major TM x GK tile.
template <int TM>
struct Stage {
  static constexpr int NU = TM / 64;
  uint4 v[NU];
};

template <int TM, int mode>
__device__ __forceinline__ void stage_load(Stage<TM> &st, const uint16_t *X, long so, long sk, int o0, int k0,
                                           int no, int ke, int tid) {
#pragma unroll
  for (int q = 0; q < Stage<TM>::NU; q++) {
    const int u = tid + 256 * q;
    uint16_t e[8];
    if constexpr (mode == LD_KVEC) {
      const int o = o0 + (u >> 2), k = k0 + (u & 3) * 8;
      if (o < no && k + 8 <= ke) {
        st.v[q] = *(const uint4 *)(X + (long)o * so + k);
        continue;
      }
#pragma unroll
      for (int j = 0; j < 8; j++) e[j] = ld1(X, so, sk, o, k + j, no, ke);
    } else if constexpr (mode == LD_OVEC) {
      const int k = k0 + u % GK, o = o0 + (u / GK) * 8;
      if (k < ke && o + 8 <= no) {
        st.v[q] = *(const uint4 *)(X + (long)k * sk + o);
        continue;
      }
#pragma unroll
      for (int j = 0; j < 8; j++) e[j] = ld1(X, so, sk, o + j, k, no, ke);
    } else {
      // element idx = tid + 256 (8 q + j) of the row-major TM x GK tile
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int idx = tid + 256 * (8 * q + j);
        e[j] = ld1(X, so, sk, o0 + idx / GK, k0 + idx % GK, no, ke);
      }
    }
    st.v[q] = pack8(e);
  }
}

// sX[o][k] (pitch GP) from a thread's staged units
template <int TM, int mode>
__device__ __forceinline__ void stage_store(const Stage<TM> &st, uint16_t *sX, int tid) {
#pragma unroll
  for (int q = 0; q < Stage<TM>::NU; q++) {
    const int u = tid + 256 * q;
    if constexpr (mode == LD_KVEC) {
      *(uint4 *)(sX + (u >> 2) * GP + (u & 3) * 8) = st.v[q];
      continue;
    }
    const uint4 v = st.v[q];
    const uint16_t e[8] = {(uint16_t)v.x, (uint16_t)(v.x >> 16), (uint16_t)v.y, (uint16_t)(v.y >> 16),
                           (uint16_t)v.z, (uint16_t)(v.z >> 16), (uint16_t)v.w, (uint16_t)(v.w >> 16)};
    if constexpr (mode == LD_OVEC) {
      const int k = u % GK, o = (u / GK) * 8;
#pragma unroll
      for (int j = 0; j < 8; j++) sX[(o + j) * GP + k] = e[j];
    } else {
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int idx = tid + 256 * (8 * q + j);
        sX[(idx / GK) * GP + idx % GK] = e[j];
      }
    }
  }
}

// A 256-thread block owns a TM x TM tile of C (TM = 64 or 128; each wave a
// TM/2 x TM/2 quarter as 2 x 2 MFMA tiles of 16 x 16 or 32 x 32).  Depth steps of
// GK are staged through two LDS buffers: the global loads of step s+1 are in
// flight while step s is multiplied, and one barrier per step separates a
// buffer's reads from its next writes.  Split K: block z takes depths
// [z kchunk, (z+1) kchunk) and writes slice z of C.
template <int TM, int AM, int BM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 128 ? 2 : 1, 8))) k_gemm_bf16(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                                   float *__restrict__ C, int M, int N, int K, long sam, long sak,
                                                   long sbk, long sbn, int ldc, int accumulate, int kchunk,
                                                   long cslice) {
  // TM = 64: each wave 2 x 2 MFMA tiles of 16 x 16 (v_mfma_f32_16x16x16_bf16);
  // TM = 128: each wave 2 x 2 tiles of 32 x 32 (v_mfma_f32_32x32x16_bf16: lane l
  // supplies rows or columns l % 32 at depths 8 (l / 32) .. +7)
  constexpr bool BIG = TM == 128;
  constexpr int IT = 2;
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][TM * GP];   // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][TM * GP];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  C += blockIdx.z * cslice;
  const int wr = wv >> 1, wc = wv & 1;
  v4f acc[IT][IT];
  v16f acc32[IT][IT];
#pragma unroll
  for (int i = 0; i < IT; i++)
#pragma unroll
    for (int j = 0; j < IT; j++) {
      if constexpr (BIG) acc32[i][j] = (v16f){0.f};
      else acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
  Stage<TM> sa, sb;
  stage_load<TM, AM>(sa, A, sam, sak, m0, kb, M, ke, tid);
  stage_load<TM, BM>(sb, B, sbn, sbk, n0, kb, N, ke, tid);
  stage_store<TM, AM>(sa, sA[0], tid);
  stage_store<TM, BM>(sb, sB[0], tid);
  __syncthreads();
  const int row = lane & 15, kq = (lane >> 4) * 4;
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    const bool more = k0 + GK < ke;
    if (more) {
      stage_load<TM, AM>(sa, A, sam, sak, m0, k0 + GK, M, ke, tid);
      stage_load<TM, BM>(sb, B, sbn, sbk, n0, k0 + GK, N, ke, tid);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      if constexpr (BIG) {
        const int r32 = lane & 31, k8 = (lane >> 5) * 8;
        v8bf a[IT], b[IT];
#pragma unroll
        for (int i = 0; i < IT; i++) {
          a[i] = *(const v8bf *)(sA[buf] + (wr * 64 + i * 32 + r32) * GP + ks + k8);
          b[i] = *(const v8bf *)(sB[buf] + (wc * 64 + i * 32 + r32) * GP + ks + k8);
        }
#pragma unroll
        for (int i = 0; i < IT; i++)
#pragma unroll
          for (int j = 0; j < IT; j++) acc32[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc32[i][j], 0, 0, 0);
      } else {
        v4s a[IT], b[IT];
#pragma unroll
        for (int i = 0; i < IT; i++) {
          a[i] = *(const v4s *)(sA[buf] + (wr * 32 + i * 16 + row) * GP + ks + kq);
          b[i] = *(const v4s *)(sB[buf] + (wc * 32 + i * 16 + row) * GP + ks + kq);
        }
#pragma unroll
        for (int i = 0; i < IT; i++)
#pragma unroll
          for (int j = 0; j < IT; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      stage_store<TM, AM>(sa, sA[buf ^ 1], tid);
      stage_store<TM, BM>(sb, sB[buf ^ 1], tid);
    }
    __syncthreads();
    buf ^= 1;
  }
  if constexpr (BIG) {
    // 32 x 32 D layout: lane l holds column l%32, value 4g+t at row 8g + 4(l/32) + t
    const int col = lane & 31, rh = (lane >> 5) * 4;
#pragma unroll
    for (int i = 0; i < IT; i++)
#pragma unroll
      for (int j = 0; j < IT; j++)
#pragma unroll
        for (int v = 0; v < 16; v++) {
          const int gm = m0 + wr * 64 + i * 32 + 8 * (v >> 2) + rh + (v & 3), gn = n0 + wc * 64 + j * 32 + col;
          if (gm < M && gn < N) {
            float *p = &C[(long)gm * ldc + gn];
            *p = accumulate ? *p + acc32[i][j][v] : acc32[i][j][v];
          }
        }
  } else {
    // 16 x 16 D layout: lane l holds column l%16, rows 4*(l/16)+t
    const int col = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < IT; i++)
#pragma unroll
      for (int j = 0; j < IT; j++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int gm = m0 + wr * 32 + i * 16 + rq + t, gn = n0 + wc * 32 + j * 16 + col;
          if (gm < M && gn < N) {
            float *p = &C[(long)gm * ldc + gn];
            *p = accumulate ? *p + acc[i][j][t] : acc[i][j][t];
          }
        }
  }
}

// launch k_gemm_bf16<TM, AM, BM> for the run-time read modes of A and B
template <int TM, int AM>
static void launch_b(int bm, dim3 g, hipStream_t s, const uint16_t *A, const uint16_t *B, float *C, int M, int N,
                     int K, long sam, long sak, long sbk, long sbn, int ldc, int accumulate, int kchunk, long cslice) {
  if (bm == LD_KVEC)
    hipLaunchKernelGGL((k_gemm_bf16<TM, AM, LD_KVEC>), g, dim3(256), 0, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc,
                       accumulate, kchunk, cslice);
  else if (bm == LD_OVEC)
    hipLaunchKernelGGL((k_gemm_bf16<TM, AM, LD_OVEC>), g, dim3(256), 0, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc,
                       accumulate, kchunk, cslice);
  else
    hipLaunchKernelGGL((k_gemm_bf16<TM, AM, LD_SCALAR>), g, dim3(256), 0, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc,
                       accumulate, kchunk, cslice);
}

template <int TM>
static void launch_gemm(int am, int bm, dim3 g, hipStream_t s, const uint16_t *A, const uint16_t *B, float *C, int M,
                        int N, int K, long sam, long sak, long sbk, long sbn, int ldc, int accumulate, int kchunk,
                        long cslice) {
  if (am == LD_KVEC) launch_b<TM, LD_KVEC>(bm, g, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, kchunk, cslice);
  else if (am == LD_OVEC) launch_b<TM, LD_OVEC>(bm, g, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, kchunk, cslice);
  else launch_b<TM, LD_SCALAR>(bm, g, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, kchunk, cslice);
}

// read mode of an operand with outer stride so and depth stride sk
static int ld_mode(const uint16_t *X, long so, long sk) {
  const bool al = ((uintptr_t)X & 15) == 0;
  if (al && sk == 1 && so % 8 == 0) return LD_KVEC;
  if (al && so == 1 && sk % 8 == 0) return LD_OVEC;
  return LD_SCALAR;
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z += b (per column); H = GELU(Z) in BF16 (act != 0) or Y = Z (output layer)
__global__ void k_bias_act(float *__restrict__ Z, const float *__restrict__ b, uint16_t *__restrict__ H, int M,
                           int N, int act) {
  const long n = (long)M * N;
  // the column by 32-bit arithmetic where the index fits (a 64-bit remainder
  // is a long instruction sequence)
  const bool i32 = n <= 0x7fffffffL;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int col = i32 ? (int)((unsigned)i % (unsigned)N) : (int)(i % N);
    const float z = Z[i] + b[col];
    Z[i] = z;
    if (act) H[i] = f2bf(gelu(z));
  }
}

// dZ = dH * GELU'(Z) in BF16, fused with the partial column sums of dZ (FP32)
// that the bias gradient needs: block (x, y) takes columns 64 x .. 64 x + 63
// of rows y R .. y R + R - 1 (R = ceil(M / gridDim.y)) with 16 waves; wave w
// takes rows w, w + 16, ... of the slice, and the 16 wave sums are added in
// wave order into part[y][n] (a fixed order).  k_splitk_sum then adds the
// slices in order.
constexpr int GB_WAVES = 16;
__global__ void __launch_bounds__(64 * GB_WAVES) k_gelu_bwd_colsum(const float *__restrict__ dH,
                                                                   const float *__restrict__ Z,
                                                                   uint16_t *__restrict__ dZb,
                                                                   float *__restrict__ part, int M, int N) {
  __shared__ float red[GB_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const int R = (M + gridDim.y - 1) / gridDim.y, r0 = blockIdx.y * R, r1 = min(M, r0 + R);
  float sum = 0.f;
  if (n < N) {
#pragma unroll 4
    for (int m = r0 + wv; m < r1; m += GB_WAVES) {
      const long i = (long)m * N + n;
      const float d = dH[i] * gelu_d(Z[i]);
      dZb[i] = f2bf(d);
      sum += d;
    }
  }
  red[wv][lane] = sum;
  __syncthreads();
  if (wv == 0 && n < N) {
    float t = 0.f;
    for (int w = 0; w < GB_WAVES; w++) t += red[w][lane];
    part[(long)blockIdx.y * N + n] = t;
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

// loss = sum of the block partials / n: one wave, lane l adds partials l, l + 64,
// ...; the lane sums are then added in lane order by lane 0 from LDS (fixed order)
__global__ void k_sum_parts(const double *__restrict__ part, int nparts, long n, float *__restrict__ out) {
  __shared__ double red[64];
  const int l = threadIdx.x;
  double s = 0;
  for (int i = l; i < nparts; i += 64) s += part[i];
  red[l] = s;
  __syncthreads();
  if (l == 0) {
    double t = 0;
    for (int i = 0; i < 64; i++) t += red[i];
    *out = (float)(t / (double)n);
  }
}

// Partial column sums of dZ[M][N]: block (x, y) adds rows y R .. y R + R - 1
// of columns 64 x .. 64 x + 63 (R = ceil(M / gridDim.y)); wave w takes rows
// w, w + 4, ... of the slice in two interleaved sums, and the four wave sums
// are added in wave order into part[y][n] (a fixed order: the result does not
// depend on timing).  k_splitk_sum then adds the slices in order.
__global__ void __launch_bounds__(256) k_colsum_part(const float *__restrict__ dZ, float *__restrict__ part, int M,
                                                     int N) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const int R = (M + gridDim.y - 1) / gridDim.y, r0 = blockIdx.y * R, r1 = min(M, r0 + R);
  float s0 = 0.f, s1 = 0.f;
  if (n < N) {
    int m = r0 + wv;
#pragma unroll 4
    for (; m + 4 < r1; m += 8) {
      s0 += dZ[(long)m * N + n];
      s1 += dZ[(long)(m + 4) * N + n];
    }
    for (; m < r1; m += 4) s0 += dZ[(long)m * N + n];
  }
  red[wv][lane] = s0 + s1;
  __syncthreads();
  if (wv == 0 && n < N) part[(long)blockIdx.y * N + n] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// C[m][n] (ldc) (+)= sum over z of P[z][m][n] (slices of M x N), in z order;
// the loads of sixteen slices are issued before their adds
__global__ void k_splitk_sum(const float *__restrict__ P, float *__restrict__ C, int M, int N, int S, int ldc,
                             int accumulate) {
  const long mn = (long)M * N;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < mn; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z0 = 0; z0 < S; z0 += 16) {
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; j++) v[j] = z0 + j < S ? P[(z0 + j) * mn + i] : 0.f;
#pragma unroll
      for (int j = 0; j < 16; j++)
        if (z0 + j < S) s += v[j];
    }
    const long o = ldc == N ? i : (i / N) * ldc + i % N;
    C[o] = accumulate ? C[o] + s : s;
  }
}

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

// AdamW on the fp32 master parameters; refresh the BF16 weight copies
__global__ void k_adamw(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ g, long n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2, const long *__restrict__ wmap, uint16_t *__restrict__ wb,
                        const long *__restrict__ wmapT, uint16_t *__restrict__ wbT) {
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
    if (w >= 0) {
      const uint16_t b = f2bf(pi);
      wb[w] = b;
      wbT[wmapT[i]] = b;
    }
  }
}

// --------------------------------------------------------------------------
hipError_t mlp_gemm(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, long sam, long sak,
                    long sbk, long sbn, int ldc, int accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  const int am = ld_mode(A, sam, sak), bm = ld_mode(B, sbn, sbk);
  // 128 x 128 tiles where they still give at least one block per CU
  if ((long)((M + 127) / 128) * ((N + 127) / 128) >= 256) {
    dim3 g((N + 127) / 128, (M + 127) / 128);
    launch_gemm<128>(am, bm, g, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, K, 0L);
  } else {
    dim3 g((N + GT - 1) / GT, (M + GT - 1) / GT);
    launch_gemm<GT>(am, bm, g, s, A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, accumulate, K, 0L);
  }
  return hipGetLastError();
}

static int blocks_for(long n);

int mlp_splitk_slices(int M, int N, int K) {
  const int tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  if (tiles >= 64 || K < 512) return 1;
  int S = 512 / tiles;
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
  launch_gemm<GT>(ld_mode(A, sam, sak), ld_mode(B, sbn, sbk), g, s, A, B, partial, M, N, K, sam, sak, sbk, sbn, N, 0, kc,
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

hipError_t mlp_gelu_bwd_colsum(const float *dH, const float *Z, uint16_t *dZb, float *db, int M, int N, float *partial,
                               int max_slices, hipStream_t s) {
  // row slices of at least 16 rows (one per wave), at most 64 of them and at
  // most max_slices (partial holds slices x N floats)
  int S = M / 16;
  if (S > 64) S = 64;
  if (S > max_slices) S = max_slices;
  if (S < 1) S = 1;
  hipLaunchKernelGGL(k_gelu_bwd_colsum, dim3((N + 63) / 64, S), dim3(64 * GB_WAVES), 0, s, dH, Z, dZb, partial, M, N);
  hipLaunchKernelGGL(k_splitk_sum, dim3(blocks_for(N)), dim3(256), 0, s, partial, db, 1, N, S, N, 0);
  return hipGetLastError();
}

hipError_t mlp_mse(const float *Y, const float *T, uint16_t *dYb, float *dYf, double *part, long n, float *loss,
                   hipStream_t s) {
  const int nb = MLP_LOSS_PARTS;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, Y, T, dYb, dYf, part, n);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, nb, n, loss);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float *dZ, float *db, int M, int N, float *partial, hipStream_t s) {
  // row slices of at least 64 rows, at most MLP_SPLITK_MAX of them (partial holds slices x N)
  int S = M / 64;
  if (S > MLP_SPLITK_MAX) S = MLP_SPLITK_MAX;
  if (S < 1) S = 1;
  hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, S), dim3(256), 0, s, dZ, partial, M, N);
  hipLaunchKernelGGL(k_splitk_sum, dim3(blocks_for(N)), dim3(256), 0, s, partial, db, 1, N, S, N, 0);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t mlp_adamw(float *p, float *m, float *v, const float *g, long n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, const long *wmap, uint16_t *wb, const long *wmapT,
                     uint16_t *wbT, hipStream_t s) {
  hipLaunchKernelGGL(k_adamw, dim3(blocks_for(n)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, wd, c1, c2, wmap, wb,
                     wmapT, wbT);
  return hipGetLastError();
}

}  // namespace fdlb
