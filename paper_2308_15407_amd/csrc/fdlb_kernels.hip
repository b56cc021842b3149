// fdlb_kernels.hip -- gfx950 kernels of one FDLB stage (Sec. III.B).
//
// A stage is two launches over a flat block map that may span many cases:
//   k_table  : per cell (16-cell tiles; 8 on small maps): moments of the stage input from the
//              partial raw sums, closure (eq:chi, eq:viscosity, eq:tau,
//              eq:prandtl), 6th-order gradients (Sec. III.B.3), the
//              Shakhov/J1 polynomial (eq:j0, eq:j1) and its per-axis lattice
//              projections (eq:hh_gk, eq:H_gk) written as tables n X_a[kx] and
//              YZ_a[ky,kz]; two extra blocks per case reduce the incoming wall
//              fluxes into the wall densities (impenetrability, Sec. III.B).
//   k_update : per (63-cell tile, kx chunk): each wave takes a contiguous
//              range of velocity rows (whole y-lines with body force), lanes
//              along cells (coalesced f[kappa][cell]); each
//              lane reconstructs one face by WENO-5 (eq:weno5_flux_x ..
//              eq:weno5_sigma) and takes its right neighbour's face by a lane
//              shuffle, adds the body force (eq:kernel_H) and the relaxation to
//              the target, applies the RK3 combination (eq:rk3) and
//              accumulates the FP64 raw moment sums of its output, reduced
//              across the block's waves in LDS into per-chunk partials.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fdlb_common.h"
#include "fdlb_host.h"

namespace fdlb {

// Pointers held in CaseDev are plain device addresses; casting them to the
// global address space lets the compiler emit global (not flat) memory
// instructions with a uniform base and 32-bit lane offsets.
#define GAS __attribute__((address_space(1)))
// constant address space: read-only for the whole kernel, so uniform
// addresses are read with scalar loads
#define CAS __attribute__((address_space(4)))
template <bool B>
struct BoolC { static constexpr bool value = B; };
template <int N>
struct IntC { static constexpr int value = N; };

template <typename T>
__device__ __forceinline__ GAS T *gp(void *p) { return (GAS T *)p; }
template <typename T>
__device__ __forceinline__ const GAS T *gp(const void *p) { return (const GAS T *)p; }
// element at a 32-bit byte offset from a (uniform) row base: lets the compiler
// use scalar-base + 32-bit vector-offset addressing
template <typename T>
__device__ __forceinline__ T ldb(const GAS T *row, unsigned bytes) {
  return *(const GAS T *)((const GAS char *)row + bytes);
}
// the same through the constant address space, for data the kernel only reads
// (its reads are free to move ahead of the kernel's global stores)
template <typename T>
__device__ __forceinline__ T ldc(const CAS T *row, unsigned bytes) {
  return *(const CAS T *)((const CAS char *)row + bytes);
}
template <typename T>
__device__ __forceinline__ void stb(GAS T *row, unsigned bytes, T v) {
  *(GAS T *)((GAS char *)row + bytes) = v;
}
// raw buffer access to one row of `bytes` bytes: the base stays in scalar
// registers, lanes supply 32-bit byte offsets, and accesses outside the row
// read zero / are dropped by the hardware range check
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const GAS void *row, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, (int)bytes, 0x00020000);
}
// off: the lane's byte offset; soff: a wave-uniform byte offset (a row)
template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, unsigned off, int soff = 0) {
  if constexpr (sizeof(T) == 8) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const v2i v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, soff, 0);
    return __builtin_bit_cast(T, v);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, soff, 0));
  }
}
template <typename T>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned off, T v) {
  if constexpr (sizeof(T) == 8) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, (int)off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)off, 0, 0);
  }
}
template <typename T>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned off, int soff, T v) {
  if constexpr (sizeof(T) == 8) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, (int)off, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)off, soff, 0);
  }
}
// value of lane + 1 (lane 63 receives 0): a wave-wide DPP shift
template <typename T>
__device__ __forceinline__ T shift_down1(T v) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned)lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
  }
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// epsilon-free WENO-5 face value in the upwind frame (eq:weno5_flux_x,
// eq:weno5_omega_x, eq:weno5_sigma).  mode 0: three candidates, 1: candidate
// 3 unavailable, 2: candidate 1 only.  The weights d_q / b_q^2 are evaluated
// as d_q prod_{r != q} b_r^2 (division free); in FP32 the indicators are first
// scaled by the largest one to keep the products in range.  Vanishing
// indicators are handled directly: the candidates with b_q = 0 share the
// weight in proportion to d_q (all zero: ideal weights).
template <typename T>
__device__ __forceinline__ T weno_face(const T v0, const T v1, const T v2, const T v3, const T v4, int mode) {
  const T F1 = v0 * (T)(1.0 / 3.0) - v1 * (T)(7.0 / 6.0) + v2 * (T)(11.0 / 6.0);
  const T F2 = -v1 * (T)(1.0 / 6.0) + v2 * (T)(5.0 / 6.0) + v3 * (T)(1.0 / 3.0);
  const T F3 = v2 * (T)(1.0 / 3.0) + v3 * (T)(5.0 / 6.0) - v4 * (T)(1.0 / 6.0);
  const T a1 = v0 - (T)2 * v1 + v2, c1 = v0 - (T)4 * v1 + (T)3 * v2;
  const T a2 = v1 - (T)2 * v2 + v3, c2 = v1 - v3;
  const T a3 = v2 - (T)2 * v3 + v4, c3 = (T)3 * v2 - (T)4 * v3 + v4;
  T b1 = (T)(13.0 / 12.0) * a1 * a1 + (T)0.25 * c1 * c1;
  T b2 = (T)(13.0 / 12.0) * a2 * a2 + (T)0.25 * c2 * c2;
  T b3 = (T)(13.0 / 12.0) * a3 * a3 + (T)0.25 * c3 * c3;
  const bool drop3 = (mode == 1);
  const T d3 = drop3 ? (T)0 : (T)0.3;
  if (drop3) b3 = (T)1;
  if (sizeof(T) == 4) {
    // scale into [0, 1]; the tiny offset keeps bmax = 0 finite (all b stay 0)
    const T bmax = fmax(fmax(b1, b2), drop3 ? b2 : b3);
    const T r = fast_rcp(bmax + (T)1e-30f);
    b1 *= r; b2 *= r;
    if (!drop3) b3 *= r;
  }
  const T p12 = b1 * b2, p13 = b1 * b3, p23 = b2 * b3;
  T w1 = (T)0.1 * p23 * p23, w2 = (T)0.6 * p13 * p13, w3 = d3 * p12 * p12;
  T ws = w1 + w2 + w3;
  // smallest normal number of T: below it the reciprocal of ws is not finite
  const T tiny = sizeof(T) == 4 ? (T)1.17549435e-38f : (T)2.2250738585072014e-308;
  if (!(ws >= tiny)) {
    // two or more indicators vanish (or the products underflow)
    const bool z1 = b1 == (T)0, z2 = b2 == (T)0, z3 = !drop3 && b3 == (T)0;
    if (z1 || z2 || z3) {
      w1 = z1 ? (T)0.1 : (T)0; w2 = z2 ? (T)0.6 : (T)0; w3 = z3 ? d3 : (T)0;
    } else {
      const bool m1 = b1 <= b2 && (drop3 || b1 <= b3);
      const bool m2 = !m1 && (drop3 || b2 <= b3);
      w1 = m1 ? (T)1 : (T)0; w2 = m2 ? (T)1 : (T)0; w3 = (!m1 && !m2) ? (T)1 : (T)0;
    }
    ws = w1 + w2 + w3;
  }
  const T r = (w1 * F1 + w2 * F2 + w3 * F3) * fast_rcp(ws);
  return (mode == 2) ? F1 : r;
}

// Face value for interior faces (all three candidates, no ghosts), written
// in the first differences e_k = v_{k+1} - v_k of the stencil: every
// candidate is v2 plus a combination of them, and so is every second
// difference in the indicators, so the face is v2 plus the weighted mean of
// the candidates' increments.  The indicators are taken as (12/13) beta_q =
// a_q^2 + (3/13) c_q^2 (a common factor, which the normalisation removes),
// scaled into [0, 1] and offset by 1e-30 (FP64) or 1e-9 (FP32), so the
// weight products neither vanish nor underflow (1e-36 > FLT_MIN) and no
// branch is needed: a candidate whose indicator is below the offset times the
// largest is weighted as if it were that fraction of it.  Where indicators
// vanish, the weights then follow the zero-set rule of weno_face to a relative
// 1e-60 (FP64) or 1e-18 (FP32) of the surviving ones.  The ideal weights d_q
// are folded into the increments (G_q = d_q (F_q - v2)) and into the
// normalising sum.
template <typename T>
__device__ __forceinline__ T weno_face_interior(const T v0, const T v1, const T v2, const T v3, const T v4) {
  constexpr T off = sizeof(T) == 4 ? (T)1e-9f : (T)1e-30;
  constexpr T tiny = sizeof(T) == 4 ? (T)1e-30f : (T)1e-300;
  const T e0 = v1 - v0, e1 = v2 - v1, e2 = v3 - v2, e3 = v4 - v3;
  const T a1 = e1 - e0, a2 = e2 - e1, a3 = e3 - e2;
  // c_q up to sign: v0 - 4 v1 + 3 v2, v1 - v3, 3 v2 - 4 v3 + v4
  const T c1 = e0 - (T)3 * e1, c2 = e1 + e2, c3 = e3 - (T)3 * e2;
  T b1 = a1 * a1 + (T)(3.0 / 13.0) * (c1 * c1);
  T b2 = a2 * a2 + (T)(3.0 / 13.0) * (c2 * c2);
  T b3 = a3 * a3 + (T)(3.0 / 13.0) * (c3 * c3);
  const T r = fast_rcp(fmax(fmax(b1, b2), b3) + tiny);
  b1 = b1 * r + off; b2 = b2 * r + off; b3 = b3 * r + off;
  const T p12 = b1 * b2, p13 = b1 * b3, p23 = b2 * b3;
  const T w1 = p23 * p23, w2 = p13 * p13, w3 = p12 * p12;
  // d_q (F_q - v2): F1 - v2 = (5 e1 - 2 e0)/6, F2 - v2 = (e1 + 2 e2)/6, F3 - v2 = (4 e2 - e3)/6
  const T G1 = e1 * (T)(0.5 / 6.0) - e0 * (T)(0.2 / 6.0);
  const T G2 = e1 * (T)(0.6 / 6.0) + e2 * (T)(1.2 / 6.0);
  const T G3 = e2 * (T)(1.2 / 6.0) - e3 * (T)(0.3 / 6.0);
  const T num = w1 * G1 + w2 * G2 + w3 * G3;
  const T den = (T)0.1 * w1 + (T)0.6 * w2 + (T)0.3 * w3;
  return v2 + num * fast_rcp(den);
}

__device__ __forceinline__ double chi_cs(double eta) {
  const double om = 1.0 - eta;
  return 0.5 * (2.0 - eta) / (om * om * om);
}

// ---------------------------------------------------------------------------
// table pass
// ---------------------------------------------------------------------------
// Wall density n_w of one wall from the stage input g (impenetrability: the
// numerical mass flux through the wall face vanishes).  Incoming populations
// reach the face through the fully interior third-order candidate; emitted
// ones carry n_w g^w.  The first 256 threads of the block take part, with the
// same summation order for any block width, so 256- and 512-thread table
// blocks give the same bits.
template <typename T>
__device__ void wall_block(const CaseDev &c, int wall, int gin) {
  __shared__ double red[256];
  const T *g = (const T *)c.f[sizeof(T) == 4 ? 1 : 0][gin];
  const int nx = c.nx, qh = c.qh, qyz = c.qyz;
  const int tid = threadIdx.x;
  double acc = 0;
  const int n_in = qh * qyz;
  if (tid < 256) {
    for (int t = tid; t < n_in; t += 256) {
      const int kx = (wall == 0 ? qh : 0) + t / qyz;
      const int kap = kx * qyz + t % qyz;
      const double p = c.lat[c.lo.px + kx];
      const T *row = g + (size_t)kap * c.nxp;
      double f0, f1, f2;
      if (wall == 0) { f0 = row[fslot(0)]; f1 = row[fslot(1)]; f2 = row[fslot(2)]; }
      else { f0 = row[fslot(nx - 1)]; f1 = row[fslot(nx - 2)]; f2 = row[fslot(nx - 3)]; }
      // the extrapolation weights sum to one: the background passes through
      const double bgk = sizeof(T) == 4 ? c.lat[c.lo.bg + kap] : 0.0;
      acc += p * (bgk + (f2 * (1.0 / 3.0) - f1 * (7.0 / 6.0) + f0 * (11.0 / 6.0)));
    }
    red[tid] = acc;
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) const_cast<CaseDev &>(c).nw[wall] = (wall == 0 ? -red[0] : red[0]) / c.wallD[wall];
}

// full-range table values Y_b(p_k), b = 0..3, for one node from the Hermite
// coefficients of g(p)(p-u)^b (recurrences in l and b; fixed-size, unrolled)
__device__ __forceinline__ void full_axis_values(double u, double T, int q, const double *__restrict__ H,
                                                 double (&Y)[4]) {
  constexpr int LM = MAXQY + 4;
  double G0[LM], G1[LM], G2[LM], G3[LM];
  G0[0] = 1.0;
  G0[1] = u;
#pragma unroll
  for (int l = 1; l < LM - 1; l++) G0[l + 1] = u * G0[l] + l * (T - 1.0) * G0[l - 1];
#pragma unroll
  for (int l = 0; l < LM - 1; l++) G1[l] = G0[l + 1] + (l > 0 ? l * G0[l - 1] : 0.0) - u * G0[l];
#pragma unroll
  for (int l = 0; l < LM - 2; l++) G2[l] = G1[l + 1] + (l > 0 ? l * G1[l - 1] : 0.0) - u * G1[l];
#pragma unroll
  for (int l = 0; l < LM - 3; l++) G3[l] = G2[l + 1] + (l > 0 ? l * G2[l - 1] : 0.0) - u * G2[l];
  Y[0] = Y[1] = Y[2] = Y[3] = 0.0;
#pragma unroll
  for (int l = 0; l < MAXQY; l++)
    if (l < q) {
      const double h = H[l];
      Y[0] += h * G0[l]; Y[1] += h * G1[l]; Y[2] += h * G2[l]; Y[3] += h * G3[l];
    }
}

// Revised Enskog average density (chi_mode 1 cases; eq:chi_ret and the
// average that follows it, reduced to the slab):
//   nbar_i = 3/(4 sigma^3) sum_j n_j int_{cell j, |x'-x_i| < sigma} (sigma^2 - (x'-x_i)^2) dx',
// with n_j the density of the stage input from the chunk partials (added in
// chunk order, as the table pass does).  One 8-wave block per NBAR_TILE cells:
// the densities and faces of the tile's window go to LDS, then each wave takes
// one cell at a time with its lanes striding over the cell's window.
template <typename T>
__global__ void __launch_bounds__(512) k_nbar(const CaseDev *__restrict__ cases, const int4 *__restrict__ map) {
  // LDS: densities [nwin] and faces [nwin + 1] of the tile's window, and the
  // centre and window range of each cell of the tile
  extern __shared__ double s_n[];
  __shared__ double s_x[NBAR_TILE];
  __shared__ int s_lo[NBAR_TILE], s_hi[NBAR_TILE];
  const int4 bm = map[blockIdx.x];
  const CaseDev &c = cases[max(bm.x, 0)];
  if (bm.x < 0) return;
  const int nx = c.nx, c0 = bm.y * NBAR_TILE, c1 = min(c0 + NBAR_TILE, nx);
  const GAS double *lat = gp<double>(c.lat);
  const int jmin = (int)lat[c.lo.wlo + c0], jmax = (int)lat[c.lo.whi + c1 - 1];
  const int nwin = jmax - jmin + 1, nch = c.nchunk;
  double *s_f = s_n + nwin;
  const double bg0 = sizeof(T) == 4 ? lat[c.lo.bgm] : 0.0;
  const int tid = threadIdx.x;
  if (tid < c1 - c0) {
    s_x[tid] = lat[c.lo.xcn + c0 + tid];
    s_lo[tid] = (int)lat[c.lo.wlo + c0 + tid];
    s_hi[tid] = (int)lat[c.lo.whi + c0 + tid];
  }
  for (int q = tid; q <= nwin; q += blockDim.x) s_f[q] = lat[c.lo.xf + jmin + q];
  // up to PB chunk loads in flight per thread (the chunk count is uniform)
  constexpr int PB = 16;
  for (int q = tid; q < nwin; q += blockDim.x) {
    const GAS double *pp = gp<double>(c.part) + jmin + q;   // raw density row of chunk 0
    double a = 0.0;
    for (int ch0 = 0; ch0 < nch; ch0 += PB) {
      double v[PB];
#pragma unroll
      for (int k = 0; k < PB; k++)
        if (ch0 + k < nch) v[k] = pp[(size_t)(ch0 + k) * NRAW * nx];
#pragma unroll
      for (int k = 0; k < PB; k++)
        if (ch0 + k < nch) a += v[k];
    }
    s_n[q] = a + bg0;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const double sg = c.sigma, s2 = sg * sg;
  for (int i = c0 + wv; i < c1; i += nwv) {
    const double x = s_x[i - c0];
    const int lo = s_lo[i - c0] - jmin, hi = s_hi[i - c0] - jmin;
    double acc = 0.0;
    for (int q = lo + lane; q <= hi; q += 64) {
      const double a = fmax(s_f[q], x - sg) - x, b = fmin(s_f[q + 1], x + sg) - x;
      acc += s_n[q] * ((s2 * b - b * b * b / 3.0) - (s2 * a - a * a * a / 3.0));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) c.nbar[i] = 3.0 / (4.0 * sg * s2) * acc;
  }
}

// WIDE = false serves half-range orders up to MAXQH with an NB-node base rule
// and the Lagrange rows in LDS; WIDE = true serves the orders above (up to
// MAXQH_WIDE) with an NB_WIDE-node base rule and the rows read from global
// memory.  Both run on the same launch map; each skips the other's cases, and
// the wall blocks of every case belong to the standard instantiation.
template <typename T, int NT, bool WIDE, int TS>
__global__ void __launch_bounds__(NT) k_table(const CaseDev *__restrict__ cases, const int4 *__restrict__ map,
                                               int mode, int gin) {
  // launch maps list only active cases; padding entries have bm.x < 0
  const int4 bm = map[blockIdx.x];
  const CaseDev &c = cases[max(bm.x, 0)];
  if (bm.x < 0) return;
  if (bm.y < 0) {
    if (!WIDE && (mode & TM_WALLS)) wall_block<T>(c, -bm.y - 1, gin);
    return;
  }
  if ((c.wide != 0) != WIDE) return;
  constexpr int NBX = WIDE ? NB_WIDE : NB;   // base rule nodes
  constexpr int W = TS + 2 * CHALO;
  __shared__ double s_m[6][W];      // n, ux, uy, T, qx, qy
  __shared__ double s_l[3][W];      // ln n, ln chi, ln T
  __shared__ double s_chi[W];       // contact value chi
  __shared__ double s_c[TS][20]; // n, ux, uy, T, invtau, C[13]
  // the raw sums of the tile and its halo first, then the base weights G
  // (rows padded by one double so that lanes reading different cells or
  // nodes fall in different banks)
  static_assert(NRAW * W <= 256, "one thread per raw moment and cell of the tile and halo");
  constexpr int SCR = NRAW * W > TS * 2 * (NBX + 1) ? NRAW * W : TS * 2 * (NBX + 1);
  __shared__ double s_scr[SCR];
  double (*s_G)[2][NBX + 1] = reinterpret_cast<double (*)[2][NBX + 1]>(s_scr);
  __shared__ double s_red[NT];
  // full-range z-axis values Z_0, Z_2 per owned cell and node (they depend on T only)
  __shared__ double s_Z[TS][MAXQY][2];
  // lattice constants, staged by one linear copy of their contiguous block
  // [p_x (2 qh) | P_m | A_m | h_Q(P_m) | lambda (qh rows of NB) | c_k (qh) | H_y | H_z];
  // the lambda rows are padded by one double in LDS (bank spread); the wide
  // instantiation leaves them in global memory and stages the rest
  constexpr int NCST = WIDE ? 3 * MAXQH_WIDE + 3 * NBX + 2 * MAXQY * MAXQY
                            : 2 * MAXQH + 3 * NB + MAXQH * (NB + 1) + MAXQH + 2 * MAXQY * MAXQY;
  __shared__ double s_cst[NCST];
  const int nx = c.nx, c0 = bm.y * TS;
  const int own = min(TS, nx - c0);
  const int tid = threadIdx.x;
  const double *lat = c.lat;
  const LatOff lo = c.lo;
  const int qh = c.qh, qy = c.qy, qz = c.qz;

  // Every global read of the kernel is issued first so that the latencies
  // overlap: the lattice constants (one contiguous block: p_x, the base
  // nodes, lambda, c_k, H_y, H_z), the metric and wall FD weights of the
  // owned cells, the average density (revised Enskog cases) and the chunk
  // partials of the tile and its halo.  Three phases follow: moments;
  // closure (first wave) beside the base weights (other waves); the X and YZ
  // tables.
  const GAS double *glat = gp<double>(lat);
  constexpr int CB = 2048 / NT;
  static_assert(CB * NT >= (WIDE ? 3 * MAXQH_WIDE + 3 * NBX : 3 * MAXQH + 3 * NB + MAXQH * NB) +
                                 2 * MAXQY * MAXQY, "constant staging");
  const int cL0 = 2 * qh + 3 * NBX, cL1 = cL0 + (WIDE ? 0 : qh * NB), ncst = cL1 + qh + qy * qy + qz * qz;
  double cv[CB];
  if (mode & TM_TABLES) {
#pragma unroll
    for (int u = 0; u < CB; u++) {
      const int it = min(tid + u * NT, ncst - 1);
      cv[u] = glat[WIDE && it >= cL0 ? lo.ck + (it - cL0) : lo.px + it];
    }
  }
  const int ci = c0 + tid;
  const double dxi_own = tid < own ? gp<double>(c.invdx)[min(ci, nx - 1)] : 0.0;
  double fwv[7];
  {
    const bool wall_cell = tid < own && !(ci >= 3 && ci <= nx - 4);
    const int r = wall_cell ? (ci < 3 ? ci : nx - 1 - ci) : 0;
#pragma unroll
    for (int jj = 0; jj < 7; jj++) fwv[jj] = wall_cell ? glat[lo.fdw + r * 7 + jj] : 0.0;
  }
  double bgs[NRAW];
#pragma unroll
  for (int m = 0; m < NRAW; m++) bgs[m] = sizeof(T) == 4 ? glat[lo.bgm + m] : 0.0;
  // revised Enskog cases: chi takes the average density of the stage input
  const bool ret = c.chi_mode == 1 && (mode & TM_PARTIALS);
  double nbv = 0.0;
  if (ret && tid < W) nbv = gp<double>(c.nbar)[min(max(c0 - CHALO + tid, 0), nx - 1)];
  // one thread per (raw moment, cell of the tile and halo) adds the chunk
  // partials in chunk order; up to PB chunk loads are in flight at a time
  // (the chunk count is uniform, so the guards are scalar branches)
  constexpr int PB = 16;
  const int pm = tid / W, pw = tid - pm * W, pcell = c0 - CHALO + pw;
  double praw = 0.0;
  if (!(mode & TM_FIELDS) && tid < NRAW * W && pcell >= 0 && pcell < nx) {
    const int nch = c.nchunk;
    const GAS double *pp = gp<double>(c.part) + (size_t)pm * nx + pcell;
    const size_t cstride = (size_t)NRAW * nx;
    for (int ch0 = 0; ch0 < nch; ch0 += PB) {
      double v[PB];
#pragma unroll
      for (int k = 0; k < PB; k++)
        if (ch0 + k < nch) v[k] = pp[(size_t)(ch0 + k) * cstride];
#pragma unroll
      for (int k = 0; k < PB; k++)
        if (ch0 + k < nch) praw += v[k];
    }
  }
  if (mode & TM_TABLES) {
#pragma unroll
    for (int u = 0; u < CB; u++) {
      const int it = tid + u * NT;
      if (it < ncst) {
        const int q = it - cL0;
        const int dst = WIDE ? it : (it < cL0 ? it : (it < cL1 ? cL0 + (q / NB) * (NB + 1) + q % NB : it + qh));
        s_cst[dst] = cv[u];
      }
    }
  }
  if (!(mode & TM_FIELDS) && tid < NRAW * W) s_scr[pm * W + pw] = praw;
  __syncthreads();

  const double *s_px = s_cst, *s_P = s_cst + 2 * qh, *s_A = s_P + NBX, *s_hQ = s_A + NBX;
  const double *s_lam = s_hQ + NBX, *s_ck = WIDE ? s_lam : s_lam + qh * (NB + 1);
  const double *s_Hy = s_ck + qh, *s_Hz = s_Hy + qy * qy;

  // ---- moments of the stage input for the tile and its halo ----
  double rmax = 0;
  if (tid < W) {
    const int cell = c0 - CHALO + tid;
    if (cell >= 0 && cell < nx) {
      double n, ux, uy, T_, qx, qy_, pxx = 0, pxy = 0, pyy = 0, pzz = 0;
      if (mode & TM_FIELDS) {
        const double *fl = c.fields;
        n = fl[cell]; ux = fl[nx + cell]; uy = fl[2 * nx + cell]; T_ = fl[3 * nx + cell];
        qx = fl[4 * nx + cell]; qy_ = fl[5 * nx + cell];   // slot 5 carries P_xy
      } else {
        double S[NRAW];
#pragma unroll
        for (int m = 0; m < NRAW; m++) S[m] = s_scr[m * W + tid];
        if (sizeof(T) == 4) {
          // FP32 storage holds f - bg: add the background's raw sums
#pragma unroll
          for (int m = 0; m < NRAW; m++) S[m] += bgs[m];
        }
        n = S[0];
        ux = S[1] / n; uy = S[2] / n;
        pxx = S[3] - n * ux * ux; pxy = S[4] - n * ux * uy; pyy = S[5] - n * uy * uy; pzz = S[6];
        const double S2 = S[3] + S[5] + S[6], u2 = ux * ux + uy * uy;
        T_ = (pxx + pyy + pzz) / (3.0 * n);
        qx = 0.5 * (S[7] - 2.0 * (ux * S[3] + uy * S[4]) - ux * S2 + 2.0 * n * ux * u2);
        qy_ = 0.5 * (S[8] - 2.0 * (ux * S[4] + uy * S[5]) - uy * S2 + 2.0 * n * uy * u2);
      }
      s_m[0][tid] = n; s_m[1][tid] = ux; s_m[2][tid] = uy; s_m[3][tid] = T_; s_m[4][tid] = qx; s_m[5][tid] = qy_;
      const double chi = chi_cs(c.eta0 * (ret ? nbv : n));
      s_chi[tid] = chi;
      s_l[0][tid] = log(n); s_l[1][tid] = log(chi); s_l[2][tid] = log(T_);
      const bool owned = tid >= CHALO && tid < CHALO + own;
      if (owned && (mode & TM_RESID)) {
        const double *mo = c.mom;
        const double dn = fabs(n - mo[cell]), dux = fabs(ux - mo[nx + cell]);
        const double duy = fabs(uy - mo[2 * nx + cell]), dT = fabs(T_ - mo[3 * nx + cell]);
        double r = fmax(fmax(dn, dux), fmax(duy, dT)) / c.dt;
        if (!(n > 0.0) || !(T_ > 0.0) || !isfinite(r) || !isfinite(qx) || !isfinite(qy_))
          r = __longlong_as_double(0x7ff8000000000000LL);
        rmax = r;
      }
      if (owned && (mode & TM_WRITE_MOM)) {
        double *mo = c.mom;
        mo[cell] = n; mo[nx + cell] = ux; mo[2 * nx + cell] = uy; mo[3 * nx + cell] = T_;
        mo[4 * nx + cell] = qx; mo[5 * nx + cell] = qy_; mo[6 * nx + cell] = pxx;
        mo[7 * nx + cell] = pxy; mo[8 * nx + cell] = pyy; mo[9 * nx + cell] = pzz;
      }
    }
  }
  if (mode & TM_RESID) {
    s_red[tid] = rmax;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double a = s_red[tid], b = s_red[tid + s];
        s_red[tid] = (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000LL) : fmax(a, b);
      }
      __syncthreads();
    }
    if (tid == 0) atomicMax(c.resid, (unsigned long long)__double_as_longlong(s_red[0]));
  }
  if (!(mode & TM_TABLES)) return;
  __syncthreads();

  // ---- closure, gradients and the target polynomial per owned cell ----
  if (tid < own) {
    const int i = c0 + tid, li = tid + CHALO;
    const double n = s_m[0][li], ux = s_m[1][li], uy = s_m[2][li], T_ = s_m[3][li];
    double C[13];
    double itau = 0.0;
#pragma unroll
    for (int q = 0; q < 13; q++) C[q] = 0.0;
    if (mode & TM_FIELDS) {
      // Grad-13-type state: 1 + Pxy xi_x xi_y/(n T^2) + qx xi_x (xi^2/T - 5)/(5 n T^2)
      const double qx = s_m[4][li], pxy = s_m[5][li];
      const double nT2 = n * T_ * T_;
      C[0] = 1.0;
      C[1] = -qx / nT2;
      C[6] = pxy / nT2;
      C[7] = qx / (5.0 * nT2 * T_);
      C[8] = C[7];
      C[9] = C[7];
    } else {
      // gradients d/dx = (d/deta)/J, 6th-order central inside, one-sided at walls
      double g[5];
#pragma unroll
      for (int q = 0; q < 5; q++) {
        const double *src = q == 0 ? s_l[0] : (q == 1 ? s_l[1] : (q == 2 ? s_l[2] : (q == 3 ? s_m[1] : s_m[2])));
        double d;
        if (i >= 3 && i <= nx - 4) {
          d = (src[li + 1] - src[li - 1]) * 0.75 - (src[li + 2] - src[li - 2]) * 0.15 +
              (src[li + 3] - src[li - 3]) * (1.0 / 60.0);
        } else if (i < 3) {
          d = 0;
          for (int jj = 0; jj < 7; jj++) d += fwv[jj] * src[li - i + jj];
        } else {
          const int r = nx - 1 - i;
          d = 0;
          for (int jj = 0; jj < 7; jj++) d -= fwv[jj] * src[li + r - jj];
        }
        g[q] = d * dxi_own;
      }
      const double eta = c.eta0 * n, chi = s_chi[li];
      const double brc = 4.0 * eta * chi;   // b rho chi
      double tau = 0.0;
      if (c.tau_pre > 0.0) {
        tau = c.tau_pre / (n * sqrt(T_)) *
              (1.0 / chi + 3.2 * eta + 64.0 / 25.0 * (1.0 + 12.0 / M_PI) * eta * eta * chi);
        itau = 1.0 / tau;
      }
      double Pr = 1.0;
      if (c.collision == 1) Pr = c.pr_fixed;
      else if (c.collision == 2)
        Pr = 2.0 / 3.0 * (1.0 + 0.8 * brc + 4.0 / 25.0 * (1.0 + 12.0 / M_PI) * brc * brc) /
             (1.0 + 1.2 * brc + 9.0 / 25.0 * (1.0 + 32.0 / (9.0 * M_PI)) * brc * brc);
      const double qx = s_m[4][li], qy_ = s_m[5][li];
      const double s0 = (1.0 - Pr) / (n * T_ * T_);
      const double A = -tau * brc;                  // tau J1 prefactor
      const double D = 2.0 * g[0] + g[1] + g[2];    // d ln(rho^2 chi T)/dx
      const double G = g[2], dux = g[3], duy = g[4];
      const double iT = 1.0 / T_;
      // coefficients of xi_x^a xi_y^b xi_z^c in 1 + S + tau J:
      // 0:000 1:100 2:010 3:200 4:020 5:002 6:110 7:300 8:120 9:102 10:210 11:030 12:012
      C[0] = 1.0 - A * dux;
      C[1] = A * (D - 1.5 * G) - s0 * qx;
      C[2] = -s0 * qy_;
      C[3] = A * 0.6 * dux * iT;
      C[4] = A * 0.2 * dux * iT;
      C[5] = C[4];
      C[6] = A * 0.4 * (c.j1_shear ? duy : 0.0) * iT;
      C[7] = A * 0.3 * G * iT + 0.2 * s0 * qx * iT;
      C[8] = C[7];
      C[9] = C[7];
      C[10] = 0.2 * s0 * qy_ * iT;
      C[11] = C[10];
      C[12] = C[10];
    }
    s_c[tid][0] = n; s_c[tid][1] = ux; s_c[tid][2] = uy; s_c[tid][3] = T_; s_c[tid][4] = itau;
#pragma unroll
    for (int q = 0; q < 13; q++) s_c[tid][5 + q] = C[q];
  } else if (tid >= 64) {
    // ---- half-range base weights per owned cell and half, and the z values
    // per owned cell and node (waves 1..) ----
    static_assert(TS <= 64, "the closure runs on the first wave");
    const int nG = own * 2 * NBX;
    for (int it = tid - 64; it < nG + own * qz; it += NT - 64) {
      if (it < nG) {
        const int cl = it / (2 * NBX), h = (it / NBX) & 1, m = it % NBX;
        const double ux = s_m[1][cl + CHALO], T_ = s_m[3][cl + CHALO];
        const double u = h == 0 ? ux : -ux;
        const double d = s_P[m] - u;
        s_G[cl][h][m] = exp(s_A[m] - d * d / (2.0 * T_)) * rsqrt(T_);
      } else {
        const int cl = (it - nG) % own, kz = (it - nG) / own;
        double Z[4];
        full_axis_values(0.0, s_m[3][cl + CHALO], qz, &s_Hz[kz * qz], Z);
        s_Z[cl][kz][0] = Z[0];
        s_Z[cl][kz][1] = Z[2];
      }
    }
  }
  __syncthreads();

  // ---- n X_a[kx] and YZ_a[ky,kz] tables, one flat item list ----
  // layout [kx][cell][a] and [yz][cell][a]: the four coefficients of a node
  // and cell are adjacent, so a reader takes them with one vector load
  // an X item is one cell and half x a pair of nodes: each base weight read
  // from LDS feeds the two dot products and the three base moments m_0..m_2
  const int nkx = c.nkx, qyz = c.qyz;
  constexpr int P = sizeof(T) == 4 ? 1 : 0;   // storage precision of this instantiation
  T *tX = (T *)c.tabX[P];
  T *tYZ = (T *)c.tabYZ[P];
  typedef T T4 __attribute__((ext_vector_type(4)));
  const int ngrp = (qh + 1) / 2;
  const int nXi = own * 2 * ngrp, nYi = own * qy;
  for (int it = tid; it < nXi + nYi; it += blockDim.x) {
    if (it < nXi) {
      const int cl = it % own, rest = it / own, h = rest & 1, k0 = 2 * (rest >> 1);   // cell fastest
      const double u = h == 0 ? s_c[cl][1] : -s_c[cl][1];
      const double *Gc = s_G[cl][h];
      double x[2] = {0.0, 0.0}, mb[3] = {0.0, 0.0, 0.0};
      if constexpr (WIDE) {
        const GAS double *l0 = glat + lo.lam + k0 * NBX, *l1 = glat + lo.lam + min(k0 + 1, qh - 1) * NBX;
#pragma unroll 8
        for (int m = 0; m < NBX; m++) {
          const double g = Gc[m];
          x[0] += g * l0[m]; x[1] += g * l1[m];
          const double d = s_P[m] - u, hv = s_hQ[m] * g;
          mb[0] += hv; mb[1] += hv * d; mb[2] += hv * d * d;
        }
      } else {
        const double *l0 = s_lam + k0 * (NB + 1), *l1 = s_lam + min(k0 + 1, qh - 1) * (NB + 1);
#pragma unroll 8
        for (int m = 0; m < NB; m++) {
          const double g = Gc[m];
          x[0] += g * l0[m]; x[1] += g * l1[m];
          const double d = s_P[m] - u, hv = s_hQ[m] * g;
          mb[0] += hv; mb[1] += hv * d; mb[2] += hv * d * d;
        }
      }
      const double sg = h ? -1.0 : 1.0, n = s_c[cl][0];
      const size_t i = (size_t)c0 + cl;
#pragma unroll
      for (int j = 0; j < 2; j++) {
        const int k = k0 + j;
        if (k < qh) {
          const int kx = h * qh + k;
          const double x0 = x[j], dk = s_px[k] - u, ck = s_ck[k];
          const double X1 = dk * x0 + ck * mb[0];
          const double X2 = dk * dk * x0 + ck * (dk * mb[0] + mb[1]);
          const double X3 = dk * dk * dk * x0 + ck * (dk * dk * mb[0] + dk * mb[1] + mb[2]);
          // FP32 storage: the a = 0 table is the deviation from the background factor
          T4 xv;
          xv.x = (T)(n * x0 - (sizeof(T) == 4 ? ((const CAS double *)lat)[lo.xbg + kx] : 0.0));
          xv.y = (T)(n * sg * X1);
          xv.z = (T)(n * X2);
          xv.w = (T)(n * sg * X3);
          *(T4 *)(tX + ((size_t)kx * nx + i) * 4) = xv;
        }
      }
    } else {
      // one item per owned cell and y node: Y_b once, then the qz YZ entries
      const int iy = it - nXi;
      const int cl = iy % own, ky = iy / own;
      double Y[4];
      full_axis_values(s_c[cl][2], s_c[cl][3], qy, &s_Hy[ky * qy], Y);
      const double *C = &s_c[cl][5];
      const size_t i = (size_t)c0 + cl;
      for (int kz = 0; kz < qz; kz++) {
        const int yz = ky * qz + kz;
        const double Z0 = s_Z[cl][kz][0], Z2 = s_Z[cl][kz][1];
        const double yz0 = C[0] * Y[0] * Z0 + C[2] * Y[1] * Z0 + C[4] * Y[2] * Z0 + C[11] * Y[3] * Z0 +
                           C[5] * Y[0] * Z2 + C[12] * Y[1] * Z2;
        const double yz1 = C[1] * Y[0] * Z0 + C[6] * Y[1] * Z0 + C[8] * Y[2] * Z0 + C[9] * Y[0] * Z2;
        const double yz2 = C[3] * Y[0] * Z0 + C[10] * Y[1] * Z0;
        const double yz3 = C[7] * Y[0] * Z0;
        T4 yv;
        yv.x = (T)(yz0 - (sizeof(T) == 4 ? ((const CAS double *)lat)[lo.yzbg + yz] : 0.0));
        yv.y = (T)yz1;
        yv.z = (T)yz2;
        yv.w = (T)yz3;
        *(T4 *)(tYZ + ((size_t)yz * nx + i) * 4) = yv;
      }
    }
  }
  if (tid < own) ((T *)c.invtau[P])[c0 + tid] = (T)s_c[tid][4];
}

// ---------------------------------------------------------------------------
// update pass
// ---------------------------------------------------------------------------
// Sum the per-wave raw moment sums of a block into the chunk's partials.
// s_acc: LDS of at least waves * NRAW * 64 doubles.
template <typename T>
__device__ __forceinline__ void block_partials(const CaseDev &c, int chunk, int c0, double (&acc)[NRAW],
                                               bool is_cell, double *s_acc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
#pragma unroll
  for (int m = 0; m < NRAW; m++) s_acc[(wv * NRAW + m) * 64 + lane] = acc[m];
  __syncthreads();
  for (int it = threadIdx.x; it < NRAW * 64; it += blockDim.x) {
    const int m = it / 64, l = it % 64;
    const int cell = c0 + l;
    if (l < UTILE && cell < c.nx) {
      double s = 0;
      for (int w = 0; w < nwv; w++) s += s_acc[(w * NRAW + m) * 64 + l];
      gp<double>(c.part)[((size_t)chunk * NRAW + m) * c.nx + cell] = s;
    }
  }
  (void)is_cell;
}

#ifndef FDLB_UNROLL_F64
#define FDLB_UNROLL_F64 1
#endif
#ifndef FDLB_UNROLL_F32
#define FDLB_UNROLL_F32 2
#endif
#ifndef FDLB_UPDATE_WPE
#define FDLB_UPDATE_WPE 4
#endif
#ifndef FDLB_UPDATE_WPE_F64
#define FDLB_UPDATE_WPE_F64 4
#endif
// body-force blocks hold every read of a y-line at once (qy rows of stencil,
// target and f^n values), so they trade occupancy for registers
#ifndef FDLB_UPDATE_WPE_FORCE
#define FDLB_UPDATE_WPE_FORCE 2
#endif
// depth of the row prefetch ring in interior update tiles
#ifndef FDLB_RING_F64
#define FDLB_RING_F64 4
#endif
#ifndef FDLB_RING_F32
#define FDLB_RING_F32 3
#endif

template <typename T, int STAGE, bool FORCE, int QYC = MAXQY>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FORCE ? FDLB_UPDATE_WPE_FORCE : (sizeof(T) == 8 ? FDLB_UPDATE_WPE_F64 : FDLB_UPDATE_WPE), 8))) k_update(const CaseDev *__restrict__ cases, const int4 *__restrict__ map) {
  extern __shared__ double lds_dyn[];
  // FP32 storage holds the deviation from the case's background populations
  constexpr bool DF = sizeof(T) == 4;
  // launch maps list only active cases; padding entries have bm.x < 0
  const int4 bm = map[blockIdx.x];
  const CaseDev &c = cases[max(bm.x, 0)];
  if (bm.x < 0) return;
  // the wave index is uniform within a wave: keep it (and everything derived
  // from it -- rows, pointers, loop bounds) in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwv = blockDim.x >> 6;
  const int nx = c.nx, qy = c.qy, qz = c.qz, qyz = c.qyz, nkx = c.nkx;
  constexpr int P = sizeof(T) == 4 ? 1 : 0;   // storage precision of this instantiation
  const GAS T *__restrict__ gin = gp<T>(c.f[P][STAGE == 1 ? 0 : (STAGE == 2 ? 1 : 2)]);
  // stage 3 writes f^{n+1} over f^n: each lane reads f^n only at the node it writes
  const GAS T *fn = gp<T>(c.f[P][0]);
  GAS T *out = gp<T>(c.f[P][STAGE == 1 ? 1 : (STAGE == 2 ? 2 : 0)]);
  const GAS T *__restrict__ tX = gp<T>(c.tabX[P]);
  const GAS T *__restrict__ tYZ = gp<T>(c.tabYZ[P]);
  const CAS T *gwL = (const CAS T *)c.gw[P][0];
  const CAS T *gwR = (const CAS T *)c.gw[P][1];
  // the projection tables are written by the table pass and only read here
  const CAS T *ctX = (const CAS T *)c.tabX[P];
  const CAS T *ctYZ = (const CAS T *)c.tabYZ[P];
  const GAS double *__restrict__ lat = gp<double>(c.lat);
  // the same constants through the constant address space: read-only for the
  // kernel, so their (uniform) reads can move ahead of the population stores
  const CAS double *clat = (const CAS double *)c.lat;
  const int c0 = bm.y * UTILE;
  const int j = c0 + lane;                       // face j (left face of cell j)
  const bool is_cell = lane < UTILE && j < nx;
  const int jc = min(j, nx - 1);
  // byte offsets of this lane's cell: in the [.][cell] tables, and as a slot
  // of the population rows (read and write)
  const unsigned bc = (unsigned)jc * (unsigned)sizeof(T);
  const unsigned bcf = (unsigned)fslot(jc) * (unsigned)sizeof(T);
  const unsigned bw = (unsigned)fslot(max(j, 0)) * (unsigned)sizeof(T);
  const int kx0 = bm.z * c.kxc, kx1 = min(kx0 + c.kxc, nkx);
  const double nwl = c.nw[0], nwr = c.nw[1];
  // 1/dx and 1/tau of the lane's cell: without body force they are loaded
  // after the table staging, so that no load is outstanding when the staging
  // loop starts
  T dxi = 0, itau = 0;
  const GAS double *__restrict__ invdx = gp<double>(c.invdx);
  const GAS T *__restrict__ invtau = gp<T>(c.invtau[P]);
  if (FORCE) { dxi = (T)invdx[jc]; itau = invtau[jc]; }
  const T dt = (T)c.dt;
  const size_t tstride = (size_t)nx;             // row stride of the [.][cell] tables
  const size_t fstride = (size_t)c.nxp;          // row stride of the population arrays (slots)
  const int c_qh = c.qh, c_kxc = c.kxc, c_tlds = c.tlds;
  const int lo_px = c.lo.px, lo_py = c.lo.py, lo_pz = c.lo.pz, lo_phi = c.lo.phi, lo_bg = c.lo.bg;
  // Stencil of the lane's face for one upwind direction (pos: p_x > 0): the
  // byte offsets of the five upwind-ordered cells, clamped into the row; the
  // flags of the three that may be ghost cells (only the emitting side of the
  // stencil can reach past a wall); the face's WENO mode (3: wall face).
  // Computed where a path needs it, so that interior tiles keep no registers
  // for it.
  struct Stencil { unsigned o[5]; bool g[3]; int mode; };
  auto stencil = [&](bool pos) {
    Stencil st;
    auto cl = [&](int x) { return (unsigned)fslot(min(max(x, 0), nx - 1)) * (unsigned)sizeof(T); };
    if (pos) {
      const int cp = j - 3;
#pragma unroll
      for (int k = 0; k < 5; k++) st.o[k] = cl(cp + k);
      st.g[0] = cp < 0; st.g[1] = cp + 1 < 0; st.g[2] = cp + 2 < 0;
      st.mode = (j == 0) ? 3 : (j == nx ? 2 : (j == nx - 1 ? 1 : 0));
    } else {
      const int cn = j + 2;
#pragma unroll
      for (int k = 0; k < 5; k++) st.o[k] = cl(cn - k);
      st.g[0] = cn >= nx; st.g[1] = cn - 1 >= nx; st.g[2] = cn - 2 >= nx;
      st.mode = (j == nx) ? 3 : (j == 0 ? 2 : (j == 1 ? 1 : 0));
    }
    return st;
  };
  double acc[NRAW];
#pragma unroll
  for (int m = 0; m < NRAW; m++) acc[m] = 0.0;

  auto finish = [&](int kap, int ky, int kz, double pxd, T cen, T L, T fnv) {
    const T adv1 = cen + dt * L;
    T o;
    if (STAGE == 1) o = adv1;
    else o = (STAGE == 2) ? (T)0.75 * fnv + (T)0.25 * adv1 : fnv * (T)(1.0 / 3.0) + (T)(2.0 / 3.0) * adv1;
    if (is_cell) stb(out + (size_t)kap * fstride, bw, o);
    {
      const double pyd = clat[lo_py + ky], pzd = clat[lo_pz + kz];
      const double p2 = pxd * pxd + pyd * pyd + pzd * pzd;
      const double od = is_cell ? (double)o : 0.0;
      acc[0] += od;
      acc[1] += pxd * od;
      acc[2] += pyd * od;
      acc[3] += (pxd * pxd) * od;
      acc[4] += (pxd * pyd) * od;
      acc[5] += (pyd * pyd) * od;
      acc[6] += (pzd * pzd) * od;
      acc[7] += (pxd * p2) * od;
      acc[8] += (pyd * p2) * od;
    }
  };
  // face value and cell-centre value of one velocity row (row is uniform)
  auto face = [&](const GAS T *row, const Stencil &st, bool pos, T fw, T &cen) -> T {
    // unconditional loads at clamped (always valid) cells, then ghost selects
    const T t0 = ldb(row, st.o[0]), t1 = ldb(row, st.o[1]), t2 = ldb(row, st.o[2]), t3 = ldb(row, st.o[3]),
            t4 = ldb(row, st.o[4]);
    const T v0 = st.g[0] ? fw : t0, v1 = st.g[1] ? fw : t1, v2 = st.g[2] ? fw : t2;
    cen = pos ? t3 : v2;
    const T w = weno_face<T>(v0, v1, v2, t3, t4, st.mode == 3 ? 0 : st.mode);
    return (st.mode == 3) ? fw : w;
  };
  // target of one node; FP32: its deviation from the background (see the row loop)
  typedef T T4 __attribute__((ext_vector_type(4)));
  auto target = [&](int kx, int yz, T X0, T X1, T X2, T X3) -> T {
    const T4 y = ldc((const CAS T4 *)(ctYZ + (size_t)yz * tstride * 4), 4 * bc);
    T F = X0 * y.x + X1 * y.y + X2 * y.z + X3 * y.w;
    if (DF) F += X0 * (T)lat[c.lo.yzbg + yz] + (T)lat[c.lo.xbg + kx] * y.x;
    return F;
  };

  if (!FORCE) {
    // Rows (velocities) of the chunk are split into contiguous ranges per
    // wave, positive-x rows first.  The row loop is unrolled by two with two
    // register sets, so the loads of row r+1 are in flight while row r is
    // computed without copies between the sets.
    const int nrows = (kx1 - kx0) * qyz;
    const int per = (nrows + nwv - 1) / nwv;
    const int r0 = min(wv * per, nrows), r1 = min(r0 + per, nrows);
    const int rsplit = min(max((c_qh - kx0) * qyz, 0), nrows);
    const int kap_base = kx0 * qyz;
    // row r of the chunk is (kl, yz) = (r / qyz, r % qyz): r / qyz as the
    // high word of r * mq with mq = ceil(2^32 / qyz), exact for r < 2^32 / qyz
    const unsigned mq = (unsigned)((((unsigned long long)1 << 32) + (unsigned)qyz - 1u) / (unsigned)qyz);
    const bool tlds = c_tlds != 0;
    typedef T T4 __attribute__((ext_vector_type(4)));
    // LDS tables of the tile, four coefficients a = 0..3 adjacent per lane:
    // sYZ[(yz * 64 + lane) * 4 + a], sX[(kl * 64 + lane) * 4 + a]
    T *sYZ = (T *)lds_dyn, *sX = sYZ + 4 * qyz * 64;
    if (tlds) {
      // table rows 0 .. qyz - 1 are YZ[yz], the rest X[kx], four coefficients
      // per cell each; each wave issues SB row loads (clamped to a valid row)
      // before it writes any of them to LDS, so their latencies overlap
      constexpr int SB = 8;
      const unsigned bj = 4u * (unsigned)min(c0 + lane, nx - 1) * (unsigned)sizeof(T);
      const int nk = kx1 - kx0, nr = qyz + nk;
      for (int base = wv; base < nr; base += SB * nwv) {
        T4 v[SB];
#pragma unroll
        for (int u = 0; u < SB; u++) {
          const int rr = min(base + u * nwv, nr - 1);
          const GAS T *src = rr < qyz ? tYZ + (size_t)rr * tstride * 4 : tX + (size_t)(kx0 + rr - qyz) * tstride * 4;
          v[u] = ldb((const GAS T4 *)src, bj);
        }
#pragma unroll
        for (int u = 0; u < SB; u++) {
          const int rr = base + u * nwv;
          if (rr < qyz) *(T4 *)(sYZ + (rr * 64 + lane) * 4) = v[u];
          else if (rr < nr) *(T4 *)(sX + ((rr - qyz) * 64 + lane) * 4) = v[u];
        }
      }
      __syncthreads();
    }
    dxi = (T)invdx[jc];
    itau = invtau[jc];
    // the RK3 weight of the advanced value (eq:rk3) folded into the lane's
    // factors: o = (1 - ws) f^n + ws cen - (p_x ws dt/dx)(fr - fh) + (ws dt/tau)(F - cen)
    constexpr double WS = STAGE == 1 ? 1.0 : (STAGE == 2 ? 0.25 : 2.0 / 3.0);
    const T adx = (T)WS * dt * dxi, ait = (T)WS * dt * itau;
    // FP32: p_x and the background factors as floats (uniform operands
    // without conversions): fpx[kx], fxb[kx], fyzb[yz]
    const CAS float *fpx = (const CAS float *)(c.lat + c.lo.f32);
    const CAS float *fxb = fpx + 2 * c_qh, *fyzb = fpx + 4 * c_qh;
    const bool interior = c0 >= 3 && c0 + 66 <= nx;
    // interior tiles: per-wave LDS row buffers after the tables.  The row load
    // takes the tile's 64 aligned slots (cells c0 .. c0+62 and the padding
    // slot); a second load brings the halo: cells c0-3 .. c0-1 on lanes 0..2
    // and c0+63 .. c0+65 on lanes 3..5 (other lanes read past the row: zero)
    T *sRow = (tlds ? sX + 4 * c_kxc * 64 : (T *)lds_dyn) + wv * 2 * ROWBUF;
    const unsigned oa = (unsigned)(64 * bm.y + lane) * (unsigned)sizeof(T);
    const unsigned oh = lane < 3 ? (unsigned)fslot(max(c0 - 3 + lane, 0)) * (unsigned)sizeof(T)
                                 : (lane < 6 ? (unsigned)fslot(min(c0 + 60 + lane, nx - 1)) * (unsigned)sizeof(T)
                                             : 0x80000000u);
    const CAS double *__restrict__ phi = (const CAS double *)(c.lat + lo_phi);
    const CAS double *__restrict__ bgc = (const CAS double *)(c.lat + lo_bg);
    const unsigned rowbytes = (unsigned)c.nxp * (unsigned)sizeof(T);
    // one buffer resource per population array over the chunk's rows: a row
    // is a scalar byte offset, a cell the lane's offset (lanes past the
    // chunk's range read zero and store nothing)
    const size_t cbase = (size_t)kap_base * fstride;
    const unsigned cbytes = (unsigned)(kx1 - kx0) * (unsigned)qyz * rowbytes;
    const auto rs_in = rsrc_of(gin + cbase, cbytes);
    const auto rs_fn = rsrc_of(fn + cbase, cbytes);
    const auto rs_out = rsrc_of(out + cbase, cbytes);
    // global loads of a row (stencil of the stage input and f^n) are issued
    // two rows ahead; the tables (LDS, short latency) are read at the start of
    // the row's arithmetic
    struct Row { T t0, t1, t2, t3, t4, fnv; };
    // POS: upwind from the left (p_x > 0); WALL: ghost cells and boundary
    // faces may occur in the tile; TL: tables from LDS
    auto rows = [&](auto posc, auto wallc, auto tlc, int ra, int rb) {
      constexpr bool POS = decltype(posc)::value, WALL = decltype(wallc)::value, TL = decltype(tlc)::value;
      if (ra >= rb) return;
      Stencil st;
      if (WALL) st = stencil(POS);
      const unsigned o0 = st.o[0], o1 = st.o[1], o2 = st.o[2], o3 = st.o[3], o4 = st.o[4];
      const bool g0 = st.g[0], g1 = st.g[1], g2 = st.g[2];
      const int mode = st.mode;
      auto load = [&](int r, Row &d) {
        const int so = (int)((unsigned)r * rowbytes);
        if (WALL) {
          d.t0 = bld<T>(rs_in, o0, so); d.t1 = bld<T>(rs_in, o1, so); d.t2 = bld<T>(rs_in, o2, so);
          d.t3 = bld<T>(rs_in, o3, so); d.t4 = bld<T>(rs_in, o4, so);
        } else {
          d.t0 = bld<T>(rs_in, oa, so);
          d.t1 = bld<T>(rs_in, oh, so);
        }
        if (STAGE != 1) d.fnv = bld<T>(rs_fn, bcf, so);
      };
      auto compute = [&](int r, const Row &d) {
        const int kap = kap_base + r;
        const int kl = (int)__umulhi((unsigned)r, mq), yz = r - kl * qyz;
        const int kx = kx0 + kl;
        const CAS double *ph = phi + (size_t)kap * 8;
        const double pxd = ph[0];
        T y0, y1, y2, y3, x0, x1, x2, x3;
        if (TL) {
          const T4 yv = *(const T4 *)(sYZ + (yz * 64 + lane) * 4);
          const T4 xv = *(const T4 *)(sX + (kl * 64 + lane) * 4);
          y0 = yv.x; y1 = yv.y; y2 = yv.z; y3 = yv.w;
          x0 = xv.x; x1 = xv.y; x2 = xv.z; x3 = xv.w;
        } else {
          const T4 yv = ldc((const CAS T4 *)(ctYZ + (size_t)yz * tstride * 4), 4 * bc);
          const T4 xv = ldc((const CAS T4 *)(ctX + (size_t)kx * tstride * 4), 4 * bc);
          y0 = yv.x; y1 = yv.y; y2 = yv.z; y3 = yv.w;
          x0 = xv.x; x1 = xv.y; x2 = xv.z; x3 = xv.w;
        }
        T v0, v1, v2, v3, v4, cen;
        T fh;
        if (WALL) {
          v0 = d.t0; v1 = d.t1; v2 = d.t2;
          const T fw = (T)((POS ? nwl : nwr) * (double)(POS ? gwL : gwR)[kap] - (DF ? bgc[kap] : 0.0));
          if (g0) v0 = fw;
          if (g1) v1 = fw;
          if (g2) v2 = fw;
          cen = POS ? d.t3 : v2;
          const T w = weno_face<T>(v0, v1, v2, d.t3, d.t4, mode == 3 ? 0 : mode);
          fh = (mode == 3) ? fw : w;
        } else {
          // the row's 69 cells pass through one of this wave's two LDS row
          // buffers (alternating by row); the five stencil values are shifted
          // reads of it.  Lanes read what other lanes wrote: the wave-scope
          // release/acquire pair orders the writes before the reads, and the
          // alternation keeps the next-but-one row's writes behind this
          // row's reads (they are separated by the next row's pair).
          // buffer index i holds cell c0-3+i; the padding slot (lane 63) goes
          // to an unused entry
          T *rb = sRow + (r & 1) * ROWBUF;
          rb[lane < 63 ? lane + 3 : 69] = d.t0;
          if (lane < 6) rb[lane < 3 ? lane : 63 + lane] = d.t1;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (POS) { v0 = rb[lane]; v1 = rb[lane + 1]; v2 = rb[lane + 2]; v3 = rb[lane + 3]; v4 = rb[lane + 4]; }
          else { v0 = rb[lane + 5]; v1 = rb[lane + 4]; v2 = rb[lane + 3]; v3 = rb[lane + 2]; v4 = rb[lane + 1]; }
          cen = POS ? v3 : v2;
          fh = weno_face_interior<T>(v0, v1, v2, v3, v4);
        }
        const T fr = shift_down1(fh);
        T F = x0 * y0 + x1 * y1 + x2 * y2 + x3 * y3;
        // FP32: F - bg = dX0 dYZ0 + dX0 yzbg + xbg dYZ0 + sum_{a>0} X_a YZ_a, every
        // term of the size of the deviation
        if (DF) F += x0 * (T)fyzb[yz] + (T)fxb[kx] * y0;
        const T pxT = DF ? (T)fpx[kx] : (T)pxd;
        T o = STAGE == 1 ? cen : (T)(1.0 - WS) * d.fnv + (T)WS * cen;
        o -= (pxT * adx) * (fr - fh);
        o += ait * (F - cen);
        // lanes without a cell store past the row range (dropped), so the
        // store needs no branch
        bst<T>(rs_out, is_cell ? bw : 0x80000000u, (int)((unsigned)r * rowbytes), o);
        // lanes that own no cell accumulate values that are never stored
        const double od = (double)o;
        acc[0] += od;
#pragma unroll
        for (int m = 1; m < NRAW; m++) acc[m] = __builtin_fma(ph[m - 1], od, acc[m]);
      };
      // a ring of D register sets: rows r+1 .. r+D-1 are in flight while row r
      // is computed (interior rows hold one value per lane plus the halo, so
      // the ring is deeper there)
      constexpr int D = WALL ? 3 : (sizeof(T) == 8 ? FDLB_RING_F64 : FDLB_RING_F32);
      // Loads are issued unconditionally (rows past the range repeat the last
      // row): every path then has the same loads in flight, so the memory
      // counter waits stay exact and do not drain the ring.
      Row ring[D];
#pragma unroll
      for (int k = 0; k < D - 1; k++) load(min(ra + k, rb - 1), ring[k]);
      int r = ra;
      // full trips: straight-line code over D rows, so the scheduler can
      // overlap the rows' dependent chains
      for (; r + D <= rb; r += D) {
#pragma unroll
        for (int k = 0; k < D; k++) {
          load(min(r + k + D - 1, rb - 1), ring[(k + D - 1) % D]);
          compute(r + k, ring[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < D; k++) {
        if (r + k < rb) {
          load(min(r + k + D - 1, rb - 1), ring[(k + D - 1) % D]);
          compute(r + k, ring[k]);
        }
      }
    };
    using TT = BoolC<true>;
    using FF = BoolC<false>;
    if (interior && tlds) {
      rows(TT(), FF(), TT(), r0, min(r1, rsplit));
      rows(FF(), FF(), TT(), max(r0, rsplit), r1);
    } else if (interior) {
      rows(TT(), FF(), FF(), r0, min(r1, rsplit));
      rows(FF(), FF(), FF(), max(r0, rsplit), r1);
    } else if (tlds) {
      rows(TT(), TT(), TT(), r0, min(r1, rsplit));
      rows(FF(), TT(), TT(), max(r0, rsplit), r1);
    } else {
      rows(TT(), TT(), FF(), r0, min(r1, rsplit));
      rows(FF(), TT(), FF(), max(r0, rsplit), r1);
    }
    // the LDS of the tables and row buffers is reused by the partial sums
    if (tlds || interior) __syncthreads();
  } else {
    // body force couples the velocities of one y-line: a wave takes whole
    // lines.  The line's rows are a compile-time count (one code path per
    // Q_y), so all its reads (stencils, targets, f^n) form straight-line code
    // and are in flight together before the first store; a row count known
    // only at run time would put a branch between the rows and serialise
    // their reads.  QYC is the largest Q_y of the launch: the instance for
    // Q_y <= 4 keeps fewer registers live than the one for Q_y <= 8.
    const T ay = (T)c.ay;
    const int nlines = (kx1 - kx0) * qz;
    // Q_y <= 4 (many lines per wave): a line's rows pass through LDS row
    // buffers, one per row, in this wave's slice of the partial-sum area
    // (NRAW x 64 doubles hold MAXQY buffers).  Buffer index i holds cell
    // c0-3+i clamped into [0, nx-1], so the five stencil values are shifted
    // reads of it and equal the clamped loads of face(); ghosts and wall
    // faces are then substituted per lane.  Per row that is one row load and
    // a six-lane halo load instead of five stencil loads, which pays where a
    // wave walks many lines; with one line per wave (Q_y up to 8 on short
    // grids) the LDS round trip lengthens the line's dependent chain, so that
    // instance reads the stencils directly.  Both give the same values.
    constexpr bool LDS_LINES = QYC <= 4;
    static_assert(MAXQY * ROWBUF <= NRAW * 64, "row buffers of a line fit the wave's partial-sum slice");
    T *sLine = (T *)(lds_dyn + (size_t)wv * NRAW * 64);
    const unsigned oa = lane < UTILE ? (unsigned)fslot(min(c0 + lane, nx - 1)) * (unsigned)sizeof(T) : 0x80000000u;
    const unsigned oh = lane < 3 ? (unsigned)fslot(max(c0 - 3 + lane, 0)) * (unsigned)sizeof(T)
                                 : (lane < 6 ? (unsigned)fslot(min(c0 + 60 + lane, nx - 1)) * (unsigned)sizeof(T)
                                             : 0x80000000u);
    const int kap_base = kx0 * qyz;
    const unsigned rowbytes = (unsigned)c.nxp * (unsigned)sizeof(T);
    const auto rs_in = rsrc_of(gin + (size_t)kap_base * fstride, (unsigned)(kx1 - kx0) * (unsigned)qyz * rowbytes);
    auto lines = [&](auto qyc) {
      constexpr int QY = decltype(qyc)::value;
      for (int line = wv; line < nlines; line += nwv) {
        const int kx = kx0 + line / qz, kz = line - (line / qz) * qz;
        const double pxd = lat[lo_px + kx];
        const bool pos = kx < c_qh;               // positive x nodes come first
        const Stencil st = stencil(pos);
        const T4 xv = ldc((const CAS T4 *)(ctX + (size_t)kx * tstride * 4), 4 * bc);
        const T X0 = xv.x, X1 = xv.y, X2 = xv.z, X3 = xv.w;
        const CAS T *gw = pos ? gwL : gwR;
        const double nw = pos ? nwl : nwr;
        T cen[QY], adv[QY], tgt[QY], fnv[QY];
        if constexpr (!LDS_LINES) {
#pragma unroll
          for (int ky = 0; ky < QY; ky++) {
            const int kap = (kx * QY + ky) * qz + kz;
            const T fw = (T)(nw * (double)gw[kap] - (DF ? lat[c.lo.bg + kap] : 0.0));
            const T fh = face(gin + (size_t)kap * fstride, st, pos, fw, cen[ky]);
            const T fr = shift_down1(fh);
            adv[ky] = -(T)pxd * dxi * (fr - fh);
            tgt[ky] = target(kx, ky * qz + kz, X0, X1, X2, X3);
            fnv[ky] = STAGE == 1 ? (T)0 : ldb(fn + (size_t)kap * fstride, bcf);
          }
        } else {
          T ra[QY], rh[QY];
#pragma unroll
          for (int ky = 0; ky < QY; ky++) {
            const int kap = (kx * QY + ky) * qz + kz;
            const int so = (int)((unsigned)(kap - kap_base) * rowbytes);
            ra[ky] = bld<T>(rs_in, oa, so);
            rh[ky] = bld<T>(rs_in, oh, so);
            tgt[ky] = target(kx, ky * qz + kz, X0, X1, X2, X3);
            fnv[ky] = STAGE == 1 ? (T)0 : ldb(fn + (size_t)kap * fstride, bcf);
          }
          // the previous line's reads of the buffers come before these writes
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int ky = 0; ky < QY; ky++) {
            T *rb = sLine + ky * ROWBUF;
            rb[lane < UTILE ? lane + 3 : ROWBUF - 3] = ra[ky];
            if (lane < 6) rb[lane < 3 ? lane : 63 + lane] = rh[ky];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int ky = 0; ky < QY; ky++) {
            const int kap = (kx * QY + ky) * qz + kz;
            const T fw = (T)(nw * (double)gw[kap] - (DF ? lat[c.lo.bg + kap] : 0.0));
            const T *rb = sLine + ky * ROWBUF;
            T v0, v1, v2, v3, v4;
            if (pos) { v0 = rb[lane]; v1 = rb[lane + 1]; v2 = rb[lane + 2]; v3 = rb[lane + 3]; v4 = rb[lane + 4]; }
            else { v0 = rb[lane + 5]; v1 = rb[lane + 4]; v2 = rb[lane + 3]; v3 = rb[lane + 2]; v4 = rb[lane + 1]; }
            if (st.g[0]) v0 = fw;
            if (st.g[1]) v1 = fw;
            if (st.g[2]) v2 = fw;
            cen[ky] = pos ? v3 : v2;
            const T w = weno_face<T>(v0, v1, v2, v3, v4, st.mode == 3 ? 0 : st.mode);
            const T fh = (st.mode == 3) ? fw : w;
            const T fr = shift_down1(fh);
            adv[ky] = -(T)pxd * dxi * (fr - fh);
          }
        }
#pragma unroll
        for (int ky = 0; ky < QY; ky++) {
          const int kap = (kx * QY + ky) * qz + kz;
          T sf = 0;
          const CAS double *km = clat + c.lo.kmat + ky * QY;
#pragma unroll
          for (int k2 = 0; k2 < QY; k2++) sf += (T)km[k2] * cen[k2];
          if (DF) sf += (T)clat[c.lo.kbg + kap];
          finish(kap, ky, kz, pxd, cen[ky], adv[ky] - ay * sf + (tgt[ky] - cen[ky]) * itau, fnv[ky]);
        }
      }
    };
    static_assert(MAXQY == 8, "one code path per full-range order 2..8");
    switch (qy) {
      case 2: lines(IntC<2>()); break;
      case 3: lines(IntC<3>()); break;
      case 4: lines(IntC<4>()); break;
      default:
        if constexpr (QYC > 4) {
          switch (qy) {
            case 5: lines(IntC<5>()); break;
            case 6: lines(IntC<6>()); break;
            case 7: lines(IntC<7>()); break;
            default: lines(IntC<8>()); break;
          }
        }
        break;
    }
  }
  block_partials<T>(c, bm.z, c0, acc, is_cell, lds_dyn);
}

// initial state from the tables: f = sum_a n X_a YZ_a (times 1 + noise)
template <typename T>
__global__ void __launch_bounds__(512) k_fill(const CaseDev *__restrict__ cases, const int4 *__restrict__ map,
                                              int use_noise) {
  const int4 bm = map[blockIdx.x];
  if (bm.x < 0) return;
  const CaseDev &c = cases[bm.x];
  if (!c.active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int nx = c.nx, qy = c.qy, qz = c.qz, qyz = c.qyz, nkx = c.nkx;
  constexpr int P = sizeof(T) == 4 ? 1 : 0;
  T *f = (T *)c.f[P][0];
  const T *tX = (const T *)c.tabX[P];
  const T *tYZ = (const T *)c.tabYZ[P];
  const double *lat = c.lat;
  const int c0 = bm.y * UTILE, j = c0 + lane;
  const bool is_cell = lane < UTILE && j < nx;
  const int jc = min(j, nx - 1);
  const int kx0 = bm.z * c.kxc, kx1 = min(kx0 + c.kxc, nkx);
  double acc[NRAW];
  for (int m = 0; m < NRAW; m++) acc[m] = 0.0;
  const int nrows = (kx1 - kx0) * qyz;
  for (int r = wv; r < nrows; r += nwv) {
    const int kx = kx0 + r / qyz, yz = r % qyz, ky = yz / qz, kz = yz % qz;
    const int kap = kx * qyz + yz;
    const T *xr = tX + ((size_t)kx * nx + jc) * 4, *yr = tYZ + ((size_t)yz * nx + jc) * 4;
    double F = 0;
    for (int a = 0; a < 4; a++) F += (double)xr[a] * (double)yr[a];
    if (sizeof(T) == 4) {
      // FP32 storage: the tables give the deviation from the background
      // (F - bg = dX0 dYZ0 + dX0 yzbg + xbg dYZ0 + sum_{a>0} X_a YZ_a)
      F += (double)xr[0] * lat[c.lo.yzbg + yz] + lat[c.lo.xbg + kx] * (double)yr[0];
      if (use_noise) F += (F + lat[c.lo.bg + kap]) * c.noise[(size_t)kap * nx + jc];
    } else if (use_noise) {
      F *= 1.0 + c.noise[(size_t)kap * nx + jc];
    }
    const T o = (T)F;
    if (is_cell) {
      f[(size_t)kap * c.nxp + fslot(j)] = o;
      const double od = (double)o, pxd = lat[c.lo.px + kx], pyd = lat[c.lo.py + ky], pzd = lat[c.lo.pz + kz];
      const double p2 = pxd * pxd + pyd * pyd + pzd * pzd;
      acc[0] += od; acc[1] += pxd * od; acc[2] += pyd * od; acc[3] += pxd * pxd * od; acc[4] += pxd * pyd * od;
      acc[5] += pyd * pyd * od; acc[6] += pzd * pzd * od; acc[7] += pxd * p2 * od; acc[8] += pyd * p2 * od;
    }
  }
  {
    __shared__ double s_acc[8 * NRAW * 64];
    block_partials<T>(c, bm.z, c0, acc, is_cell, s_acc);
  }
}

// partial raw sums of f^n (after an upload)
template <typename T>
__global__ void __launch_bounds__(512) k_partials(const CaseDev *__restrict__ cases, const int4 *__restrict__ map) {
  const int4 bm = map[blockIdx.x];
  if (bm.x < 0) return;
  const CaseDev &c = cases[bm.x];
  if (!c.active) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int nx = c.nx, qz = c.qz, qyz = c.qyz, nkx = c.nkx;
  constexpr int P = sizeof(T) == 4 ? 1 : 0;
  const T *f = (const T *)c.f[P][0];
  const double *lat = c.lat;
  const int c0 = bm.y * UTILE, j = c0 + lane;
  const bool is_cell = lane < UTILE && j < nx;
  const int jc = min(j, nx - 1);
  const int kx0 = bm.z * c.kxc, kx1 = min(kx0 + c.kxc, nkx);
  double acc[NRAW];
  for (int m = 0; m < NRAW; m++) acc[m] = 0.0;
  const int nrows = (kx1 - kx0) * qyz;
  for (int r = wv; r < nrows; r += nwv) {
    const int kx = kx0 + r / qyz, yz = r % qyz, ky = yz / qz, kz = yz % qz;
    const int kap = kx * qyz + yz;
    if (is_cell) {
      const double od = (double)f[(size_t)kap * c.nxp + fslot(jc)];
      const double pxd = lat[c.lo.px + kx], pyd = lat[c.lo.py + ky], pzd = lat[c.lo.pz + kz];
      const double p2 = pxd * pxd + pyd * pyd + pzd * pzd;
      acc[0] += od; acc[1] += pxd * od; acc[2] += pyd * od; acc[3] += pxd * pxd * od; acc[4] += pxd * pyd * od;
      acc[5] += pyd * pyd * od; acc[6] += pzd * pzd * od; acc[7] += pxd * p2 * od; acc[8] += pyd * p2 * od;
    }
  }
  {
    __shared__ double s_acc[8 * NRAW * 64];
    block_partials<T>(c, bm.z, c0, acc, is_cell, s_acc);
  }
}

__global__ void k_zero_resid(const CaseDev *__restrict__ cases, int ncases) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncases) *cases[i].resid = 0ull;
}

__global__ void k_scale(double *__restrict__ x, double a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] *= a;
}

// FP32 deviation storage of case c -> FP64 populations (f = bg + g)
__global__ void k_promote(const CaseDev *__restrict__ cases, int ci) {
  const CaseDev &c = cases[ci];
  const float *g = (const float *)c.f[1][0];
  double *f = (double *)c.f[0][0];
  const double *bg = c.lat + c.lo.bg;
  const size_t n = (size_t)c.K * c.nxp;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    f[i] = (double)g[i] + bg[i / c.nxp];
}

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// plain device copy used to calibrate memory-traffic counters
__global__ void __launch_bounds__(256) k_copy_probe(const double4 *__restrict__ src, double4 *__restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// plain launch, or (timing) with events recorded at the kernel's own start and end
template <typename K, typename... A>
static void launch_k(K kern, dim3 g, dim3 b, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1, A... args) {
  if (e0) hipExtLaunchKernelGGL(kern, g, b, (uint32_t)lds, s, e0, e1, 0u, args...);
  else hipLaunchKernelGGL(kern, g, b, lds, s, args...);
}

hipError_t launch_nbar(int prec, const CaseDev *cases, const int *map, int nblocks, size_t lds, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (lds == 0 || lds > NBAR_LDS_MAX) return hipErrorInvalidValue;
  const int4 *m = (const int4 *)map;
  if (prec == 0) hipLaunchKernelGGL(k_nbar<double>, dim3(nblocks), dim3(512), lds, s, cases, m);
  else hipLaunchKernelGGL(k_nbar<float>, dim3(nblocks), dim3(512), lds, s, cases, m);
  return hipGetLastError();
}

hipError_t launch_table(int prec, const CaseDev *cases, const int *map, int nblocks, int mode, int gin,
                        bool wide, int tile, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nblocks <= 0) return hipSuccess;
  const int4 *m = (const int4 *)map;
  if (tile == CTILE_SMALL) {
    // small maps (built with CTILE_SMALL cells per block; never with wide cases)
    if (wide || nblocks > TABLE_WIDE_MAX) return hipErrorInvalidValue;
    if (prec == 0) launch_k(k_table<double, 512, false, CTILE_SMALL>, dim3(nblocks), dim3(512), 0, s, e0, e1, cases, m, mode, gin);
    else launch_k(k_table<float, 512, false, CTILE_SMALL>, dim3(nblocks), dim3(512), 0, s, e0, e1, cases, m, mode, gin);
    return hipGetLastError();
  }
  if (tile != CTILE) return hipErrorInvalidValue;
  // small maps are latency-bound: twice the threads per block shorten the
  // per-phase work of each thread; large maps keep more blocks resident
  hipEvent_t e1s = wide ? nullptr : e1;
  if (nblocks <= TABLE_WIDE_MAX) {
    if (prec == 0) launch_k(k_table<double, 512, false, CTILE>, dim3(nblocks), dim3(512), 0, s, e0, e1s, cases, m, mode, gin);
    else launch_k(k_table<float, 512, false, CTILE>, dim3(nblocks), dim3(512), 0, s, e0, e1s, cases, m, mode, gin);
  } else {
    if (prec == 0) launch_k(k_table<double, 256, false, CTILE>, dim3(nblocks), dim3(256), 0, s, e0, e1s, cases, m, mode, gin);
    else launch_k(k_table<float, 256, false, CTILE>, dim3(nblocks), dim3(256), 0, s, e0, e1s, cases, m, mode, gin);
  }
  // orders above MAXQH: a second pass over the same map (after the first, so
  // the wall fluxes are in place)
  if (wide) {
    if (prec == 0) hipLaunchKernelGGL((k_table<double, 512, true, CTILE>), dim3(nblocks), dim3(512), 0, s, cases, m, mode, gin);
    else hipLaunchKernelGGL((k_table<float, 512, true, CTILE>), dim3(nblocks), dim3(512), 0, s, cases, m, mode, gin);
    if (e1) { hipError_t r = hipEventRecord(e1, s); if (r != hipSuccess) return r; }
  }
  return hipGetLastError();
}

template <typename T, bool FORCE, int QYC = MAXQY>
static void upd(int stage, dim3 g, dim3 b, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                const CaseDev *cases, const int4 *map) {
  if (stage == 1) launch_k(k_update<T, 1, FORCE, QYC>, g, b, lds, s, e0, e1, cases, map);
  else if (stage == 2) launch_k(k_update<T, 2, FORCE, QYC>, g, b, lds, s, e0, e1, cases, map);
  else launch_k(k_update<T, 3, FORCE, QYC>, g, b, lds, s, e0, e1, cases, map);
}

size_t update_lds_bytes(int prec, int qyz, int kxc, int waves, bool tlds) {
  const size_t part = (size_t)waves * NRAW * 64 * sizeof(double);
  const size_t tab = ((tlds ? (size_t)4 * (qyz + kxc) * 64 : 0) + (size_t)waves * 2 * ROWBUF) * (prec == 0 ? 8 : 4);
  return part > tab ? part : tab;
}

hipError_t launch_update(int prec, int stage, const CaseDev *cases, const int *map, int nblocks, int waves,
                         int force, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nblocks <= 0) return hipSuccess;
  if (lds > UPDATE_LDS_MAX || lds < (size_t)waves * NRAW * 64 * sizeof(double)) return hipErrorInvalidValue;
  const dim3 g(nblocks), b(64 * waves);
  const int4 *m = (const int4 *)map;
  // force: 0 none; otherwise the largest Q_y of the launch's cases
  if (force > MAXQY) return hipErrorInvalidValue;
  if (prec == 0) {
    if (force > 4) upd<double, true, 8>(stage, g, b, lds, s, e0, e1, cases, m);
    else if (force) upd<double, true, 4>(stage, g, b, lds, s, e0, e1, cases, m);
    else upd<double, false>(stage, g, b, lds, s, e0, e1, cases, m);
  } else {
    if (force > 4) upd<float, true, 8>(stage, g, b, lds, s, e0, e1, cases, m);
    else if (force) upd<float, true, 4>(stage, g, b, lds, s, e0, e1, cases, m);
    else upd<float, false>(stage, g, b, lds, s, e0, e1, cases, m);
  }
  return hipGetLastError();
}

hipError_t launch_fill(int prec, const CaseDev *cases, const int *map, int nblocks, int waves, int use_noise,
                       hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_fill<double>, dim3(nblocks), dim3(64 * waves), 0, s, cases, (const int4 *)map, use_noise);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(nblocks), dim3(64 * waves), 0, s, cases, (const int4 *)map, use_noise);
  return hipGetLastError();
}

hipError_t launch_partials(int prec, const CaseDev *cases, const int *map, int nblocks, int waves, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_partials<double>, dim3(nblocks), dim3(64 * waves), 0, s, cases, (const int4 *)map);
  else
    hipLaunchKernelGGL(k_partials<float>, dim3(nblocks), dim3(64 * waves), 0, s, cases, (const int4 *)map);
  return hipGetLastError();
}

hipError_t launch_zero_resid(const CaseDev *cases, int ncases, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_resid, dim3((ncases + 255) / 256), dim3(256), 0, s, cases, ncases);
  return hipGetLastError();
}

// dir 0: float -> double, dir 1: double -> float
hipError_t launch_convert(int dir, const void *src, void *dst, size_t n, hipStream_t s) {
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  if (n == 0) return hipSuccess;
  if (dir == 0)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, s, (const float *)src, (double *)dst, n);
  else
    hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, s, (const double *)src, (float *)dst, n);
  return hipGetLastError();
}

hipError_t launch_promote(const CaseDev *cases, int c, size_t n, hipStream_t s) {
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_promote, dim3(blocks), dim3(256), 0, s, cases, c);
  return hipGetLastError();
}

hipError_t launch_scale(void *x, double a, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_scale, dim3(blocks), dim3(256), 0, s, (double *)x, a, n);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / sizeof(double4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_probe, dim3(2048), dim3(256), 0, s, (const double4 *)src, (double4 *)dst, n);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// reduced models (Sec. II.B): one fused kernel per RK stage
// ---------------------------------------------------------------------------
// Revised Enskog average density of reduced cases (chi_mode 1): the window
// sums of k_nbar, with the density of each window cell summed over the phi
// rows of the stage input.  One 8-wave block per NBAR_TILE cells.
__global__ void __launch_bounds__(512) k_r1_nbar(const R1Dev *__restrict__ cases, const int2 *__restrict__ map,
                                                 int stage) {
  extern __shared__ double s_n[];   // densities [nwin] and faces [nwin + 1] of the tile's window
  __shared__ double s_x[NBAR_TILE];
  __shared__ int s_lo[NBAR_TILE], s_hi[NBAR_TILE];
  const int2 bm = map[blockIdx.x];
  const R1Dev &c = cases[bm.x];
  const int nx = c.nx, c0 = bm.y * NBAR_TILE, c1 = min(c0 + NBAR_TILE, nx), Kh = 2 * c.qh * c.qy;
  const double *lat = c.lat;
  const int jmin = (int)lat[c.lo.wlo + c0], jmax = (int)lat[c.lo.whi + c1 - 1];
  const int nwin = jmax - jmin + 1;
  double *s_f = s_n + nwin;
  const double *gin = stage == 1 ? c.f : (stage == 2 ? c.g1 : c.g2);
  const int tid = threadIdx.x;
  if (tid < c1 - c0) {
    s_x[tid] = lat[c.lo.xcn + c0 + tid];
    s_lo[tid] = (int)lat[c.lo.wlo + c0 + tid];
    s_hi[tid] = (int)lat[c.lo.whi + c0 + tid];
  }
  for (int q = tid; q <= nwin; q += blockDim.x) s_f[q] = lat[c.lo.xf + jmin + q];
  for (int q = tid; q < nwin; q += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < Kh; r++) a += gin[(size_t)r * nx + jmin + q];
    s_n[q] = a;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const double sg = c.sigma, s2 = sg * sg;
  for (int i = c0 + wv; i < c1; i += nwv) {
    const double x = s_x[i - c0];
    const int lo = s_lo[i - c0] - jmin, hi = s_hi[i - c0] - jmin;
    double acc = 0.0;
    for (int q = lo + lane; q <= hi; q += 64) {
      const double a = fmax(s_f[q], x - sg) - x, b = fmin(s_f[q + 1], x + sg) - x;
      acc += s_n[q] * ((s2 * b - b * b * b / 3.0) - (s2 * a - a * a * a / 3.0));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) c.nbar[i] = 3.0 / (4.0 * sg * s2) * acc;
  }
}

// A block owns TS cells of one case.  It stages phi and theta of its cells and
// a halo of R1_HALO cells per side in LDS, and then, without going back to
// memory: the moments (eq:macro1D, eq:macro2D) of every staged cell, the wall
// densities (tiles whose stencils reach a wall), the closure and the targets
// of its cells (phi^S + tau J1^phi and theta^S + tau J1^theta as polynomials
// in xi times the Maxwellian, projected per axis), and the update of every
// row of its cells: WENO-5 advection with the diffuse-wall rules of the 3D
// pass, the body force on the y-nodes (2D), relaxation and the TVD-RK3
// combination (eq:rk3).  D is the dimension of the reduced model, RM the
// largest row count of the launch (it sizes the LDS) and TS the cells per
// block (32 up to 128 rows, 16 up to 256, 4 above; 8 on small maps of at most
// 256 rows).
template <int STAGE, int RM, int D, int TS>
__global__ void __launch_bounds__(512) k_r1_stage(const R1Dev *__restrict__ cases, const int2 *__restrict__ map) {
  constexpr int W = TS + 2 * R1_HALO, QYM = D == 2 ? MAXQY : 1;
  const int2 bm = map[blockIdx.x];
  const R1Dev &c = cases[bm.x];
  __shared__ double s_g[RM][W];
  __shared__ double s_t[RM][TS];
  __shared__ double s_G[TS][2][NB + 1];
  __shared__ double s_m[6][W];              // n, u_x, u_y, T, q_x, q_y
  __shared__ double s_l[3][W];              // ln n, ln chi, ln T
  __shared__ double s_c[TS][2];             // n, 1/tau
  __shared__ double s_y[TS][2][4][QYM];     // per y-node: sum_b P_ab Y_b (phi, theta)
  __shared__ double s_nw[2];
  __shared__ double s_lam[D == 2 ? MAXQH : RM / 4][NB + 1];   // Lagrange rows (padded: bank spread)
  __shared__ double s_bh[2][NB];            // base nodes P_m and h_Q(P_m)
  __shared__ double s_px[2 * MAXQH], s_py[QYM], s_km[QYM * QYM];   // x-nodes, y-nodes, force matrix
  __shared__ unsigned char s_rk[D == 2 ? RM / 2 : 1][2];             // 2D: phi row -> (kx, ky)
  const int nx = c.nx, qh = c.qh, qy = D == 1 ? 1 : c.qy, Q2 = 2 * qh, Kh = Q2 * qy, R = c.R;
  // node indices of a phi row without a division in the row loops
  auto kx_of = [&](int r) -> int { return D == 2 ? s_rk[r][0] : r; };
  auto ky_of = [&](int r) -> int { return D == 2 ? s_rk[r][1] : 0; };
  const int c0 = bm.y * TS, own = min(TS, nx - c0);
  const int tid = threadIdx.x;
  const double *lat = c.lat;
  const LatOff lo = c.lo;
  const double *gin = STAGE == 1 ? c.f : (STAGE == 2 ? c.g1 : c.g2);
  double *gout = STAGE == 1 ? c.g1 : (STAGE == 2 ? c.g2 : c.f);
  constexpr int SW = 4, NS = TS / SW;   // update strips: 4 cells of one row

  for (int it = tid; it < R * W; it += blockDim.x) {
    const int r = it / W, w = it - r * W, cell = c0 - R1_HALO + w;
    s_g[r][w] = (cell >= 0 && cell < nx) ? gin[(size_t)r * nx + cell] : 0.0;
  }
  for (int it = tid; it < qh * NB; it += blockDim.x) s_lam[it / NB][it % NB] = lat[lo.lam + it];
  for (int it = tid; it < NB; it += blockDim.x) { s_bh[0][it] = lat[lo.bP + it]; s_bh[1][it] = lat[lo.hQ + it]; }
  if (tid < Q2) s_px[tid] = lat[lo.px + tid];
  if (D == 2 && tid < qy) s_py[tid] = lat[lo.py + tid];
  if (D == 2 && tid < qy * qy) s_km[tid] = lat[lo.kmat + tid];
  if (D == 2)
    for (int it = tid; it < Kh; it += blockDim.x) {
      const int kx = it / qy;
      s_rk[it][0] = (unsigned char)kx; s_rk[it][1] = (unsigned char)(it - kx * qy);
    }
  __syncthreads();

  // moments of the staged cells (8 lanes per cell, each summing every 8th
  // phi row, then a butterfly over the 8 lanes); wall densities in the tiles
  // whose stencils reach a wall
  static_assert(8 * W <= 448, "moment lanes stay below the wall threads");
  if (tid < 8 * W) {
    const int wc = tid >> 3, sub = tid & 7, cell = c0 - R1_HALO + wc;
    const bool live = cell >= 0 && cell < nx;   // uniform over the 8 lanes of a cell
    double n = 0.0, jx = 0.0, jy = 0.0;
    if (live)
      for (int r = sub; r < Kh; r += 8) {
        const double v = s_g[r][wc];
        n += v; jx += s_px[kx_of(r)] * v;
        if (D == 2) jy += s_py[ky_of(r)] * v;
      }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      n += __shfl_xor(n, off, 64); jx += __shfl_xor(jx, off, 64); jy += __shfl_xor(jy, off, 64);
    }
    const double ux = live ? jx / n : 0.0, uy = live ? jy / n : 0.0;
    double pin = 0.0, th = 0.0, qx = 0.0, qy_ = 0.0;   // pin: sum of |xi_in-plane|^2 phi
    if (live)
      for (int r = sub; r < Kh; r += 8) {
        const double cx = s_px[kx_of(r)] - ux, cy = D == 2 ? s_py[ky_of(r)] - uy : 0.0;
        const double ph = s_g[r][wc], tt = s_g[Kh + r][wc], c2 = cx * cx + cy * cy;
        pin += c2 * ph; th += tt;
        qx += cx * (0.5 * c2 * ph + 0.5 * tt);
        if (D == 2) qy_ += cy * (0.5 * c2 * ph + 0.5 * tt);
      }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      pin += __shfl_xor(pin, off, 64); th += __shfl_xor(th, off, 64);
      qx += __shfl_xor(qx, off, 64); qy_ += __shfl_xor(qy_, off, 64);
    }
    if (live && sub == 0) {
      const double T_ = (pin + th) / (3.0 * n);
      s_m[0][wc] = n; s_m[1][wc] = ux; s_m[2][wc] = uy; s_m[3][wc] = T_; s_m[4][wc] = qx; s_m[5][wc] = qy_;
      // revised Enskog cases take chi at the average density of the stage input
      const double nc = c.chi_mode == 1 ? c.nbar[cell] : n;
      s_l[0][wc] = log(n); s_l[1][wc] = log(chi_cs(c.eta0 * nc)); s_l[2][wc] = log(T_);
    }
  } else if (tid >= 448) {
    // impenetrability: the incoming phi rows reach the wall face through the
    // fully interior candidate; n_w makes the net mass flux vanish.  Every
    // tile whose stencils reach a wall's ghosts (cells within 3 of it) takes
    // that wall's density; the cells it needs are staged.  The last wave
    // sums it: lanes 0-31 the left wall, 32-63 the right, each over every
    // 32nd phi row, then a butterfly within the half.
    const int wall = (tid - 448) >> 5, ln = tid & 31;
    const bool here = wall == 0 ? c0 < 3 : c0 + own + 2 >= nx;   // uniform over the half
    double in = 0.0;
    if (here) {
      const int w0 = wall == 0 ? R1_HALO : nx - 1 - c0 + R1_HALO;   // the wall cell
      const int st = wall == 0 ? 1 : -1;                             // into the domain
      for (int r = ln; r < Kh; r += 32) {
        const double p = s_px[kx_of(r)];
        if ((wall == 0) != (p < 0.0)) continue;
        const double v0 = s_g[r][w0 + 2 * st], v1 = s_g[r][w0 + st], v2 = s_g[r][w0];
        in += p * (v0 * (1.0 / 3.0) - v1 * (7.0 / 6.0) + v2 * (11.0 / 6.0));
      }
    }
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) in += __shfl_xor(in, off, 64);
    if (here && ln == 0) s_nw[wall] = -in / c.wallD[wall];
  }
  __syncthreads();

  // closure and the target polynomials per owned cell, folded with the y
  // projections into the per-node factors s_y
  if (tid < own) {
    const int i = c0 + tid, li = tid + R1_HALO;
    double g[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
      const double *src = q < 3 ? s_l[q] : (q == 3 ? s_m[1] : s_m[2]);
      double d = 0.0;
      if (q == 4 && D == 1) { g[q] = 0.0; continue; }
      if (i >= 3 && i <= nx - 4) {
        d = (src[li + 1] - src[li - 1]) * 0.75 - (src[li + 2] - src[li - 2]) * 0.15 +
            (src[li + 3] - src[li - 3]) * (1.0 / 60.0);
      } else if (i < 3) {
        for (int jj = 0; jj < 7; jj++) d += lat[lo.fdw + i * 7 + jj] * src[li - i + jj];
      } else {
        const int r = nx - 1 - i;
        for (int jj = 0; jj < 7; jj++) d -= lat[lo.fdw + r * 7 + jj] * src[li + r - jj];
      }
      g[q] = d * c.invdx[i];
    }
    const double n = s_m[0][li], uy = s_m[2][li], T_ = s_m[3][li], qx = s_m[4][li], qy_ = s_m[5][li];
    // b rho stays local; chi enters tau, Pr, the J1 prefactor and dln chi
    const double eta = c.eta0 * n, chi = chi_cs(c.chi_mode == 1 ? c.eta0 * c.nbar[i] : eta), brc = 4.0 * eta * chi;
    double tau = 0.0, itau = 0.0;
    if (c.tau_pre > 0.0) {
      tau = c.tau_pre / (n * sqrt(T_)) *
            (1.0 / chi + 3.2 * eta + 64.0 / 25.0 * (1.0 + 12.0 / M_PI) * eta * eta * chi);
      itau = 1.0 / tau;
    }
    double Pr = 1.0;
    if (c.collision == 1) Pr = c.pr_fixed;
    else if (c.collision == 2)
      Pr = 2.0 / 3.0 * (1.0 + 0.8 * brc + 4.0 / 25.0 * (1.0 + 12.0 / M_PI) * brc * brc) /
           (1.0 + 1.2 * brc + 9.0 / 25.0 * (1.0 + 32.0 / (9.0 * M_PI)) * brc * brc);
    const double s0 = (1.0 - Pr) / (5.0 * n * T_ * T_), iT = 1.0 / T_;
    const bool j1 = itau > 0.0 && brc > 0.0;
    const double A = j1 ? -tau * brc : 0.0, g1 = g[1] + 2.0 * g[0];   // dln chi + 2 dln rho
    if (D == 1) {
      // phi: 1 + s0 (xi^2/T - 3) xi q_x + tau J1^phi / f^MB; theta / (2T):
      // 1 + s0 (xi^2/T - 1) xi q_x + tau J1^theta / (2T f^MB)
      const double cp[4] = {1.0 - A * 0.6 * g[3], -3.0 * s0 * qx + A * (g1 + 0.1 * g[2]), A * 0.6 * g[3] * iT,
                            s0 * qx * iT + A * 0.3 * g[2] * iT};
      const double ct[4] = {1.0 - A * 0.2 * g[3], -s0 * qx + A * (g1 + 0.7 * g[2]), A * 0.6 * g[3] * iT,
                            s0 * qx * iT + A * 0.3 * g[2] * iT};
#pragma unroll
      for (int a = 0; a < 4; a++) { s_y[tid][0][a][0] = cp[a]; s_y[tid][1][a][0] = 2.0 * T_ * ct[a]; }
    } else {
      // P[w][a][b]: coefficient of xi_x^a xi_y^b in phi^S_2D + tau J1^phi_2D
      // (w = 0) and in (theta^S_2D + tau J1^theta_2D) / T (w = 1), with the
      // 3D operator's (2/5)(xi_x xi_y / T) du_y/dx term when j1_shear = 1
      double P[2][4][4];
#pragma unroll
      for (int w = 0; w < 2; w++) {
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
          for (int b = 0; b < 4; b++) P[w][a][b] = 0.0;
        const double cq = w == 0 ? 4.0 : 2.0, cu = w == 0 ? 2.0 : 1.0, cT = w == 0 ? -2.0 / 3.0 : 4.0 / 3.0;
        P[w][0][0] = 1.0 - A * 0.4 * cu * g[3];
        P[w][3][0] = s0 * qx * iT + A * 0.3 * iT * g[2];
        P[w][1][2] = s0 * qx * iT + A * 0.3 * iT * g[2];
        P[w][1][0] = -cq * s0 * qx + A * (g1 + 0.3 * cT * g[2]);
        P[w][2][1] = s0 * qy_ * iT;
        P[w][0][3] = s0 * qy_ * iT;
        P[w][0][1] = -cq * s0 * qy_;
        P[w][2][0] = A * 0.6 * iT * g[3];
        P[w][0][2] = A * 0.2 * iT * g[3];
        P[w][1][1] = c.j1_shear ? A * 0.4 * iT * g[4] : 0.0;
      }
      for (int ky = 0; ky < qy; ky++) {
        double Y[4];
        full_axis_values(uy, T_, qy, lat + lo.Hy + ky * qy, Y);
#pragma unroll
        for (int w = 0; w < 2; w++)
#pragma unroll
          for (int a = 0; a < 4; a++)
            s_y[tid][w][a][ky] = (w == 0 ? 1.0 : T_) *
                                 (P[w][a][0] * Y[0] + P[w][a][1] * Y[1] + P[w][a][2] * Y[2] + P[w][a][3] * Y[3]);
      }
    }
    s_c[tid][0] = n; s_c[tid][1] = itau;
  } else if (tid >= 64) {
    // half-range base weights per owned cell and half
    for (int it = tid - 64; it < own * 2 * NB; it += blockDim.x - 64) {
      const int cl = it / (2 * NB), h = (it / NB) & 1, m = it % NB;
      const int w = cl + R1_HALO;
      const double u = h == 0 ? s_m[1][w] : -s_m[1][w], T_ = s_m[3][w];
      const double d = s_bh[0][m] - u;
      s_G[cl][h][m] = exp(lat[lo.bA + m] - d * d / (2.0 * T_)) * rsqrt(T_);
    }
  }
  __syncthreads();

  // targets: X_a[k] = Proj[g (p - u)^a] at x-node k (both halves), then per
  // y-node phi_t = n sum_a X_a s_y[0][a] and theta_t = n sum_a X_a s_y[1][a];
  // an item is one cell and half and a pair of x-nodes, which share the
  // base-weight reads
  const int npair = (qh + 1) / 2;
  for (int it = tid; it < own * 2 * npair; it += blockDim.x) {
    const int cl = it % own, hk = it / own, h = hk / npair, k0 = 2 * (hk - h * npair);
    const int k1 = min(k0 + 1, qh - 1);
    const double u = h == 0 ? s_m[1][cl + R1_HALO] : -s_m[1][cl + R1_HALO];
    const double *Gc = s_G[cl][h];
    const double *l0 = s_lam[k0], *l1 = s_lam[k1];
    double x0a = 0.0, x0b = 0.0, mb0 = 0.0, mb1 = 0.0, mb2 = 0.0;
#pragma unroll 8
    for (int m = 0; m < NB; m++) {
      const double gv = Gc[m], d = s_bh[0][m] - u, hv = s_bh[1][m] * gv;
      x0a += gv * l0[m]; x0b += gv * l1[m];
      mb0 += hv; mb1 += hv * d; mb2 += hv * d * d;
    }
    const double sg = h ? -1.0 : 1.0, n = s_c[cl][0];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int k = k0 + j;
      if (k >= qh) break;
      const double x0 = j == 0 ? x0a : x0b;
      const double dk = s_px[k] - u, ck = lat[lo.ck + k];
      const double X[4] = {x0, sg * (dk * x0 + ck * mb0), dk * dk * x0 + ck * (dk * mb0 + mb1),
                           sg * (dk * dk * dk * x0 + ck * (dk * dk * mb0 + dk * mb1 + mb2))};
      const int kx = h * qh + k;
      for (int ky = 0; ky < qy; ky++) {
        double tp = 0.0, tt = 0.0;
#pragma unroll
        for (int a = 0; a < 4; a++) { tp += s_y[cl][0][a][D == 2 ? ky : 0] * X[a]; tt += s_y[cl][1][a][D == 2 ? ky : 0] * X[a]; }
        s_t[kx * qy + ky][cl] = n * tp;
        s_t[Kh + kx * qy + ky][cl] = n * tt;
      }
    }
  }
  __syncthreads();

  // advection, body force, relaxation and the RK combination: a thread takes
  // one row and a strip of 4 owned cells, reconstructing the strip's 5 faces once
  const double nwl = c0 < 3 ? s_nw[0] : 0.0, nwr = c0 + own + 2 >= nx ? s_nw[1] : 0.0;
  for (int it = tid; it < R * NS; it += blockDim.x) {
    const int r = it / NS, q = it - r * NS, cl0 = q * SW;
    if (cl0 >= own) continue;
    const int ncl = min(SW, own - cl0);
    const int rh = r < Kh ? r : r - Kh, ky = ky_of(rh);
    const double p = s_px[kx_of(rh)];
    const double *row = s_g[r];
    const double fwl = nwl * c.gw[r], fwr = nwr * c.gw[R + r];
    // face j (left face of cell j) in the upwind frame, with the wall rules:
    // emitted populations take n_w g^w at the wall face and as ghosts; at the
    // first interior faces of an incoming population the candidates that
    // would reach past the wall are dropped; faces clear of both walls use
    // the branch-free interior form
    auto face = [&](int j) -> double {
      if (p > 0.0) {
        if (j >= 3 && j <= nx - 2) {
          const int b = j - c0 + R1_HALO;
          return weno_face_interior<double>(row[b - 3], row[b - 2], row[b - 1], row[b], row[b + 1]);
        }
        if (j == 0) return fwl;
        double v[5];
#pragma unroll
        for (int s2 = 0; s2 < 5; s2++) {
          const int cc = j - 3 + s2;
          v[s2] = cc < 0 ? fwl : (cc >= nx ? 0.0 : row[cc - c0 + R1_HALO]);
        }
        const int mode = j == nx ? 2 : (j == nx - 1 ? 1 : 0);
        return weno_face<double>(v[0], v[1], v[2], v[3], v[4], mode);
      }
      if (j >= 2 && j <= nx - 3) {
        const int b = j - c0 + R1_HALO;
        return weno_face_interior<double>(row[b + 2], row[b + 1], row[b], row[b - 1], row[b - 2]);
      }
      if (j == nx) return fwr;
      double v[5];
#pragma unroll
      for (int s2 = 0; s2 < 5; s2++) {
        const int cc = j + 2 - s2;
        v[s2] = cc >= nx ? fwr : (cc < 0 ? 0.0 : row[cc - c0 + R1_HALO]);
      }
      const int mode = j == 0 ? 2 : (j == 1 ? 1 : 0);
      return weno_face<double>(v[0], v[1], v[2], v[3], v[4], mode);
    };
    double fl = face(c0 + cl0);
#pragma unroll
    for (int u = 0; u < SW; u++) {
      if (u >= ncl) break;
      const int cl = cl0 + u, i = c0 + cl;
      const double fr = face(i + 1);
      const double cen = row[cl + R1_HALO];
      double L = (s_t[r][cl] - cen) * s_c[cl][1] - p * (fr - fl) * c.invdx[i];
      if (D == 2 && c.ay != 0.0) {
        // -a_y d/dp_y on the y-nodes of this x-node and population (App. A kernel)
        double sF = 0.0;
        for (int k2 = 0; k2 < qy; k2++) sF += s_km[ky * qy + k2] * s_g[r - ky + k2][cl + R1_HALO];
        L -= c.ay * sF;
      }
      const double adv = cen + c.dt * L;
      double o;
      if (STAGE == 1) o = adv;
      else {
        const double fn = c.f[(size_t)r * nx + i];
        o = STAGE == 2 ? 0.75 * fn + 0.25 * adv : fn * (1.0 / 3.0) + (2.0 / 3.0) * adv;
      }
      gout[(size_t)r * nx + i] = o;
      fl = fr;
    }
  }
}

// moments [FDLB_NMOM][nx] of the reduced state f^n: n, u_x, u_y, T, q_x, q_y,
// P_xx, P_xy, P_yy, P_zz (1D: u_y = q_y = P_xy = 0 and P_yy = P_zz = half the
// theta sum; 2D: P_zz = the theta sum)
__global__ void k_r1_moments(const R1Dev *__restrict__ cases, int c_idx) {
  const R1Dev &c = cases[c_idx];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.nx) return;
  const int nx = c.nx, qy = c.qy, Kh = 2 * c.qh * qy;
  const double *px = c.lat + c.lo.px, *py = c.lat + c.lo.py;
  const bool two = c.dim == 2;
  double n = 0.0, jx = 0.0, jy = 0.0;
  for (int r = 0; r < Kh; r++) {
    const double v = c.f[(size_t)r * nx + i];
    n += v; jx += px[r / qy] * v;
    if (two) jy += py[r % qy] * v;
  }
  const double ux = jx / n, uy = jy / n;
  double pxx = 0.0, pxy = 0.0, pyy = 0.0, th = 0.0, qx = 0.0, qy_ = 0.0;
  for (int r = 0; r < Kh; r++) {
    const double cx = px[r / qy] - ux, cy = two ? py[r % qy] - uy : 0.0;
    const double ph = c.f[(size_t)r * nx + i], tt = c.f[(size_t)(Kh + r) * nx + i], c2 = cx * cx + cy * cy;
    pxx += cx * cx * ph; pxy += cx * cy * ph; pyy += cy * cy * ph; th += tt;
    qx += cx * (0.5 * c2 * ph + 0.5 * tt); qy_ += cy * (0.5 * c2 * ph + 0.5 * tt);
  }
  double *mo = c.mom;
  mo[i] = n; mo[nx + i] = ux; mo[2 * nx + i] = uy; mo[3 * nx + i] = (pxx + pyy + th) / (3.0 * n);
  mo[4 * nx + i] = qx; mo[5 * nx + i] = qy_; mo[6 * nx + i] = pxx; mo[7 * nx + i] = pxy;
  mo[8 * nx + i] = two ? pyy : 0.5 * th; mo[9 * nx + i] = two ? th : 0.5 * th;
}

template <int RM, int D, int TS>
static void r1_launch(int stage, const R1Dev *cases, const int2 *m, int nblocks, hipStream_t s) {
  if (stage == 1) hipLaunchKernelGGL((k_r1_stage<1, RM, D, TS>), dim3(nblocks), dim3(512), 0, s, cases, m);
  else if (stage == 2) hipLaunchKernelGGL((k_r1_stage<2, RM, D, TS>), dim3(nblocks), dim3(512), 0, s, cases, m);
  else hipLaunchKernelGGL((k_r1_stage<3, RM, D, TS>), dim3(nblocks), dim3(512), 0, s, cases, m);
}

// cells per block: 32 up to 128 rows, 16 up to 256, 4 above; maps of at most
// 256 rows that would have at most R1_SMALL_MAP blocks take CTILE_SMALL
// cells per block (latency-bound sizes)
int r1_tile(int rmax, int total_cells) {
  if (rmax > R1_RMAX) return R1_TILE_BIG;
  const int t = rmax <= 128 ? R1_TILE : R1_TILE_2;
  return (total_cells + t - 1) / t <= R1_SMALL_MAP ? CTILE_SMALL : t;
}

template <int RM, int D>
static bool r1_by_tile(int stage, const R1Dev *cases, const int2 *m, int nblocks, int tile, hipStream_t s) {
  if constexpr (RM > R1_RMAX) {
    // the largest row counts take 4-cell tiles only (the LDS holds RM rows)
    if (tile != R1_TILE_BIG) return false;
    r1_launch<RM, D, R1_TILE_BIG>(stage, cases, m, nblocks, s);
  } else {
    constexpr int TL = RM <= 128 ? R1_TILE : R1_TILE_2;
    if (tile == TL) r1_launch<RM, D, TL>(stage, cases, m, nblocks, s);
    else if (tile == CTILE_SMALL) r1_launch<RM, D, CTILE_SMALL>(stage, cases, m, nblocks, s);
    else return false;
  }
  return true;
}

// one stage of one group: the instantiation that holds the group's rows
static bool r1_group_stage(int stage, const R1Dev *cases, const R1Group &g, int dim, hipStream_t s) {
  const int2 *m = (const int2 *)g.map;
  if (dim == 1) {
    if (g.rmax <= 64) return r1_by_tile<64, 1>(stage, cases, m, g.nblocks, g.tile, s);
    if (g.rmax <= 4 * MAXQH) return r1_by_tile<4 * MAXQH, 1>(stage, cases, m, g.nblocks, g.tile, s);
  } else if (dim == 2) {
    if (g.rmax <= 128) return r1_by_tile<128, 2>(stage, cases, m, g.nblocks, g.tile, s);
    if (g.rmax <= R1_RMAX) return r1_by_tile<R1_RMAX, 2>(stage, cases, m, g.nblocks, g.tile, s);
    if (g.rmax <= R1_RMAX_BIG) return r1_by_tile<R1_RMAX_BIG, 2>(stage, cases, m, g.nblocks, g.tile, s);
  }
  return false;
}

hipError_t launch_r1_step(const R1Dev *cases, const R1Group *groups, int ngroups, int dim, const int *map_n,
                          int nblocks_n, size_t lds_n, long nsteps, hipStream_t s) {
  if (nblocks_n > 0 && (lds_n == 0 || lds_n > NBAR_LDS_MAX)) return hipErrorInvalidValue;
  const int2 *mn = (const int2 *)map_n;
  // check every group's launch shape before the first launch
  for (int gi = 0; gi < ngroups; gi++) {
    const R1Group &g = groups[gi];
    if (g.nblocks == 0) continue;
    if (g.nblocks < 0 || !g.map || g.rmax <= 0 || g.rmax > (dim == 1 ? 4 * MAXQH : R1_RMAX_BIG)) return hipErrorInvalidValue;
    if (g.rmax > R1_RMAX ? g.tile != R1_TILE_BIG
                         : (g.tile != CTILE_SMALL && g.tile != (g.rmax <= 128 ? R1_TILE : R1_TILE_2)))
      return hipErrorInvalidValue;
  }
  for (long k = 0; k < nsteps; k++)
    for (int stage = 1; stage <= 3; stage++) {
      if (nblocks_n > 0) hipLaunchKernelGGL(k_r1_nbar, dim3(nblocks_n), dim3(512), lds_n, s, cases, mn, stage);
      // the groups hold different cases: their launches of a stage are independent
      for (int gi = 0; gi < ngroups; gi++)
        if (groups[gi].nblocks > 0 && !r1_group_stage(stage, cases, groups[gi], dim, s)) return hipErrorInvalidValue;
    }
  return hipGetLastError();
}

hipError_t launch_r1_moments(const R1Dev *cases, int c, int nx, hipStream_t s) {
  hipLaunchKernelGGL(k_r1_moments, dim3((nx + 255) / 256), dim3(256), 0, s, cases, c);
  return hipGetLastError();
}

}  // namespace fdlb
