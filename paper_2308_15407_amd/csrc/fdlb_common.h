// fdlb_common.h -- data layout shared by the host driver and the gfx950
// kernels of the FDLB channel solver, plus the per-axis projection formulas
// used both on the host (wall tables) and on the device (per-cell tables).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdlb {

constexpr int NB = 48;         // nodes of the half-range base rule used for projections
constexpr int MAXQH = 32;      // largest half-range order per half of the standard tables
// Orders above MAXQH (quadrature convergence studies) use the wide table
// kernel: a base rule of NB_WIDE nodes, exact to degree 2 NB_WIDE - 1, so
// that the projections onto h_l, l < Q, alias only through expansion terms of
// degree >= 2 NB_WIDE - Q + 1 (>= 89 at Q = MAXQH_WIDE), which are below
// rounding for the Maxwellians of wall temperature ratios up to 3.
constexpr int MAXQH_WIDE = 200;
constexpr int NB_WIDE = 144;
__host__ __device__ inline int base_nodes(int qh) { return qh > MAXQH ? NB_WIDE : NB; }
constexpr int MAXQY = 8;       // largest full-range order on y and z
constexpr int UTILE = 63;      // cells owned by one update wave (64 faces)
#ifndef FDLB_CTILE
#define FDLB_CTILE 16
#endif
constexpr int CTILE = FDLB_CTILE;  // cells per table block
// Table maps that would have at most SMALL_TABLE_MAP blocks of CTILE cells use
// blocks of CTILE_SMALL cells instead: twice the blocks, each with half the
// work, for small cases whose table pass is latency-bound (a 512-cell case:
// 66 blocks of 8 cells instead of 34 of 16).
constexpr int CTILE_SMALL = 8;
#ifndef FDLB_SMALL_TABLE_MAP
#define FDLB_SMALL_TABLE_MAP 64
#endif
constexpr int SMALL_TABLE_MAP = FDLB_SMALL_TABLE_MAP;
// the same rule for the reduced models' stage kernel, with its own threshold
constexpr int R1_SMALL_MAP = 32;
constexpr int CHALO = 6;       // moment halo of a table block
#ifndef FDLB_TABLE_WIDE_MAX
#define FDLB_TABLE_WIDE_MAX 128
#endif
constexpr int TABLE_WIDE_MAX = FDLB_TABLE_WIDE_MAX;  // table maps up to this many blocks use 512 threads
constexpr int NRAW = 9;        // raw moment sums per cell
constexpr int ROWBUF = 72;     // LDS row buffer of an interior update tile (69 cells, padded); two per wave

// Populations are stored per velocity in 64-slot tiles holding 63 cells each
// (one padding slot), so that the rows an update tile reads start on a
// 64-element boundary: cell i lives in slot i + i / 63.
__host__ __device__ inline int fslot(int cell) { return cell + cell / UTILE; }
__host__ __device__ inline int fslots(int nx) { return 64 * ((nx + UTILE - 1) / UTILE); }

// Offsets (in doubles) of the lattice constants of one case.
// px, bP, bA, hQ, lam, ck, Hy, Hz are contiguous in that order.
struct LatOff {
  int px, py, pz;   // node coordinates: [2qh], [qy], [qz]
  int kmat;         // momentum-derivative kernel [qy*qy] (App. A)
  int bP, bA;       // base rule nodes P_m and A_m = ln W_m + P_m^2/2, [nb] each
  int lam;          // Lagrange basis of the lattice nodes at the base nodes [qh*nb]
  int hQ;           // h_Q at the base nodes [nb]
  int ck;           // 1/h_Q'(p_k) [qh]
  int Hy, Hz;       // w_k He_l(p_k)/l!  [qy*qy], [qz*qz]
  int nb;           // nodes of the base rule (NB or NB_WIDE)
  int fdw;          // one-sided 7-point first-derivative weights, rows for cells 0,1,2 [3*7]
  int xf, xcn;      // cell faces [nx+1] and centres [nx]
  int wlo, whi;     // per cell, the first and last cell its averaging window overlaps [nx] each
  int phi;          // moment weights of every velocity [K][8] (64-byte rows): px, py, px^2, px py,
                    // py^2, pz^2, px |p|^2, py |p|^2 (the weight of the density sum is 1)
  int bg;           // background populations [K] (the case's uniform initial state); FP32 storage
                    // holds f - bg
  int kbg;          // body-force kernel applied to the background [K]
  int bgm;          // raw moment sums of the background [NRAW]
  int xbg, yzbg;    // factors of the background, bg[kappa] = xbg[kx] yzbg[ky*qz+kz]: n_init X^0[kx]
                    // [2qh] and Y^0[ky] Z^0[kz] [qyz]; FP32 tables hold n X_0 - xbg and YZ_0 - yzbg
  int f32;          // FP32 copies of px [2qh], xbg [2qh] and yzbg [qyz], two to a double slot
                    // (uniform operands of the FP32 update without conversions)
  int total;
};

// One case as the kernels see it (lives in device memory).
struct CaseDev {
  int nx, qh, qy, qz, K, nkx, qyz;
  int nxp;              // slots per velocity row of the population arrays (fslots(nx))
  int nchunk, kxc, ntile_u, ntile_c;
  int prec;             // active storage: 0 double, 1 float
  int collision, j1_shear;
  int active;
  int tlds;             // update blocks stage the projection tables of their tile in LDS
  int wide;             // the x tables use the NB_WIDE base rule (the wide table pass)
  double eta0, kn, chi0, pr_fixed, ay, dt;
  double tau_pre;       // (5 sqrt(2 pi)/16) Kn chi0 ; 0 when Kn = infinity
  double wallD[2];      // sum over emitted nodes of p_x g^w (left, right)
  int chi_mode;         // 0: chi(eta0 n); 1: chi(eta0 nbar), the revised Enskog average
  double sigma;         // molecular diameter in units of the channel width (1/R)
  double *nbar;         // [nx] average density of the current stage input (chi_mode 1)
  double nw[2];         // wall densities of the current stage input, written by the table
                        // pass's wall blocks; kept in the record so the update reads them
                        // with the other fields
  double *lat;          // lattice constants
  LatOff lo;
  double *invdx;        // [nx] 1/(J_i deta)
  void *f[2][3];        // populations f^n, f^(1), f^(2) per storage precision, [K][nxp] slots
  void *tabX[2];        // n X_a[kx] at [a][kx][cell]
  void *tabYZ[2];       // YZ_a[ky*qz+kz] at [a][yz][cell]
  void *invtau[2];      // [nx]
  void *gw[2][2];       // projected wall Maxwellians (n = 1) [K], per precision, per wall
  double *part;         // partial raw sums [nchunk][NRAW][nx]
  double *mom;          // [10][nx] moments of f^n (as of the last stage-1 table pass)
  unsigned long long *resid;  // residual bits (max of non-negative doubles)
  double *fields;       // staging [6][nx] for set_state
  double *noise;        // staging [K][nx] for set_state (may be unused)
};

// One case of a reduced model (Sec. II.B): phi and theta on the 2 qh x-nodes
// (1D flows, qy = 1) or the 2 qh x qy (x, y) nodes (2D flows).  Rows of the
// [R][nx] arrays: phi (kx, ky) at kx qy + ky, then theta; R = 4 qh qy.
constexpr int R1_TILE = 32;    // cells per block of the reduced stage kernel (up to 128 rows)
constexpr int R1_TILE_2 = 16;  // cells per block for 129..256 rows
constexpr int R1_RMAX = 256;
constexpr int R1_TILE_BIG = 4; // cells per block for 257..R1_RMAX_BIG rows (2D, qx_half qy <= 160)
constexpr int R1_RMAX_BIG = 640;   // rows of a reduced case
constexpr int R1_HALO = 6;     // moment halo (the one-sided wall stencils reach 6 cells)
struct R1Dev {
  int nx, qh, qy, R;
  int dim;              // 1 or 2
  int collision, j1_shear;
  double pr_fixed, eta0, tau_pre, dt, ay;
  const double *lat;    // lattice constants of the case (px, base rule, lambda, c_k, FD weights)
  LatOff lo;
  const double *invdx;  // [nx] 1 / (cell width)
  const double *gw;     // [2][R] wall phi/theta at n = 1 (left, right)
  double wallD[2];      // sum over the emitted phi rows of p_x g^w (left, right)
  double *f, *g1, *g2;  // [R][nx] f^n and the two RK stage states
  double *mom;          // [FDLB_NMOM][nx]
  int chi_mode;         // 0: chi(eta0 n); 1: chi(eta0 nbar), the revised Enskog average
  double sigma;         // molecular diameter (chi_mode 1)
  double *nbar;         // [nx] average density of the stage input (chi_mode 1)
};

// ---------------------------------------------------------------------------
// projection formulas
// ---------------------------------------------------------------------------

// Half-range table of g(p) (p-u)^a, a = 0..3, at the positive nodes p_k for the
// positive half line (with a full-range x rule, App. A, the same formulas on
// the full-range family give the full-range projection at the positive nodes).  With the base-rule weights G_m = W_m g(P_m)/omega(P_m)
// the Lagrange identity gives X_0[k] = sum_m G_m l_k(P_m); higher powers use
// (p-u)^a l_k(p) = (p_k-u)^a l_k(p) + h_Q(p)/h_Q'(p_k) sum_{b<a} (p_k-u)^{a-1-b} (p-u)^b.
// The negative half follows from X^-_a(u) = (-1)^a X^+_a(-u).
__host__ __device__ inline double base_weight(const double *lat, const LatOff &lo, int m, double u,
                                              double T, double rsT) {
  double d = lat[lo.bP + m] - u;
  return exp(lat[lo.bA + m] - d * d / (2.0 * T)) * rsT;
}

// full-range Hermite coefficients G^{(b)}_l = int g (p-u)^b He_l(p) dp, b=0..3, l<=L
template <int LMAX>
__host__ __device__ inline void hermite_coeffs(double u, double T, int L, double G[4][LMAX + 4]) {
  G[0][0] = 1.0;
  G[0][1] = u;
  for (int l = 1; l < L + 3; l++) G[0][l + 1] = u * G[0][l] + l * (T - 1.0) * G[0][l - 1];
  for (int b = 1; b < 4; b++)
    for (int l = 0; l <= L + 3 - b; l++)
      G[b][l] = G[b - 1][l + 1] + (l > 0 ? l * G[b - 1][l - 1] : 0.0) - u * G[b - 1][l];
}

// Host-side full table of the half-range projection of g (p-u)^a (both halves,
// 2qh entries, positive half first) -- used for the wall Maxwellians.
inline void host_half_table(const double *lat, const LatOff &lo, int qh, double u, double T, int a,
                            double *X) {
  double rsT = 1.0 / sqrt(T);
  const int nb = lo.nb;
  for (int side = 0; side < 2; side++) {
    double us = side == 0 ? u : -u;
    double G[NB_WIDE], mb[3] = {0, 0, 0};
    for (int m = 0; m < nb; m++) G[m] = base_weight(lat, lo, m, us, T, rsT);
    for (int m = 0; m < nb; m++) {
      double d = lat[lo.bP + m] - us, h = lat[lo.hQ + m] * G[m];
      mb[0] += h; mb[1] += h * d; mb[2] += h * d * d;
    }
    for (int k = 0; k < qh; k++) {
      double x0 = 0;
      for (int m = 0; m < nb; m++) x0 += G[m] * lat[lo.lam + k * nb + m];
      double dk = lat[lo.px + k] - us, ck = lat[lo.ck + k];
      double v;
      if (a == 0) v = x0;
      else if (a == 1) v = dk * x0 + ck * mb[0];
      else if (a == 2) v = dk * dk * x0 + ck * (dk * mb[0] + mb[1]);
      else v = dk * dk * dk * x0 + ck * (dk * dk * mb[0] + dk * mb[1] + mb[2]);
      X[side * qh + k] = (side == 1 && (a & 1)) ? -v : v;
    }
  }
}

inline void host_full_table(const double *H, int q, double u, double T, int b, double *Y) {
  double G[4][MAXQY + 4];
  hermite_coeffs<MAXQY>(u, T, q - 1, G);
  for (int k = 0; k < q; k++) {
    double s = 0;
    for (int l = 0; l < q; l++) s += H[k * q + l] * G[b][l];
    Y[k] = s;
  }
}

}  // namespace fdlb
