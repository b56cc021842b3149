// lattice.cpp -- host construction of the velocity lattice, projection
// constants, grid metric and finite-difference weights for one case.
//
// Route (independent of how the paper states the rules): the half-range
// recurrence coefficients come from a discretised Stieltjes procedure in long
// double on a composite Gauss-Legendre discretisation of the half-range weight
// exp(-p^2/2)/sqrt(2 pi) on [0, inf) (Sec. III.A.2, eq:hh_ortho); nodes are the
// eigenvalues of the Jacobi matrix found by Sturm-sequence bisection and the
// weights are Christoffel numbers 1/sum_l h_l(p_k)^2.  Full-range
// Gauss-Hermite rules (App. A) use the known Jacobi matrix of the normal
// density (alpha_l = sqrt(l), beta = 0) with the same eigen/weight route.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fdlb_common.h"
#include "fdlb_host.h"

namespace fdlb {

typedef long double ld;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton on P_n (long double)
static void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
  x.assign(n, 0); w.assign(n, 0);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; i++) {
    ld z = cosl(pi * (i + 0.75L) / (n + 0.5L)), dp = 0;
    for (int it = 0; it < 100; it++) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; k++) { ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-20L) break;
    }
    ld p0 = 1, p1 = z;
    for (int k = 2; k <= n; k++) { ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = z; w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// recurrence coefficients of the orthonormal polynomials of the half-range
// weight: p h_l = a[l+1] h_{l+1} + b[l] h_l + a[l] h_{l-1}, h_0 = 1/sqrt(mu0)
// (composite Gauss-Legendre on [0, PMAX]: h_l^2 times the weight is below
// 1e-100 of its mass beyond PMAX for every l <= L; the panels keep a few
// half-oscillations of h_L each)
static void half_range_recurrence(int L, std::vector<ld> &a, std::vector<ld> &b, ld &mu0) {
  const bool high = L > 64;
  const int NP = high ? 160 : 64, NG = 24;
  const ld PMAX = high ? 64.0L : 32.0L, pi = 3.141592653589793238462643383279502884L;
  std::vector<ld> gx, gw;
  gauss_legendre(NG, gx, gw);
  std::vector<ld> X, W;
  for (int p = 0; p < NP; p++) {
    ld lo = PMAX * p / NP, hi = PMAX * (p + 1) / NP;
    for (int g = 0; g < NG; g++) {
      ld xx = lo + (hi - lo) * (gx[g] + 1) / 2;
      X.push_back(xx);
      W.push_back(gw[g] * (hi - lo) / 2 * expl(-xx * xx / 2) / sqrtl(2 * pi));
    }
  }
  size_t N = X.size();
  std::vector<ld> hm1(N, 0), h0(N), h1(N);
  mu0 = 0;
  for (size_t i = 0; i < N; i++) mu0 += W[i];
  for (size_t i = 0; i < N; i++) h0[i] = 1 / sqrtl(mu0);
  a.assign(L + 1, 0); b.assign(L + 1, 0);
  for (int l = 0; l <= L; l++) {
    ld s = 0;
    for (size_t i = 0; i < N; i++) s += W[i] * X[i] * h0[i] * h0[i];
    b[l] = s;
    if (l == L) break;
    ld nrm = 0;
    for (size_t i = 0; i < N; i++) {
      h1[i] = (X[i] - b[l]) * h0[i] - a[l] * hm1[i];
      nrm += W[i] * h1[i] * h1[i];
    }
    a[l + 1] = sqrtl(nrm);
    for (size_t i = 0; i < N; i++) { hm1[i] = h0[i]; h0[i] = h1[i] / a[l + 1]; }
  }
}

// eigenvalues of the symmetric tridiagonal (diag b[0..n-1], offdiag a[1..n-1])
// by Sturm-sequence bisection, ascending
static void jacobi_eigs(int n, const std::vector<ld> &a, const std::vector<ld> &b, std::vector<ld> &ev) {
  ld lo = 1e30L, hi = -1e30L;
  for (int i = 0; i < n; i++) {
    ld r = (i > 0 ? fabsl(a[i]) : 0) + (i + 1 < n ? fabsl(a[i + 1]) : 0);
    lo = fminl(lo, b[i] - r); hi = fmaxl(hi, b[i] + r);
  }
  auto count_below = [&](ld x) {
    int c = 0; ld d = 1;
    for (int i = 0; i < n; i++) {
      ld off = i > 0 ? a[i] * a[i] : 0;
      d = (b[i] - x) - (i > 0 ? off / d : 0);
      if (d == 0) d = -1e-300L;
      if (d < 0) c++;
    }
    return c;
  };
  ev.assign(n, 0);
  for (int k = 0; k < n; k++) {
    ld l = lo, h = hi;
    for (int it = 0; it < 200; it++) {
      ld m = (l + h) / 2;
      if (count_below(m) > k) h = m; else l = m;
      if (h - l <= 1e-21L * (1 + fabsl(m))) break;
    }
    ev[k] = (l + h) / 2;
  }
}

// orthonormal polynomial values h_0..h_L at x from the recurrence
static void ortho_vals(ld x, int L, const std::vector<ld> &a, const std::vector<ld> &b, ld mu0, ld *h) {
  h[0] = 1 / sqrtl(mu0);
  if (L >= 1) h[1] = (x - b[0]) * h[0] / a[1];
  for (int l = 1; l < L; l++) h[l + 1] = ((x - b[l]) * h[l] - a[l] * h[l - 1]) / a[l + 1];
}

static void ortho_derivs(ld x, int L, const std::vector<ld> &a, const std::vector<ld> &b, ld mu0, ld *h, ld *dh) {
  ortho_vals(x, L, a, b, mu0, h);
  dh[0] = 0;
  if (L >= 1) dh[1] = h[0] / a[1];
  for (int l = 1; l < L; l++) dh[l + 1] = ((x - b[l]) * dh[l] + h[l] - a[l] * dh[l - 1]) / a[l + 1];
}

static void gauss_rule(int Q, const std::vector<ld> &a, const std::vector<ld> &b, ld mu0,
                       std::vector<ld> &x, std::vector<ld> &w) {
  jacobi_eigs(Q, a, b, x);
  w.assign(Q, 0);
  std::vector<ld> h(Q + 1);
  for (int k = 0; k < Q; k++) {
    ortho_vals(x[k], Q - 1, a, b, mu0, h.data());
    ld s = 0;
    for (int l = 0; l < Q; l++) s += h[l] * h[l];
    w[k] = 1 / s;
  }
}

// first-derivative weights at x0 on points xs[0..n-1]: derivative of the
// Lagrange basis, l_j'(x0) = sum_{m != j} 1/(x_j - x_m) prod_{l != j,m} (x0 - x_l)/(x_j - x_l)
static void lagrange_d1(ld x0, const ld *xs, int n, ld *c1) {
  for (int j = 0; j < n; j++) {
    ld s = 0;
    for (int m = 0; m < n; m++) {
      if (m == j) continue;
      ld t = 1 / (xs[j] - xs[m]);
      for (int l = 0; l < n; l++)
        if (l != j && l != m) t *= (x0 - xs[l]) / (xs[j] - xs[l]);
      s += t;
    }
    c1[j] = s;
  }
}

static double chi_cs(double eta) { return 0.5 * (2 - eta) / ((1 - eta) * (1 - eta) * (1 - eta)); }

int validate(const fdlb_params &p, std::string &why, double *sigma, double *R) {
  if (!(p.nx >= 7)) { why = "nx must be >= 7"; return -1; }
  if (p.qx_half < 1 || p.qx_half > MAXQH_WIDE) { why = "qx_half must be in [1, 200]"; return -1; }
  if (p.qy < 2 || p.qy > MAXQY || p.qz < 2 || p.qz > MAXQY) { why = "qy, qz must be in [2, 8]"; return -1; }
  if (!(p.eta0 >= 0 && p.eta0 < 0.5)) { why = "eta0 must be in [0, 0.5)"; return -1; }
  if (p.kn <= 0 && p.eta0 > 0) { why = "Kn = infinity requires eta0 = 0"; return -1; }
  if (p.collision < 0 || p.collision > 2) { why = "unknown collision model"; return -1; }
  if (p.collision == 1 && !(p.pr_fixed > 0)) { why = "pr_fixed must be positive"; return -1; }
  if (p.grid != 0 && p.grid != 1) { why = "unknown grid"; return -1; }
  if (p.grid == 1 && !(p.stretch > 0)) { why = "tanh grid needs stretch > 0"; return -1; }
  if (p.precision != 0 && p.precision != 1) { why = "unknown precision"; return -1; }
  if (p.x_rule != 0 && p.x_rule != 1) { why = "x_rule must be 0 (half-range) or 1 (full-range)"; return -1; }
  if (p.x_rule == 1 && 2 * p.qx_half > MAXQH_WIDE) { why = "full-range x rule: 2 qx_half must be <= 200"; return -1; }
  if (p.chi_mode != 0 && p.chi_mode != 1) { why = "chi_mode must be 0 (local) or 1 (revised Enskog average)"; return -1; }
  if (p.chi_mode == 1 && p.nx > 4000) { why = "chi_mode 1 supports nx <= 4000 (averaging windows are staged in LDS)"; return -1; }
  if (!(p.t_left > 0 && p.t_right > 0 && p.t_init > 0 && p.n_init > 0)) { why = "temperatures and density must be positive"; return -1; }
  if (!(p.dt > 0) && !(p.cfl > 0)) { why = "need cfl > 0 or dt > 0"; return -1; }
  double s = 0, r = INFINITY;
  if (p.eta0 > 0) {
    r = 1.0 / (6.0 * sqrt(2.0) * p.eta0 * chi_cs(p.eta0) * p.kn);
    if (!(r > 1.0)) { why = "confinement ratio R <= 1 (channel narrower than a molecule)"; return -1; }
    s = 1.0 / r;
  }
  if (sigma) *sigma = s;
  if (R) *R = r;
  return 0;
}

// Build every host-side constant of one case.
int build_case(const fdlb_params &p, CaseHost &c, std::string &why) {
  double sigma, R;
  if (validate(p, why, &sigma, &R)) return -1;
  c.p = p;
  c.nx = p.nx; c.qh = p.qx_half; c.qy = p.qy; c.qz = p.qz;
  c.K = 2 * c.qh * c.qy * c.qz;
  c.nxp = fslots(c.nx);
  c.sigma = sigma; c.R = R; c.Lc = 1.0 - sigma;
  c.chi0 = chi_cs(p.eta0);
  // x rule: half-range of order Q per half (Sec. III.A.2), or full-range of
  // order 2Q (App. A; its projections alias through terms of degree >= 2 nb - 2Q,
  // so it always takes the NB_WIDE base rule)
  const bool full_x = p.x_rule == 1;
  const int Q = c.qh, QX = full_x ? 2 * Q : Q, nb = full_x ? NB_WIDE : base_nodes(Q);
  c.wide = nb == NB_WIDE;
  // lattice offsets
  LatOff &o = c.lo;
  int off = 0;
  // p_x .. H_z form one contiguous block in this order (the table kernel
  // stages it with a single linear copy)
  o.px = off; off += 2 * Q;
  o.bP = off; off += nb;
  o.bA = off; off += nb;
  o.hQ = off; off += nb;
  o.lam = off; off += Q * nb;
  o.ck = off; off += Q;
  o.Hy = off; off += c.qy * c.qy;
  o.Hz = off; off += c.qz * c.qz;
  o.nb = nb;
  o.py = off; off += c.qy;
  o.pz = off; off += c.qz;
  o.kmat = off; off += c.qy * c.qy;
  o.fdw = off; off += 3 * 7;
  o.xf = off; off += c.nx + 1;     // cell faces
  o.xcn = off; off += c.nx;        // cell centres
  o.wlo = off; off += c.nx;        // first and last cell of each averaging window
  o.whi = off; off += c.nx;
  off = (off + 7) & ~7;   // 64-byte aligned rows (one scalar load per velocity)
  o.phi = off; off += c.K * 8;
  o.bg = off; off += c.K;
  o.kbg = off; off += c.K;
  o.bgm = off; off += NRAW;
  o.xbg = off; off += 2 * Q;
  o.yzbg = off; off += c.qy * c.qz;
  o.f32 = off; off += (4 * Q + c.qy * c.qz + 1) / 2;
  o.total = off;
  c.lat.assign(off, 0.0);
  double *L = c.lat.data();

  // x rule and the base rule of order nb: the half-range family, or the
  // full-range one (normal density, alpha_l = sqrt(l), beta = 0, mu0 = 1); the
  // lattice holds the Q positive nodes p_k (ascending) and their mirror images
  std::vector<ld> a, b, xq, wq, xb, wb;
  ld mu0;
  int Lmax = std::max(nb, QX) + 2;
  if (full_x) {
    a.assign(Lmax + 1, 0); b.assign(Lmax + 1, 0); mu0 = 1;
    for (int l = 1; l <= Lmax; l++) a[l] = sqrtl((ld)l);
  } else {
    half_range_recurrence(Lmax, a, b, mu0);
  }
  gauss_rule(QX, a, b, mu0, xq, wq);
  gauss_rule(nb, a, b, mu0, xb, wb);
  const int k0 = QX - Q;   // first positive node
  c.wx.assign(2 * Q, 0);
  for (int k = 0; k < Q; k++) {
    L[o.px + k] = (double)xq[k0 + k]; L[o.px + Q + k] = -(double)xq[k0 + k];
    c.wx[k] = c.wx[Q + k] = (double)wq[k0 + k];
  }
  std::vector<ld> h(Lmax + 2), dh(Lmax + 2), hb(Lmax + 2);
  // Lagrange basis of the QX lattice nodes at the base nodes (Christoffel-Darboux
  // sum), kept for the positive nodes
  std::vector<std::vector<ld>> hk(Q, std::vector<ld>(QX + 1));
  for (int k = 0; k < Q; k++) {
    ortho_derivs(xq[k0 + k], QX, a, b, mu0, h.data(), dh.data());
    for (int l = 0; l <= QX; l++) hk[k][l] = h[l];
    L[o.ck + k] = (double)(1 / dh[QX]);
  }
  for (int m = 0; m < nb; m++) {
    ortho_vals(xb[m], QX, a, b, mu0, hb.data());
    L[o.bP + m] = (double)xb[m];
    L[o.bA + m] = (double)(logl(wb[m]) + xb[m] * xb[m] / 2);
    L[o.hQ + m] = (double)hb[QX];
    for (int k = 0; k < Q; k++) {
      ld s = 0;
      for (int l = 0; l < QX; l++) s += hk[k][l] * hb[l];
      L[o.lam + k * nb + m] = (double)(wq[k0 + k] * s);
    }
  }
  // full-range rules on y and z (normal density, alpha_l = sqrt(l), beta = 0)
  auto gh = [&](int q, int poff, int hoff, std::vector<double> &wout) {
    std::vector<ld> ga(q + 2, 0), gb(q + 2, 0), x, w;
    for (int l = 1; l <= q + 1; l++) ga[l] = sqrtl((ld)l);
    gauss_rule(q, ga, gb, 1.0L, x, w);
    wout.assign(q, 0);
    for (int k = 0; k < q; k++) {
      L[poff + k] = (double)x[k]; wout[k] = (double)w[k];
      // w_k He_l(p_k) / l!
      ld he[MAXQY + 2];
      he[0] = 1; he[1] = x[k];
      for (int l = 1; l < q; l++) he[l + 1] = x[k] * he[l] - l * he[l - 1];
      ld fact = 1;
      for (int l = 0; l < q; l++) {
        L[hoff + k * q + l] = (double)(w[k] * he[l] / fact);
        fact *= (l + 1);
      }
    }
  };
  gh(c.qy, o.py, o.Hy, c.wy);
  gh(c.qz, o.pz, o.Hz, c.wz);
  // momentum-derivative kernel K_{k,k'} = -w_k sum_{l=0}^{q-2} He_{l+1}(p_k) He_l(p_k') / l!
  {
    std::vector<std::vector<ld>> he(c.qy, std::vector<ld>(c.qy + 1));
    for (int k = 0; k < c.qy; k++) {
      ld xk = L[o.py + k];
      he[k][0] = 1; he[k][1] = xk;
      for (int l = 1; l < c.qy; l++) he[k][l + 1] = xk * he[k][l] - l * he[k][l - 1];
    }
    for (int k = 0; k < c.qy; k++)
      for (int k2 = 0; k2 < c.qy; k2++) {
        ld s = 0, fact = 1;
        for (int l = 0; l <= c.qy - 2; l++) { s += he[k][l + 1] * he[k2][l] / fact; fact *= (l + 1); }
        L[o.kmat + k * c.qy + k2] = (double)(-c.wy[k] * s);
      }
  }
  // one-sided 7-point first-derivative weights for the three wall-adjacent cells
  for (int r = 0; r < 3; r++) {
    ld xs[7], w7[7];
    for (int j = 0; j < 7; j++) xs[j] = j;
    lagrange_d1((ld)r, xs, 7, w7);
    for (int j = 0; j < 7; j++) L[o.fdw + r * 7 + j] = (double)w7[j];
  }
  // moment weights per velocity
  for (int kx = 0; kx < 2 * Q; kx++)
    for (int ky = 0; ky < c.qy; ky++)
      for (int kz = 0; kz < c.qz; kz++) {
        const int kap = (kx * c.qy + ky) * c.qz + kz;
        const double px = L[o.px + kx], py = L[o.py + ky], pz = L[o.pz + kz];
        const double p2 = px * px + py * py + pz * pz;
        double *ph = &L[o.phi + kap * 8];
        ph[0] = px; ph[1] = py; ph[2] = px * px; ph[3] = px * py; ph[4] = py * py; ph[5] = pz * pz;
        ph[6] = px * p2; ph[7] = py * p2;
      }
  // grid: eta_i = -1 + (i + 1/2) deta; x = (L_c/2) eta or (L_c/2) tanh(d eta)/tanh(d)
  c.deta = 2.0 / c.nx;
  c.x.assign(c.nx, 0); c.jac.assign(c.nx, 0); c.invdx.assign(c.nx, 0);
  double hmin = 1e300;
  for (int i = 0; i < c.nx; i++) {
    double eta = -1 + (i + 0.5) * c.deta;
    if (p.grid == 1) {
      double d = p.stretch, th = tanh(d), ch = cosh(d * eta);
      c.x[i] = 0.5 * c.Lc * tanh(d * eta) / th;
      c.jac[i] = 0.5 * c.Lc * d / (ch * ch * th);
    } else {
      c.x[i] = 0.5 * c.Lc * eta;
      c.jac[i] = 0.5 * c.Lc;
    }
    c.invdx[i] = 1.0 / (c.jac[i] * c.deta);
    hmin = fmin(hmin, c.jac[i] * c.deta);
  }
  c.dt = p.dt > 0 ? p.dt : p.cfl * hmin / fabs(L[o.px + Q - 1]);
  // averaging geometry of the revised Enskog contact value (faces, centres and
  // the cells each window |x' - x_i| < sigma overlaps; ranges stored as doubles)
  for (int j = 0; j <= c.nx; j++) {
    const double eta = -1 + j * c.deta;
    L[o.xf + j] = p.grid == 1 ? 0.5 * c.Lc * tanh(p.stretch * eta) / tanh(p.stretch) : 0.5 * c.Lc * eta;
  }
  for (int i = 0; i < c.nx; i++) {
    L[o.xcn + i] = c.x[i];
    int lo = i, hi = i;
    while (lo > 0 && L[o.xf + lo] > c.x[i] - sigma) lo--;
    while (hi < c.nx - 1 && L[o.xf + hi + 1] < c.x[i] + sigma) hi++;
    L[o.wlo + i] = lo; L[o.whi + i] = hi;
  }
  // wall Maxwellians at (u_x = 0, u_y = U_w, T_w) with n = 1, and the emitted flux
  // denominators sum_{emitted} p_x g^w
  for (int wall = 0; wall < 2; wall++) {
    double Tw = wall == 0 ? p.t_left : p.t_right, Uw = wall == 0 ? p.uy_left : p.uy_right;
    std::vector<double> X(2 * Q), Y(c.qy), Z(c.qz);
    host_half_table(L, o, Q, 0.0, Tw, 0, X.data());
    host_full_table(&L[o.Hy], c.qy, Uw, Tw, 0, Y.data());
    host_full_table(&L[o.Hz], c.qz, 0.0, Tw, 0, Z.data());
    c.gw[wall].assign(c.K, 0);
    double den = 0;
    for (int kx = 0; kx < 2 * Q; kx++)
      for (int ky = 0; ky < c.qy; ky++)
        for (int kz = 0; kz < c.qz; kz++) {
          int kap = (kx * c.qy + ky) * c.qz + kz;
          double v = X[kx] * Y[ky] * Z[kz];
          c.gw[wall][kap] = v;
          double pxv = L[o.px + kx];
          if ((wall == 0 && pxv > 0) || (wall == 1 && pxv < 0)) den += fabs(pxv) * v;
        }
    c.wallD[wall] = den;
  }
  // background: the projected uniform initial state n_init f^MB(u_y = uy_init, T = t_init)
  {
    std::vector<double> X(2 * Q), Y(c.qy), Z(c.qz);
    host_half_table(L, o, Q, 0.0, p.t_init, 0, X.data());
    host_full_table(&L[o.Hy], c.qy, p.uy_init, p.t_init, 0, Y.data());
    host_full_table(&L[o.Hz], c.qz, 0.0, p.t_init, 0, Z.data());
    for (int m = 0; m < NRAW; m++) L[o.bgm + m] = 0;
    for (int kx = 0; kx < 2 * Q; kx++) L[o.xbg + kx] = p.n_init * X[kx];
    for (int ky = 0; ky < c.qy; ky++)
      for (int kz = 0; kz < c.qz; kz++) L[o.yzbg + ky * c.qz + kz] = Y[ky] * Z[kz];
    for (int kx = 0; kx < 2 * Q; kx++)
      for (int ky = 0; ky < c.qy; ky++)
        for (int kz = 0; kz < c.qz; kz++) {
          const int kap = (kx * c.qy + ky) * c.qz + kz;
          const double b = L[o.xbg + kx] * L[o.yzbg + ky * c.qz + kz];
          L[o.bg + kap] = b;
          L[o.bgm] += b;
          for (int m = 1; m < NRAW; m++) L[o.bgm + m] += L[o.phi + kap * 8 + m - 1] * b;
        }
    for (int kx = 0; kx < 2 * Q; kx++)
      for (int ky = 0; ky < c.qy; ky++)
        for (int kz = 0; kz < c.qz; kz++) {
          double sf = 0;
          for (int k2 = 0; k2 < c.qy; k2++) sf += L[o.kmat + ky * c.qy + k2] * L[o.bg + (kx * c.qy + k2) * c.qz + kz];
          L[o.kbg + (kx * c.qy + ky) * c.qz + kz] = sf;
        }
  }
  {
    std::vector<float> f(4 * Q + c.qy * c.qz);
    for (int kx = 0; kx < 2 * Q; kx++) {
      f[kx] = (float)L[o.px + kx];
      f[2 * Q + kx] = (float)L[o.xbg + kx];
    }
    for (int yz = 0; yz < c.qy * c.qz; yz++) f[4 * Q + yz] = (float)L[o.yzbg + yz];
    std::memcpy(&L[o.f32], f.data(), f.size() * sizeof(float));
  }
  return 0;
}

}  // namespace fdlb
