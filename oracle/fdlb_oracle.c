/*
 * fdlb_oracle.c -- plain FP64 CPU oracle for the finite-difference lattice
 * Boltzmann (FDLB) time step of Busuioc & Sofonea, "Bounded flows of dense
 * gases" (arXiv 2308.15407).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or generator with
 * the GPU path.
 *
 * The oracle takes the method's steps in the paper's order and notation with
 * plain loops and no blocking or fusion:
 *   - velocity space (Sec. III.A): half-range Hermite polynomials h_l built by
 *     orthonormalisation w.r.t. the half-range weight (eq:hh_ortho) with
 *     monomial coefficients h_{l,s} (eq:hh_exp) in quad precision; nodes are
 *     the positive roots of h_Q; weights from eq:hh_wk; full-range nodes are
 *     the roots of He_Q with weights eq:H_wk (App. A);
 *   - equilibrium-type targets: the half-range expansion coefficients
 *     (eq:hh_F / eq:hh_gk) and full-range coefficients (eq:g_H / eq:H_gk) of
 *     Maxwellian x polynomial, evaluated into weighted populations (eq:hh_fk);
 *   - moments (eq:macro_LB, Sec. II moments) as plain two-pass sums;
 *   - collision: Shakhov target (eq:j0) and the first-order Enskog
 *     correction J1 (eq:j1), transport data eq:chi, eq:viscosity, eq:prandtl,
 *     eq:tau and the Kn definition (Sec. II.A);
 *   - WENO-5 advection (eq:weno5_flux_x, eq:weno5_omega_x, eq:weno5_sigma),
 *     6th-order central gradients (Sec. III.B.3), diffuse walls (Sec. III.B),
 *     TVD Runge-Kutta (eq:rk3) on the cast form eq:cast.
 * Points where the paper is silent or garbled follow the readings listed in
 * the design notes (units, tau, collision modes, weight sign, expansion
 * normalisation, projection of the Shakhov/J1 polynomials, wall treatment,
 * stretched grid, residual).
 *
 * Pins (tests/test_oracle_pins.py) fix the quadratures, projections, chi, tau,
 * Pr, the force kernel, the target's conservation and balance laws, WENO, FD6,
 * RK3, Maxwellian invariance, wall mass conservation, symmetry, the dilute
 * limit and the free-molecular heat flux.  Parity unpinned: dense steady
 * profiles at finite Kn in general, for which no independent values exist.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared fdlb_oracle.c -lquadmath -lm
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 qf;

#define ORC_MAXQ 72   /* largest half-range order supported by the oracle */

/* ------------------------------------------------------------------------ */
/* parameters (mirrored by a ctypes Structure in oracle/oracle.py)          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int flow;                 /* 0 Fourier, 1 Couette, 2 Poiseuille (metadata) */
  double kn;                /* Knudsen number (Sec. II.A); <=0 means infinity */
  double eta0;              /* mean reduced density */
  double t_left, t_right;   /* wall temperatures */
  double uy_left, uy_right; /* wall tangential velocities */
  double ay;                /* body acceleration along y */
  double n_init, t_init, uy_init;
  int nx, grid;             /* grid: 0 uniform, 1 tanh-stretched */
  double stretch;
  int qx_half, qy, qz;
  int collision;            /* 0 BGK, 1 Shakhov fixed Pr, 2 Shakhov dense Pr */
  double pr_fixed;
  int chi_mode, j1_shear;
  double cfl, dt;
} orc_params;

typedef struct {
  orc_params p;
  int nx, qh, qy, qz, K, kx_n;
  /* half-range polynomials: coefficient h_{l,s} at hq[l*(qh+2)+s], l<=qh+1 */
  qf *hq;
  qf *hpk;                  /* h_l(p_k) at the positive nodes, [l*qh+k] */
  double *px, *wx;          /* [2qh] x nodes (positive half first) + weights */
  double *py, *wy, *pz, *wz;
  double *kmat;             /* [qy*qy] momentum-derivative kernel (App. A) */
  /* grid */
  double sigma, Lc, deta, dt, chi0;
  double *xc, *jac;         /* cell centres and metric dx/deta */
  /* state and scratch */
  double *f, *f1, *f2, *Lg;
  double *gw_l, *gw_r;      /* projected wall Maxwellians (n = 1), [K] */
  long steps;
  double resid, prev_mom_valid;
  double *prev_mom;         /* [4][nx] n, ux, uy, T of the previous step */
} orc_t;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */
static qf q_pi(void) { return M_PIq; }

/* half-range moment of the weight omega(p) = exp(-p^2/2)/sqrt(2 pi) on [0,inf):
   mu_s = 2^{s/2} Gamma((s+1)/2) / (2 sqrt(pi)) */
static qf hr_moment(int s) {
  return powq(2.0Q, (qf)s / 2) * tgammaq(((qf)s + 1) / 2) / (2 * sqrtq(q_pi()));
}

/* inner product of two monomial-coefficient polynomials w.r.t. omega on [0,inf) */
static qf hr_inner(const qf *a, int da, const qf *b, int db) {
  qf s = 0;
  for (int i = 0; i <= da; i++)
    for (int j = 0; j <= db; j++) s += a[i] * b[j] * hr_moment(i + j);
  return s;
}

static qf poly_eval_q(const qf *c, int deg, qf x) {
  qf r = 0;
  for (int i = deg; i >= 0; i--) r = r * x + c[i];
  return r;
}

/* Build h_0..h_{L} (orthonormal w.r.t. omega on [0,inf), eq:hh_ortho) as
   monomial coefficients (eq:hh_exp) by Gram-Schmidt of p*h_{l-1} against all
   previous polynomials (done twice for cleanliness), in quad precision.
   out[l*(L+1)+s] = h_{l,s}. */
static void hr_polys(int L, qf *out) {
  int W = L + 1;
  memset(out, 0, sizeof(qf) * W * W);
  out[0] = 1 / sqrtq(hr_moment(0));
  qf *v = (qf *)calloc(W, sizeof(qf));
  for (int l = 1; l <= L; l++) {
    memset(v, 0, sizeof(qf) * W);
    for (int s = 0; s < l; s++) v[s + 1] = out[(l - 1) * W + s]; /* p*h_{l-1} */
    for (int pass = 0; pass < 2; pass++)
      for (int m = 0; m < l; m++) {
        qf c = hr_inner(v, l, &out[m * W], m);
        for (int s = 0; s <= m; s++) v[s] -= c * out[m * W + s];
      }
    qf nrm = sqrtq(hr_inner(v, l, v, l));
    for (int s = 0; s <= l; s++) out[l * W + s] = v[s] / nrm;
  }
  free(v);
}

/* all real roots of a polynomial known to have n simple roots in (lo,hi):
   sign-change scan on a fine grid, then bisection in quad precision */
static int poly_roots(const qf *c, int deg, double lo, double hi, int n, double *roots) {
  int found = 0, NG = 200000;
  qf prevx = lo, prevv = poly_eval_q(c, deg, lo);
  for (int g = 1; g <= NG && found < n; g++) {
    qf x = lo + (hi - lo) * (qf)g / NG;
    qf v = poly_eval_q(c, deg, x);
    if (v == 0) { roots[found++] = (double)x; prevx = x; prevv = v; continue; }
    if ((prevv < 0 && v > 0) || (prevv > 0 && v < 0)) {
      qf a = prevx, b = x, fa = prevv;
      for (int it = 0; it < 200; it++) {
        qf m = (a + b) / 2, fm = poly_eval_q(c, deg, m);
        if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else b = m;
      }
      roots[found++] = (double)((a + b) / 2);
    }
    prevx = x; prevv = v;
  }
  return found;
}

/* probabilists' Hermite He_l(x) by its defining recurrence */
static qf he_q(int l, qf x) {
  qf a = 1, b = x;
  if (l == 0) return a;
  for (int k = 1; k < l; k++) { qf c = x * b - k * a; a = b; b = c; }
  return b;
}
static double he_d(int l, double x) {
  double a = 1, b = x;
  if (l == 0) return a;
  for (int k = 1; k < l; k++) { double c = x * b - k * a; a = b; b = c; }
  return b;
}

static double factorial(int n) { double r = 1; for (int i = 2; i <= n; i++) r *= i; return r; }

/* Full-range Gauss-Hermite rule of order Q (App. A): nodes are the roots of
   He_Q, weights w_k = Q! / He_{Q+1}(p_k)^2 (eq:H_wk). */
int orc_gh_rule(int Q, double *nodes, double *weights) {
  qf *c = (qf *)calloc(Q + 1, sizeof(qf));
  /* monomial coefficients of He_Q from the recurrence */
  qf *a = (qf *)calloc(Q + 2, sizeof(qf)), *b = (qf *)calloc(Q + 2, sizeof(qf)),
     *t = (qf *)calloc(Q + 2, sizeof(qf));
  a[0] = 1; if (Q >= 1) { b[1] = 1; }
  if (Q == 0) { c[0] = 1; }
  else {
    for (int k = 1; k < Q; k++) {
      memset(t, 0, sizeof(qf) * (Q + 2));
      for (int s = 0; s <= k; s++) t[s + 1] += b[s];
      for (int s = 0; s <= k; s++) t[s] -= k * a[s];
      memcpy(a, b, sizeof(qf) * (Q + 2)); memcpy(b, t, sizeof(qf) * (Q + 2));
    }
    for (int s = 0; s <= Q; s++) c[s] = b[s];
  }
  double bound = 2.0 * sqrt((double)Q) + 4.0;
  int n = poly_roots(c, Q, -bound, bound, Q, nodes);
  for (int k = 0; k < n; k++) {
    qf h = he_q(Q + 1, (qf)nodes[k]);
    weights[k] = (double)(tgammaq((qf)Q + 1) / (h * h));
  }
  free(a); free(b); free(t); free(c);
  return n == Q ? 0 : -1;
}

/* Half-range Gauss-Hermite rule of order Q (Sec. III.A.2): nodes are the
   positive roots of h_Q; weights from eq:hh_wk with the weight function
   exp(-p^2/2)/sqrt(2 pi):
     w_k = p_k a_Q^2 / ( h_{Q+1}(p_k)^2 [ p_k + h_Q(0)^2 / sqrt(2 pi) ] ),
   a_Q = h_{Q+1,Q+1} / h_{Q,Q}.   hcoef (optional) receives h_{l,s}. */
int orc_hr_rule(int Q, double *nodes, double *weights, qf *hcoef_out) {
  int W = Q + 2;
  qf *h = (qf *)malloc(sizeof(qf) * W * W);
  hr_polys(Q + 1, h);
  double bound = 2.5 * sqrt((double)Q) + 6.0;
  int n = poly_roots(&h[Q * W], Q, 0.0, bound, Q, nodes);
  qf aQ = h[(Q + 1) * W + Q + 1] / h[Q * W + Q];
  qf hq0 = h[Q * W + 0];
  for (int k = 0; k < n; k++) {
    qf pk = nodes[k];
    qf hn = poly_eval_q(&h[(Q + 1) * W], Q + 1, pk);
    weights[k] = (double)(pk * aQ * aQ / (hn * hn * (pk + hq0 * hq0 / sqrtq(2 * q_pi()))));
  }
  if (hcoef_out) memcpy(hcoef_out, h, sizeof(qf) * W * W);
  free(h);
  return n == Q ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* projections of Maxwellian x monomial onto the lattice                   */
/* ------------------------------------------------------------------------ */

/* E_s(a) = int_0^inf g(p) (p-u)^a p^s dp for the 1D Maxwellian
   g = exp(-(p-u)^2/(2T))/sqrt(2 pi T), s = 0..smax, in quad precision.
   Raw truncated moments I_j = int_0^inf g p^j obey
   I_0 = erfc(-u/sqrt(2T))/2, I_1 = u I_0 + T g(0), I_j = u I_{j-1} + (j-1) T I_{j-2}. */
static void trunc_moments(qf u, qf T, int a, int smax, qf *E) {
  int J = smax + a;
  qf *I = (qf *)malloc(sizeof(qf) * (J + 1));
  qf g0 = expq(-u * u / (2 * T)) / sqrtq(2 * q_pi() * T);
  I[0] = erfcq(-u / sqrtq(2 * T)) / 2;
  if (J >= 1) I[1] = u * I[0] + T * g0;
  for (int j = 2; j <= J; j++) I[j] = u * I[j - 1] + (j - 1) * T * I[j - 2];
  for (int s = 0; s <= smax; s++) {
    qf acc = 0, binom = 1;
    for (int i = 0; i <= a; i++) {
      /* binom = C(a,i) */
      acc += binom * powq(-u, a - i) * I[s + i];
      binom = binom * (a - i) / (i + 1);
    }
    E[s] = acc;
  }
  free(I);
}

/* Half-range projection of g(p) (p-u)^a, evaluated as weighted populations
   at the 2Q x-nodes (positive half first):
     + half:  X[k]   = w_k sum_{l<Q} G^+_l h_l(p_k),  G^+_l = int_0^inf g (p-u)^a h_l(p) dp
     - half:  X[Q+k] = w_k sum_{l<Q} G^-_l h_l(p_k),  G^-_l = int_{-inf}^0 g (p-u)^a h_l(-p) dp
   (eq:hh_F, eq:hh_gk, eq:hh_fk; orthonormal expansion truncated at l = Q-1). */
static void project_half(const orc_t *o, double u, double T, int a, double *X) {
  int Q = o->qh, W = Q + 2;
  qf E[ORC_MAXQ + 4], G[ORC_MAXQ + 4];
  for (int side = 0; side < 2; side++) {
    /* - half: substitute p -> -s: G^-_l(a; u) = (-1)^a G^+_l(a; -u) */
    qf us = side == 0 ? (qf)u : -(qf)u;
    trunc_moments(us, (qf)T, a, Q - 1, E);
    for (int l = 0; l < Q; l++) {
      qf acc = 0;
      for (int s = 0; s <= l; s++) acc += o->hq[l * W + s] * E[s];
      G[l] = (side == 1 && (a & 1)) ? -acc : acc;
    }
    for (int k = 0; k < Q; k++) {
      qf acc = 0;
      for (int l = 0; l < Q; l++) acc += G[l] * o->hpk[l * Q + k];
      X[side * Q + k] = (double)((qf)o->wx[k] * acc);
    }
  }
}

/* Full-range projection of g(p) (p-u)^b at Q Gauss-Hermite nodes, truncated
   at N = Q-1 (eq:H_gk):  Y[k] = w_k sum_{l<=N} He_l(p_k) G^{(b)}_l / l!,
   G^{(b)}_l = int g (p-u)^b He_l(p) dp.  For b = 0 this is the closed form
   eq:g_H; for b > 0 the integral is evaluated exactly by a 24-point
   Gauss-Hermite rule in the variable t = (p-u)/sqrt(T). */
static double gh24_t[24], gh24_w[24];
static int gh24_ready = 0;
static void project_full(const double *nodes, const double *w, int Q, double u, double T, int b, double *Y) {
  if (!gh24_ready) { orc_gh_rule(24, gh24_t, gh24_w); gh24_ready = 1; }
  int N = Q - 1;
  double G[64];
  for (int l = 0; l <= N; l++) {
    if (b == 0) {
      /* eq:g_H: G_l = sum_s l!/(2^s s! (l-2s)!) (T-1)^s u^(l-2s) */
      double acc = 0;
      for (int s = 0; 2 * s <= l; s++)
        acc += factorial(l) / (pow(2.0, s) * factorial(s) * factorial(l - 2 * s)) * pow(T - 1, s) * pow(u, l - 2 * s);
      G[l] = acc;
    } else {
      double acc = 0, sT = sqrt(T);
      for (int m = 0; m < 24; m++) {
        double t = gh24_t[m];
        acc += gh24_w[m] * pow(sT * t, b) * he_d(l, u + sT * t);
      }
      G[l] = acc;
    }
  }
  for (int k = 0; k < Q; k++) {
    double acc = 0;
    for (int l = 0; l <= N; l++) acc += he_d(l, nodes[k]) * G[l] / factorial(l);
    Y[k] = w[k] * acc;
  }
}

/* ------------------------------------------------------------------------ */
/* transport data (Sec. II.A)                                              */
/* ------------------------------------------------------------------------ */
double orc_chi(double eta) { return 0.5 * (2 - eta) / ((1 - eta) * (1 - eta) * (1 - eta)); } /* eq:chi */

/* dense Prandtl number, eq:prandtl, as a function of b rho chi */
double orc_pr_dense(double brc) {
  double num = 1 + 0.8 * brc + 4.0 / 25.0 * (1 + 12 / M_PI) * brc * brc;
  double den = 1 + 1.2 * brc + 9.0 / 25.0 * (1 + 32 / (9 * M_PI)) * brc * brc;
  return 2.0 / 3.0 * num / den;
}

/* relaxation time tau = mu / P_i (eq:tau) with mu from eq:viscosity and mu_0,
   expressed through Kn = 1/(sqrt2 pi sigma^2 n0 chi(n0) L) with n0 = L = 1:
   tau = (5 sqrt(2 pi)/16) Kn chi0 /(n sqrt T) [1/chi + (4/5) b rho + (4/25)(1+12/pi)(b rho)^2 chi],
   b rho = 4 eta.   kn <= 0 encodes Kn = infinity (then 1/tau = 0). */
double orc_inv_tau(double kn, double chi0, double n, double T, double eta) {
  if (kn <= 0) return 0.0;
  double chi = orc_chi(eta), br = 4 * eta;
  double bracket = 1 / chi + 0.8 * br + 4.0 / 25.0 * (1 + 12 / M_PI) * br * br * chi;
  double tau = 5 * sqrt(2 * M_PI) / 16 * kn * chi0 / (n * sqrt(T)) * bracket;
  return 1 / tau;
}

/* ------------------------------------------------------------------------ */
/* polynomials in the peculiar velocity xi = (xi_x, xi_y, xi_z), deg <= 3   */
/* ------------------------------------------------------------------------ */
typedef struct { double c[4][4][4]; } poly3;
static void p3_zero(poly3 *p) { memset(p, 0, sizeof(*p)); }
/* r += s * (x * y) with degrees kept <= 3 (aborts on overflow of degree) */
static int p3_mul_add(poly3 *r, const poly3 *x, const poly3 *y, double s) {
  for (int a1 = 0; a1 < 4; a1++) for (int b1 = 0; b1 < 4; b1++) for (int c1 = 0; c1 < 4; c1++) {
    double xv = x->c[a1][b1][c1]; if (xv == 0) continue;
    for (int a2 = 0; a2 < 4; a2++) for (int b2 = 0; b2 < 4; b2++) for (int c2 = 0; c2 < 4; c2++) {
      double yv = y->c[a2][b2][c2]; if (yv == 0) continue;
      if (a1 + a2 > 3 || b1 + b2 > 3 || c1 + c2 > 3) return -1;
      r->c[a1 + a2][b1 + b2][c1 + c2] += s * xv * yv;
    }
  }
  return 0;
}

/* Projected target n * Proj[ f^MB(u,T) * P(xi) ] at every lattice node of
   one cell.  The projection is taken per axis (x half-range, y and z full
   range) on the product of the three 1D Maxwellians, term by term in the
   monomials of P. */
static void project_poly(const orc_t *o, double n, double ux, double uy, double T, const poly3 *P, double *out) {
  int Q2 = 2 * o->qh, qy = o->qy, qz = o->qz;
  double X[4][2 * ORC_MAXQ], Y[4][16], Z[4][16];
  for (int a = 0; a < 4; a++) {
    int need = 0;
    for (int b = 0; b < 4; b++) for (int c = 0; c < 4; c++) if (P->c[a][b][c] != 0) need = 1;
    if (need) project_half(o, ux, T, a, X[a]);
  }
  for (int b = 0; b < 4; b++) project_full(o->py, o->wy, qy, uy, T, b, Y[b]);
  for (int c = 0; c < 4; c++) project_full(o->pz, o->wz, qz, 0.0, T, c, Z[c]);
  for (int kx = 0; kx < Q2; kx++)
    for (int ky = 0; ky < qy; ky++)
      for (int kz = 0; kz < qz; kz++) {
        double acc = 0;
        for (int a = 0; a < 4; a++) for (int b = 0; b < 4; b++) for (int c = 0; c < 4; c++) {
          double cf = P->c[a][b][c];
          if (cf != 0) acc += cf * X[a][kx] * Y[b][ky] * Z[c][kz];
        }
        out[(kx * qy + ky) * qz + kz] = n * acc;
      }
}

/* ------------------------------------------------------------------------ */
/* moments (eq:macro_LB), two-pass                                          */
/* ------------------------------------------------------------------------ */
typedef struct { double n, ux, uy, T, qx, qy, pxx, pxy, pyy, pzz; } moms;

static double node_px(const orc_t *o, int kap) { return o->px[kap / (o->qy * o->qz)]; }
static double node_py(const orc_t *o, int kap) { return o->py[(kap / o->qz) % o->qy]; }
static double node_pz(const orc_t *o, int kap) { return o->pz[kap % o->qz]; }

static moms cell_moments(const orc_t *o, const double *g, int i) {
  moms m; memset(&m, 0, sizeof(m));
  int nx = o->nx;
  double n = 0, jx = 0, jy = 0;
  for (int k = 0; k < o->K; k++) {
    double f = g[(size_t)k * nx + i];
    n += f; jx += node_px(o, k) * f; jy += node_py(o, k) * f;
  }
  m.n = n; m.ux = jx / n; m.uy = jy / n;
  double e = 0, qx = 0, qy = 0, pxx = 0, pxy = 0, pyy = 0, pzz = 0;
  for (int k = 0; k < o->K; k++) {
    double f = g[(size_t)k * nx + i];
    double cx = node_px(o, k) - m.ux, cy = node_py(o, k) - m.uy, cz = node_pz(o, k);
    double c2 = cx * cx + cy * cy + cz * cz;
    e += c2 * f;
    qx += 0.5 * cx * c2 * f; qy += 0.5 * cy * c2 * f;
    pxx += cx * cx * f; pxy += cx * cy * f; pyy += cy * cy * f; pzz += cz * cz * f;
  }
  m.T = e / (3 * n);
  m.qx = qx; m.qy = qy; m.pxx = pxx; m.pxy = pxy; m.pyy = pyy; m.pzz = pzz;
  return m;
}

/* ------------------------------------------------------------------------ */
/* finite differences (Sec. III.B.3)                                       */
/* ------------------------------------------------------------------------ */
/* weights of the first derivative at point `at` of a 7-point stencil on
   integer positions 0..6, from the Taylor (Vandermonde) conditions
   sum_j c_j (j-at)^m = delta_{m1}, m = 0..6, solved by Gaussian elimination. */
static void fd_weights7(int at, double *c) {
  double A[7][8];
  for (int m = 0; m < 7; m++) {
    for (int j = 0; j < 7; j++) A[m][j] = pow((double)(j - at), m);
    A[m][7] = (m == 1) ? 1.0 : 0.0;
  }
  for (int col = 0; col < 7; col++) {
    int piv = col;
    for (int r = col + 1; r < 7; r++) if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    for (int j = 0; j < 8; j++) { double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
    for (int r = 0; r < 7; r++) if (r != col) {
      double fct = A[r][col] / A[col][col];
      for (int j = 0; j < 8; j++) A[r][j] -= fct * A[col][j];
    }
  }
  for (int j = 0; j < 7; j++) c[j] = A[j][7] / A[j][j];
}

/* d/deta of a cell field q[0..nx-1] at cell i (unit spacing in index):
   interior: the paper's 6th-order central stencil; the three cells next to
   each wall: one-sided 7-point stencils inside the domain. */
static double ddeta(const double *q, int nx, int i) {
  if (i >= 3 && i <= nx - 4) {
    return -q[i - 3] / 60 + 3 * q[i - 2] / 20 - 3 * q[i - 1] / 4 + 3 * q[i + 1] / 4 - 3 * q[i + 2] / 20 + q[i + 3] / 60;
  }
  double c[7];
  if (i < 3) { fd_weights7(i, c); double s = 0; for (int j = 0; j < 7; j++) s += c[j] * q[j]; return s; }
  fd_weights7(i - (nx - 7), c);
  double s = 0; for (int j = 0; j < 7; j++) s += c[j] * q[nx - 7 + j]; return s;
}

/* ------------------------------------------------------------------------ */
/* WENO-5 face reconstruction (eq:weno5_flux_x .. eq:weno5_sigma)          */
/* ------------------------------------------------------------------------ */
enum { W_FULL = 0, W_DROP3 = 1, W_ONLY1 = 2 };

/* v[0..4] = f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2} in the upwind frame.
   mode W_DROP3: candidate 3 unavailable (its stencil leaves the domain), the
   ideal weights of candidates 1 and 2 are renormalised.  W_ONLY1: only the
   fully interior candidate 1.  Vanishing smoothness indicators are handled
   directly: the weights are distributed over the zero-indicator candidates in
   proportion to their ideal weights. */
double orc_weno(const double *v, int mode) {
  double F1 = v[0] / 3 - 7 * v[1] / 6 + 11 * v[2] / 6;
  double F2 = -v[1] / 6 + 5 * v[2] / 6 + v[3] / 3;
  double F3 = v[2] / 3 + 5 * v[3] / 6 - v[4] / 6;
  if (mode == W_ONLY1) return F1;
  double b1 = 13.0 / 12 * pow(v[0] - 2 * v[1] + v[2], 2) + 0.25 * pow(v[0] - 4 * v[1] + 3 * v[2], 2);
  double b2 = 13.0 / 12 * pow(v[1] - 2 * v[2] + v[3], 2) + 0.25 * pow(v[1] - v[3], 2);
  double b3 = 13.0 / 12 * pow(v[2] - 2 * v[3] + v[4], 2) + 0.25 * pow(3 * v[2] - 4 * v[3] + v[4], 2);
  double d[3] = {0.1, 0.6, 0.3}, b[3] = {b1, b2, b3}, F[3] = {F1, F2, F3};
  int nq = (mode == W_DROP3) ? 2 : 3;
  double dsum = 0; for (int q = 0; q < nq; q++) dsum += d[q];
  for (int q = 0; q < nq; q++) d[q] /= dsum;
  int nz = 0; double dz = 0;
  for (int q = 0; q < nq; q++) if (b[q] == 0) { nz++; dz += d[q]; }
  double w[3] = {0, 0, 0};
  if (nz > 0) {
    for (int q = 0; q < nq; q++) w[q] = (b[q] == 0) ? d[q] / dz : 0;
  } else {
    double s = 0;
    for (int q = 0; q < nq; q++) { w[q] = d[q] / (b[q] * b[q]); s += w[q]; }
    for (int q = 0; q < nq; q++) w[q] /= s;
  }
  double r = 0; for (int q = 0; q < nq; q++) r += w[q] * F[q];
  return r;
}

/* ------------------------------------------------------------------------ */
/* setup                                                                    */
/* ------------------------------------------------------------------------ */
static void fill_wall(orc_t *o, double T, double U, double *gw) {
  poly3 one; p3_zero(&one); one.c[0][0][0] = 1;
  project_poly(o, 1.0, 0.0, U, T, &one, gw);
}

void orc_destroy(orc_t *o) {
  if (!o) return;
  free(o->hq); free(o->hpk); free(o->px); free(o->wx); free(o->py); free(o->wy); free(o->pz); free(o->wz);
  free(o->kmat); free(o->xc); free(o->jac); free(o->f); free(o->f1); free(o->f2); free(o->Lg);
  free(o->gw_l); free(o->gw_r); free(o->prev_mom); free(o);
}

orc_t *orc_create(const orc_params *p) {
  if (p->nx < 7 || p->qx_half < 1 || p->qx_half > ORC_MAXQ || p->qy < 2 || p->qy > 16 || p->qz < 2 || p->qz > 16) return NULL;
  if (p->eta0 < 0 || p->eta0 >= 0.5) return NULL;
  orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
  o->p = *p;
  o->nx = p->nx; o->qh = p->qx_half; o->qy = p->qy; o->qz = p->qz;
  o->K = 2 * o->qh * o->qy * o->qz;
  int Q = o->qh, W = Q + 2;
  o->hq = (qf *)malloc(sizeof(qf) * W * W);
  o->px = (double *)malloc(sizeof(double) * 2 * Q); o->wx = (double *)malloc(sizeof(double) * 2 * Q);
  double *nd = (double *)malloc(sizeof(double) * Q), *wt = (double *)malloc(sizeof(double) * Q);
  if (orc_hr_rule(Q, nd, wt, o->hq) != 0) { free(nd); free(wt); orc_destroy(o); return NULL; }
  for (int k = 0; k < Q; k++) { o->px[k] = nd[k]; o->px[Q + k] = -nd[k]; o->wx[k] = wt[k]; o->wx[Q + k] = wt[k]; }
  free(nd); free(wt);
  o->hpk = (qf *)malloc(sizeof(qf) * Q * Q);
  for (int l = 0; l < Q; l++)
    for (int k = 0; k < Q; k++) o->hpk[l * Q + k] = poly_eval_q(&o->hq[l * W], l, (qf)o->px[k]);
  o->py = (double *)malloc(sizeof(double) * o->qy); o->wy = (double *)malloc(sizeof(double) * o->qy);
  o->pz = (double *)malloc(sizeof(double) * o->qz); o->wz = (double *)malloc(sizeof(double) * o->qz);
  if (orc_gh_rule(o->qy, o->py, o->wy) || orc_gh_rule(o->qz, o->pz, o->wz)) { orc_destroy(o); return NULL; }
  /* momentum-derivative kernel (eq:kernel_H), p0 = 1:
     K_{k,k'} = -w_k sum_{l=0}^{Q-2} He_{l+1}(p_k) He_l(p_k') / l! */
  o->kmat = (double *)calloc(o->qy * o->qy, sizeof(double));
  for (int k = 0; k < o->qy; k++)
    for (int k2 = 0; k2 < o->qy; k2++) {
      double s = 0;
      for (int l = 0; l <= o->qy - 2; l++) s += he_d(l + 1, o->py[k]) * he_d(l, o->py[k2]) / factorial(l);
      o->kmat[k * o->qy + k2] = -o->wy[k] * s;
    }
  /* geometry (Sec. IV): L = 1, sigma = 1/R, R = 1/(6 sqrt2 eta0 chi0 Kn), L_c = 1 - sigma */
  o->chi0 = orc_chi(p->eta0);
  if (p->eta0 > 0) {
    if (p->kn <= 0) { orc_destroy(o); return NULL; }
    double R = 1.0 / (6 * sqrt(2.0) * p->eta0 * o->chi0 * p->kn);
    if (R <= 1) { orc_destroy(o); return NULL; }
    o->sigma = 1.0 / R;
  } else o->sigma = 0;
  o->Lc = 1 - o->sigma;
  int nx = o->nx;
  o->deta = 2.0 / nx;
  o->xc = (double *)malloc(sizeof(double) * nx); o->jac = (double *)malloc(sizeof(double) * nx);
  for (int i = 0; i < nx; i++) {
    double eta = -1 + (i + 0.5) * o->deta;
    if (p->grid == 1 && p->stretch > 0) {
      double d = p->stretch, th = tanh(d);
      o->xc[i] = 0.5 * o->Lc * tanh(d * eta) / th;
      double ch = cosh(d * eta);
      o->jac[i] = 0.5 * o->Lc * d / (ch * ch * th);
    } else { o->xc[i] = 0.5 * o->Lc * eta; o->jac[i] = 0.5 * o->Lc; }
  }
  if (p->dt > 0) o->dt = p->dt;
  else {
    double hmin = 1e300, pmax = 0;
    for (int i = 0; i < nx; i++) if (o->jac[i] * o->deta < hmin) hmin = o->jac[i] * o->deta;
    for (int k = 0; k < 2 * Q; k++) if (fabs(o->px[k]) > pmax) pmax = fabs(o->px[k]);
    o->dt = p->cfl * hmin / pmax;
  }
  size_t N = (size_t)o->K * nx;
  o->f = (double *)calloc(N, sizeof(double)); o->f1 = (double *)calloc(N, sizeof(double));
  o->f2 = (double *)calloc(N, sizeof(double)); o->Lg = (double *)calloc(N, sizeof(double));
  o->gw_l = (double *)malloc(sizeof(double) * o->K); o->gw_r = (double *)malloc(sizeof(double) * o->K);
  fill_wall(o, p->t_left, p->uy_left, o->gw_l);
  fill_wall(o, p->t_right, p->uy_right, o->gw_r);
  o->prev_mom = (double *)calloc(4 * nx, sizeof(double));
  return o;
}

/* initial state: Grad-13-type distribution
   f = n Proj[ f^MB(u,T) (1 + Pxy xi_x xi_y /(n T^2) + qx xi_x (xi^2/T - 5)/(5 n T^2)) ] (1 + noise) */
void orc_set_state(orc_t *o, const double *fields, const double *noise) {
  int nx = o->nx;
  double *cellf = (double *)malloc(sizeof(double) * o->K);
  for (int i = 0; i < nx; i++) {
    double n = fields[i], ux = fields[nx + i], uy = fields[2 * nx + i], T = fields[3 * nx + i];
    double qx = fields[4 * nx + i], pxy = fields[5 * nx + i];
    poly3 P; p3_zero(&P);
    P.c[0][0][0] = 1;
    P.c[1][1][0] += pxy / (n * T * T);
    /* qx xi_x (xi_x^2 + xi_y^2 + xi_z^2)/(5 n T^3) - qx xi_x /(n T^2) */
    double c3 = qx / (5 * n * T * T * T);
    P.c[3][0][0] += c3; P.c[1][2][0] += c3; P.c[1][0][2] += c3;
    P.c[1][0][0] += -qx / (n * T * T);
    project_poly(o, n, ux, uy, T, &P, cellf);
    for (int k = 0; k < o->K; k++) {
      double v = cellf[k];
      if (noise) v *= 1 + noise[(size_t)k * nx + i];
      o->f[(size_t)k * nx + i] = v;
    }
  }
  free(cellf);
  o->steps = 0; o->prev_mom_valid = 0; o->resid = 0;
}

void orc_set_uniform(orc_t *o) {
  int nx = o->nx;
  double *fl = (double *)calloc(6 * nx, sizeof(double));
  for (int i = 0; i < nx; i++) { fl[i] = o->p.n_init; fl[2 * nx + i] = o->p.uy_init; fl[3 * nx + i] = o->p.t_init; }
  orc_set_state(o, fl, NULL);
  free(fl);
}

/* ------------------------------------------------------------------------ */
/* the right-hand side L[g] of eq:cast                                     */
/* ------------------------------------------------------------------------ */
/* Target polynomial P(xi) = 1 + S(xi) + tau J(xi): Shakhov factor (eq:j0 and
   the f^S definition) and J1 of eq:j1 divided by f^MB, with x-gradients only. */
static void target_poly(const orc_t *o, const moms *m, double dlnn, double dlnchi, double dlnT,
                        double dux, double duy, double *inv_tau_out, poly3 *P) {
  double n = m->n, T = m->T;
  double eta = o->p.eta0 * n;
  double chi = orc_chi(eta);
  double brho = 4 * eta;                    /* b rho = 4 eta */
  double inv_tau = orc_inv_tau(o->p.kn, o->chi0, n, T, eta);
  *inv_tau_out = inv_tau;
  double Pr = 1.0;
  if (o->p.collision == 1) Pr = o->p.pr_fixed;
  else if (o->p.collision == 2) Pr = orc_pr_dense(brho * chi);
  p3_zero(P);
  P->c[0][0][0] = 1;
  /* Shakhov: (1-Pr)/(P_i T) (xi^2/(5T) - 1) (xi . q), P_i = n T */
  if (Pr != 1.0) {
    poly3 A, B; p3_zero(&A); p3_zero(&B);
    A.c[2][0][0] = A.c[0][2][0] = A.c[0][0][2] = 1 / (5 * T); A.c[0][0][0] = -1;
    B.c[1][0][0] = m->qx; B.c[0][1][0] = m->qy;
    p3_mul_add(P, &A, &B, (1 - Pr) / (n * T * T));
  }
  /* J1 / f^MB = -b rho chi { xi.[grad ln(rho^2 chi T) + 3/5 (zeta^2 - 5/2) grad ln T]
                            + 2/5 [ 2 zeta zeta : grad u + (zeta^2 - 5/2) div u ] },
     zeta = xi / sqrt(2T); only x-derivatives are non-zero.  tau multiplies it
     so that -(f - f^S)/tau + J1 = (n Proj[f^MB P] - f)/tau. */
  if (inv_tau > 0 && brho > 0) {
    double tau = 1 / inv_tau;
    double pre = -brho * chi * tau;
    double grad_main = 2 * dlnn + dlnchi + dlnT;       /* d/dx ln(rho^2 chi T) */
    poly3 J; p3_zero(&J);
    poly3 z2; p3_zero(&z2);                             /* zeta^2 - 5/2 */
    z2.c[2][0][0] = z2.c[0][2][0] = z2.c[0][0][2] = 1 / (2 * T); z2.c[0][0][0] = -2.5;
    poly3 xix; p3_zero(&xix); xix.c[1][0][0] = 1;
    J.c[1][0][0] += grad_main;
    p3_mul_add(&J, &xix, &z2, 0.6 * dlnT);
    /* 2 zeta zeta : grad u = 2 (xi_x^2/(2T)) du_x/dx + 2 (xi_x xi_y/(2T)) du_y/dx */
    J.c[2][0][0] += 0.4 * (2 * dux / (2 * T));
    if (o->p.j1_shear) J.c[1][1][0] += 0.4 * (2 * duy / (2 * T));
    for (int a = 0; a < 4; a++) for (int b = 0; b < 4; b++) for (int c = 0; c < 4; c++)
      J.c[a][b][c] += 0.4 * dux * z2.c[a][b][c];
    for (int a = 0; a < 4; a++) for (int b = 0; b < 4; b++) for (int c = 0; c < 4; c++)
      P->c[a][b][c] += pre * J.c[a][b][c];
  }
}

/* L[g] into out; also returns the wall densities n_w used */
static void rhs(orc_t *o, const double *g, double *out, double *nw_l, double *nw_r) {
  int nx = o->nx, K = o->K, Q = o->qh, qyz = o->qy * o->qz;
  moms *M = (moms *)malloc(sizeof(moms) * nx);
  double *lnn = (double *)malloc(sizeof(double) * nx), *lnchi = (double *)malloc(sizeof(double) * nx),
         *lnT = (double *)malloc(sizeof(double) * nx), *ux = (double *)malloc(sizeof(double) * nx),
         *uy = (double *)malloc(sizeof(double) * nx);
  for (int i = 0; i < nx; i++) {
    M[i] = cell_moments(o, g, i);
    lnn[i] = log(M[i].n); lnchi[i] = log(orc_chi(o->p.eta0 * M[i].n)); lnT[i] = log(M[i].T);
    ux[i] = M[i].ux; uy[i] = M[i].uy;
  }
  /* wall densities from impenetrability: zero numerical mass flux through
     each wall face; incoming populations use the interior candidate 1 */
  double in_l = 0, out_l = 0, in_r = 0, out_r = 0;
  for (int k = 0; k < K; k++) {
    double p = node_px(o, k);
    const double *row = &g[(size_t)k * nx];
    if (p < 0) {
      double v[5] = {row[2], row[1], row[0], 0, 0};
      in_l += p * orc_weno(v, W_ONLY1);
      out_r += p * o->gw_r[k];
    } else {
      double v[5] = {row[nx - 3], row[nx - 2], row[nx - 1], 0, 0};
      in_r += p * orc_weno(v, W_ONLY1);
      out_l += p * o->gw_l[k];
    }
  }
  double nwl = -in_l / out_l, nwr = -in_r / out_r;
  if (nw_l) *nw_l = nwl;
  if (nw_r) *nw_r = nwr;
  double *tgt = (double *)malloc(sizeof(double) * K);
  double *face = (double *)malloc(sizeof(double) * (nx + 1));
  for (int i = 0; i < nx; i++) {
    double dlnn = ddeta(lnn, nx, i) / (o->deta * o->jac[i]);
    double dlnchi = ddeta(lnchi, nx, i) / (o->deta * o->jac[i]);
    double dlnT = ddeta(lnT, nx, i) / (o->deta * o->jac[i]);
    double dux = ddeta(ux, nx, i) / (o->deta * o->jac[i]);
    double duy = ddeta(uy, nx, i) / (o->deta * o->jac[i]);
    poly3 P; double inv_tau;
    target_poly(o, &M[i], dlnn, dlnchi, dlnT, dux, duy, &inv_tau, &P);
    project_poly(o, M[i].n, M[i].ux, M[i].uy, M[i].T, &P, tgt);
    for (int k = 0; k < K; k++) out[(size_t)k * nx + i] = (tgt[k] - g[(size_t)k * nx + i]) * inv_tau;
  }
  /* advection: face values f^_{j}, j = 0..nx (face j is the left face of cell j) */
  for (int k = 0; k < K; k++) {
    double p = node_px(o, k);
    const double *row = &g[(size_t)k * nx];
    double fwl = nwl * o->gw_l[k], fwr = nwr * o->gw_r[k];
    for (int j = 0; j <= nx; j++) {
      double v[5]; int mode = W_FULL;
      if (p > 0) {
        if (j == 0) { face[j] = fwl; continue; }
        /* upwind cell j-1; stencil j-3..j+1, ghosts left of the wall = f^w */
        for (int s = 0; s < 5; s++) {
          int c = j - 3 + s;
          v[s] = c < 0 ? fwl : (c >= nx ? 0.0 : row[c]);
        }
        if (j == nx) mode = W_ONLY1; else if (j == nx - 1) mode = W_DROP3;
      } else {
        if (j == nx) { face[j] = fwr; continue; }
        /* upwind cell j; mirrored stencil j+2, j+1, j, j-1, j-2 */
        for (int s = 0; s < 5; s++) {
          int c = j + 2 - s;
          v[s] = c >= nx ? fwr : (c < 0 ? 0.0 : row[c]);
        }
        if (j == 0) mode = W_ONLY1; else if (j == 1) mode = W_DROP3;
      }
      face[j] = orc_weno(v, mode);
    }
    for (int i = 0; i < nx; i++)
      out[(size_t)k * nx + i] -= p * (face[i + 1] - face[i]) / (o->jac[i] * o->deta);
  }
  /* body force: F . grad_p f moved to the right-hand side: -a_y (d f/d p_y) */
  if (o->p.ay != 0) {
    for (int i = 0; i < nx; i++)
      for (int kx = 0; kx < 2 * Q; kx++)
        for (int kz = 0; kz < o->qz; kz++)
          for (int ky = 0; ky < o->qy; ky++) {
            double s = 0;
            for (int k2 = 0; k2 < o->qy; k2++)
              s += o->kmat[ky * o->qy + k2] * g[(size_t)((kx * o->qy + k2) * o->qz + kz) * nx + i];
            out[(size_t)((kx * o->qy + ky) * o->qz + kz) * nx + i] -= o->p.ay * s;
          }
  }
  (void)qyz;
  free(M); free(lnn); free(lnchi); free(lnT); free(ux); free(uy); free(tgt); free(face);
}

/* one TVD-RK3 step (eq:rk3) */
static void rk3_step(orc_t *o) {
  size_t N = (size_t)o->K * o->nx;
  double dt = o->dt;
  rhs(o, o->f, o->Lg, NULL, NULL);
  for (size_t j = 0; j < N; j++) o->f1[j] = o->f[j] + dt * o->Lg[j];
  rhs(o, o->f1, o->Lg, NULL, NULL);
  for (size_t j = 0; j < N; j++) o->f2[j] = 0.75 * o->f[j] + 0.25 * o->f1[j] + 0.25 * dt * o->Lg[j];
  rhs(o, o->f2, o->Lg, NULL, NULL);
  for (size_t j = 0; j < N; j++) o->f[j] = o->f[j] / 3 + 2.0 / 3.0 * o->f2[j] + 2.0 / 3.0 * dt * o->Lg[j];
  o->steps++;
}

/* residual: max over n, u_x, u_y, T and cells of |M^{s} - M^{s-1}| / dt */
static double step_with_resid(orc_t *o) {
  int nx = o->nx;
  double *a = (double *)malloc(sizeof(double) * 4 * nx);
  for (int i = 0; i < nx; i++) {
    moms m = cell_moments(o, o->f, i);
    a[i] = m.n; a[nx + i] = m.ux; a[2 * nx + i] = m.uy; a[3 * nx + i] = m.T;
  }
  rk3_step(o);
  double r = 0;
  for (int i = 0; i < nx; i++) {
    moms m = cell_moments(o, o->f, i);
    double d[4] = {m.n - a[i], m.ux - a[nx + i], m.uy - a[2 * nx + i], m.T - a[3 * nx + i]};
    for (int q = 0; q < 4; q++) if (fabs(d[q]) / o->dt > r) r = fabs(d[q]) / o->dt;
  }
  free(a);
  o->resid = r;
  return r;
}

/* ------------------------------------------------------------------------ */
/* exported API                                                             */
/* ------------------------------------------------------------------------ */
int orc_K(const orc_t *o) { return o->K; }
double orc_dt(const orc_t *o) { return o->dt; }
double orc_sigma(const orc_t *o) { return o->sigma; }
double orc_Lc(const orc_t *o) { return o->Lc; }
long orc_steps(const orc_t *o) { return o->steps; }

void orc_step(orc_t *o, long nsteps) { for (long s = 0; s < nsteps; s++) rk3_step(o); }

double orc_step_resid(orc_t *o) { return step_with_resid(o); }

/* run until the residual drops below tol (checked every step) or max_steps */
long orc_run_to_steady(orc_t *o, double tol, long max_steps, double *resid_out) {
  long s = 0; double r = 1e300;
  while (s < max_steps) { r = step_with_resid(o); s++; if (r < tol) break; }
  if (resid_out) *resid_out = r;
  return s;
}

/* moments [10][nx]: n, ux, uy, T, qx, qy, Pxx, Pxy, Pyy, Pzz */
void orc_moments(const orc_t *o, double *out) {
  int nx = o->nx;
  for (int i = 0; i < nx; i++) {
    moms m = cell_moments(o, o->f, i);
    double v[10] = {m.n, m.ux, m.uy, m.T, m.qx, m.qy, m.pxx, m.pxy, m.pyy, m.pzz};
    for (int q = 0; q < 10; q++) out[q * nx + i] = v[q];
  }
}

void orc_get_f(const orc_t *o, double *out) { memcpy(out, o->f, sizeof(double) * o->K * o->nx); }
void orc_set_f(orc_t *o, const double *in) { memcpy(o->f, in, sizeof(double) * o->K * o->nx); }

void orc_lattice(const orc_t *o, double *px, double *py, double *pz, double *w) {
  for (int k = 0; k < o->K; k++) {
    int kx = k / (o->qy * o->qz), ky = (k / o->qz) % o->qy, kz = k % o->qz;
    px[k] = o->px[kx]; py[k] = o->py[ky]; pz[k] = o->pz[kz];
    w[k] = o->wx[kx] * o->wy[ky] * o->wz[kz];
  }
}

void orc_grid(const orc_t *o, double *x, double *jac) {
  memcpy(x, o->xc, sizeof(double) * o->nx); memcpy(jac, o->jac, sizeof(double) * o->nx);
}

/* L[f] of the current state plus the wall densities (for unit checks) */
void orc_rhs(orc_t *o, double *out, double *nw) { rhs(o, o->f, out, &nw[0], &nw[1]); }

/* half-range projection table of g (p-u)^a for a standalone lattice order */
int orc_project_half_table(int Q, double u, double T, int a, double *out) {
  orc_params p; memset(&p, 0, sizeof(p));
  p.nx = 7; p.qx_half = Q; p.qy = 2; p.qz = 2; p.kn = 1; p.cfl = 0.5;
  orc_t *o = orc_create(&p);
  if (!o) return -1;
  project_half(o, u, T, a, out);
  orc_destroy(o);
  return 0;
}

int orc_project_full_table(int Q, double u, double T, int b, double *out) {
  double *nd = (double *)malloc(sizeof(double) * Q), *w = (double *)malloc(sizeof(double) * Q);
  if (orc_gh_rule(Q, nd, w)) { free(nd); free(w); return -1; }
  project_full(nd, w, Q, u, T, b, out);
  free(nd); free(w);
  return 0;
}

int orc_kmat_table(const orc_t *o, double *out) { memcpy(out, o->kmat, sizeof(double) * o->qy * o->qy); return 0; }

void orc_fd_weights7(int at, double *c) { fd_weights7(at, c); }
double orc_ddeta(const double *q, int nx, int i) { return ddeta(q, nx, i); }

/* target F at every node of one cell from given moments and gradients */
void orc_target(const orc_t *o, const double *mom10, const double *grad5, double *out, double *inv_tau) {
  moms m; m.n = mom10[0]; m.ux = mom10[1]; m.uy = mom10[2]; m.T = mom10[3]; m.qx = mom10[4]; m.qy = mom10[5];
  poly3 P;
  target_poly(o, &m, grad5[0], grad5[1], grad5[2], grad5[3], grad5[4], inv_tau, &P);
  project_poly(o, m.n, m.ux, m.uy, m.T, &P, out);
}
