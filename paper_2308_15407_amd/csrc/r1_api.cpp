// r1_api.cpp -- host side of the reduced models (Sec. II.B): phi and theta on
// the 2 qx_half x-nodes (1D flows: the Fourier flow) or on the 2 qx_half x qy
// (x, y) nodes (2D flows: Couette and Poiseuille), advanced by one fused
// kernel per TVD-RK3 stage (k_r1_stage).  The lattice, the grid and the
// finite-difference weights come from the same case construction as the 3D
// path; the z velocity set (and the y set in 1D) is not used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fdlb_common.h"
#include "fdlb_host.h"

using namespace fdlb;

#define R1CHK(expr)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return api_fail(FDLB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct fdlb_r1_ctx {
  std::vector<CaseHost> cases;
  std::vector<R1Dev> hdev;
  hipStream_t stream = nullptr;
  R1Dev *d_cases = nullptr;
  int *d_map = nullptr;
  R1Group grp[2] = {};   // cases of at most R1_RMAX rows, then the larger ones
  int rmax = 0;    // the largest row count of the cases
  int *d_mapN = nullptr;   // averaged-density blocks of the chi_mode 1 cases
  int nN = 0;
  size_t ldsN = 0;
  int dim = 0;     // 1 or 2, the same for every case
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// dimension of the reduced model of a case: the Fourier flow is 1D, the
// Couette and Poiseuille flows 2D
static int r1_dim(const fdlb_params &p) { return p.flow == 0 ? 1 : 2; }
static int r1_rows(const CaseHost &c, int dim) { return 4 * c.qh * (dim == 2 ? c.qy : 1); }

// the parameters the reduced model accepts, and the case built from them
static int r1_case(const fdlb_params &p, CaseHost &c, std::string &why) {
  const int dim = r1_dim(p);
  if (p.qx_half > MAXQH) { why = "reduced model: qx_half must be in [1, 32]"; return -1; }
  if (dim == 1 && (p.uy_left != 0 || p.uy_right != 0 || p.uy_init != 0 || p.ay != 0)) {
    why = "reduced 1D model (Fourier flow): no y-motion (walls, initial state) and no body force";
    return -1;
  }
  if (dim == 2 && 4 * p.qx_half * p.qy > R1_RMAX_BIG) {
    why = "reduced 2D model: 4 qx_half qy must be <= 640";
    return -1;
  }
  if (p.precision != FDLB_F64) { why = "reduced model: FP64 storage only"; return -1; }
  if (p.x_rule != 0) { why = "reduced model: half-range x rule only"; return -1; }
  fdlb_params q = p;
  if (dim == 1) q.qy = 2;
  q.qz = 2;   // transverse sets of the shared construction that are not used here
  return build_case(q, c, why);
}

// bytes of one case's arrays: lattice, 1/dx, wall rows, f / g1 / g2, moments
static size_t r1_case_bytes(const CaseHost &c) {
  const size_t R = r1_rows(c, r1_dim(c.p));
  return al256(sizeof(double) * c.lat.size()) + al256(sizeof(double) * c.nx) + al256(sizeof(double) * 2 * R) +
         3 * al256(sizeof(double) * R * c.nx) + al256(sizeof(double) * FDLB_NMOM * c.nx) +
         (c.p.chi_mode == 1 ? al256(sizeof(double) * c.nx) : 0);
}

static size_t r1_tiles(const CaseHost &c, int tile) { return (c.nx + tile - 1) / tile; }

// phi and theta of the state with fields (n, u_x, u_y, T, q_x, P_xy) per
// cell: the Grad-13-type distribution integrated over the dropped axes, with
// s = q_x / (5 n T^2):
//   1D: phi = n Proj[g (1 + s xi (xi^2/T - 3))], theta = 2T n Proj[g (1 + s xi (xi^2/T - 1))]
//   2D: phi = n Proj[g (1 + P_xy xi_x xi_y/(n T^2) + s xi_x ((xi_x^2 + xi_y^2)/T - 4))],
//       theta = T n Proj[g (1 + P_xy xi_x xi_y/(n T^2) + s xi_x ((xi_x^2 + xi_y^2)/T - 2))]
// optionally times (1 + noise) node by node
static void r1_fill(const CaseHost &c, const double *fields, const double *noise, std::vector<double> &f) {
  const int dim = r1_dim(c.p), nx = c.nx, Q = c.qh, Q2 = 2 * Q, qy = dim == 2 ? c.qy : 1, Kh = Q2 * qy;
  f.assign((size_t)2 * Kh * nx, 0.0);
  std::vector<double> X[4], Y[4];
  for (int a = 0; a < 4; a++) { X[a].assign(Q2, 0.0); Y[a].assign(qy, 0.0); }
  for (int i = 0; i < nx; i++) {
    const double n = fields[i], ux = fields[nx + i], uy = fields[2 * nx + i], T = fields[3 * nx + i];
    const double qx = fields[4 * nx + i], pxy = fields[5 * nx + i];
    for (int a = 0; a < 4; a++) host_half_table(c.lat.data(), c.lo, Q, ux, T, a, X[a].data());
    const double s = qx / (5.0 * n * T * T);
    if (dim == 1) {
      for (int k = 0; k < Q2; k++) {
        f[(size_t)k * nx + i] = n * (X[0][k] - 3.0 * s * X[1][k] + s / T * X[3][k]);
        f[(size_t)(Q2 + k) * nx + i] = 2.0 * T * n * (X[0][k] - s * X[1][k] + s / T * X[3][k]);
      }
      continue;
    }
    for (int b = 0; b < 4; b++) host_full_table(&c.lat[c.lo.Hy], qy, uy, T, b, Y[b].data());
    const double sxy = pxy / (n * T * T);
    for (int kx = 0; kx < Q2; kx++)
      for (int ky = 0; ky < qy; ky++) {
        const double base = X[0][kx] * Y[0][ky] + sxy * X[1][kx] * Y[1][ky] + s / T * X[3][kx] * Y[0][ky] +
                            s / T * X[1][kx] * Y[2][ky];
        f[(size_t)(kx * qy + ky) * nx + i] = n * (base - 4.0 * s * X[1][kx] * Y[0][ky]);
        f[(size_t)(Kh + kx * qy + ky) * nx + i] = T * n * (base - 2.0 * s * X[1][kx] * Y[0][ky]);
      }
  }
  if (noise)
    for (size_t j = 0; j < f.size(); j++) f[j] *= 1.0 + noise[j];
}

extern "C" size_t fdlb_r1_workspace_bytes(const fdlb_params *cases, int ncases) {
  if (!cases || ncases <= 0) { api_fail(FDLB_EINVAL, "no cases"); return 0; }
  size_t total = al256(sizeof(R1Dev) * ncases), tiles = 0;
  for (int i = 0; i < ncases; i++) {
    CaseHost c;
    std::string why;
    if (r1_case(cases[i], c, why)) { api_fail(FDLB_EINVAL, "case " + std::to_string(i) + ": " + why); return 0; }
    if (r1_dim(cases[i]) != r1_dim(cases[0])) {
      api_fail(FDLB_EINVAL, "reduced model: a batch holds cases of one dimension (Fourier, or Couette/Poiseuille)");
      return 0;
    }
    total += r1_case_bytes(c);
    tiles += r1_tiles(c, R1_TILE_BIG);   // the smallest tile bounds the map
    if (c.p.chi_mode == 1) tiles += r1_tiles(c, NBAR_TILE);
  }
  return total + al256(sizeof(int) * 2 * tiles) + 256;   // two map regions, each 256-byte aligned
}

extern "C" int fdlb_r1_init(const fdlb_params *cases, int ncases, void *dev_workspace, size_t bytes,
                            void *hip_stream, fdlb_r1_handle *out) {
  if (!out) return api_fail(FDLB_EINVAL, "null output handle");
  *out = nullptr;
  const size_t need = fdlb_r1_workspace_bytes(cases, ncases);
  if (need == 0) return FDLB_EINVAL;
  if (!dev_workspace || bytes < need)
    return api_fail(FDLB_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes, need " + std::to_string(need));
  fdlb_r1_ctx *h = new fdlb_r1_ctx();
  h->stream = (hipStream_t)hip_stream;
  h->cases.resize(ncases);
  h->hdev.resize(ncases);
  char *ws = (char *)dev_workspace;
  size_t off = 0;
  auto take = [&](size_t nbytes) { char *p = ws + off; off += al256(nbytes); return p; };
  h->d_cases = (R1Dev *)take(sizeof(R1Dev) * ncases);
  std::vector<int> map, mapN;
  auto bail = [&](int code) { delete h; return code; };
  h->dim = r1_dim(cases[0]);
  int cells[2] = {0, 0};
  for (int i = 0; i < ncases; i++) {
    CaseHost &c = h->cases[i];
    std::string why;
    if (r1_case(cases[i], c, why)) return bail(api_fail(FDLB_EINVAL, why));
    const int rows = r1_rows(c, h->dim), g = rows > R1_RMAX;
    h->rmax = std::max(h->rmax, rows);
    h->grp[g].rmax = std::max(h->grp[g].rmax, rows);
    cells[g] += c.nx;
  }
  for (int g = 0; g < 2; g++)
    if (cells[g] > 0) h->grp[g].tile = r1_tile(h->grp[g].rmax, cells[g]);
  std::vector<int> mapg[2];
  for (int i = 0; i < ncases; i++) {
    CaseHost &c = h->cases[i];
    const int nx = c.nx, Q = c.qh, Q2 = 2 * Q, qy = h->dim == 2 ? c.qy : 1, Kh = Q2 * qy, R = 2 * Kh;
    R1Dev &d = h->hdev[i];
    memset(&d, 0, sizeof(d));
    d.nx = nx; d.qh = Q; d.qy = qy; d.R = R; d.dim = h->dim;
    d.collision = c.p.collision; d.j1_shear = c.p.j1_shear; d.pr_fixed = c.p.pr_fixed; d.eta0 = c.p.eta0;
    d.dt = c.dt; d.ay = c.p.ay;
    d.tau_pre = c.p.kn > 0 ? 5.0 * sqrt(2.0 * M_PI) / 16.0 * c.p.kn * c.chi0 : 0.0;
    d.lo = c.lo;
    double *lat = (double *)take(sizeof(double) * c.lat.size());
    double *invdx = (double *)take(sizeof(double) * nx);
    double *gw = (double *)take(sizeof(double) * 2 * R);
    d.f = (double *)take(sizeof(double) * R * nx);
    d.g1 = (double *)take(sizeof(double) * R * nx);
    d.g2 = (double *)take(sizeof(double) * R * nx);
    d.mom = (double *)take(sizeof(double) * FDLB_NMOM * nx);
    d.chi_mode = c.p.chi_mode;
    d.sigma = c.sigma;
    if (c.p.chi_mode == 1) d.nbar = (double *)take(sizeof(double) * nx);
    d.lat = lat; d.invdx = invdx; d.gw = gw;
    // wall rows at n = 1: phi_w = Proj[g(0, T_w)] (times Proj[g(U_w, T_w)] on
    // the y-nodes in 2D), theta_w = 2 T_w phi_w (1D) or T_w phi_w (2D);
    // wallD = the emitted mass flux per unit n_w
    std::vector<double> hgw(2 * R), X(Q2), Y(qy, 1.0);
    for (int w = 0; w < 2; w++) {
      const double Tw = w == 0 ? c.p.t_left : c.p.t_right, Uw = w == 0 ? c.p.uy_left : c.p.uy_right;
      host_half_table(c.lat.data(), c.lo, Q, 0.0, Tw, 0, X.data());
      if (h->dim == 2) host_full_table(&c.lat[c.lo.Hy], qy, Uw, Tw, 0, Y.data());
      const double tf = h->dim == 2 ? Tw : 2.0 * Tw;
      double D = 0.0;
      for (int kx = 0; kx < Q2; kx++)
        for (int ky = 0; ky < qy; ky++) {
          const double v = X[kx] * Y[ky];
          hgw[w * R + kx * qy + ky] = v;
          hgw[w * R + Kh + kx * qy + ky] = tf * v;
          const double p = c.lat[c.lo.px + kx];
          if ((w == 0) == (p > 0.0)) D += p * v;
        }
      d.wallD[w] = D;
    }
    R1CHK(hipMemcpyAsync(lat, c.lat.data(), sizeof(double) * c.lat.size(), hipMemcpyHostToDevice, h->stream));
    R1CHK(hipMemcpyAsync(invdx, c.invdx.data(), sizeof(double) * nx, hipMemcpyHostToDevice, h->stream));
    R1CHK(hipMemcpyAsync(gw, hgw.data(), sizeof(double) * 2 * R, hipMemcpyHostToDevice, h->stream));
    std::vector<double> fields((size_t)6 * nx, 0.0), f;
    for (int k = 0; k < nx; k++) {
      fields[k] = c.p.n_init; fields[2 * nx + k] = h->dim == 2 ? c.p.uy_init : 0.0; fields[3 * nx + k] = c.p.t_init;
    }
    r1_fill(c, fields.data(), nullptr, f);
    R1CHK(hipMemcpyAsync(d.f, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, h->stream));
    R1CHK(hipStreamSynchronize(h->stream));
    R1Group &grp = h->grp[r1_rows(c, h->dim) > R1_RMAX];
    std::vector<int> &mg = mapg[&grp - h->grp];
    for (size_t t = 0; t < r1_tiles(c, grp.tile); t++) { mg.push_back(i); mg.push_back((int)t); }
    if (c.p.chi_mode == 1) {
      // averaged-density blocks: the LDS holds the densities and faces of a tile's window
      for (int t = 0; t * NBAR_TILE < nx; t++) {
        const int i0 = t * NBAR_TILE, i1 = std::min(i0 + NBAR_TILE, nx) - 1;
        const size_t wlen = (size_t)(c.lat[c.lo.whi + i1] - c.lat[c.lo.wlo + i0]) + 1;
        h->ldsN = std::max(h->ldsN, sizeof(double) * (2 * wlen + 1));
        mapN.push_back(i); mapN.push_back(t);
      }
    }
  }
  map = mapg[0];
  map.insert(map.end(), mapg[1].begin(), mapg[1].end());
  h->d_map = (int *)take(sizeof(int) * map.size());
  h->grp[0].map = h->d_map;
  h->grp[0].nblocks = (int)(mapg[0].size() / 2);
  h->grp[1].map = h->d_map + mapg[0].size();
  h->grp[1].nblocks = (int)(mapg[1].size() / 2);
  h->nN = (int)(mapN.size() / 2);
  if (h->nN > 0) h->d_mapN = (int *)take(sizeof(int) * mapN.size());
  if (off > bytes) return bail(api_fail(FDLB_ENOMEM, "workspace layout exceeds the buffer"));
  if (h->ldsN > NBAR_LDS_MAX) return bail(api_fail(FDLB_EINVAL, "revised Enskog window too wide for the LDS"));
  R1CHK(hipMemcpyAsync(h->d_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice, h->stream));
  if (h->nN > 0)
    R1CHK(hipMemcpyAsync(h->d_mapN, mapN.data(), sizeof(int) * mapN.size(), hipMemcpyHostToDevice, h->stream));
  R1CHK(hipMemcpyAsync(h->d_cases, h->hdev.data(), sizeof(R1Dev) * ncases, hipMemcpyHostToDevice, h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  *out = h;
  return FDLB_OK;
}

extern "C" int fdlb_r1_step(fdlb_r1_handle h, long nsteps) {
  if (!h || nsteps < 0) return api_fail(FDLB_EINVAL, "null handle or negative step count");
  R1CHK(launch_r1_step(h->d_cases, h->grp, 2, h->dim, h->d_mapN, h->nN, h->ldsN, nsteps, h->stream));
  return FDLB_OK;
}

extern "C" int fdlb_r1_moments(fdlb_r1_handle h, int c, double *host_out) {
  if (!h || c < 0 || c >= (int)h->cases.size() || !host_out) return api_fail(FDLB_EINVAL, "bad handle, case or output");
  const int nx = h->cases[c].nx;
  R1CHK(launch_r1_moments(h->d_cases, c, nx, h->stream));
  R1CHK(hipMemcpyAsync(host_out, h->hdev[c].mom, sizeof(double) * FDLB_NMOM * nx, hipMemcpyDeviceToHost, h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  return FDLB_OK;
}

extern "C" int fdlb_r1_set_state(fdlb_r1_handle h, int c, const double *fields, const double *noise) {
  if (!h || c < 0 || c >= (int)h->cases.size() || !fields) return api_fail(FDLB_EINVAL, "bad handle, case or fields");
  const CaseHost &ch = h->cases[c];
  for (int i = 0; i < ch.nx; i++)
    if (!(fields[i] > 0) || !(fields[3 * ch.nx + i] > 0)) return api_fail(FDLB_EINVAL, "fields need n > 0 and T > 0");
  std::vector<double> f;
  r1_fill(ch, fields, noise, f);
  R1CHK(hipMemcpyAsync(h->hdev[c].f, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  return FDLB_OK;
}

extern "C" int fdlb_r1_get_f(fdlb_r1_handle h, int c, double *host_f) {
  if (!h || c < 0 || c >= (int)h->cases.size() || !host_f) return api_fail(FDLB_EINVAL, "bad handle, case or output");
  const CaseHost &ch = h->cases[c];
  R1CHK(hipMemcpyAsync(host_f, h->hdev[c].f, sizeof(double) * h->hdev[c].R * ch.nx, hipMemcpyDeviceToHost,
                       h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  return FDLB_OK;
}

extern "C" int fdlb_r1_dt(fdlb_r1_handle h, int c, double *dt) {
  if (!h || c < 0 || c >= (int)h->cases.size() || !dt) return api_fail(FDLB_EINVAL, "bad handle, case or output");
  *dt = h->cases[c].dt;
  return FDLB_OK;
}

extern "C" void fdlb_r1_destroy(fdlb_r1_handle h) { delete h; }
