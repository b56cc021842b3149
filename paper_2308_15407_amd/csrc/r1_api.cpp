// r1_api.cpp -- host side of the reduced 1D model of the Fourier flow
// (Sec. II.B, 1D flows): phi and theta on the 2 qx_half x-nodes, advanced by
// one fused kernel per TVD-RK3 stage (k_r1_stage).  The lattice, the grid and
// the finite-difference weights come from the same case construction as the
// 3D path; the y and z velocity sets are not used.
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
  int nmap = 0;
  int rmax = 0;    // the largest row count (4 qx_half) of the cases
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// the parameters the reduced model accepts, and the case built from them
static int r1_case(const fdlb_params &p, CaseHost &c, std::string &why) {
  if (p.qx_half > MAXQH) { why = "reduced 1D model: qx_half must be in [1, 32]"; return -1; }
  if (p.uy_left != 0 || p.uy_right != 0 || p.uy_init != 0 || p.ay != 0) {
    why = "reduced 1D model: no y-motion (walls, initial state) and no body force";
    return -1;
  }
  if (p.chi_mode != 0) { why = "reduced 1D model: local contact value only (chi_mode 0)"; return -1; }
  if (p.precision != FDLB_F64) { why = "reduced 1D model: FP64 storage only"; return -1; }
  fdlb_params q = p;
  q.qy = 2; q.qz = 2;   // the transverse sets of the shared construction (unused here)
  return build_case(q, c, why);
}

// bytes of one case's arrays: lattice, 1/dx, wall rows, f / g1 / g2, moments
static size_t r1_case_bytes(const CaseHost &c) {
  const size_t R = 4 * c.qh;
  return al256(sizeof(double) * c.lat.size()) + al256(sizeof(double) * c.nx) + al256(sizeof(double) * 2 * R) +
         3 * al256(sizeof(double) * R * c.nx) + al256(sizeof(double) * FDLB_NMOM * c.nx);
}

static size_t r1_tiles(const CaseHost &c) { return (c.nx + R1_TILE - 1) / R1_TILE; }

// phi and theta of the state with fields (n, u_x, T, q_x) per cell: the
// Grad-13-type distribution integrated over p_y and p_z,
//   phi = n Proj[g (1 + s xi (xi^2/T - 3))], theta = 2T n Proj[g (1 + s xi (xi^2/T - 1))],
// s = q_x / (5 n T^2), optionally times (1 + noise) node by node
static void r1_fill(const CaseHost &c, const double *fields, const double *noise, std::vector<double> &f) {
  const int nx = c.nx, Q = c.qh, Q2 = 2 * Q, R = 4 * Q;
  f.assign((size_t)R * nx, 0.0);
  std::vector<double> X[4];
  for (int a = 0; a < 4; a++) X[a].assign(Q2, 0.0);
  for (int i = 0; i < nx; i++) {
    const double n = fields[i], ux = fields[nx + i], T = fields[3 * nx + i], qx = fields[4 * nx + i];
    for (int a = 0; a < 4; a++) host_half_table(c.lat.data(), c.lo, Q, ux, T, a, X[a].data());
    const double s = qx / (5.0 * n * T * T);
    for (int k = 0; k < Q2; k++) {
      f[(size_t)k * nx + i] = n * (X[0][k] - 3.0 * s * X[1][k] + s / T * X[3][k]);
      f[(size_t)(Q2 + k) * nx + i] = 2.0 * T * n * (X[0][k] - s * X[1][k] + s / T * X[3][k]);
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
    total += r1_case_bytes(c);
    tiles += r1_tiles(c);
  }
  return total + al256(sizeof(int) * 2 * tiles);
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
  std::vector<int> map;
  auto bail = [&](int code) { delete h; return code; };
  for (int i = 0; i < ncases; i++) {
    CaseHost &c = h->cases[i];
    std::string why;
    if (r1_case(cases[i], c, why)) return bail(api_fail(FDLB_EINVAL, why));
    const int nx = c.nx, Q = c.qh, Q2 = 2 * Q, R = 4 * Q;
    h->rmax = std::max(h->rmax, R);
    R1Dev &d = h->hdev[i];
    memset(&d, 0, sizeof(d));
    d.nx = nx; d.qh = Q; d.R = R;
    d.collision = c.p.collision; d.pr_fixed = c.p.pr_fixed; d.eta0 = c.p.eta0; d.dt = c.dt;
    d.tau_pre = c.p.kn > 0 ? 5.0 * sqrt(2.0 * M_PI) / 16.0 * c.p.kn * c.chi0 : 0.0;
    d.lo = c.lo;
    double *lat = (double *)take(sizeof(double) * c.lat.size());
    double *invdx = (double *)take(sizeof(double) * nx);
    double *gw = (double *)take(sizeof(double) * 2 * R);
    d.f = (double *)take(sizeof(double) * R * nx);
    d.g1 = (double *)take(sizeof(double) * R * nx);
    d.g2 = (double *)take(sizeof(double) * R * nx);
    d.mom = (double *)take(sizeof(double) * FDLB_NMOM * nx);
    d.lat = lat; d.invdx = invdx; d.gw = gw;
    // wall rows at n = 1: phi_w = Proj[g(0, T_w)], theta_w = 2 T_w phi_w;
    // wallD = the emitted mass flux per unit n_w
    std::vector<double> hgw(2 * R), X(Q2);
    for (int w = 0; w < 2; w++) {
      const double Tw = w == 0 ? c.p.t_left : c.p.t_right;
      host_half_table(c.lat.data(), c.lo, Q, 0.0, Tw, 0, X.data());
      double D = 0.0;
      for (int k = 0; k < Q2; k++) {
        hgw[w * R + k] = X[k];
        hgw[w * R + Q2 + k] = 2.0 * Tw * X[k];
        const double p = c.lat[c.lo.px + k];
        if ((w == 0) == (p > 0.0)) D += p * X[k];
      }
      d.wallD[w] = D;
    }
    R1CHK(hipMemcpyAsync(lat, c.lat.data(), sizeof(double) * c.lat.size(), hipMemcpyHostToDevice, h->stream));
    R1CHK(hipMemcpyAsync(invdx, c.invdx.data(), sizeof(double) * nx, hipMemcpyHostToDevice, h->stream));
    R1CHK(hipMemcpyAsync(gw, hgw.data(), sizeof(double) * 2 * R, hipMemcpyHostToDevice, h->stream));
    std::vector<double> fields((size_t)6 * nx, 0.0), f;
    for (int k = 0; k < nx; k++) { fields[k] = c.p.n_init; fields[3 * nx + k] = c.p.t_init; }
    r1_fill(c, fields.data(), nullptr, f);
    R1CHK(hipMemcpyAsync(d.f, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, h->stream));
    R1CHK(hipStreamSynchronize(h->stream));
    for (size_t t = 0; t < r1_tiles(c); t++) { map.push_back(i); map.push_back((int)t); }
  }
  h->d_map = (int *)take(sizeof(int) * map.size());
  h->nmap = (int)(map.size() / 2);
  if (off > bytes) return bail(api_fail(FDLB_ENOMEM, "workspace layout exceeds the buffer"));
  R1CHK(hipMemcpyAsync(h->d_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice, h->stream));
  R1CHK(hipMemcpyAsync(h->d_cases, h->hdev.data(), sizeof(R1Dev) * ncases, hipMemcpyHostToDevice, h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  *out = h;
  return FDLB_OK;
}

extern "C" int fdlb_r1_step(fdlb_r1_handle h, long nsteps) {
  if (!h || nsteps < 0) return api_fail(FDLB_EINVAL, "null handle or negative step count");
  R1CHK(launch_r1_step(h->d_cases, h->d_map, h->nmap, h->rmax, nsteps, h->stream));
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
  R1CHK(hipMemcpyAsync(host_f, h->hdev[c].f, sizeof(double) * 4 * ch.qh * ch.nx, hipMemcpyDeviceToHost, h->stream));
  R1CHK(hipStreamSynchronize(h->stream));
  return FDLB_OK;
}

extern "C" int fdlb_r1_dt(fdlb_r1_handle h, int c, double *dt) {
  if (!h || c < 0 || c >= (int)h->cases.size() || !dt) return api_fail(FDLB_EINVAL, "bad handle, case or output");
  *dt = h->cases[c].dt;
  return FDLB_OK;
}

extern "C" void fdlb_r1_destroy(fdlb_r1_handle h) { delete h; }
