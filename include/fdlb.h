/*
 * fdlb.h -- C ABI of the MI355X (gfx950) finite-difference lattice Boltzmann
 * (FDLB) solver for the simplified Enskog equation on a 1D wall-bounded
 * channel (Busuioc & Sofonea, "Bounded flows of dense gases", arXiv 2308.15407).
 *
 * What one time step computes (paper references):
 *   - moments of the weighted populations on the mixed half-range (x) /
 *     full-range (y, z) Gauss-Hermite lattice (eq:macro_LB, Sec. III.A);
 *   - the Carnahan-Starling contact value chi (eq:chi), relaxation time
 *     (eq:viscosity, eq:tau, Kn definition of Sec. II.A) and Prandtl number
 *     (eq:prandtl);
 *   - the Shakhov target (eq:j0) plus the first-order Enskog correction J1
 *     (eq:j1) from 6th-order gradients of ln n, ln chi, ln T, u (Sec. III.B.3),
 *     projected per axis onto the lattice (eq:hh_gk, eq:H_gk);
 *   - WENO-5 advection (eq:weno5_flux_x .. eq:weno5_sigma) with diffuse
 *     walls whose density follows from impenetrability (Sec. III.B), the
 *     body-force kernel of App. A (eq:kernel_H), advanced by TVD-RK3 (eq:rk3).
 *
 * Conventions
 *   - Reduced units m = k_B = 1; plate separation L = 1; sigma = 1/R with
 *     R = 1/(6 sqrt2 eta0 chi(eta0) Kn); computational width L_c = 1 - sigma.
 *   - Velocity index kappa = ((kx*qy) + ky)*qz + kz, kx < qx_half are the
 *     positive x nodes; populations stored structure-of-arrays f[kappa][cell].
 *   - All host-side numbers are double.  Every call returns FDLB_OK (0) or a
 *     negative fdlb_status; fdlb_last_error() returns a thread-local message.
 *   - Memory: the caller owns one device workspace (size from
 *     fdlb_workspace_bytes) and the HIP stream; the library never calls
 *     hipMalloc for them.  The handle owns host-side tables only.
 *   - Calls are stream-ordered on the caller's stream.  Functions returning
 *     host data (moments, residuals, state) synchronise that stream.
 */
#ifndef FDLB_H
#define FDLB_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fdlb_status {
  FDLB_OK = 0,
  FDLB_EINVAL = -1,     /* invalid parameters or arguments */
  FDLB_EHIP = -2,       /* a HIP runtime call failed */
  FDLB_ENOMEM = -3,     /* workspace too small */
  FDLB_ENONFINITE = -4, /* non-finite or non-positive n or T detected */
  FDLB_ESTALL = -5,     /* residual stalled or max_steps reached (outputs filled) */
  FDLB_ESTATE = -6      /* call not valid in the handle's current state */
};

enum fdlb_flow { FDLB_FOURIER = 0, FDLB_COUETTE = 1, FDLB_POISEUILLE = 2 };
enum fdlb_collision { FDLB_BGK = 0, FDLB_SHAKHOV_FIXED_PR = 1, FDLB_SHAKHOV_DENSE_PR = 2 };
enum fdlb_grid { FDLB_GRID_UNIFORM = 0, FDLB_GRID_TANH = 1 };
enum fdlb_precision { FDLB_F64 = 0, FDLB_F32_BULK = 1 };
enum fdlb_x_rule { FDLB_X_HALF_RANGE = 0, FDLB_X_FULL_RANGE = 1 };

/* Problem statement of one channel case (Sec. II.A, Sec. IV, Table tab:quad). */
typedef struct {
  int flow;                  /* fdlb_flow; metadata (walls and force define the physics) */
  double kn;                 /* Knudsen number; <= 0 encodes Kn = infinity (requires eta0 == 0) */
  double eta0;               /* mean reduced density, [0, 0.5) */
  double t_left, t_right;    /* wall temperatures */
  double uy_left, uy_right;  /* wall velocities along y */
  double ay;                 /* body acceleration along y (Poiseuille) */
  double n_init, t_init, uy_init; /* uniform initial state (projected Maxwellian) */
  int nx, grid;              /* cells (>= 7) and fdlb_grid */
  double stretch;            /* tanh map parameter delta for FDLB_GRID_TANH */
  int qx_half, qy, qz;       /* half-range order per half (1..200); full-range orders (2..8) */
  int collision;             /* fdlb_collision */
  double pr_fixed;           /* Prandtl number for FDLB_SHAKHOV_FIXED_PR */
  int chi_mode;              /* 0: local Carnahan-Starling chi(eta0 n(x)) (eq:chi); 1: revised
                                Enskog theory, chi(eta0 nbar(x)) with the Fischer-Methfessel
                                average density (eq:chi_ret) over |x'-x| < sigma, n = 0 outside
                                the accessible width; nx <= 4000.  With 1 the layered density
                                of a dense case can leave the residual of fdlb_run_to_steady
                                stalled at 1e-6 .. 1e-4 (WENO weights switching at its
                                extrema) while the moments have settled */
  int j1_shear;              /* 1: keep the xi_x xi_y du_y/dx term of J1 (3D operator) */
  double cfl, dt;            /* dt > 0 overrides dt = cfl * min cell / max |p_x| */
  int precision;             /* fdlb_precision */
  int x_rule;                /* fdlb_x_rule: FDLB_X_HALF_RANGE (0, the method, Sec. III.A.2) or
                                FDLB_X_FULL_RANGE (1): a full-range Gauss-Hermite rule of order
                                2*qx_half on x, the comparison of App. A (fig:full_vs_half);
                                2*qx_half <= 200; the lattice keeps the same layout (kx <
                                qx_half are the positive nodes, kx >= qx_half their mirror
                                images) and the projections are the full-range ones
                                (eq:g_H, eq:H_gk); not available for the reduced models */
} fdlb_params;

typedef struct fdlb_ctx *fdlb_handle;

/* Number of moment fields returned per cell: n, u_x, u_y, T, q_x, q_y,
   P_xx, P_xy, P_yy, P_zz (kinetic parts, eq:macro_LB). */
#define FDLB_NMOM 10

/* Device workspace bytes for ncases cases (0 when a case is invalid;
   fdlb_last_error() names it). */
size_t fdlb_workspace_bytes(const fdlb_params *cases, int ncases);

/* Validate one case and report derived quantities: out[0] = sigma,
   out[1] = L_c, out[2] = dt, out[3] = K (velocities), out[4] = R. */
int fdlb_case_info(const fdlb_params *p, double *out5);

/* Host-only helpers (no device needed): the velocity set px, py, pz and
   lattice weights w ([K] each) and the grid (cell centres x[nx], metric
   dx/deta jac[nx]) that a case would use. */
int fdlb_case_lattice(const fdlb_params *p, double *px, double *py, double *pz, double *w);
int fdlb_case_grid(const fdlb_params *p, double *x, double *jac);

/* Set up ncases independent cases in dev_workspace (bytes long, device
   memory owned by the caller) on hip_stream (a hipStream_t, may be NULL for
   the default stream).  Builds the lattice, grid and constant tables on the
   host, uploads them, and sets every case to its uniform initial state.  The
   single-case solver is a batch of one. */
int fdlb_init(const fdlb_params *cases, int ncases, void *dev_workspace, size_t bytes,
              void *hip_stream, fdlb_handle *out);

/* Variant of fdlb_init for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the workspace is a device array of FDLB_STATIC_WORKSPACE_BYTES
   that the library reserves per GPU when its code object loads and keeps until
   the process ends; this call allocates no device memory.  The cases are set
   up on hip_stream of the current device as by fdlb_init, and every other call
   takes the handle as usual.  One live handle per device holds the array:
   FDLB_ESTATE while an earlier handle from this call on the same device is
   not destroyed (its state lives in the same memory; two handles would race),
   FDLB_ENOMEM when fdlb_workspace_bytes of the cases exceeds the array (the
   C1-C3 workloads fit in either precision; large cases need fdlb_init),
   FDLB_EINVAL for invalid cases, FDLB_EHIP if the array's address cannot be
   obtained.  Each set-up overwrites everything it uses, so the contents a
   previous handle left do not matter. */
#define FDLB_STATIC_WORKSPACE_BYTES (32u << 20)
int fdlb_init_static(const fdlb_params *cases, int ncases, void *hip_stream, fdlb_handle *out);

/* Advance every active case by nsteps TVD-RK3 steps (asynchronous). */
int fdlb_step(fdlb_handle h, long nsteps);

/* Moments of case `c` into host_out[FDLB_NMOM][nx] (synchronises). */
int fdlb_moments(fdlb_handle h, int c, double *host_out);

/* Cell centres x[nx] and metric dx/deta[nx] of case c. */
int fdlb_grid_coords(fdlb_handle h, int c, double *x, double *jac);

/* Velocity set of case c: px, py, pz and lattice weights w, each [K]. */
int fdlb_lattice(fdlb_handle h, int c, double *px, double *py, double *pz, double *w);

/* Geometry of case c: out3[0] = sigma, out3[1] = L_c, out3[2] = R. */
int fdlb_geometry(fdlb_handle h, int c, double *out3);

/* Time step of case c. */
int fdlb_dt(fdlb_handle h, int c, double *dt);

/* Run all cases until the steady-state residual
   r = max over n, u_x, u_y, T and cells of |M^{s} - M^{s-1}| / dt
   drops below tol, checked every check_every steps (converged cases stop
   advancing).  steps_out[ncases] and resid_out[ncases] receive the step
   count and last residual.  Returns FDLB_ESTALL if some case did not
   converge within max_steps (outputs still filled).  An FDLB_F32_BULK case
   is promoted to FP64 storage, with the mass it started the call with, when
   its residual stalls (fdlb_set_stall_checks), falls below tol or reaches
   exactly 0 (a fixed point of the FP32 map, whose sub-ulp increments are
   lost), and finishes in FP64: the converged state is an FP64 one. */
int fdlb_run_to_steady(fdlb_handle h, double tol, long max_steps, long check_every,
                       long *steps_out, double *resid_out);

/* Residual of the last completed step of every case (synchronises):
   resid_out[ncases]. */
int fdlb_residual(fdlb_handle h, double *resid_out);

/* Replace the state of case c by the Grad-13-type distribution
   f = n Proj[f^MB(n,u,T) (1 + Pxy xi_x xi_y/(n T^2) + qx xi_x (xi^2/T - 5)/(5 n T^2))]
   from host fields[6][nx] = n, u_x, u_y, T, q_x, P_xy, optionally multiplied
   node by node by (1 + noise[K][nx]) (noise may be NULL). */
int fdlb_set_state(fdlb_handle h, int c, const double *fields, const double *noise);

/* Copy the populations of case c to / from host memory as double [K][nx]. */
int fdlb_get_f(fdlb_handle h, int c, double *host_f);
int fdlb_set_f(fdlb_handle h, int c, const double *host_f);

/* Promote case c from FP32-bulk to FP64 storage now (no-op for FP64 cases):
   the FP64 populations are the FP32 state, which holds f minus the case's
   background populations, plus that background.  Later steps run in FP64.
   Rebuilds the launch maps (drops captured graphs); synchronises. */
int fdlb_promote(fdlb_handle h, int c);

/* Stall rule of fdlb_run_to_steady for FP32-bulk cases: a case whose residual
   has not dropped below 0.9 x its best value for `checks` consecutive checks
   is promoted to FP64 (default 20; checks >= 1). */
int fdlb_set_stall_checks(fdlb_handle h, int checks);

/* When on, fdlb_run_to_steady gives a case whose moments turn non-finite one
   restart from its uniform initial state (same batch, steps keep counting)
   instead of retiring it; for warm starts that may be unstable.  Default off. */
int fdlb_set_restart_on_nonfinite(fdlb_handle h, int on);

/* Restarts of each case in the last fdlb_run_to_steady: out[ncases]. */
int fdlb_restarts(fdlb_handle h, long *out);

/* Precision currently used for the bulk of case c (fdlb_precision). */
int fdlb_case_precision(fdlb_handle h, int c, int *precision);

/* Kernel tuning for all cases: kx values per velocity chunk (0 = automatic)
   and waves per update block (1, 2, 4 or 8).  Rebuilds the launch maps and
   drops captured graphs. */
int fdlb_set_tiling(fdlb_handle h, int kx_per_chunk, int waves_per_block);

/* Capture nsteps steps in a HIP graph that fdlb_step replays (0 disables). */
int fdlb_set_graph_steps(fdlb_handle h, int nsteps);

/* Measurement: runs nrep ordinary steps with HIP events on the caller's
   stream around every table and update launch, and returns the mean device
   time in ms per launch as the kernels run in sequence: ms_out[7] = table pass
   (summed over launch groups), update stages 1-3 of FP64 cases, update stages
   1-3 of FP32-bulk cases.  Advances the state by nrep steps (synchronises). */
int fdlb_profile(fdlb_handle h, int nrep, double *ms_out);

/* Measurement: plain device-to-device copy of `bytes` (a multiple of 32) on
   the given stream, used to calibrate hardware traffic counters. */
int fdlb_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------------
   Warm-start network: a multilayer perceptron (n_in -> depth hidden layers of
   `width` with GELU -> n_out), BF16 weights and activations with FP32
   accumulation (MFMA), FP32 master weights, MSE loss and AdamW, trained and
   evaluated by the library's own kernels.  Parameters are one flat FP32
   vector: for each layer W[out][in] row-major, then b[out].  x, t, y are
   device pointers to FP32 row-major [batch][n_in] / [batch][n_out].
   ------------------------------------------------------------------------ */
typedef struct fdlb_mlp_ctx *fdlb_mlp;
size_t fdlb_mlp_workspace_bytes(int n_in, int width, int depth, int n_out, int max_batch);
int fdlb_mlp_init(int n_in, int width, int depth, int n_out, int max_batch, void *dev_workspace, size_t bytes,
                  void *hip_stream, fdlb_mlp *out);
int fdlb_mlp_num_params(fdlb_mlp h, long *n);
int fdlb_mlp_set_params(fdlb_mlp h, const float *host_params);   /* resets the optimiser state */
int fdlb_mlp_get_params(fdlb_mlp h, float *host_params);
int fdlb_mlp_forward(fdlb_mlp h, const float *x_dev, int batch, float *y_dev);
/* forward + backward without an update: mean squared error and its gradient
   with respect to every parameter (grad_host[num_params], may be NULL) */
int fdlb_mlp_loss_grad(fdlb_mlp h, const float *x_dev, const float *t_dev, int batch, float *loss_host,
                       float *grad_host);
/* one AdamW step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay);
   loss_host may be NULL to stay asynchronous */
int fdlb_mlp_train_step(fdlb_mlp h, const float *x_dev, const float *t_dev, int batch, float lr,
                        float weight_decay, float *loss_host);
/* C[M][N] (ldc) = A * B for BF16 A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (synchronises) */
int fdlb_mlp_gemm_bf16(const void *A, const void *B, float *C, int M, int N, int K, long sam, long sak, long sbk,
                       long sbn, int ldc, void *hip_stream);
void fdlb_mlp_destroy(fdlb_mlp h);
const char *fdlb_mlp_last_error(void);

/* Release host-side state (the caller still owns the workspace). */
void fdlb_destroy(fdlb_handle h);

/* ---- reduced models (Sec. II.B) ------------------------------------------
   The paper's own formulation of the channel flows, chosen by the flow field:
   - Fourier (flow 0), 1D: phi = int f dp_y dp_z and theta = int (p_y^2 +
     p_z^2) f dp_y dp_z on the 2 qx_half half-range x-nodes (eq:evolution_1D,
     moments eq:macro1D).  Walls and initial state at u_y = 0, a_y = 0; qy is
     ignored.  Rows: [0, 2 qx_half) phi, then theta.
   - Couette and Poiseuille (flows 1, 2), 2D: phi = int f dp_z and theta =
     int p_z^2 f dp_z on the 2 qx_half x qy (x, y) nodes (eq:evolution_2D with
     the body force, moments eq:macro2D), 4 qx_half qy <= 640.  Rows: phi
     (kx, ky) at kx qy + ky, then theta in the same order.
   Every case: precision FDLB_F64, qx_half <= 32; chi_mode 0 or 1 (the
   revised Enskog average, by its own pass over the phi rows before each
   stage; nx <= 4000); qz is ignored; one dimension per batch.  Cases of at
   most 256 rows and those above launch as two groups, one after the other
   in each stage, each with the tile of its largest row count (32 cells up
   to 128 rows, 16 up to 256, 4 above); results do not depend on the tile.  State layout: [rows][nx] doubles, x-nodes in
   the order of fdlb_case_lattice's, cells contiguous.  Each TVD-RK3 step is
   three launches of one fused kernel; the calls follow the 3D solver's
   conventions (caller-owned workspace, stream, error codes). */
typedef struct fdlb_r1_ctx *fdlb_r1_handle;
/* Device workspace bytes for ncases reduced cases (0 when a case is invalid
   or the batch mixes dimensions). */
size_t fdlb_r1_workspace_bytes(const fdlb_params *cases, int ncases);
/* Set up the cases in dev_workspace on hip_stream, each at its uniform
   initial state (n_init, T_init at rest). */
int fdlb_r1_init(const fdlb_params *cases, int ncases, void *dev_workspace, size_t bytes,
                 void *hip_stream, fdlb_r1_handle *out);
/* Advance every case by nsteps steps (asynchronous). */
int fdlb_r1_step(fdlb_r1_handle h, long nsteps);
/* Moments of case c into host_out[FDLB_NMOM][nx] (1D: u_y, q_y, P_xy are 0
   and P_yy = P_zz = half the theta sum; 2D: P_zz is the theta sum)
   (synchronises). */
int fdlb_r1_moments(fdlb_r1_handle h, int c, double *host_out);
/* Replace the state of case c by the reduced Grad-13-type state of host
   fields[6][nx] (n, u_x, u_y, T, q_x, P_xy; 1D ignores u_y and P_xy),
   optionally times (1 + noise[rows][nx]) (synchronises). */
int fdlb_r1_set_state(fdlb_r1_handle h, int c, const double *fields, const double *noise);
/* Copy phi and theta of case c to host_f[rows][nx] (synchronises). */
int fdlb_r1_get_f(fdlb_r1_handle h, int c, double *host_f);
/* Time step of case c. */
int fdlb_r1_dt(fdlb_r1_handle h, int c, double *dt);
void fdlb_r1_destroy(fdlb_r1_handle h);

const char *fdlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
