"""ctypes binding of libfdlb.so (include/fdlb.h): same names, argument marshalling only.

Every step of the time integration runs in the library's gfx950 kernels; this
module converts Python/numpy/torch arguments and raises on negative status.
The library must have been built (``paper_2308_15407_amd.build.build()``); there
is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FDLB_LIB", os.path.join(HERE, "libfdlb.so"))

FDLB_OK, FDLB_EINVAL, FDLB_EHIP, FDLB_ENOMEM, FDLB_ENONFINITE, FDLB_ESTALL, FDLB_ESTATE = 0, -1, -2, -3, -4, -5, -6
FDLB_NMOM = 10
FDLB_STATIC_WORKSPACE_BYTES = 32 << 20   # include/fdlb.h
MOMENT_NAMES = ("n", "ux", "uy", "T", "qx", "qy", "Pxx", "Pxy", "Pyy", "Pzz")

# every symbol declared in include/fdlb.h
EXPORTS = ("fdlb_workspace_bytes", "fdlb_case_info", "fdlb_case_lattice", "fdlb_case_grid", "fdlb_init",
           "fdlb_init_static",
           "fdlb_step", "fdlb_moments", "fdlb_grid_coords", "fdlb_lattice", "fdlb_geometry", "fdlb_dt",
           "fdlb_run_to_steady",
           "fdlb_residual", "fdlb_set_state", "fdlb_get_f", "fdlb_set_f", "fdlb_promote",
           "fdlb_set_restart_on_nonfinite", "fdlb_restarts",
           "fdlb_set_stall_checks", "fdlb_case_precision",
           "fdlb_set_tiling", "fdlb_set_graph_steps", "fdlb_profile", "fdlb_copy_probe", "fdlb_destroy",
           "fdlb_last_error", "fdlb_mlp_workspace_bytes", "fdlb_mlp_init", "fdlb_mlp_num_params",
           "fdlb_mlp_set_params", "fdlb_mlp_get_params", "fdlb_mlp_forward", "fdlb_mlp_loss_grad",
           "fdlb_mlp_train_step", "fdlb_mlp_gemm_bf16", "fdlb_mlp_destroy", "fdlb_mlp_last_error",
           "fdlb_r1_workspace_bytes", "fdlb_r1_init", "fdlb_r1_step", "fdlb_r1_moments", "fdlb_r1_set_state",
           "fdlb_r1_get_f", "fdlb_r1_dt", "fdlb_r1_destroy")


class FdlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fdlb error %d: %s" % (code, msg))
        self.code = code


class fdlb_params(C.Structure):
    _fields_ = [("flow", C.c_int), ("kn", C.c_double), ("eta0", C.c_double),
                ("t_left", C.c_double), ("t_right", C.c_double),
                ("uy_left", C.c_double), ("uy_right", C.c_double), ("ay", C.c_double),
                ("n_init", C.c_double), ("t_init", C.c_double), ("uy_init", C.c_double),
                ("nx", C.c_int), ("grid", C.c_int), ("stretch", C.c_double),
                ("qx_half", C.c_int), ("qy", C.c_int), ("qz", C.c_int),
                ("collision", C.c_int), ("pr_fixed", C.c_double),
                ("chi_mode", C.c_int), ("j1_shear", C.c_int),
                ("cfl", C.c_double), ("dt", C.c_double), ("precision", C.c_int), ("x_rule", C.c_int)]


PARAM_DEFAULTS = dict(flow=0, kn=0.1, eta0=0.05, t_left=1.0, t_right=1.0, uy_left=0.0, uy_right=0.0, ay=0.0,
                      n_init=1.0, t_init=1.0, uy_init=0.0, nx=64, grid=0, stretch=0.0, qx_half=4, qy=3, qz=3,
                      collision=0, pr_fixed=2.0 / 3.0, chi_mode=0, j1_shear=1, cfl=0.5, dt=0.0, precision=0,
                      x_rule=0)


def make_params(d):
    full = dict(PARAM_DEFAULTS)
    d = {k: v for k, v in d.items() if not k.startswith("_")}   # caller bookkeeping keys
    unknown = set(d) - set(full)
    if unknown:
        raise TypeError("unknown case parameters: %s" % sorted(unknown))
    full.update(d)
    return fdlb_params(**full)


_lib = None


def lib():
    """Load libfdlb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own libamdhip64.so.7: load it first so that this
        # library binds to the same HIP runtime as the tensors it is handed
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfdlb.so is not built; run paper_2308_15407_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P, I, D, Z = C.c_void_p, C.c_int, C.c_double, C.c_size_t
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(fdlb_params)
        L.fdlb_workspace_bytes.restype = Z
        L.fdlb_workspace_bytes.argtypes = [pp, I]
        L.fdlb_case_info.argtypes = [pp, dp]
        L.fdlb_case_lattice.argtypes = [pp, dp, dp, dp, dp]
        L.fdlb_case_grid.argtypes = [pp, dp, dp]
        L.fdlb_init.argtypes = [pp, I, P, Z, P, C.POINTER(P)]
        L.fdlb_init_static.argtypes = [pp, I, P, C.POINTER(P)]
        L.fdlb_step.argtypes = [P, C.c_long]
        L.fdlb_moments.argtypes = [P, I, dp]
        L.fdlb_grid_coords.argtypes = [P, I, dp, dp]
        L.fdlb_lattice.argtypes = [P, I, dp, dp, dp, dp]
        L.fdlb_dt.argtypes = [P, I, dp]
        L.fdlb_run_to_steady.argtypes = [P, D, C.c_long, C.c_long, C.POINTER(C.c_long), dp]
        L.fdlb_residual.argtypes = [P, dp]
        L.fdlb_set_state.argtypes = [P, I, dp, dp]
        L.fdlb_get_f.argtypes = [P, I, dp]
        L.fdlb_set_f.argtypes = [P, I, dp]
        L.fdlb_case_precision.argtypes = [P, I, C.POINTER(I)]
        L.fdlb_promote.argtypes = [P, I]
        L.fdlb_geometry.argtypes = [P, I, dp]
        L.fdlb_set_restart_on_nonfinite.argtypes = [P, I]
        L.fdlb_restarts.argtypes = [P, C.POINTER(C.c_long)]
        L.fdlb_set_stall_checks.argtypes = [P, I]
        L.fdlb_set_tiling.argtypes = [P, I, I]
        L.fdlb_set_graph_steps.argtypes = [P, I]
        L.fdlb_profile.argtypes = [P, I, dp]
        L.fdlb_copy_probe.argtypes = [P, P, Z, P]
        L.fdlb_destroy.argtypes = [P]
        L.fdlb_destroy.restype = None
        L.fdlb_last_error.restype = C.c_char_p
        fp = C.POINTER(C.c_float)
        L.fdlb_mlp_workspace_bytes.restype = Z
        L.fdlb_mlp_workspace_bytes.argtypes = [I, I, I, I, I]
        L.fdlb_mlp_init.argtypes = [I, I, I, I, I, P, Z, P, C.POINTER(P)]
        L.fdlb_mlp_num_params.argtypes = [P, C.POINTER(C.c_long)]
        L.fdlb_mlp_set_params.argtypes = [P, fp]
        L.fdlb_mlp_get_params.argtypes = [P, fp]
        L.fdlb_mlp_forward.argtypes = [P, P, I, P]
        L.fdlb_mlp_loss_grad.argtypes = [P, P, P, I, fp, fp]
        L.fdlb_mlp_train_step.argtypes = [P, P, P, I, C.c_float, C.c_float, fp]
        L.fdlb_mlp_gemm_bf16.argtypes = [P, P, P, I, I, I, C.c_long, C.c_long, C.c_long, C.c_long, I, P]
        L.fdlb_mlp_destroy.argtypes = [P]
        L.fdlb_mlp_destroy.restype = None
        L.fdlb_mlp_last_error.restype = C.c_char_p
        L.fdlb_r1_workspace_bytes.restype = Z
        L.fdlb_r1_workspace_bytes.argtypes = [pp, I]
        L.fdlb_r1_init.argtypes = [pp, I, P, Z, P, C.POINTER(P)]
        L.fdlb_r1_step.argtypes = [P, C.c_long]
        L.fdlb_r1_moments.argtypes = [P, I, dp]
        L.fdlb_r1_set_state.argtypes = [P, I, dp, dp]
        L.fdlb_r1_get_f.argtypes = [P, I, dp]
        L.fdlb_r1_dt.argtypes = [P, I, dp]
        L.fdlb_r1_destroy.argtypes = [P]
        L.fdlb_r1_destroy.restype = None
        for name in EXPORTS:
            if name not in ("fdlb_workspace_bytes", "fdlb_destroy", "fdlb_last_error", "fdlb_mlp_workspace_bytes",
                            "fdlb_mlp_destroy", "fdlb_mlp_last_error", "fdlb_r1_workspace_bytes", "fdlb_r1_destroy"):
                getattr(L, name).restype = I
        _lib = L
    return _lib


def _chk(code, allow=()):
    if code != FDLB_OK and code not in allow:
        raise FdlbError(code, lib().fdlb_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _params_array(cases):
    arr = (fdlb_params * len(cases))()
    for i, d in enumerate(cases):
        arr[i] = make_params(d)
    return arr


def fdlb_workspace_bytes(cases):
    arr = _params_array(cases)
    n = lib().fdlb_workspace_bytes(arr, len(cases))
    if n == 0:
        raise FdlbError(FDLB_EINVAL, lib().fdlb_last_error().decode())
    return n


def fdlb_case_info(case):
    out = np.zeros(5)
    p = make_params(case)
    _chk(lib().fdlb_case_info(C.byref(p), _dptr(out)))
    return dict(sigma=out[0], Lc=out[1], dt=out[2], K=int(out[3]), R=out[4])


def fdlb_case_lattice(case):
    p = make_params(case)
    K = 2 * p.qx_half * p.qy * p.qz
    px, py, pz, w = (np.zeros(K) for _ in range(4))
    _chk(lib().fdlb_case_lattice(C.byref(p), _dptr(px), _dptr(py), _dptr(pz), _dptr(w)))
    return px, py, pz, w


def fdlb_case_grid(case):
    p = make_params(case)
    x, j = np.zeros(p.nx), np.zeros(p.nx)
    _chk(lib().fdlb_case_grid(C.byref(p), _dptr(x), _dptr(j)))
    return x, j


def fdlb_init(cases, workspace_ptr, nbytes, stream_ptr):
    arr = _params_array(cases)
    h = C.c_void_p()
    _chk(lib().fdlb_init(arr, len(cases), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def fdlb_init_static(cases, stream_ptr):
    """fdlb_init on the library's static device workspace (no allocation)."""
    arr = _params_array(cases)
    h = C.c_void_p()
    _chk(lib().fdlb_init_static(arr, len(cases), C.c_void_p(stream_ptr), C.byref(h)))
    return h


def fdlb_step(h, nsteps):
    _chk(lib().fdlb_step(h, int(nsteps)))


def fdlb_moments(h, c, nx):
    out = np.zeros((FDLB_NMOM, nx))
    _chk(lib().fdlb_moments(h, c, _dptr(out)))
    return out


def fdlb_grid_coords(h, c, nx):
    x, j = np.zeros(nx), np.zeros(nx)
    _chk(lib().fdlb_grid_coords(h, c, _dptr(x), _dptr(j)))
    return x, j


def fdlb_lattice(h, c, K):
    px, py, pz, w = (np.zeros(K) for _ in range(4))
    _chk(lib().fdlb_lattice(h, c, _dptr(px), _dptr(py), _dptr(pz), _dptr(w)))
    return px, py, pz, w


def fdlb_set_restart_on_nonfinite(h, on):
    _chk(lib().fdlb_set_restart_on_nonfinite(h, 1 if on else 0))


def fdlb_restarts(h, ncases):
    out = (C.c_long * ncases)()
    _chk(lib().fdlb_restarts(h, out))
    return np.array(list(out))


def fdlb_geometry(h, c):
    out = np.zeros(3)
    _chk(lib().fdlb_geometry(h, c, _dptr(out)))
    return {"sigma": out[0], "Lc": out[1], "R": out[2]}


def fdlb_dt(h, c):
    d = C.c_double()
    _chk(lib().fdlb_dt(h, c, C.byref(d)))
    return d.value


def fdlb_run_to_steady(h, ncases, tol, max_steps, check_every):
    steps = (C.c_long * ncases)()
    res = np.zeros(ncases)
    code = _chk(lib().fdlb_run_to_steady(h, tol, int(max_steps), int(check_every), steps, _dptr(res)),
                allow=(FDLB_ESTALL, FDLB_ENONFINITE))
    return np.array(list(steps)), res, code


def fdlb_residual(h, ncases):
    out = np.zeros(ncases)
    _chk(lib().fdlb_residual(h, _dptr(out)))
    return out


def fdlb_set_state(h, c, fields, noise=None):
    fields = np.ascontiguousarray(fields, dtype=np.float64)
    noise = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
    _chk(lib().fdlb_set_state(h, c, _dptr(fields), _dptr(noise)))


def fdlb_get_f(h, c, K, nx):
    out = np.zeros((K, nx))
    _chk(lib().fdlb_get_f(h, c, _dptr(out)))
    return out


def fdlb_set_f(h, c, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _chk(lib().fdlb_set_f(h, c, _dptr(f)))


def fdlb_promote(h, c):
    _chk(lib().fdlb_promote(h, c))


def fdlb_set_stall_checks(h, checks):
    _chk(lib().fdlb_set_stall_checks(h, checks))


def fdlb_case_precision(h, c):
    p = C.c_int()
    _chk(lib().fdlb_case_precision(h, c, C.byref(p)))
    return p.value


def fdlb_set_tiling(h, kx_per_chunk, waves):
    _chk(lib().fdlb_set_tiling(h, int(kx_per_chunk), int(waves)))


def fdlb_set_graph_steps(h, nsteps):
    _chk(lib().fdlb_set_graph_steps(h, int(nsteps)))


def fdlb_profile(h, nrep):
    out = np.zeros(7)
    _chk(lib().fdlb_profile(h, int(nrep), _dptr(out)))
    return out


def fdlb_copy_probe(src_ptr, dst_ptr, nbytes, stream_ptr):
    _chk(lib().fdlb_copy_probe(C.c_void_p(src_ptr), C.c_void_p(dst_ptr), int(nbytes), C.c_void_p(stream_ptr)))


def fdlb_destroy(h):
    lib().fdlb_destroy(h)


# --------------------------------------------------------------------------
# warm-start network
# --------------------------------------------------------------------------
def _mchk(code):
    if code != FDLB_OK:
        raise FdlbError(code, lib().fdlb_mlp_last_error().decode())


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def fdlb_mlp_workspace_bytes(n_in, width, depth, n_out, max_batch):
    return lib().fdlb_mlp_workspace_bytes(n_in, width, depth, n_out, max_batch)


def fdlb_mlp_init(n_in, width, depth, n_out, max_batch, ws_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _mchk(lib().fdlb_mlp_init(n_in, width, depth, n_out, max_batch, C.c_void_p(ws_ptr), nbytes,
                              C.c_void_p(stream_ptr), C.byref(h)))
    return h


def fdlb_mlp_num_params(h):
    n = C.c_long()
    _mchk(lib().fdlb_mlp_num_params(h, C.byref(n)))
    return n.value


def fdlb_mlp_set_params(h, params):
    params = np.ascontiguousarray(params, dtype=np.float32)
    _mchk(lib().fdlb_mlp_set_params(h, _fptr(params)))


def fdlb_mlp_get_params(h, n):
    out = np.zeros(n, dtype=np.float32)
    _mchk(lib().fdlb_mlp_get_params(h, _fptr(out)))
    return out


def fdlb_mlp_forward(h, x_ptr, batch, y_ptr):
    _mchk(lib().fdlb_mlp_forward(h, C.c_void_p(x_ptr), batch, C.c_void_p(y_ptr)))


def fdlb_mlp_loss_grad(h, x_ptr, t_ptr, batch, nparams):
    loss = np.zeros(1, dtype=np.float32)
    grad = np.zeros(nparams, dtype=np.float32)
    _mchk(lib().fdlb_mlp_loss_grad(h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), batch, _fptr(loss), _fptr(grad)))
    return float(loss[0]), grad


def fdlb_mlp_train_step(h, x_ptr, t_ptr, batch, lr, wd, want_loss=False):
    loss = np.zeros(1, dtype=np.float32) if want_loss else None
    _mchk(lib().fdlb_mlp_train_step(h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), batch, lr, wd, _fptr(loss)))
    return float(loss[0]) if want_loss else None


def fdlb_mlp_gemm_bf16(a_ptr, b_ptr, c_ptr, M, N, K, sam, sak, sbk, sbn, ldc, stream_ptr):
    _mchk(lib().fdlb_mlp_gemm_bf16(C.c_void_p(a_ptr), C.c_void_p(b_ptr), C.c_void_p(c_ptr), M, N, K, sam, sak, sbk,
                                   sbn, ldc, C.c_void_p(stream_ptr)))


def fdlb_mlp_destroy(h):
    lib().fdlb_mlp_destroy(h)


# ---- reduced 1D model (phi, theta on the x-nodes) ----------------------------
def fdlb_r1_workspace_bytes(cases):
    arr = _params_array(cases)
    n = lib().fdlb_r1_workspace_bytes(arr, len(cases))
    if n == 0:
        raise FdlbError(FDLB_EINVAL, lib().fdlb_last_error().decode())
    return n


def fdlb_r1_init(cases, workspace_ptr, nbytes, stream_ptr):
    arr = _params_array(cases)
    h = C.c_void_p()
    _chk(lib().fdlb_r1_init(arr, len(cases), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def fdlb_r1_step(h, nsteps):
    _chk(lib().fdlb_r1_step(h, int(nsteps)))


def fdlb_r1_moments(h, c, nx):
    out = np.zeros((FDLB_NMOM, nx))
    _chk(lib().fdlb_r1_moments(h, c, _dptr(out)))
    return out


def fdlb_r1_set_state(h, c, fields, noise=None):
    fields = np.ascontiguousarray(fields, dtype=np.float64)
    noise = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
    _chk(lib().fdlb_r1_set_state(h, c, _dptr(fields), _dptr(noise)))


def fdlb_r1_get_f(h, c, rows, nx):
    out = np.zeros((rows, nx))
    _chk(lib().fdlb_r1_get_f(h, c, _dptr(out)))
    return out


def fdlb_r1_dt(h, c):
    out = C.c_double()
    _chk(lib().fdlb_r1_dt(h, c, C.byref(out)))
    return out.value


def fdlb_r1_destroy(h):
    lib().fdlb_r1_destroy(h)
