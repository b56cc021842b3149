"""ctypes binding of the plain FP64 CPU oracle (fdlb_oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle exists to check the GPU path.  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this module.  It shares no code with the product package.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdlb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile the oracle (gcc, -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [("flow", C.c_int), ("kn", C.c_double), ("eta0", C.c_double),
                ("t_left", C.c_double), ("t_right", C.c_double),
                ("uy_left", C.c_double), ("uy_right", C.c_double), ("ay", C.c_double),
                ("n_init", C.c_double), ("t_init", C.c_double), ("uy_init", C.c_double),
                ("nx", C.c_int), ("grid", C.c_int), ("stretch", C.c_double),
                ("qx_half", C.c_int), ("qy", C.c_int), ("qz", C.c_int),
                ("collision", C.c_int), ("pr_fixed", C.c_double),
                ("chi_mode", C.c_int), ("j1_shear", C.c_int),
                ("cfl", C.c_double), ("dt", C.c_double), ("x_rule", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P, D, I = C.c_void_p, C.c_double, C.c_int
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(OrcParams)]
        L.orc_destroy.argtypes = [P]
        L.orc_threads.restype = I
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [I]
        for name, res in [("orc_K", I), ("orc_dt", D), ("orc_sigma", D), ("orc_Lc", D), ("orc_steps", C.c_long)]:
            getattr(L, name).restype = res
            getattr(L, name).argtypes = [P]
        L.orc_set_state.argtypes = [P, dp, P]
        L.orc_set_uniform.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_long]
        L.orc_step_resid.restype = D
        L.orc_step_resid.argtypes = [P]
        L.orc_run_to_steady.restype = C.c_long
        L.orc_run_to_steady.argtypes = [P, D, C.c_long, C.POINTER(D)]
        L.orc_moments.argtypes = [P, dp]
        L.orc_get_f.argtypes = [P, dp]
        L.orc_set_f.argtypes = [P, dp]
        L.orc_lattice.argtypes = [P, dp, dp, dp, dp]
        L.orc_grid.argtypes = [P, dp, dp]
        L.orc_rhs.argtypes = [P, dp, dp]
        L.orc_face_fluxes.argtypes = [P, dp, dp, dp]
        L.orc_gh_rule.restype = I
        L.orc_gh_rule.argtypes = [I, dp, dp]
        L.orc_gh_rule_n.restype = I
        L.orc_gh_rule_n.argtypes = [I, dp, dp]
        L.orc_project_fullx_table.restype = I
        L.orc_project_fullx_table.argtypes = [I, D, D, I, dp]
        L.orc_hr_rule.restype = I
        L.orc_hr_rule.argtypes = [I, dp, dp, P]
        L.orc_project_half_table.restype = I
        L.orc_project_half_table.argtypes = [I, D, D, I, dp]
        L.orc_project_full_table.restype = I
        L.orc_project_full_table.argtypes = [I, D, D, I, dp]
        L.orc_kmat_table.restype = I
        L.orc_kmat_table.argtypes = [P, dp]
        L.orc_fd_weights7.argtypes = [I, dp]
        L.orc_weno.restype = D
        L.orc_weno.argtypes = [dp, I]
        L.orc_chi.restype = D
        L.orc_chi.argtypes = [D]
        L.orc_pr_dense.restype = D
        L.orc_pr_dense.argtypes = [D]
        L.orc_inv_tau.restype = D
        L.orc_inv_tau.argtypes = [D, D, D, D, D]
        L.orc_nbar.argtypes = [P, dp, dp]
        L.orc_nbar.restype = None
        L.orc_target.argtypes = [P, dp, dp, dp, C.POINTER(D)]
        L.orc_create_reduced1d.restype = P
        L.orc_set_weno_ideal.argtypes = [P, I]
        L.orc_set_weno_ideal.restype = None
        L.orc_create_reduced1d.argtypes = [C.POINTER(OrcParams)]
        L.orc_create_reduced2d.restype = P
        L.orc_create_reduced2d.argtypes = [C.POINTER(OrcParams)]
        _lib = L
    return _lib


DEFAULTS = dict(flow=0, kn=0.1, eta0=0.05, t_left=1.0, t_right=1.0, uy_left=0.0, uy_right=0.0,
                ay=0.0, n_init=1.0, t_init=1.0, uy_init=0.0, nx=64, grid=0, stretch=0.0,
                qx_half=4, qy=3, qz=3, collision=0, pr_fixed=2.0 / 3.0, chi_mode=0, j1_shear=1,
                cfl=0.5, dt=0.0, x_rule=0)


class Oracle:
    """One FDLB case on the CPU in FP64 (see fdlb_oracle.c).  reduced1d=True
    builds the paper's reduced 1D model of the Fourier flow instead: phi and
    theta on the 2 qx_half x-nodes (rows 0..2Q-1 and 2Q..4Q-1 of get_f);
    reduced2d=True the reduced 2D model: phi and theta on the 2 qx_half x qy
    (x, y) nodes (rows kx*qy + ky, then the theta rows)."""

    def __init__(self, reduced1d=False, reduced2d=False, **kw):
        d = dict(DEFAULTS)
        unknown = set(kw) - set(d)
        if unknown:
            raise TypeError("unknown oracle parameters: %s" % sorted(unknown))
        d.update(kw)
        self.params = d
        self._p = OrcParams(**d)
        self.reduced1d, self.reduced2d = bool(reduced1d), bool(reduced2d)
        create = lib().orc_create_reduced2d if reduced2d else (lib().orc_create_reduced1d if reduced1d
                                                                 else lib().orc_create)
        self._h = create(C.byref(self._p))
        if not self._h:
            raise ValueError("oracle rejected parameters %r" % d)
        self.nx = d["nx"]
        self.K = lib().orc_K(self._h)
        lib().orc_set_uniform(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def dt(self):
        return lib().orc_dt(self._h)

    @property
    def sigma(self):
        return lib().orc_sigma(self._h)

    @property
    def Lc(self):
        return lib().orc_Lc(self._h)

    @property
    def steps(self):
        return lib().orc_steps(self._h)

    def set_state(self, fields, noise=None):
        fields = np.ascontiguousarray(fields, dtype=np.float64).reshape(6, self.nx)
        if noise is None:
            lib().orc_set_state(self._h, fields, None)
        else:
            noise = np.ascontiguousarray(noise, dtype=np.float64).reshape(self.K, self.nx)
            lib().orc_set_state(self._h, fields, noise.ctypes.data_as(C.c_void_p))

    def set_weno_ideal(self, on=True):
        """Advect with the ideal (linear) WENO weights: a switch for the
        cross-check between the 3D lattice and the reduced model only."""
        lib().orc_set_weno_ideal(self._h, 1 if on else 0)

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def step_resid(self):
        return lib().orc_step_resid(self._h)

    def run_to_steady(self, tol, max_steps):
        r = C.c_double()
        s = lib().orc_run_to_steady(self._h, tol, int(max_steps), C.byref(r))
        return s, r.value

    def moments(self):
        out = np.zeros((10, self.nx))
        lib().orc_moments(self._h, out)
        return out

    def get_f(self):
        out = np.zeros((self.K, self.nx))
        lib().orc_get_f(self._h, out)
        return out

    def set_f(self, f):
        lib().orc_set_f(self._h, np.ascontiguousarray(f, dtype=np.float64).reshape(self.K, self.nx))

    def lattice(self):
        px, py, pz, w = (np.zeros(self.K) for _ in range(4))
        lib().orc_lattice(self._h, px, py, pz, w)
        return px, py, pz, w

    def grid(self):
        x, j = np.zeros(self.nx), np.zeros(self.nx)
        lib().orc_grid(self._h, x, j)
        return x, j

    def rhs(self):
        out = np.zeros((self.K, self.nx))
        nw = np.zeros(2)
        lib().orc_rhs(self._h, out, nw)
        return out, nw

    def face_fluxes(self):
        """Numerical face fluxes of the current state, each [nx + 1]: mass
        sum p_x f^, x-momentum sum p_x^2 f^ and y-momentum sum p_x p_y f^."""
        m, px, py = (np.zeros(self.nx + 1) for _ in range(3))
        lib().orc_face_fluxes(self._h, m, px, py)
        return m, px, py

    def kmat(self):
        out = np.zeros(self.params["qy"] ** 2)
        lib().orc_kmat_table(self._h, out)
        return out.reshape(self.params["qy"], self.params["qy"])

    def nbar(self, n):
        """Revised-Enskog (Fischer-Methfessel) average density of a cell-average
        density profile n[nx] on this oracle's grid."""
        n = np.ascontiguousarray(n, dtype=np.float64)
        out = np.zeros(self.params["nx"])
        lib().orc_nbar(self._h, n, out)
        return out

    def target(self, mom6, grad5):
        out = np.zeros(self.K)
        it = C.c_double()
        lib().orc_target(self._h, np.ascontiguousarray(mom6, dtype=np.float64),
                         np.ascontiguousarray(grad5, dtype=np.float64), out, C.byref(it))
        return out, it.value


def gh_rule(Q):
    n, w = np.zeros(Q), np.zeros(Q)
    if lib().orc_gh_rule(Q, n, w):
        raise RuntimeError("gh rule failed")
    return n, w


def gh_rule_n(Q):
    """Full-range rule of order Q <= 96 from the scaled Hermite recurrence
    (the x rule of x_rule = 1)."""
    n, w = np.zeros(Q), np.zeros(Q)
    if lib().orc_gh_rule_n(Q, n, w):
        raise RuntimeError("gh rule failed")
    return n, w


def project_fullx(qh, u, T, a):
    """Full-range x projection of g (p-u)^a at the 2 qh nodes of an x_rule = 1
    lattice (positive nodes first, then their mirror images)."""
    out = np.zeros(2 * qh)
    if lib().orc_project_fullx_table(qh, u, T, a, out):
        raise RuntimeError("projection failed")
    return out


def hr_rule(Q):
    n, w = np.zeros(Q), np.zeros(Q)
    if lib().orc_hr_rule(Q, n, w, None):
        raise RuntimeError("half-range rule failed")
    return n, w


def project_half(Q, u, T, a):
    out = np.zeros(2 * Q)
    if lib().orc_project_half_table(Q, u, T, a, out):
        raise RuntimeError("projection failed")
    return out


def project_full(Q, u, T, b):
    out = np.zeros(Q)
    if lib().orc_project_full_table(Q, u, T, b, out):
        raise RuntimeError("projection failed")
    return out


def fd_weights7(at):
    c = np.zeros(7)
    lib().orc_fd_weights7(at, c)
    return c


def weno(v, mode=0):
    return lib().orc_weno(np.ascontiguousarray(v, dtype=np.float64), mode)


def chi(eta):
    return lib().orc_chi(eta)


def pr_dense(brc):
    return lib().orc_pr_dense(brc)


def inv_tau(kn, chi0, n, T, eta):
    return lib().orc_inv_tau(kn, chi0, n, T, eta)
