"""Linear stability of the dense-gas model about the gas at rest (CPU, oracle).

The mass-flow-rate sweep (Sec. IV, Poiseuille flow, fig:poisseuille_mfr)
cannot reach mean reduced densities above about 0.25: such cases blow up in
the oracle and on the GPU alike, at any time step.  These tests pin where
that comes from:

* the velocity-discrete model with exact spatial derivatives (the kinetic
  equation with the Shakhov target and J1, linearised about n = T = 1, u = 0
  for a Fourier mode e^{ikx}) has no growing mode at any k, at the densities
  that fail;
* the discretised right-hand side L[f] of the oracle (WENO-5 advection, FD6
  gradients for J1, diffuse walls), linearised about the same state between
  walls at T = 1, has growing modes for eta0 >= 0.25 but none at 0.2, and
  their growth rate doubles when the grid is refined twice, so that a finer
  grid (toward the paper's sigma/100) makes it worse;
* the growing modes sit at the walls (amplitude halving per cell inward) and
  appear only as J1 (proportional to b rho chi) grows with the density.

The instability is a property of the semi-discrete scheme at these
densities, not of the explicit time step and not of a reading of the
paper's formulas (the dense transport coefficients it implies are pinned in
test_oracle_pins.py)."""
import math

import numpy as np
import pytest

import fdlb_inputs as I
from oracle import oracle as O


def _kn(eta0, R):
    return 1.0 / (6 * math.sqrt(2) * eta0 * O.chi(eta0) * R)


def _cfg(eta0, R, nx):
    return dict(I.BASE, flow=I.FOURIER, kn=_kn(eta0, R), eta0=eta0, nx=nx, qx_half=4, qy=3, qz=3,
                collision=I.SHAKHOV_DENSE)


def _continuous_growth(eta0, R, ks):
    """max Re(lambda) of A(k) = -i k p_x - 1/tau + (1/tau) dF/dm M + (i k / tau) dF/dg G M,
    the Jacobians of the target F with respect to the moments m = (n, u_x, u_y,
    T, q_x, q_y) and to the gradients g = (ln n, ln chi, ln T, u_x, u_y)', taken
    by central differences of the oracle's target; M maps f to m, G maps m to
    the gradient amplitudes (chi local: dln chi = eta (3/(1-eta) - 1/(2-eta)) dln n)."""
    o = O.Oracle(**_cfg(eta0, R, 16))
    px, py, pz, _ = o.lattice()
    m0 = np.array([1.0, 0, 0, 1.0, 0, 0])
    f0, itau = o.target(m0, np.zeros(5))

    def moments(f):
        n = f.sum()
        ux, uy = (px * f).sum() / n, (py * f).sum() / n
        cx, cy = px - ux, py - uy
        c2 = cx ** 2 + cy ** 2 + pz ** 2
        return np.array([n, ux, uy, (c2 * f).sum() / (3 * n), 0.5 * (cx * c2 * f).sum(), 0.5 * (cy * c2 * f).sum()])

    eps, K = 1e-7, o.K
    M = np.array([(moments(f0 + eps * e) - moments(f0 - eps * e)) / (2 * eps) for e in np.eye(K)]).T
    dFm = np.array([(o.target(m0 + eps * e, np.zeros(5))[0] - o.target(m0 - eps * e, np.zeros(5))[0]) / (2 * eps)
                    for e in np.eye(6)]).T
    dFg = np.array([(o.target(m0, eps * e)[0] - o.target(m0, -eps * e)[0]) / (2 * eps) for e in np.eye(5)]).T
    G = np.zeros((5, 6))
    G[0, 0] = 1.0
    G[1, 0] = eta0 * (3 / (1 - eta0) - 1 / (2 - eta0))
    G[2, 3] = G[3, 1] = G[4, 2] = 1.0
    worst = -np.inf
    for k in ks:
        A = -1j * k * np.diag(px) - itau * np.eye(K) + itau * (dFm @ M) + itau * 1j * k * (dFg @ G @ M)
        worst = max(worst, np.max(np.linalg.eigvals(A).real))
    return worst


def _discrete_growth(eta0, R, nx):
    """max Re(lambda) of the Jacobian of the oracle's L[f] (reduced 1D form of
    the Fourier channel, walls at T = 1) at the uniform rest state, which is an
    exact steady state of the discrete equations."""
    o = O.Oracle(reduced1d=True, **_cfg(eta0, R, nx))
    f0 = o.get_f().copy()
    flat = f0.ravel()
    L0, _ = o.rhs()
    assert np.max(np.abs(L0)) < 1e-10
    J = np.zeros((flat.size, flat.size))
    for j in range(flat.size):
        h = 1e-6 * max(abs(flat[j]), 1e-3)
        e = flat.copy()
        e[j] += h
        o.set_f(e.reshape(f0.shape))
        Lp, _ = o.rhs()
        e[j] -= 2 * h
        o.set_f(e.reshape(f0.shape))
        Lm, _ = o.rhs()
        J[:, j] = (Lp - Lm).ravel() / (2 * h)
    o.set_f(f0)
    return np.max(np.linalg.eigvals(J).real)


@pytest.mark.parametrize("eta0,R", [(0.2, 10), (0.3, 10), (0.367, 10), (0.397, 5)])
def test_continuous_model_has_no_growing_mode(eta0, R):
    ks = np.concatenate([np.linspace(0.5, 60, 25), np.logspace(2, math.log10(5000), 20)])
    g = _continuous_growth(eta0, R, ks)
    print("eta0 %.3f R %d: max Re(lambda) over k = %.2e" % (eta0, R, g), flush=True)
    assert g < 1e-6


def test_discretised_operator_is_unstable_above_eta0_025_and_worse_on_finer_grids():
    stable = _discrete_growth(0.2, 10, 24)
    g24, g48 = _discrete_growth(0.3, 10, 24), _discrete_growth(0.3, 10, 48)
    print("R 10: eta0 0.2 nx 24: %.2e; eta0 0.3: nx 24 %.3g, nx 48 %.3g" % (stable, g24, g48), flush=True)
    assert stable < 1e-6
    assert g24 > 1.0
    assert 1.8 < g48 / g24 < 3.0       # grid-scale growth: proportional to 1 / dx
