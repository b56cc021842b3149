"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This module holds workload parameters and random draws only -- no arithmetic of
the method itself.  Every consumer (tests, bench, training-data generation)
turns these plain numbers into states with its own implementation.

Workloads (stand-ins for the paper's Fourier / Couette / Poiseuille channel
runs of Sec. IV; no dataset is involved):
  C1  Fourier, uniform Nx=64, Q_x^h=4 x Q_y=3 x Q_z=3 (K=72), Kn=0.1, eta0=0.05,
      walls T=1.0 / 1.1 at rest, initial n=1, u=0, T=1.05, BGK + J1, CFL 0.5.
  C2  Couette, Nx=256 wall-refined (tanh map, delta=1.5), 8 x 4 x 4 (K=256),
      Kn=0.1, eta0=0.2, walls T=1 moving at u_y=-/+0.2, Shakhov Pr=2/3.
  C3  Poiseuille, Nx=512 wall-refined, 16 x 6 x 4 (K=768), Kn=0.05, eta0=0.3,
      a_y=0.05, walls T=1 at rest, Shakhov with the dense Prandtl number.
  C4  sweep generator: flow uniform over {F, C, P}, Kn log-uniform [0.01, 1],
      eta0 uniform [0.01, 0.35], Nx in {64,128,256,512}, Q_x^h in {4,8,12,16},
      Q_y = Q_z = 4, wall dT / speed / force uniform in the stated ranges.
"""
import numpy as np

FOURIER, COUETTE, POISEUILLE = 0, 1, 2
BGK, SHAKHOV_FIXED, SHAKHOV_DENSE = 0, 1, 2
GRID_UNIFORM, GRID_TANH = 0, 1

BASE = dict(flow=FOURIER, kn=0.1, eta0=0.05, t_left=1.0, t_right=1.0, uy_left=0.0, uy_right=0.0,
            ay=0.0, n_init=1.0, t_init=1.0, uy_init=0.0, nx=64, grid=GRID_UNIFORM, stretch=0.0,
            qx_half=4, qy=3, qz=3, collision=BGK, pr_fixed=2.0 / 3.0, chi_mode=0, j1_shear=1,
            cfl=0.5, dt=0.0, x_rule=0)


def config(name, **over):
    """Parameter dict of a named workload, with optional overrides."""
    d = dict(BASE)
    if name == "C1":
        d.update(flow=FOURIER, kn=0.1, eta0=0.05, t_left=1.0, t_right=1.1, n_init=1.0,
                 t_init=1.05, nx=64, qx_half=4, qy=3, qz=3, collision=BGK)
    elif name == "C2":
        d.update(flow=COUETTE, kn=0.1, eta0=0.2, t_left=1.0, t_right=1.0, uy_left=-0.2,
                 uy_right=0.2, nx=256, grid=GRID_TANH, stretch=1.5, qx_half=8, qy=4, qz=4,
                 collision=SHAKHOV_FIXED, pr_fixed=2.0 / 3.0)
    elif name == "C3":
        d.update(flow=POISEUILLE, kn=0.05, eta0=0.3, ay=0.05, nx=512, grid=GRID_TANH,
                 stretch=1.5, qx_half=16, qy=6, qz=4, collision=SHAKHOV_DENSE)
    elif name == "R2":
        # single large Fourier-type case used to size the memory-bound roofline
        d.update(flow=FOURIER, kn=0.1, eta0=0.05, t_left=1.0, t_right=1.1, t_init=1.05,
                 nx=32768, qx_half=16, qy=4, qz=4, collision=BGK)
    else:
        raise KeyError(name)
    d.update(over)
    return d


def c4_draws(seed, n):
    """Raw seeded draws of the sweep generator (no acceptance test applied)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        out.append(dict(
            flow=int(rng.integers(0, 3)),
            kn=float(10.0 ** rng.uniform(-2.0, 0.0)),
            eta0=float(rng.uniform(0.01, 0.35)),
            nx=int(rng.choice([64, 128, 256, 512])),
            qx_half=int(rng.choice([4, 8, 12, 16])),
            dT=float(rng.uniform(0.05, 0.3)),
            speed=float(rng.uniform(0.05, 0.3)),
            force=float(rng.uniform(0.01, 0.1)),
        ))
    return out


def c4_params(draw):
    """Map one sweep draw to case parameters (FP32-bulk, dense-Pr Shakhov)."""
    d = dict(BASE)
    d.update(flow=draw["flow"], kn=draw["kn"], eta0=draw["eta0"], nx=draw["nx"],
             qx_half=draw["qx_half"], qy=4, qz=4, collision=SHAKHOV_DENSE,
             grid=GRID_TANH if draw["nx"] >= 256 else GRID_UNIFORM,
             stretch=1.5 if draw["nx"] >= 256 else 0.0)
    if draw["flow"] == FOURIER:
        d.update(t_left=1.0, t_right=1.0 + draw["dT"], t_init=1.0 + 0.5 * draw["dT"])
    elif draw["flow"] == COUETTE:
        d.update(uy_left=-draw["speed"], uy_right=draw["speed"])
    else:
        d.update(ay=draw["force"])
    return d


def smooth_fields(seed, nx, amp=0.05, n_modes=3):
    """Six smooth random cell fields (n, u_x, u_y, T, q_x, P_xy) around the rest
    state n = T = 1: low-order Fourier modes in the cell index."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = (np.arange(nx) + 0.5) / nx
    fields = np.zeros((6, nx))
    base = [1.0, 0.0, 0.0, 1.0, 0.0, 0.0]
    for f in range(6):
        acc = np.full(nx, base[f])
        for m in range(1, n_modes + 1):
            a, ph = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
            acc += amp * a * np.sin(np.pi * m * s + ph) / m
        fields[f] = acc
    return fields


def noise(seed, K, nx, eps=1e-3):
    """Multiplicative per-node perturbation (1 + noise), uniform in [-eps, eps]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-eps, eps, size=(K, nx))
