"""The C-ABI library builds, loads, and exports every symbol of include/fdlb.h
(host-side checks only; no device calls)."""
import math
import os
import re

import numpy as np
import pytest

import fdlb_inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fdlb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdlb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2308_15407_amd import fdlb as F
    L = F.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(F.EXPORTS)


def test_validation_errors():
    from paper_2308_15407_amd import fdlb as F
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, nx=5))
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, eta0=0.3, kn=1.0))      # R < 1
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, kn=0.0, eta0=0.1))      # Kn = inf needs eta0 = 0
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, qy=9))
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, qx_half=201))               # above the wide tables
    assert F.fdlb_case_info(dict(I.BASE, qx_half=200, qy=2, qz=2))["K"] == 1600
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, chi_mode=2))                # unknown contact value
    with pytest.raises(F.FdlbError):
        F.fdlb_case_info(dict(I.BASE, chi_mode=1, nx=4096))       # averaging windows in LDS
    assert F.fdlb_case_info(dict(I.BASE, chi_mode=1, nx=4000))["K"] == 72
    assert F.fdlb_case_info(I.config("C1"))["K"] == 72


@pytest.mark.parametrize("name", ["C1", "C2", "C3"])
def test_host_lattice_and_grid_match_oracle(name):
    """Independent construction routes (Stieltjes/Sturm/Christoffel here,
    roots of h_Q with the paper's weight formula in the oracle) agree."""
    from paper_2308_15407_amd import fdlb as F
    from oracle import oracle as O
    cfg = I.config(name)
    o = O.Oracle(**cfg)
    px, py, pz, w = F.fdlb_case_lattice(cfg)
    opx, opy, opz, ow = o.lattice()
    assert np.max(np.abs(px - opx)) < 1e-14
    assert np.max(np.abs(py - opy)) < 1e-14 and np.max(np.abs(pz - opz)) < 1e-14
    assert np.max(np.abs(w - ow) / ow) < 1e-13
    x, j = F.fdlb_case_grid(cfg)
    ox, oj = o.grid()
    assert np.allclose(x, ox, rtol=0, atol=1e-15) and np.allclose(j, oj, rtol=0, atol=1e-15)
    info = F.fdlb_case_info(cfg)
    assert info["dt"] == pytest.approx(o.dt, rel=1e-15)
    assert info["sigma"] == pytest.approx(o.sigma, rel=1e-14)


def test_workspace_grows_with_cases():
    from paper_2308_15407_amd import fdlb as F
    a = F.fdlb_workspace_bytes([I.config("C1")])
    b = F.fdlb_workspace_bytes([I.config("C1"), I.config("C2")])
    assert b > a > 0


def test_sweep_batch_is_seeded_and_valid():
    """The sweep batch: 256 accepted draws (R >= 2), identical on every call,
    spanning the generator's grid sizes and half-range orders."""
    from paper_2308_15407_amd import fdlb as F, sweep
    a = sweep.sweep_cases(256)
    b = sweep.sweep_cases(256)
    assert len(a) == 256 and a == b
    assert all(F.fdlb_case_info(c)["R"] >= 2.0 for c in a)
    assert {c["nx"] for c in a} == {64, 128, 256, 512}
    assert {c["qx_half"] for c in a} == {4, 8, 12, 16}
    assert all(c["precision"] == 1 and c["qy"] == 4 and c["qz"] == 4 for c in a)
    assert {c["flow"] for c in a} == {0, 1, 2}


@pytest.mark.parametrize("Q", [33, 40, 64, 100, 150, 200])
def test_wide_half_range_rule_is_exact(Q):
    """Orders above 32 (the wide tables): sum_k w_k p_k^s over the positive
    x-nodes equals the half-range moment 2^((s-1)/2) Gamma((s+1)/2)/sqrt(2 pi)
    of the weight exp(-p^2/2)/sqrt(2 pi) for every s < 2Q (Gauss exactness,
    Sec. III.A.2).  Compared in log form (the moments reach 1e600)."""
    from paper_2308_15407_amd import fdlb as F
    px, _, _, w = F.fdlb_case_lattice(dict(I.BASE, qx_half=Q, qy=2, qz=2, nx=16))
    p = px.reshape(2 * Q, -1)[:Q, 0]
    wx = w.reshape(2 * Q, -1).sum(axis=1)[:Q]
    assert np.all(p > 0) and np.all(np.diff(p) > 0) and np.all(wx > 0)
    assert np.allclose(px.reshape(2 * Q, -1)[Q:, 0], -p, rtol=0, atol=0)
    for s in range(2 * Q):
        lg = (s - 1) / 2 * math.log(2) + math.lgamma((s + 1) / 2) - 0.5 * math.log(2 * math.pi)
        ratio = np.sum(wx * np.exp(s * np.log(p) - lg))
        assert abs(ratio - 1) < 5e-16 * (40 + s * math.log(p[-1])), (s, ratio)


@pytest.mark.parametrize("Q", [40, 48])
def test_wide_host_lattice_matches_oracle(Q):
    """The wide rule (Stieltjes/Sturm/Christoffel on the finer discretisation)
    against the oracle's roots of h_Q with the paper's weight formula."""
    from paper_2308_15407_amd import fdlb as F
    from oracle import oracle as O
    px, _, _, w = F.fdlb_case_lattice(dict(I.BASE, qx_half=Q, qy=2, qz=2, nx=16))
    p, ow = O.hr_rule(Q)
    assert np.max(np.abs(px.reshape(2 * Q, -1)[:Q, 0] - p)) < 1e-13
    assert np.max(np.abs(w.reshape(2 * Q, -1).sum(axis=1)[:Q] - ow) / ow) < 1e-12


def test_reduced_model_validation():
    """The reduced 1D model takes Fourier-type cases only (host-side checks)."""
    from paper_2308_15407_amd import fdlb as F
    ok = dict(I.BASE, nx=32, qx_half=8)
    assert F.fdlb_r1_workspace_bytes([ok, dict(ok, qx_half=32)]) > 0
    assert F.fdlb_r1_workspace_bytes([dict(ok, chi_mode=1)]) > 0
    for bad in (dict(ok, uy_left=0.1), dict(ok, ay=1e-3), dict(ok, chi_mode=1, nx=4096), dict(ok, precision=1),
                dict(ok, qx_half=33), dict(ok, nx=5)):
        with pytest.raises(F.FdlbError):
            F.fdlb_r1_workspace_bytes([bad])
    # 2D (Couette, Poiseuille): 4 qx_half qy <= 640, one dimension per batch
    ok2 = dict(I.BASE, flow=I.POISEUILLE, nx=32, qx_half=8, qy=5, ay=1e-3)
    assert F.fdlb_r1_workspace_bytes([ok2, dict(ok2, flow=I.COUETTE, uy_left=0.2, qx_half=16, qy=4)]) > 0
    assert F.fdlb_r1_workspace_bytes([ok2, dict(ok2, qx_half=29), dict(ok2, qx_half=32)]) > 0
    for bad in ([dict(ok2, qx_half=32, qy=6)], [ok, ok2]):
        with pytest.raises(F.FdlbError):
            F.fdlb_r1_workspace_bytes(bad)
