"""Host logic of the quadrature convergence study (no GPU): the Knudsen
number of (R, eta0), the grid, the error measure, the order selection, and the
committed results."""
import json
import math
import os

import numpy as np
import pytest

from paper_2308_15407_amd import mfr_study as M
from paper_2308_15407_amd import quad_study as Q


def test_kn_for_inverts_the_density_relation():
    """Kn(R, eta0) and the flow-rate study's eta0(R, Kn) are inverse maps of
    Kn = 1/(6 sqrt2 eta0 chi(eta0) R)."""
    for R in Q.R_VALUES:
        for eta0 in Q.ETA_VALUES:
            kn = Q.kn_for(R, eta0)
            old = M.ETA_MAX
            try:
                M.ETA_MAX = 0.45
                assert M.eta0_for(R, kn) == pytest.approx(eta0, rel=1e-12)
            finally:
                M.ETA_MAX = old
    # dilute limit: chi -> 1
    assert Q.kn_for(10.0, 1e-9) * 6 * math.sqrt(2) * 1e-9 * 10 == pytest.approx(1.0, rel=1e-8)


def test_grid_spacing_is_the_stated_fraction_of_sigma():
    from paper_2308_15407_amd import fdlb as F
    for R in Q.R_VALUES:
        c = Q.case("couette", R, 0.1, 8)
        x, jac = F.fdlb_case_grid(c)
        sigma = F.fdlb_case_info(c)["sigma"]
        dx = np.diff(x)
        assert np.allclose(dx, sigma / Q.CELLS_PER_SIGMA, rtol=1e-12)
        assert F.fdlb_case_info(c)["R"] == pytest.approx(R, rel=1e-12)


def test_every_study_case_is_valid():
    from paper_2308_15407_amd import fdlb as F
    for flow in Q.FLOWS:
        for q in (Q.Q_SCAN[0], Q.Q_SCAN[-1], Q.Q_REF):
            info = F.fdlb_case_info(Q.case(flow, 10.0, 0.2, q))
            spec = Q.FLOWS[flow]["case"]
            assert info["K"] == 2 * q * spec["qy"] * spec["qz"]


def test_eps_and_q_min():
    ref = np.array([0.0, 1.0, 2.0, 1.0])
    assert Q.eps(ref + [0, 0.02, 0, 0], ref) == pytest.approx(0.01)
    assert Q.eps(ref - [0.04, 0, 0, 0], ref) == pytest.approx(0.02)   # either sign counts
    qs = [4, 6, 8, 10, 12]
    assert Q.q_min(qs, [0.3, 0.005, 0.02, 0.004, 0.001]) == 10      # a later excursion resets
    assert Q.q_min(qs, [0.3, 0.05, 0.009, 0.004, 0.001]) == 8
    assert Q.q_min(qs, [0.3, 0.05, 0.02, 0.04, 0.011]) is None


def test_committed_results_are_consistent():
    path = Q.DEFAULT_OUT
    if not os.path.exists(path):
        pytest.skip("no committed results")
    res = json.load(open(path))
    assert res["q_ref"] == Q.Q_REF
    for flow, d in res["flows"].items():
        for R, by_eta in d["R"].items():
            for eta0, e in by_eta.items():
                assert e["q_min"] == Q.q_min(e["q"], e["eps"])
                # a settled case has no spread; an averaged one reports its spread
                for ok, sp in zip(e["converged"] + [e["converged_ref"]], e["spread"] + [e["spread_ref"]]):
                    assert (ok and sp == 0.0) or (not ok and 0.0 < sp < Q.EPS_LIMIT), (flow, R, eta0, sp)
                bound = [x + sp + e["spread_ref"] for x, sp in zip(e["eps"], e["spread"])]
                assert e["q_min_bound"] == Q.q_min(e["q"], bound)
                # the error falls by an order of magnitude or more over the scanned orders
                assert e["eps"][-1] < 0.1 * e["eps"][0], (flow, R, eta0)


def test_finer_grid_keeps_the_dense_orders_and_raises_the_rarefied_ones():
    """Poiseuille at 20 cells per sigma against 10: the dense orders stay, the
    rarefied ones grow by at most a few (toward the paper's grid of 100)."""
    fine_path = os.path.join(Q.HERE, "quad_results_poiseuille_cps20.json")
    if not (os.path.exists(fine_path) and os.path.exists(Q.DEFAULT_OUT)):
        pytest.skip("no committed results")
    fine = json.load(open(fine_path))["flows"]["poiseuille"]["R"]
    base = json.load(open(Q.DEFAULT_OUT))["flows"]["poiseuille"]["R"]
    for R, by_eta in fine.items():
        for eta0, e in by_eta.items():
            b = base[R][eta0]
            assert e["q_min"] == Q.q_min(e["q"], e["eps"])
            if float(eta0) >= 0.1:
                assert e["q_min"] == b["q_min"], (R, eta0)
            else:
                assert b["q_min"] <= e["q_min"] <= b["q_min"] + 4, (R, eta0, b["q_min"], e["q_min"])


def test_paper_grid_reproduces_the_rarefied_poiseuille_order():
    """The rarefied narrow Poiseuille cell of Table tab:quad (R = 4, eta0 =
    0.01) on the paper's grid, sigma/100 (Nx = 300): the smallest order with
    eps below 1 % is 29, the paper's value; the same cell needs 22 at 10 and
    24 at 20 cells per sigma, so the grid accounts for the difference."""
    path = os.path.join(Q.HERE, "quad_results_poiseuille_r4_cps100.json")
    if not os.path.exists(path):
        pytest.skip("no committed results")
    res = json.load(open(path))
    assert res["cells_per_sigma"] == 100
    e = res["flows"]["poiseuille"]["R"]["4"]["0.01"]
    assert e["nx"] == Q.nx_for(4.0, 100) == 300
    assert e["converged_ref"] and all(e["converged"])
    assert e["q_min"] == Q.q_min(e["q"], e["eps"]) == 29
    coarse = [json.load(open(p))["flows"]["poiseuille"]["R"]["4"]["0.01"]["q_min"]
              for p in (Q.DEFAULT_OUT, os.path.join(Q.HERE, "quad_results_poiseuille_cps20.json"))]
    assert coarse == [22, 24]


def test_wide_rarefied_poiseuille_order_has_converged_in_the_grid():
    """R = 10, eta0 = 0.01 at 50 cells per sigma (Nx = 450): the order stays
    at 13, as at 20 cells per sigma (12 at 10); the paper lists 15, so here the
    grid does not account for the difference."""
    path = os.path.join(Q.HERE, "quad_results_poiseuille_r10_cps50.json")
    if not os.path.exists(path):
        pytest.skip("no committed results")
    res = json.load(open(path))
    assert res["cells_per_sigma"] == 50
    e = res["flows"]["poiseuille"]["R"]["10"]["0.01"]
    assert e["nx"] == Q.nx_for(10.0, 50) == 450
    assert e["converged_ref"] and all(e["converged"])
    assert e["q_min"] == Q.q_min(e["q"], e["eps"]) == 13
    cps20 = json.load(open(os.path.join(Q.HERE, "quad_results_poiseuille_cps20.json")))
    assert cps20["flows"]["poiseuille"]["R"]["10"]["0.01"]["q_min"] == 13


def test_paper_grid_with_the_revised_contact_value():
    """The same rarefied narrow Poiseuille cell (R = 4, eta0 = 0.01, sigma/100)
    with the revised Enskog contact value (chi_mode 1): the residual stalls,
    so the profiles are window means with a reported spread; the order is 29
    either way (also with eps raised by both spreads), and eps differs from
    the local-chi run by a few per cent at most."""
    path = os.path.join(Q.HERE, "quad_results_poiseuille_r4_cps100_chi1.json")
    if not os.path.exists(path):
        pytest.skip("no committed results")
    res = json.load(open(path))
    assert res["cells_per_sigma"] == 100 and res["flows"]["poiseuille"]["chi_mode"] == 1
    e = res["flows"]["poiseuille"]["R"]["4"]["0.01"]
    assert e["nx"] == 300
    assert e["q_min"] == Q.q_min(e["q"], e["eps"]) == 29
    assert e["q_min_bound"] == 29
    for ok, sp in zip(e["converged"] + [e["converged_ref"]], e["spread"] + [e["spread_ref"]]):
        assert (ok and sp == 0.0) or (not ok and 0.0 < sp < 1e-5)
    local = json.load(open(os.path.join(Q.HERE, "quad_results_poiseuille_r4_cps100.json")))
    e0 = local["flows"]["poiseuille"]["R"]["4"]["0.01"]
    assert e0["q"] == e["q"]
    assert np.allclose(e["eps"], e0["eps"], rtol=0.05)
