"""The Poiseuille mass-flow-rate study: its inputs and normalisation (CPU), and
the trends of the committed results (written on the GPU by
`python -m paper_2308_15407_amd.mfr_study run`)."""
import json
import math

import numpy as np
import pytest

from paper_2308_15407_amd import mfr_study as M


def test_eta0_inverts_the_knudsen_definition():
    """Kn = 1/(6 sqrt2 eta0 chi(eta0) R) (Sec. II.A) round trip."""
    for R, kn in ((2.0, 0.3), (5.0, 0.07), (20.0, 0.02), (10.0, 1.2)):
        e = M.eta0_for(R, kn)
        assert e is not None
        assert abs(1.0 / (6 * math.sqrt(2.0) * e * M.chi_cs(e) * R) - kn) < 1e-12 * kn
    assert M.eta0_for(2.0, 0.01) is None          # would need eta0 above the cap


class _FakeSolver:
    """Cell averages of n = 1 + 0.1 x^2 and u_y = c (L^2/4 - x^2) on a
    stretched grid; the flow rate integral has a closed form."""
    def __init__(self, nx=400, Lc=0.8, c=0.3):
        eta_f = np.linspace(-1, 1, nx + 1)
        xf = 0.5 * Lc * np.tanh(1.2 * eta_f) / np.tanh(1.2)
        self.xf, self.nx, self.Lc, self.c = xf, nx, Lc, c

    def grid(self, i):
        xc = 0.5 * (self.xf[1:] + self.xf[:-1])
        jac = np.diff(self.xf) / (2.0 / self.nx)
        return xc, jac

    def moments(self, i):
        a, b = self.xf[:-1], self.xf[1:]
        # exact cell averages of n and of n u_y divided by n (so n u_y averages exactly)
        F_n = lambda x: x + 0.1 * x ** 3 / 3
        h = self.Lc / 2
        F_nu = lambda x: self.c * (h * h * x - x ** 3 / 3 + 0.1 * (h * h * x ** 3 / 3 - x ** 5 / 5))
        n = (F_n(b) - F_n(a)) / (b - a)
        nu = (F_nu(b) - F_nu(a)) / (b - a)
        m = np.zeros((10, self.nx))
        m[0], m[2] = n, nu / n
        return m


def test_mfr_normalisation():
    """m_dot/m_dot0 = int n u_y dx / (a L_c^2) with m_dot0 = n0 a L_c^2 / v_m."""
    s = _FakeSolver()
    h = s.Lc / 2
    exact = s.c * (2 * h ** 3 - 2 * h ** 3 / 3 + 0.1 * (2 * h ** 5 / 3 - 2 * h ** 5 / 5))
    assert abs(M.mfr(s, 0) - exact / (M.AY * s.Lc ** 2)) < 1e-12 * exact / (M.AY * s.Lc ** 2)


def test_committed_results_show_the_knudsen_minimum_only_for_wide_channels():
    """The paper's qualitative statements (the mass flow rate subsection):
    for R > 5 the flow rate has a local maximum in the slip regime and a
    Knudsen minimum; for R <= 5 it only increases with Kn."""
    d = json.load(open(M.DEFAULT_OUT))["R"]
    settled = {}
    for R, v in d.items():
        ok = [i for i, st in enumerate(v["steps"]) if st > 0]
        settled[float(R)] = (np.array(v["kn"])[ok], np.array(v["mfr"])[ok])
    for R in (2.0, 5.0):
        kn, m = settled[R]
        assert np.all(np.diff(m) > 0), R
    for R in (10.0, 20.0):
        kn, m = settled[R]
        imin = int(np.argmin(m[kn > 0.1]))
        assert 0 < imin < int(np.sum(kn > 0.1)) - 1, R      # interior Knudsen minimum
    kn, m = settled[10.0]
    imax = int(np.argmax(m))
    assert 0 < imax and kn[imax] < 0.2                      # slip-regime maximum


def test_committed_order_scan_converges_in_q():
    """The order dependence (the figure's panel (b)): every case settled; at
    moderate Kn all orders agree to 0.5 %, and at the largest Kn the low orders
    deviate while the highest two agree to 1e-3."""
    import os
    path = M.DEFAULT_QSCAN_OUT
    if not os.path.exists(path):
        pytest.skip("no committed order scan")
    res = json.load(open(path))
    qs = sorted(res["Q"], key=int)
    ref = res["Q"][qs[-1]]
    for q in qs:
        d = res["Q"][q]
        assert d["kn"] == ref["kn"]
        assert all(s > 0 for s in d["steps"]), q
        for kn, m, mr in zip(d["kn"], d["mfr"], ref["mfr"]):
            if kn <= 1.0:
                assert abs(m - mr) < 5e-3 * mr, (q, kn, m, mr)
    last = [res["Q"][q]["mfr"][-1] for q in qs]
    assert abs(last[-1] - last[-2]) < 1e-3 * last[-1]
    assert abs(last[0] - last[-1]) > 10 * abs(last[-2] - last[-1])


def test_reduced_form_flow_rates_agree_with_the_lattice():
    """The same cases (Q_x^h = 16 below Kn = 0.5, 32 above) solved in the
    paper's reduced 2D form and on the 3D lattice: two discretisations of one
    model that differ only through the nonlinear WENO weights.  Settled flow
    rates agree to 1e-5 in the rarefied cases, to 3e-4 below eta0 = 0.1 and to
    5e-3 in the dense cases, where the layered density makes the weights
    matter most."""
    import os
    if not (os.path.exists(M.DEFAULT_REDUCED_OUT) and os.path.exists(M.DEFAULT_OUT)):
        pytest.skip("no committed results")
    red = json.load(open(M.DEFAULT_REDUCED_OUT))
    lat = json.load(open(M.DEFAULT_OUT))
    n = 0
    for R, d in red["R"].items():
        d3 = lat["R"][R]
        for kn, eta0, m, st in zip(d["kn"], d["eta0"], d["mfr"], d["steps"]):
            i = d3["kn"].index(kn)
            if st <= 0 or d3["steps"][i] <= 0:
                continue
            rel = abs(m - d3["mfr"][i]) / d3["mfr"][i]
            assert rel < (1e-5 if kn >= 0.5 else 3e-4 if eta0 < 0.1 else 5e-3), (R, kn, eta0, rel)
            n += 1
    assert n >= 32
