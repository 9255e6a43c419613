"""Pins of the oracle's energy sub-problem (DG-P1 in energy, section 3.2; CN, section 3.3).

* exactness of the semi-discrete operator on globally linear fluence with a
  linear stopping power, against scipy quadrature of the exact derivative
  (this pins both rows, including the sign of the lower-face term of the
  psi^2 row);
* the group-by-group CN solve against a dense LAPACK solve of the same system;
* number balance of one CN step (bottom outflow and removal only);
* the CSDA closed form of the Bragg-Kleeman law for the mean energy, with
  second-order convergence in the group width.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def _orc(oracle_mod, inputs, **kw):
    c = inputs.small(**kw)
    return c, oracle_mod.Oracle(c["grid"], c["phys"])


@pytest.mark.parametrize("kappa0", [0.0, 0.02])
def test_operator_exact_on_linear_fluence(oracle_mod, inputs, kappa0):
    c, o = _orc(oracle_mod, inputs, ng=9, e_hi=45.0)
    o.ph["kappa0"] = kappa0
    o.kappa[:] = 0.0 if kappa0 == 0 else o.kappa * (kappa0 / inputs.PHYS["kappa0"])
    s0, s1 = 3.0, -0.04            # linear S(E) = s0 + s1 E (positive on [0,45])
    a0, b0 = 2.0, 0.3              # psi(E) = a0 + b0 E
    o.S_face[:] = s0 + s1 * o.E_face
    x1 = a0 + b0 * o.E_mid
    x2 = b0 * o.dE / 2.0
    rho = 1.3
    r1, r2 = o.energy_rhs_line(rho, x1, x2)
    dflux = lambda e: rho * (s1 * (a0 + b0 * e) + (s0 + s1 * e) * b0)   # d/dE (rho S psi)
    for g in range(o.G - 1):      # the top group has no inflow from above
        lo, hi, d, Em = o.E_face[g], o.E_face[g + 1], o.dE[g], o.E_mid[g]
        m1 = integrate.quad(dflux, lo, hi)[0] / d
        m2 = 3.0 / d * integrate.quad(lambda e: dflux(e) * 2.0 * (e - Em) / d, lo, hi)[0]
        sct = rho * o.kappa[g]
        assert r1[g] == pytest.approx(m1 - sct * x1[g], rel=1e-12, abs=1e-12)
        assert r2[g] == pytest.approx(m2 - sct * x2[g], rel=1e-12, abs=1e-12)


def test_constant_fluence_constant_stopping_is_steady(oracle_mod, inputs):
    c, o = _orc(oracle_mod, inputs, ng=8)
    o.kappa[:] = 0
    o.S_face[:] = 5.0
    r1, r2 = o.energy_rhs_line(1.0, np.full(o.G, 4.0), np.zeros(o.G))
    assert np.allclose(r1[:-1], 0, atol=1e-13) and np.allclose(r2[:-1], 0, atol=1e-13)


def _dense_operator(o, rho):
    G = o.G
    A = np.zeros((2 * G, 2 * G))
    for col in range(2 * G):
        e = np.zeros(2 * G)
        e[col] = 1.0
        r1, r2 = o.energy_rhs_line(rho, e[:G], e[G:])
        A[:G, col], A[G:, col] = r1, r2
    return A


@pytest.mark.parametrize("with_source", [False, True])
def test_cn_step_equals_dense_solve(oracle_mod, inputs, with_source):
    c, o = _orc(oracle_mod, inputs, nx=3, ny=2, nth=4, ng=7, seed=1)
    rho = c["rho"][0].reshape(-1)
    st = inputs.random_state(o.gen_shape, 11, positive=False)
    Qn = Qs = None
    if with_source:
        Qn = inputs.random_state((o.G, o.NA, o.NP), 12)
        Qs = inputs.random_state((o.G, o.NA, o.NP), 13)
    h = 0.07
    ref = st.copy()
    o.energy_cn(st, rho, h, Qn, Qs)
    for a in range(o.NA):
        for pq in range(o.NP):
            A = _dense_operator(o, rho[pq])
            x = np.concatenate([ref[:, 0, a, pq], ref[:, 1, a, pq]])
            b = (np.eye(2 * o.G) + 0.5 * h * A) @ x
            if with_source:
                b[:o.G] += 0.5 * h * (Qn[:, a, pq] + Qs[:, a, pq])
            y = np.linalg.solve(np.eye(2 * o.G) - 0.5 * h * A, b)
            got = np.concatenate([st[:, 0, a, pq], st[:, 1, a, pq]])
            assert np.allclose(got, y, rtol=1e-12, atol=1e-12 * abs(y).max())


def test_cn_number_balance(oracle_mod, inputs):
    """sum_g dE psi1 changes only by the bottom-face outflow rho S_1/2 (psi1_1 - psi2_1) and removal."""
    c, o = _orc(oracle_mod, inputs, nx=2, ny=2, nth=4, ng=10, seed=2)
    rho = c["rho"][0].reshape(-1)
    st = inputs.random_state(o.gen_shape, 5)
    h = 0.05
    n0 = (st[:, 0] * o.dE[:, None, None]).sum(0)
    out0 = rho * o.S_face[0] * (st[0, 0] - st[0, 1])
    rem0 = rho * (o.kappa[:, None, None] * o.dE[:, None, None] * st[:, 0]).sum(0)
    o.energy_cn(st, rho, h)
    n1 = (st[:, 0] * o.dE[:, None, None]).sum(0)
    out1 = rho * o.S_face[0] * (st[0, 0] - st[0, 1])
    rem1 = rho * (o.kappa[:, None, None] * o.dE[:, None, None] * st[:, 0]).sum(0)
    assert np.allclose(n1 - n0, -0.5 * h * (out0 + out1 + rem0 + rem1), rtol=1e-12, atol=1e-13)


def _csda_mean_energy(ph, e0, sig, z):
    """Mean energy at depth z of protons with a Gaussian initial energy, each following
    R(E(z)) = R(E_i) - z (Bragg-Kleeman), over the protons not yet stopped."""
    al, p = ph["bk_alpha"], ph["bk_p"]
    pdf = lambda e: math.exp(-0.5 * ((e - e0) / sig) ** 2)
    Ez = lambda e: ((al * e ** p - z) / al) ** (1 / p)
    emin = (z / al) ** (1 / p)
    lo, hi = max(emin, e0 - 8 * sig), e0 + 8 * sig
    num = integrate.quad(lambda e: pdf(e) * Ez(e), lo, hi, epsabs=0, epsrel=1e-12)[0]
    den = integrate.quad(pdf, lo, hi, epsabs=0, epsrel=1e-12)[0]
    return num / den


def test_csda_mean_energy_second_order_in_group_width(oracle_mod, inputs):
    """kappa = 0: the fluence-weighted mean energy follows the Bragg-Kleeman closed form;
    the error falls ~4x per halving of dE (the paper's second order in energy)."""
    ph = dict(inputs.PHYS)
    ph["kappa0"] = 0.0
    e0, depth, nz = 60.0, 1.5, 60
    exact = _csda_mean_energy(ph, e0, 1.0, depth)
    errs = []
    for G in (40, 80, 160):
        g = inputs.grid(1, 1, 4, G, nz, 1, 1.0, 1.0, 0.1, 0.0, 80.0, depth)
        o = oracle_mod.Oracle(g, ph)
        st = o.initial(inputs.beam(e0))[0]
        rho = np.ones(1)
        h = depth / nz
        for _ in range(2 * nz):
            o.energy_cn(st, rho, h / 2)
        n = o.number_content(st).sum()
        e = o.energy_content(st).sum()
        errs.append(abs(e / n - exact))
    assert errs[-1] < 2e-3 * exact
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 3.0 and r2 > 3.0, (errs, r1, r2)


def test_range_of_monoenergetic_beam(oracle_mod, inputs):
    """Number-fluence 50 % depth -> Bragg-Kleeman range R0 = alpha E0^p (kappa = 0)."""
    ph = dict(inputs.PHYS)
    ph["kappa0"] = 0.0
    e0 = 50.0
    R0 = ph["bk_alpha"] * e0 ** ph["bk_p"]
    nz = 300
    depth = 1.2 * R0
    g = inputs.grid(1, 1, 4, 200, nz, 1, 1.0, 1.0, 0.1, 0.0, 60.0, depth)
    o = oracle_mod.Oracle(g, ph)
    st = o.initial(inputs.beam(e0, sigma_e=0.3))[0]
    h = depth / nz
    prev, z50 = 1.0, None
    for s in range(nz):
        o.energy_cn(st, np.ones(1), h / 2)
        o.energy_cn(st, np.ones(1), h / 2)
        n = o.number_content(st).sum()
        if prev >= 0.5 > n:
            z50 = (s + (prev - 0.5) / (prev - n)) * h
            break
        prev = n
    assert z50 is not None and abs(z50 - R0) < 0.01 * R0, (z50, R0)
