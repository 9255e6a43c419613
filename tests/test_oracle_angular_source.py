"""Pins of the oracle's angular diffusion step (section 3.4, eq:(sd), eq:(eqn_fly)) and of
the catastrophic source (Remark after the Strang scheme; App. A.4).

Angular: the sine-transform CN step equals a dense LAPACK solve with the
textbook 5-point Laplacian; the second angular moment grows by exactly
2 D h M0 per axis (the Fermi-Eyges angular variance of the discrete step).
Source: removed number equals injected number; a brute-force quintuple sum of
the definition; energy transfer ratio of the exponential law.
"""
import numpy as np
import pytest


def _lap5(m, d):
    T = (np.diag(-2.0 * np.ones(m)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)) / d ** 2
    I = np.eye(m)
    return np.kron(T, I) + np.kron(I, T)


@pytest.mark.parametrize("nth", [4, 7, 8])
def test_angular_cn_equals_dense_solve(oracle_mod, inputs, nth):
    c = inputs.small(nx=3, ny=2, nth=nth, ng=4, seed=3)
    o = oracle_mod.Oracle(c["grid"], c["phys"])
    rho = c["rho"][0].reshape(-1)
    st = inputs.random_state(o.gen_shape, 21, positive=False)
    ref = st.copy()
    h = 0.3
    o.angular_cn(st, rho, h)
    L = _lap5(o.m, o.dth)
    for g in range(o.G):
        for pq in range(o.NP):
            D = rho[pq] * o.sig_tr[g] / 2.0
            Aop = D * L
            I = np.eye(o.NA)
            for l in range(2):
                y = np.linalg.solve(I - 0.5 * h * Aop, (I + 0.5 * h * Aop) @ ref[g, l, :, pq])
                assert np.allclose(st[g, l, :, pq], y, rtol=1e-11, atol=1e-12 * abs(y).max())


def test_angular_second_moment_identity(oracle_mod, inputs):
    g = inputs.grid(1, 1, 40, 3, 1, 1, 1.0, 1.0, 0.4, 60.0, 120.0, 1.0)
    o = oracle_mod.Oracle(g, inputs.PHYS)
    th = o.theta()
    U, V = np.meshgrid(th, th, indexing="ij")
    s0 = 0.03
    plane = np.exp(-(U ** 2 + V ** 2) / (2 * s0 ** 2)).reshape(-1)
    st = np.zeros(o.gen_shape)
    st[:, 0, :, 0] = plane
    st[:, 1, :, 0] = 0.5 * plane
    rho = np.array([1.1])
    h = 1.0
    m0 = plane.sum()
    m2u = (plane * U.reshape(-1) ** 2).sum()
    o.angular_cn(st, rho, h)
    for g in range(o.G):
        D = rho[0] * o.sig_tr[g] / 2
        out = st[g, 0, :, 0]
        assert abs(out.sum() - m0) < 1e-12 * m0
        assert abs((out * U.reshape(-1) ** 2).sum() - (m2u + 2 * D * h * m0)) < 1e-11 * m2u
        assert abs((out * V.reshape(-1) ** 2).sum() - (m2u + 2 * D * h * m0)) < 1e-11 * m2u


def test_source_number_balance_and_brute_force(oracle_mod, inputs):
    c = inputs.small(nx=2, ny=3, nth=5, ng=6, seed=5)
    o = oracle_mod.Oracle(c["grid"], c["phys"])
    rho = c["rho"][0].reshape(-1)
    prev = inputs.random_state(o.gen_shape, 31)
    Q = o.source(prev, rho)
    # injected number = removed number, per voxel
    inj = (Q * o.dE[:, None, None]).sum(axis=(0, 1))
    rem = rho * (o.kappa[:, None, None] * o.dE[:, None, None] * prev[:, 0]).sum(axis=(0, 1))
    assert np.allclose(inj, rem, rtol=1e-13)
    # brute-force sum of the definition
    ref = np.zeros_like(Q)
    for g in range(o.G):
        for a in range(o.NA):
            for pq in range(o.NP):
                s = 0.0
                for gs in range(g, o.G):
                    for ap in range(o.NA):
                        s += o.P1[gs, g] * o.P2[ap, a] * o.kappa[gs] * prev[gs, 0, ap, pq] * o.dE[gs] / o.dE[g]
                ref[g, a, pq] = rho[pq] * s
    assert np.allclose(Q, ref, rtol=1e-12, atol=1e-15)


def test_source_energy_shape(oracle_mod, inputs):
    """A source line in one group g' feeds group g with weight exp(-lambda (E_g' - E_g))."""
    c = inputs.small(nx=1, ny=1, nth=4, ng=8, e_hi=40)
    o = oracle_mod.Oracle(c["grid"], c["phys"])
    prev = np.zeros(o.gen_shape)
    gs = 6
    prev[gs, 0, :, 0] = 1.0
    Q = o.source(prev, np.ones(1))
    per_g = (Q[:, :, 0] * o.dE[:, None]).sum(1)
    lam = c["phys"]["lambda_nuc"]
    assert np.all(per_g[gs + 1:] == 0)
    assert np.allclose(per_g[1:gs + 1] / per_g[:gs], np.exp(lam * np.diff(o.E_mid)[:gs]), rtol=1e-12)
