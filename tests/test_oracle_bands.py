"""Pins of the oracle's group-dependent nuclear kernel (App. A.4: P1 with the exponential rate lambda and
P2_g with the Gamma-law alpha, beta fitted group by group; here each group takes the parameters of the
nearest of the anchor energies, inputs.NUC_BANDS):

  * one band whose parameters are the single ones gives bitwise the single-parameter tables;
  * every group is assigned the nearest anchor;
  * P1 rows keep the exponential ratio of their source group's band and sum to one;
  * every P2_b equals the Gamma density of the deflection angle (scipy), normalised over destinations;
  * the banded source equals a brute-force quintuple sum of its definition with P2 of the destination
    group's band, and injects exactly the removed number.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2504_00340_amd import inputs as I


def _banded(**kw):
    return dict(I.PHYS, **I.NUC_BANDS, **kw)


def test_one_band_equals_single_parameters():
    c = I.small(nx=2, ny=2, nth=6, ng=9, e_hi=40.0, seed=1)
    o0 = O.Oracle(c["grid"], c["phys"])
    ph1 = dict(c["phys"], nuc_bands=1, nuc_e=[20.0], nuc_lambda=[c["phys"]["lambda_nuc"]],
               nuc_alpha=[c["phys"]["gamma_a"]], nuc_beta=[c["phys"]["gamma_b"]])
    o1 = O.Oracle(c["grid"], ph1)
    assert np.array_equal(o0.P1, o1.P1) and np.array_equal(o0.P2, o1.P2)
    assert np.all(o1.band == 0)


def _grid():
    # groups across all four bands: 40 groups on [0, 240] MeV
    return I.grid(2, 3, 6, 40, 1, 2, 1.0, 1.0, 0.15, 0.0, 240.0, 0.1)


def test_band_of_every_group_is_the_nearest_anchor():
    o = O.Oracle(_grid(), _banded())
    anchors = np.array(I.NUC_BANDS["nuc_e"])
    ref = np.argmin(np.abs(o.E_mid[:, None] - anchors[None, :]), axis=1)
    assert np.array_equal(o.band, ref)
    assert set(o.band) == {0, 1, 2, 3}


def test_banded_energy_transfer_rows():
    o = O.Oracle(_grid(), _banded())
    lam = np.array(I.NUC_BANDS["nuc_lambda"])
    assert np.allclose(o.P1.sum(axis=1), 1.0, rtol=1e-13)
    for gs in range(1, o.G):
        row = o.P1[gs, :gs + 1]
        r = row[1:] / row[:-1]
        assert np.allclose(r, np.exp(lam[o.band[gs]] * np.diff(o.E_mid[:gs + 1])), rtol=1e-12), gs
        assert np.all(o.P1[gs, gs + 1:] == 0)


def test_banded_angular_laws_are_gamma_densities():
    o = O.Oracle(_grid(), _banded())
    th = o.theta()
    U, V = np.meshgrid(th, th, indexing="ij")
    u, v = U.reshape(-1), V.reshape(-1)
    for b in range(4):
        al, be = I.NUC_BANDS["nuc_alpha"][b], I.NUC_BANDS["nuc_beta"][b]
        for s in (0, o.NA // 2, o.NA - 3):
            cosang = (1 + u * u[s] + v * v[s]) / np.sqrt((1 + u * u + v * v) * (1 + u[s] ** 2 + v[s] ** 2))
            ang = np.arccos(np.clip(cosang, -1.0, 1.0))
            f = stats.gamma.pdf(ang, a=al, scale=1.0 / be)
            assert np.allclose(o.P2[b, s], f / f.sum(), rtol=1e-7, atol=1e-12), (b, s)
    assert np.allclose(o.P2.sum(axis=2), 1.0, rtol=1e-13)


def test_banded_source_brute_force_and_number_balance():
    g = I.grid(2, 2, 5, 8, 1, 2, 1.0, 1.0, 0.15, 40.0, 200.0, 0.1)
    o = O.Oracle(g, _banded())
    assert len(set(o.band)) >= 3
    rho = np.array([1.0, 1.4, 0.7, 1.9])
    prev = I.random_state(o.gen_shape, 41)
    Q = o.source(prev, rho)
    inj = (Q * o.dE[:, None, None]).sum(axis=(0, 1))
    rem = rho * (o.kappa[:, None, None] * o.dE[:, None, None] * prev[:, 0]).sum(axis=(0, 1))
    assert np.allclose(inj, rem, rtol=1e-13)
    ref = np.zeros_like(Q)
    for gd in range(o.G):
        P2 = o.P2[o.band[gd]]
        for a in range(o.NA):
            for pq in range(o.NP):
                s = 0.0
                for gs in range(gd, o.G):
                    for ap in range(o.NA):
                        s += o.P1[gs, gd] * P2[ap, a] * o.kappa[gs] * prev[gs, 0, ap, pq] * o.dE[gs] / o.dE[gd]
                ref[gd, a, pq] = rho[pq] * s
    assert np.allclose(Q, ref, rtol=1e-12, atol=1e-15)
