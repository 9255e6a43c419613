"""Pins of the oracle's energy straggling (section 3.2's straggling operator (1/2) d^2/dE^2 (T psi),
split into (1/2) d/dE (T dpsi/dE) by the symmetric interior penalty method and (1/2) d/dE (T' psi)
treated like the stopping term; App. A.2's Williams coefficient T(E)).

  * T(E) tends to Bohr's classical value 4 pi r_e^2 (m_e c^2)^2 N_A Z/A at high energy, from above;
  * T'(E) equals a central difference of T(E);
  * the whole energy operator equals an independent assembly of its weak form (DG-P1 on each group,
    upwind flux for the first-order part, SIPG bilinear form for the second-order part), computed
    here by Gauss quadrature from the basis functions;
  * the SIPG part is symmetric and dissipative in the mass inner product, and conserves number;
  * the block-tridiagonal CN step equals a dense LAPACK solve of the same system;
  * through a thin slab the energy variance grows by the integral of rho T (the straggling's
    closed form, corrected to first order for the stopping-power slope), and the mean energy, the
    number and the stopping are left alone.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_00340_amd import inputs as I

# CODATA constants written out here, independently of the oracle
R_E, MEC2, N_A = 2.8179403262e-13, 0.51099895, 6.02214076e23


def _zoa(material):
    if material == 0:
        return (2 * 1.008 / 18.015) * 1 / 1.008 + (15.999 / 18.015) * 8 / 15.999
    if material == 1:   # bone of the paper's material table
        w = [0.042, 0.194, 0.040, 0.425, 0.001, 0.002, 0.092, 0.003, 0.201]
        za = [1 / 1.008, 6 / 12.011, 7 / 14.007, 8 / 15.999, 11 / 22.990, 12 / 24.305, 15 / 30.974, 16 / 32.06,
              20 / 40.078]
        return sum(a * b for a, b in zip(w, za))
    raise ValueError


@pytest.mark.parametrize("material", [0, 1])
def test_williams_tends_to_bohr(material):
    bohr = 4 * np.pi * R_E ** 2 * MEC2 ** 2 * N_A * _zoa(material)
    for E, lo, hi in ((250.0, 1.0, 1.01), (100.0, 1.0, 1.02), (5.0, 1.05, 1.8)):
        r = O.williams(material, E) / bohr
        print(material, E, r)
        assert lo < r < hi, (E, r)
    # the quantum correction shrinks monotonically with the velocity
    e = np.linspace(2.0, 250.0, 60)
    t = np.array([O.williams(material, x) for x in e])
    assert np.all(np.diff(t) < 0)


@pytest.mark.parametrize("material", [0, 1, 2])
def test_williams_derivative(material):
    for E in (3.0, 20.0, 80.0, 150.0, 240.0):
        d = 1e-3 * E
        fd = (O.williams(material, E + d) - O.williams(material, E - d)) / (2 * d)
        assert abs(O.williams_deriv(material, E) - fd) <= 1e-6 * abs(fd), (E, O.williams_deriv(material, E), fd)


def _phys(**kw):
    return dict(dict(I.PHYS, stopping=I.STOP_BETHE, straggling=1), **kw)


def _weak_form_matrix(o, phys, rho):
    """The energy operator of one line assembled from its weak form: rows (group e, test function i) =
    (2i - 1)/dE_e times  int_K phi_i rho [d/dE (c psi) + (1/2) d/dE (T dpsi/dE)] - sigma int_K phi_i psi,
    with c = S + T'/2 and T linear in every group from their face values, the first-order part taken with
    the upwind (upper-group) trace on every face and zero inflow above the top face, the second-order
    part by the symmetric interior penalty form with penalty 2 T_f / h_f on interior faces only.  Volume
    integrals by 6-point Gauss-Legendre; unknowns ordered [psi1_0, psi2_0, psi1_1, ...]."""
    G = o.G
    Ef, dE, Em = o.E_face, o.dE, o.E_mid
    S = np.array([O.stopping(phys, x) for x in Ef])
    T = o.T_face.copy()
    Tp = o.Tp_face.copy()
    c = S + 0.5 * Tp
    xg, wg = np.polynomial.legendre.leggauss(6)

    def phi(i, e, E):          # basis i (0: 1, 1: linear) of group e at energy E, and its derivative
        if i == 0:
            return np.ones_like(E), np.zeros_like(E)
        return 2 * (E - Em[e]) / dE[e], np.full_like(E, 2 / dE[e])

    def trace(e, top):          # values of the two basis functions of group e at its top / bottom face
        return np.array([1.0, 1.0 if top else -1.0])

    A = np.zeros((2 * G, 2 * G))
    for e in range(G):
        E = Em[e] + 0.5 * dE[e] * xg
        w = 0.5 * dE[e] * wg
        lin = lambda f: f[e] + (f[e + 1] - f[e]) * (E - Ef[e]) / dE[e]
        cE, TE = lin(c), lin(T)
        kap = o.kappa[e]
        for i in range(2):
            vi, di = phi(i, e, E)
            for j in range(2):
                vj, dj = phi(j, e, E)
                # - int c psi phi_i' - sigma/rho int psi phi_i - (1/2) int T psi' phi_i'
                A[2 * e + i, 2 * e + j] += np.sum(w * (-cE * vj * di - kap * vj * vi - 0.5 * TE * dj * di))
    # first-order flux through face f: c_f * (trace of the group above f at its bottom)
    for f in range(G + 1):
        up = f if f < G else None
        if up is None:
            continue
        flux = c[f] * trace(up, False)               # coefficients on psi_up
        for e, top in ((f - 1, True), (f, False)):   # groups that have f as top / bottom face
            if e < 0 or e >= G:
                continue
            sgn = 1.0 if top else -1.0
            for i in range(2):
                A[2 * e + i, 2 * up:2 * up + 2] += sgn * trace(e, top)[i] * flux
    # SIPG: -(1/2) [ - {T psi'}[phi] - {T phi'}[psi] + pen [psi][phi] ] on interior faces
    for f in range(1, G):
        lo, hi = f - 1, f
        pen = 2.0 * T[f] / (0.5 * (dE[lo] + dE[hi]))
        jump = np.zeros(2 * G)         # [psi] = psi(lo, top) - psi(hi, bottom) as a row over unknowns
        jump[2 * lo:2 * lo + 2] += trace(lo, True)
        jump[2 * hi:2 * hi + 2] -= trace(hi, False)
        avgd = np.zeros(2 * G)         # {T psi'} = T_f (psi'_lo + psi'_hi)/2
        avgd[2 * lo + 1] += 0.5 * T[f] * 2 / dE[lo]
        avgd[2 * hi + 1] += 0.5 * T[f] * 2 / dE[hi]
        for e, tr in ((lo, trace(lo, True)), (hi, -trace(hi, False))):   # [phi_i] of the test functions
            for i in range(2):
                jphi = tr[i]
                dphi = 0.5 * T[f] * (2 / dE[e] if i == 1 else 0.0)            # {T phi_i'}
                A[2 * e + i] += -0.5 * (-avgd * jphi - dphi * jump + pen * jump * jphi)
    A *= rho
    for e in range(G):
        A[2 * e] *= 1.0 / dE[e]
        A[2 * e + 1] *= 3.0 / dE[e]
    return A


@pytest.mark.parametrize("material,ng,lo,hi", [(0, 9, 0.0, 40.0), (1, 7, 60.0, 110.0)])
def test_operator_equals_weak_form_assembly(material, ng, lo, hi):
    g = I.grid(1, 1, 4, ng, 1, 1, 1.0, 1.0, 0.1, lo, hi, 0.1)
    ph = _phys(material=material)
    o = O.Oracle(g, ph)
    rho = 1.37
    A = _weak_form_matrix(o, ph, rho)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = rng.standard_normal(2 * ng)
        o1, o2 = o.energy_rhs_line(rho, x[0::2], x[1::2])
        ref = A @ x
        got = np.empty(2 * ng)
        got[0::2], got[1::2] = o1, o2
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), np.abs(got - ref).max()
    # without straggling the same assembly with T = 0 is the plain operator
    o0 = O.Oracle(g, dict(ph, straggling=0))
    A0 = _weak_form_matrix(o0, dict(ph, straggling=0), rho)
    x = rng.standard_normal(2 * ng)
    o1, o2 = o0.energy_rhs_line(rho, x[0::2], x[1::2])
    assert np.allclose(np.c_[o1, o2].reshape(-1), A0 @ x, rtol=1e-12, atol=1e-12)


def _operator_matrix(o, rho):
    """The energy operator of one line as a matrix, read off the oracle's line operator applied to unit
    vectors (unknowns ordered [psi1_0, psi2_0, psi1_1, ...])."""
    G = o.G
    D = np.zeros((2 * G, 2 * G))
    for j in range(2 * G):
        x = np.zeros(2 * G)
        x[j] = 1.0
        o1, o2 = o.energy_rhs_line(rho, x[0::2], x[1::2])
        D[0::2, j], D[1::2, j] = o1, o2
    return D


def test_sipg_part_symmetric_dissipative_conservative():
    """With the drift removed (T' = 0 everywhere is the case for a constant T: water above 250 MeV is
    close, so use the difference of two operators that share the drift), M D_T is symmetric and
    negative semi-definite, and its psi1 rows conserve number."""
    g = I.grid(1, 1, 4, 10, 1, 1, 1.0, 1.0, 0.1, 40.0, 90.0, 0.1)
    ph = _phys()
    o = O.Oracle(g, ph)
    G = o.G
    A = _weak_form_matrix(o, ph, 1.0)
    # the same assembly with T set to zero but the drift kept
    o_d = O.Oracle(g, ph)
    o_d.T_face[:] = 0.0
    Ad = _weak_form_matrix(o_d, ph, 1.0)
    DT = A - Ad
    M = np.diag(np.ravel([[d, d / 3] for d in o.dE]))
    MD = M @ DT
    assert np.allclose(MD, MD.T, atol=1e-13 * np.abs(MD).max())
    ev = np.linalg.eigvalsh(0.5 * (MD + MD.T))
    assert ev.max() <= 1e-12 * np.abs(ev).max(), ev.max()
    assert ev.min() < -1e-6 * np.abs(ev).max()      # it does diffuse
    # number: sum_g dE_g psi1_g is not changed by the SIPG part
    assert np.allclose(o.dE @ DT[0::2], 0.0, atol=1e-13 * np.abs(DT).max())


def test_cn_step_equals_dense_solve():
    c = I.small(nx=2, ny=1, nth=4, ng=8, e0=32.0, e_hi=40.0, seed=2)
    ph = _phys()
    o = O.Oracle(c["grid"], ph)
    rho = c["rho"][0].reshape(-1)
    st = I.random_state(o.gen_shape, 5, positive=False)
    Qn = I.random_state((o.G, o.NA, o.NP), 6) * 0.1
    Qs = I.random_state((o.G, o.NA, o.NP), 7) * 0.1
    ref = st.copy()
    h = 0.07
    o.energy_cn(st, rho, h, Qn, Qs)
    G = o.G
    for pq in range(o.NP):
        D = _operator_matrix(o, rho[pq])
        Id = np.eye(2 * G)
        for a in range(o.NA):
            x0 = np.ravel(np.c_[ref[:, 0, a, pq], ref[:, 1, a, pq]])
            q = np.zeros(2 * G)
            q[0::2] = Qn[:, a, pq] + Qs[:, a, pq]
            y = np.linalg.solve(Id - 0.5 * h * D, (Id + 0.5 * h * D) @ x0 + 0.5 * h * q)
            got = np.ravel(np.c_[st[:, 0, a, pq], st[:, 1, a, pq]])
            assert np.allclose(got, y, rtol=1e-11, atol=1e-12 * np.abs(y).max())


def _moments(o, st):
    """Number, mean energy and energy variance of one line of DG-P1 coefficients [G, 2]."""
    p1, p2 = st[:, 0], st[:, 1]
    n = np.sum(o.dE * p1)
    m1 = np.sum(o.dE * (o.E_mid * p1 + o.dE * p2 / 6))
    m2 = np.sum(p1 * (o.dE * o.E_mid ** 2 + o.dE ** 3 / 12) + p2 * o.E_mid * o.dE ** 2 / 3)
    mean = m1 / n
    return n, mean, m2 / n - mean ** 2


def test_energy_variance_grows_by_rho_T_dz():
    """A 150 MeV beam (sigma_E = 1 MeV) through 0.5 cm of water, energy sub-steps only, no nuclear
    removal.  The straggling adds d var / dz = rho T to the variance, which the stopping-power slope S'
    then stretches: to first order Delta var(z) = rho T z (1 - S' rho z) (here S' < 0).  Measured with
    and without straggling on 0.1 MeV groups; the upwind numerical diffusion of the scheme is common to
    both and cancels in the difference.  The mean energy moves by far less than the variance."""
    rho, z, n = 1.0, 0.5, 100
    g = I.grid(1, 1, 4, 300, 1, 1, 2.0, 2.0, 0.1, 130.0, 160.0, z / n)
    out = {}
    for st_on in (0, 1):
        ph = dict(_phys(straggling=st_on), kappa0=0.0)
        o = O.Oracle(g, ph)
        s0 = o.initial(I.beam(150.0))[0]
        for _ in range(n):
            o.energy_cn(s0, np.array([rho]), z / n)
        c = o.NA // 2
        out[st_on] = _moments(o, s0[:, :, c, 0])
        out["o"] = o
    (n0, m0, v0), (n1, m1, v1) = out[0], out[1]
    ph = _phys()
    Em = 0.5 * (150.0 + m1)
    T = O.williams(0, Em)
    d = 0.5
    Sp = (O.stopping(ph, Em + d) - O.stopping(ph, Em - d)) / (2 * d)
    expect = rho * T * z * (1 - Sp * rho * z)
    print("var growth", v1 - v0, "expected", expect, "mean shift", m1 - m0, "number", n0, n1)
    assert abs((v1 - v0) - expect) <= 0.01 * expect
    assert abs(m1 - m0) <= 0.01 * expect
    assert abs(n1 - n0) <= 1e-13 * n0
