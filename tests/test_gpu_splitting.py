"""The HIP path's higher-order splitting in depth (Richardson-extrapolated Strang steps, pbs_set_splitting
(ctx, 4)) against the oracle's extrapolated march (section 5's extension): ragged grids, the VALU and the
MFMA source products, two and three generations; FP64 <= 1e-12, FP32 dose <= 1e-4.  Chunked stepping is
bitwise one run, and the FP64 march converges at fourth order in depth."""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _solver(c, prec, order=4):
    from paper_2504_00340_amd.pbsplit import Solver

    s = Solver(c["grid"], c["phys"], precision=prec, order=order)
    s.set_phantom(c["rho"])
    s.set_beam(c["beam"])
    return s


CASES = [dict(nx=6, ny=7, nth=6, ng=10, nz=5, ngen=3, seed=31), dict(nx=9, ny=70, nth=8, ng=8, nz=4, ngen=2, seed=32),
         dict(nx=5, ny=6, nth=16, ng=9, nz=4, ngen=3, seed=33)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", CASES, ids=lambda d: "x".join(str(d[k]) for k in ("nx", "ny", "nth", "ng", "ngen")))
def test_extrapolated_march_matches_oracle(case, prec, tol):
    from oracle import oracle as O

    c = I.small(e0=32.0, e_hi=40.0, depth=1.0, **case)
    print("case extrapolated march", prec, case, flush=True)
    dref, fref = O.Oracle(c["grid"], c["phys"]).run(c["beam"], c["rho"], order=4)
    s = _solver(c, prec)
    s.run()
    d, st = s.dose(), s.state()
    s.close()
    print(prec, "dose", _rel(d, dref), "state", _rel(st, fref), flush=True)
    assert _rel(d, dref) <= tol
    assert _rel(st, fref) <= (tol if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_extrapolated_chunks_are_bitwise_one_run(prec):
    c = I.small(e0=32.0, e_hi=40.0, depth=1.0, **CASES[2])
    a = _solver(c, prec)
    a.run()
    b = _solver(c, prec)
    for n in (1, 0, 2, 1):
        b.step(n)
    b.run()
    assert np.array_equal(a.dose(), b.dose()) and np.array_equal(a.state(), b.state())
    a.close()
    b.close()


def test_fourth_order_in_depth_fp64():
    """The integrated fluence after 1.2 cm of water at 50 MeV (the convergence set-up of section 4) with 3,
    6, 12, 24 steps: successive differences fall by about 2^4 (Strang: 2^2)."""
    g0 = I.grid(6, 6, 6, 16, 1, 2, 0.9, 0.9, 0.12, 0.0, 56.0, 1.2)
    out = {}
    for order in (2, 4):
        res = {}
        for nz in (3, 6, 12, 24):
            g = dict(g0, nz=nz, dz=1.2 / nz)
            s = _solver(dict(grid=g, phys=dict(I.PHYS), beam=I.beam(50.0, sigma_x=0.25, sigma_y=0.25),
                             rho=np.ones((nz, 6, 6))), "fp64", order)
            s.run()
            res[nz] = s.state().sum(axis=(2, 4))     # [gen, G, 2]
            s.close()
        e = [np.abs(res[n] - res[2 * n]).sum() for n in (3, 6, 12)]
        out[order] = (e[0] / e[1], e[1] / e[2])
        print("order", order, "errors", e, "ratios", out[order], flush=True)
    assert all(3.0 < r < 5.0 for r in out[2][1:])
    assert all(11.0 < r < 20.0 for r in out[4])
