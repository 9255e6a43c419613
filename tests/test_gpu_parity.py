"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sub-steps on ragged grids (lateral tiles partly filled, ny > 64 so the row sweep spans two
segments, several generations), the full march on configuration 1, chunked stepping, and
error behaviour.  FP64 instantiation: <= 1e-12 relative; FP32: <= 1e-5 (sub-steps, as rel-L2 and
as max |got - ref| <= tol * max |ref_k| per generation) and dose rel-L2 <= 1e-4 (march), the tolerance
stated for the FP32 path.
"""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I

pytestmark = pytest.mark.gpu


def _solver(c, prec):
    from paper_2504_00340_amd.pbsplit import Solver

    s = Solver(c["grid"], c["phys"], precision=prec)
    s.set_phantom(c["rho"])
    s.set_beam(c["beam"])
    return s


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


TOL = {"fp64": 1e-12, "fp32": 1e-5}
RAGGED = [dict(nx=6, ny=5, nth=6, ng=7, ngen=3, seed=1),
          dict(nx=9, ny=70, nth=8, ng=5, ngen=2, seed=2),
          dict(nx=33, ny=31, nth=4, ng=9, ngen=1, seed=3),
          # source product on the MFMA path (>= 128 angular unknowns), partial lateral tiles
          dict(nx=5, ny=7, nth=16, ng=4, ngen=3, seed=4),
          dict(nx=4, ny=9, nth=32, ng=3, ngen=2, seed=5),
          # row-affine transport sweeps (ny = 64 / 32, nx a multiple of 8)
          dict(nx=16, ny=64, nth=6, ng=3, ngen=2, seed=6),
          dict(nx=8, ny=32, nth=16, ng=3, ngen=2, seed=7),
          # two-segment row-affine sweeps (ny = 96 / 128, nx a multiple of 8); at ny = 96 two planes per wave,
          # with odd angle counts (pairs straddle slabs and mirrorings) and nx a multiple of 4 only
          dict(nx=8, ny=96, nth=6, ng=3, ngen=2, seed=8),
          dict(nx=16, ny=128, nth=4, ng=2, ngen=2, seed=9),
          dict(nx=12, ny=96, nth=16, ng=2, ngen=1, seed=10),
          dict(nx=4, ny=96, nth=4, ng=3, ngen=2, seed=11)]


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", RAGGED, ids=lambda d: "x".join(str(d[k]) for k in ("nx", "ny", "nth", "ng", "ngen")))
def test_substeps_match_oracle(O, prec, shape):
    c = I.small(nz=3, **shape)
    print("case", prec, shape, flush=True)
    o = O.Oracle(c["grid"], c["phys"])
    s = _solver(c, prec)
    st = I.random_state(s.state_shape, 100 + shape["seed"])
    # make the psi^2 coefficients O(0.3) of psi^1 as in the physical states
    st[:, :, 1] *= 0.3
    vol = o.dx * o.dy * c["grid"]["dz"]
    for op, h in (("T", 0.037), ("A", 0.061), ("E", 0.045)):
        s.set_state(st)
        ref = st.copy()
        rho = np.ascontiguousarray(c["rho"][1].reshape(-1))
        if op == "T":
            s.apply(2, 1, h)
            for k in range(ref.shape[0]):
                o.transport_cn(ref[k], h)
        elif op == "A":
            s.apply(3, 1, h)
            for k in range(ref.shape[0]):
                o.angular_cn(ref[k], rho, h)
        else:
            s.set_beam(c["beam"])   # zero the dose
            s.set_state(st)
            s.apply(1, 1, h)
            dep = o.energy_all(ref, rho, h)
            dose = s.dose()
            assert _rel(dose[1].reshape(-1), dep / (rho * vol)) < TOL[prec], op
            assert np.all(dose[0] == 0) and np.all(dose[2] == 0)
        got = s.state()
        assert _rel(got, ref) < TOL[prec], (op, _rel(got, ref))
        # element by element, per generation: a wrong boundary lane, sweep seam or padded tile shows here
        for k in range(ref.shape[0]):
            d = np.abs(got[k] - ref[k])
            i = int(np.argmax(d))
            e = float(d.flat[i] / max(np.abs(ref[k]).max(), 1e-300))
            assert e <= TOL[prec], (op, k, e, np.unravel_index(i, ref[k].shape))
    s.close()


@pytest.fixture(scope="module")
def c1_ref(O):
    c = I.config1()
    o = O.Oracle(c["grid"], c["phys"])
    dose, fin = o.run(c["beam"], c["rho"])
    return c, dose, fin


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_config1_march_matches_oracle(c1_ref, prec, tol):
    c, dose_ref, fin_ref = c1_ref
    s = _solver(c, prec)
    s.run()
    dose = s.dose()
    print(prec, "dose rel-L2", _rel(dose, dose_ref), "state", _rel(s.state(), fin_ref), flush=True)
    assert _rel(dose, dose_ref) < tol
    assert _rel(s.state(), fin_ref) < (tol if prec == "fp64" else 1e-3)
    s.close()


def test_ragged_march_fp64(O):
    c = I.small(nx=9, ny=70, nth=6, ng=10, nz=6, ngen=3, e0=32.0, e_hi=40.0, depth=1.5, seed=4)
    o = O.Oracle(c["grid"], c["phys"])
    dref, fref = o.run(c["beam"], c["rho"])
    s = _solver(c, "fp64")
    s.run()
    assert _rel(s.dose(), dref) < 1e-12
    assert _rel(s.state(), fref) < 1e-12
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_march_with_mfma_source_product(O, prec, tol):
    c = I.small(nx=6, ny=7, nth=16, ng=10, nz=5, ngen=3, e0=32.0, e_hi=40.0, depth=1.2, seed=6)
    o = O.Oracle(c["grid"], c["phys"])
    dref, fref = o.run(c["beam"], c["rho"])
    s = _solver(c, prec)
    s.run()
    print(prec, _rel(s.dose(), dref), _rel(s.state(), fref), flush=True)
    assert _rel(s.dose(), dref) < tol
    assert _rel(s.state(), fref) < 10 * tol
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_schedules_are_bitwise_equal(prec):
    """The two-stream march (each generation's T A T beside the energy chain) gives bitwise the one-stream
    march, chunked or not, on the MFMA source-product path with three generations."""
    from paper_2504_00340_amd.pbsplit import PBS_SCHED_ONE_STREAM, PBS_SCHED_TWO_STREAMS

    c = I.small(nx=6, ny=7, nth=16, ng=10, nz=5, ngen=3, e0=32.0, e_hi=40.0, depth=1.2, seed=6)
    out = []
    for mode, chunks in ((PBS_SCHED_ONE_STREAM, (5,)), (PBS_SCHED_TWO_STREAMS, (5,)), (PBS_SCHED_TWO_STREAMS, (2, 0, 3))):
        s = _solver(c, prec)
        s.set_schedule(mode)
        for n in chunks:
            s.step(n)
        s.run()
        out.append((s.dose(), s.state()))
        s.close()
    for d, st in out[1:]:
        assert np.array_equal(d, out[0][0])
        assert np.array_equal(st, out[0][1])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_chunked_stepping_is_bitwise_equal(prec):
    c = I.config1()
    a = _solver(c, prec)
    a.run()
    b = _solver(c, prec)
    for n in (1, 7, 30, 0, 22):
        b.step(n)
    b.run()
    assert np.array_equal(a.dose(), b.dose())
    assert np.array_equal(a.state(), b.state())
    # deterministic run to run
    a.set_beam(c["beam"])
    a.run()
    assert np.array_equal(a.dose(), b.dose())
    a.close()
    b.close()


def test_error_paths():
    from paper_2504_00340_amd.pbsplit import PbsError, PBS_EINVAL, PBS_ESTATE

    c = I.config1()
    s = _solver(c, "fp32")
    with pytest.raises(PbsError) as e:
        s.step(-1)
    assert e.value.code == PBS_EINVAL
    with pytest.raises(PbsError) as e:
        s.step(c["grid"]["nz"] + 1)
    assert e.value.code == PBS_EINVAL
    bad = c["rho"].copy()
    bad[3, 2, 1] = np.nan
    with pytest.raises(PbsError):
        s.set_phantom(bad)
    bad[3, 2, 1] = -1.0
    with pytest.raises(PbsError):
        s.set_phantom(bad)
    with pytest.raises(PbsError):
        s.set_phantom(c["rho"][:-1])
    s.run()
    with pytest.raises(PbsError) as e:
        s.step(1)
    assert e.value.code == PBS_ESTATE
    with pytest.raises(PbsError):
        s.apply(9, 0, 0.1)
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_bethe_stopping_march_matches_oracle(O, prec, tol):
    """The Bethe-Bloch stopping power of App. A.1 (host tables of the library against the oracle's own);
    the model switch must change the result (here by about 3 % of the dose)."""
    c = I.small(nx=6, ny=7, nth=16, ng=10, nz=5, ngen=3, e0=32.0, e_hi=40.0, depth=1.2, seed=6)
    c["phys"] = dict(c["phys"], stopping=I.STOP_BETHE)
    print("case", prec, "Bethe-Bloch stopping", flush=True)
    dref, fref = O.Oracle(c["grid"], c["phys"]).run(c["beam"], c["rho"])
    dbk, _ = O.Oracle(c["grid"], dict(c["phys"], stopping=I.STOP_BRAGG_KLEEMAN)).run(c["beam"], c["rho"])
    assert _rel(dbk, dref) > 1e-3
    s = _solver(c, prec)
    s.run()
    print(prec, _rel(s.dose(), dref), _rel(s.state(), fref), flush=True)
    assert _rel(s.dose(), dref) < tol
    assert _rel(s.state(), fref) < 10 * tol
    s.close()


def test_voxel_phantom_entry_equals_resampled_densities():
    """pbs_set_phantom_voxels (nearest-voxel resampling in the library) gives bitwise the march of
    pbs_set_phantom with the densities of the batched plan's own sampling of its shared phantom."""
    from paper_2504_00340_amd.pbsplit import Solver

    cfg = I.config4(seed=0, nbeams=2)
    b = cfg["beams"][1]
    g = dict(b["grid"], nz=40, ng=24, dz=b["grid"]["dz"])
    out = []
    for mode in ("voxels", "direct"):
        s = Solver(g, cfg["phys"], precision="fp32")
        if mode == "voxels":
            s.set_phantom_voxels(cfg["phantom"], (0.0875, 0.1, 0.1), (-6.4 - b["spot"][0], -6.4 - b["spot"][1]))
        else:
            s.set_phantom(b["rho"][:40])
        s.set_beam(b["beam"])
        s.run()
        out.append(s.dose())
        s.close()
    assert np.array_equal(out[0], out[1])
