"""pbs_bind_static: the allocation-free binding (the library's own per-GPU scratch array instead of a
caller workspace) gives bitwise the same march as pbs_bind, on two bindings in a row (the second one a
smaller grid), invalidates the context bound before it, and refuses a grid whose workspace exceeds the
scratch."""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(c, prec, static):
    from paper_2504_00340_amd.pbsplit import Solver

    s = Solver(c["grid"], c["phys"], precision=prec, static_scratch=static)
    s.set_phantom(c["rho"])
    s.set_beam(c["beam"])
    s.step(3)
    s.run()
    return s, s.dose(), s.state()


def test_static_scratch_matches_workspace_binding():
    from oracle import oracle as O
    from paper_2504_00340_amd.pbsplit import PBS_EINVAL, PBS_ESTATE, PBS_STATIC_SCRATCH_BYTES, PbsError, Solver

    big = I.config1()
    small = I.small(nx=10, ny=9, nth=8, ng=12, nz=6, ngen=2, e0=30.0, e_hi=40.0, depth=1.2, seed=5)
    print("case no-alloc: config 1 (16x16, 8x8 angles, 48 groups, 80 steps) fp32, then ragged 10x9 fp64",
          flush=True)
    # first binding: config 1 in FP32
    wa, da, sa = _run(big, "fp32", False)
    wa.close()
    sb, db, stb = _run(big, "fp32", True)
    assert sb.ws_bytes <= PBS_STATIC_SCRATCH_BYTES
    assert np.array_equal(db, da) and np.array_equal(stb, sa)
    # second binding, a smaller grid in FP64: the scratch keeps the first call's contents
    wc, dc, sc = _run(small, "fp64", False)
    wc.close()
    sd, dd, std_ = _run(small, "fp64", True)
    assert np.array_equal(dd, dc) and np.array_equal(std_, sc)
    ref, _ = O.Oracle(small["grid"], small["phys"]).run(small["beam"], small["rho"])
    err = float(np.linalg.norm(dd - ref) / np.linalg.norm(ref))
    print(f"no-alloc fp64 ragged: dose rel-L2 vs oracle {err:.2e}", flush=True)
    assert err < 1e-12
    # the first static context lost the scratch to the second
    with pytest.raises(PbsError) as e:
        sb.dose()
    assert e.value.code == PBS_ESTATE
    sb.close()
    # the second one still works: a new beam on it is again bitwise the workspace result
    sd.set_beam(small["beam"])
    sd.run()
    assert np.array_equal(sd.dose(), dc)
    sd.close()
    # a workspace beyond the scratch is refused with the sizes in the message
    c5 = I.config5(100000)
    with pytest.raises(PbsError) as e:
        Solver(c5["grid"], c5["phys"], precision="fp32", static_scratch=True)
    assert e.value.code == PBS_EINVAL and "exceeds the static scratch" in str(e.value)
