"""The HIP path against values the paper prints, at a size the CPU oracle does not reach: the
230 MeV row of the table of crucial IDD positions in water (tests/golden/idd_positions_water.txt,
section 4), with the rows the oracle itself is pinned to at 50 and 100 MeV (there the HIP path also
equals the oracle, tests/test_gpu_parity.py).

Same set-up and 2 % tolerance as tests/test_oracle_golden.py: a 34.6 cm march of 865 steps (0.04 cm)
with 1 MeV groups, 4 x 4 lateral cells on +-2 cm and 11 x 11 angular nodes on +-0.3 rad, with either
stopping-power model.  Measured at 230 MeV with the range fit: BP +1.0 %, P90 +1.1 %, D90 +1.0 %, D20
+0.9 % (halving dz and the groups moves them by <= 0.7 %); with the paper's Bethe-Bloch form (App. A.1):
BP -0.18 %, P90 -0.01 %, D90 -0.23 %, D20 -0.34 %.
The lateral sigma of the 230 MeV column is not pinned: with the Highland scattering power used here the
result depends on the angular box (0.64 to 0.76 cm at 32 cm for +-0.1 to +-0.15 rad against 0.757).
"""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I
from test_oracle_golden import _table, idd_positions

pytestmark = pytest.mark.gpu

CASES = [(50, 2.6, 104, 60, 60.0), (100, 8.4, 210, 110, 110.0), (230, 34.6, 865, 240, 240.0)]


@pytest.mark.parametrize("stopping", [I.STOP_BRAGG_KLEEMAN, I.STOP_BETHE], ids=["bragg_kleeman", "bethe"])
@pytest.mark.parametrize("e0,depth,nz,ng,ehi", CASES, ids=["50MeV", "100MeV", "230MeV"])
def test_idd_positions_match_the_paper(e0, depth, nz, ng, ehi, stopping):
    from paper_2504_00340_amd.pbsplit import Solver

    ref = _table()[e0]
    g = I.grid(4, 4, 12, ng, nz, 2, 2.0, 2.0, 0.3, 0.0, ehi, depth)
    print("case", e0, "MeV, stopping model", stopping, flush=True)
    s = Solver(g, dict(I.PHYS, stopping=stopping), "fp32")
    s.set_phantom(I.water(g))
    s.set_beam(I.beam(float(e0)))
    s.run()
    dose = s.dose()
    s.close()
    z = (np.arange(nz) + 0.5) * g["dz"]
    got = idd_positions(z, dose.sum(axis=(1, 2)))
    print(e0, stopping, {k: round(float(v), 3) for k, v in got.items()}, ref, flush=True)
    for key in ("BP", "P90", "D90", "D20"):
        assert abs(got[key] - ref[key]) <= 0.02 * ref[key], (key, got[key], ref[key])
