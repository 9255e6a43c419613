"""The oracle with the paper's own physics of App. A.1-A.3 -- Bethe-Bloch stopping power summed over the
elements of the medium, Williams straggling, screened-Rutherford momentum-transfer cross section -- against
what the paper prints for water and bone (section 4's material table: bone of density 1.757 with its
composition):

  * the screened-Rutherford sigma_tr of water lies near the Highland scattering power (an independent
    multiple-scattering model) over the therapeutic range;
  * the characteristic positions of the integrated depth dose in bone (tests/golden/idd_positions_bone.txt)
    and water (tests/golden/idd_positions_water.txt) at 50 and 100 MeV, within 2 % / 1.5 %;
  * the lateral sigma of the dose in bone (tests/golden/lateral_sigma_bone.txt) and water
    (tests/golden/lateral_sigma_water.txt) within 2.5 %, and at 100 MeV its growth sigma^2 - sigma_0^2 at
    the depth near the peak within 15 % (the Highland form with water's radiation length misses the bone
    value by about 40 %).
The air table is not pinned: the Fokker-Planck step with the full momentum-transfer cross section spreads
a pencil beam in 40 cm of air about 2.4 times more (in sigma^2 - sigma_0^2) than the paper prints.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2504_00340_amd import inputs as I
from test_oracle_golden import idd_positions

HERE = os.path.dirname(__file__)


def _idd_table(name):
    rows = {}
    for line in open(os.path.join(HERE, "golden", name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        v = [float(x) for x in f[2:]]
        rows[int(f[1])] = dict(BP=v[1], P90=v[3], D90=v[5], D20=v[7])
    return rows


def _sigma_table(name):
    rows = {}
    for line in open(os.path.join(HERE, "golden", name)):
        if line.startswith("#") or not line.strip():
            continue
        e0, z, _, d = line.split()
        rows.setdefault(int(e0), []).append((float(z), float(d)))
    return rows


def test_rutherford_close_to_highland_in_water():
    for E in (20.0, 50.0, 100.0, 150.0, 230.0):
        r = O.rutherford(0, E) / O.scatpower(I.PHYS, E)
        print(E, r)
        assert 1.0 < r < 1.2, (E, r)


# (medium, density, E0, depth, steps, groups, upper energy): about 0.026 g/cm^2 per step, 1 MeV groups
IDD_CASES = [(I.MAT_BONE, 1.757, 50, 1.6, 107, 60, 60.0), (I.MAT_BONE, 1.757, 100, 5.2, 208, 110, 110.0),
             (I.MAT_WATER, 1.0, 50, 2.6, 104, 60, 60.0), (I.MAT_WATER, 1.0, 100, 8.4, 210, 110, 110.0)]


@pytest.mark.parametrize("mat,rho,e0,depth,nz,ng,ehi", IDD_CASES,
                         ids=["bone-50MeV", "bone-100MeV", "water-50MeV", "water-100MeV"])
def test_idd_positions_with_the_papers_physics(mat, rho, e0, depth, nz, ng, ehi):
    """Measured: bone within +0.1 % .. +1.8 % (D20 at 100 MeV), water within -1.4 % .. +0.3 %."""
    ref = _idd_table("idd_positions_bone.txt" if mat == I.MAT_BONE else "idd_positions_water.txt")[e0]
    g = I.grid(4, 4, 12, ng, nz, 2, 2.0, 2.0, 0.3, 0.0, ehi, depth)
    dose, _ = Oracle(g, I.paper_physics(mat)).run(I.beam(float(e0)), np.full((nz, 4, 4), rho))
    got = idd_positions((np.arange(nz) + 0.5) * g["dz"], dose.sum(axis=(1, 2)))
    print(mat, e0, {k: round(v, 3) for k, v in got.items()}, ref)
    tol = 0.02 if mat == I.MAT_BONE else 0.015
    for key in ("BP", "P90", "D90", "D20"):
        assert abs(got[key] - ref[key]) <= tol * ref[key], (key, got[key], ref[key])


# (medium, density, E0, depth, steps, groups, upper energy); 40 cells of 0.1 cm across x, one across y,
# 10 x 10 angular nodes on +-0.3 rad, as for the water table with the Highland form
SIGMA_CASES = [(I.MAT_BONE, 1.757, 50, 1.4, 93, 60, 60.0), (I.MAT_BONE, 1.757, 100, 4.8, 96, 55, 110.0),
               (I.MAT_WATER, 1.0, 50, 2.2, 88, 60, 60.0), (I.MAT_WATER, 1.0, 100, 7.6, 95, 55, 110.0)]


@pytest.mark.parametrize("mat,rho,e0,depth,nz,ng,ehi", SIGMA_CASES,
                         ids=["bone-50MeV", "bone-100MeV", "water-50MeV", "water-100MeV"])
def test_lateral_sigma_with_the_papers_physics(mat, rho, e0, depth, nz, ng, ehi):
    """Measured: within 1 % everywhere; the growth near the peak -10 % (bone, 100 MeV), -4 % (water)."""
    tab = _sigma_table("lateral_sigma_bone.txt" if mat == I.MAT_BONE else "lateral_sigma_water.txt")[e0]
    xh = 2.0
    g = I.grid(40, 1, 10, ng, nz, 2, xh, 8.0, 0.3, 0.0, ehi, depth)
    dose, _ = Oracle(g, I.paper_physics(mat)).run(I.beam(float(e0)), np.full((nz, 40, 1), rho))
    dx = 2 * xh / g["nx"]
    x = -xh + (np.arange(g["nx"]) + 0.5) * dx
    z = (np.arange(nz) + 0.5) * g["dz"]

    def sigma(k):
        d = dose[k, :, 0]
        m = (x * d).sum() / d.sum()
        return np.sqrt((x * x * d).sum() / d.sum() - m * m - dx * dx / 12)

    for depth_z, ref in tab:
        k = int(np.searchsorted(z, depth_z)) - 1
        w = (depth_z - z[k]) / (z[k + 1] - z[k])
        got = (1 - w) * sigma(k) + w * sigma(k + 1)
        print(mat, e0, depth_z, round(got, 4), ref)
        assert abs(got - ref) <= 0.025 * ref, (depth_z, got, ref)
    if e0 == 100:   # at 50 MeV the growth is a few 1e-3 cm^2, within the cell-width correction
        growth, ref_growth = got ** 2 - 0.09, ref ** 2 - 0.09
        assert abs(growth - ref_growth) <= 0.15 * ref_growth, (growth, ref_growth)
