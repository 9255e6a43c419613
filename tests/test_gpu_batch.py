"""Batched beams (many pencil beams of one shape class in one graph launch per wave) through the
C ABI: every beam's dose is bitwise the single-beam dose, and one beam matches the FP64 oracle."""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I

pytestmark = pytest.mark.gpu


def _beams(n=5, seed=11, nx=10, ny=10):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        G = int(rng.integers(16, 40))
        nz = int(rng.integers(3, 9))
        e0 = float(rng.uniform(25.0, 38.0))
        g = I.grid(nx, ny, 16, G, nz, 2, 1.0, 1.0, 0.15, 0.0, e0 + 6.0, 0.15 * nz)
        b = I.beam(e0, x0=float(rng.uniform(-0.2, 0.2)), y0=float(rng.uniform(-0.2, 0.2)), sigma_x=0.25, sigma_y=0.3)
        rho = rng.uniform(0.7, 1.6, size=(nz, nx, ny))
        out.append(dict(grid=g, beam=b, rho=rho))
    return out


@pytest.mark.parametrize("wave,nx,ny", [(0, 10, 10), (2, 10, 10), (0, 8, 96), (0, 16, 32)])
def test_batch_equals_single_beam_runs(wave, nx, ny):
    """The 8 x 96 case runs the two-segment row sweep, the 16 x 32 case the two-plane one."""
    from paper_2504_00340_amd.pbsplit import Batch, Solver

    beams = _beams(3, nx=nx, ny=ny) if (nx, ny) != (10, 10) else _beams()
    bt = Batch(beams, I.PHYS, wave=wave)
    if wave:
        bt.prepare()             # tuning and capture ahead of the run; without it the first run does them
    bt.run()
    first = [bt.dose(i) for i in range(len(beams))]
    bt.run()                     # replays the graphs captured by the first run
    tu = bt.tuning()
    print("tuning", tu, flush=True)
    assert tu["gemm_kernel"] in ("global", "lds256", "lds128") and tu["tpass_waves_per_block"] in (1, 2, 4)
    assert tu["apass_cells_per_block"] in (8, 16, 32)
    for i, b in enumerate(beams):
        s = Solver(b["grid"], I.PHYS, precision="fp32")
        s.set_phantom(b["rho"])
        s.set_beam(b["beam"])
        s.run()
        ref = s.dose()
        s.close()
        got = bt.dose(i)
        print(i, b["grid"]["ng"], b["grid"]["nz"], float(np.abs(got - ref).max()), flush=True)
        assert np.array_equal(got, ref), i
        assert np.array_equal(first[i], got), i
    bt.close()


def test_batch_beam_matches_oracle():
    from oracle import oracle as O
    from paper_2504_00340_amd.pbsplit import Batch

    beams = _beams(3, seed=12)
    bt = Batch(beams, I.PHYS, wave=0)
    bt.run()
    b = beams[1]
    ref, _ = O.Oracle(b["grid"], I.PHYS).run(b["beam"], b["rho"])
    got = bt.dose(1)
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("batch beam vs oracle", rel, flush=True)
    assert rel < 1e-4
    bt.close()
