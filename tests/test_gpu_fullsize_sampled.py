"""Configurations 3 and 2 at their full sizes -- 96 x 96 cells, 32 x 32 angular nodes, 160 groups, two
generations (the bench's headline), and 64 x 64 cells, 128 groups, four generations (its second march) --
with sampled outputs checked against the FP64 oracle, through the kernels and launch shapes the bench times.

One seeded random state goes through each sub-step on the GPU (FP32 context, one-product BF16 source
product), starting from that same state every time: T over dz/2, A over dz, E's opening half-step over
dz/2 (with the source of generation 1 from generation 0).  The oracle recomputes sampled outputs one by
one from the seeded state:
  * T (section 3.4's upwind sweep with the superbee limiter) acts on every (group, coefficient, angle)
    plane on its own, so the oracle sweeps whole 96 x 96 planes: every mirroring of the two angular
    directions, the theta = 0 node, the first and last groups, and the two planes that share one wave of
    the two-plane sweep across a slab boundary (961 nodes per slab is odd);
  * A (section 3.4's angular CN step) and E (section 3.2's energy CN step, eq:(0041-d), with the source of
    the Remark after the scheme) act on one lateral cell at a time, so the oracle runs them on a window grid
    made of the sampled cells with those cells' densities: the corners, both sides of the seams between
    32-cell tiles and of the 64-column seam of the row sweep, and interior cells; the dose of those cells
    (the deposit of the E step) too.
Bound: per generation, max |got - ref| <= 1e-5 max |ref| over the sampled outputs (FP32; the same bound as
the sub-step tests on small grids).  The host holds the FP64 state (45 GB for configuration 3) twice at the
peak.
"""
import numpy as np
import pytest

from paper_2504_00340_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["config3", "config2"])
def test_fullsize_config_substeps_sampled_against_oracle(name):
    from oracle import oracle as O
    from paper_2504_00340_amd.pbsplit import Solver

    c = I.config3(0) if name == "config3" else I.config2("water")
    g = c["grid"]
    nx, ny, G, ngen = g["nx"], g["ny"], g["ng"], g["ngen"]
    o = O.Oracle(g, c["phys"])
    m, NA = o.m, o.NA
    th = o.theta()
    dz = g["dz"]
    layer = 1
    rho = np.ascontiguousarray(c["rho"][layer].reshape(-1))

    # sampled lateral cells pq = p ny + q: corners, tile seams (q 31 | 32), the sweep's 64-column seam,
    # the last tile, interior
    cells = [0, ny - 1, (nx - 1) * ny, nx * ny - 1, 40 * ny + 31, 40 * ny + 32, (nx - 1) * ny + 40, 55 * ny + 7]
    cells += [17 * ny + 63, 17 * ny + 64] if ny > 64 else [17 * ny + ny - 2]
    # sampled planes (k, g, l, a); a = i m + j with theta_x = th[i], theta_y = th[j]
    c0 = (m // 2) * m + m // 2
    planes = [(0, 100, 0, c0), (0, 100, 0, 0), (0, 100, 1, m - 1), (1, 20, 0, (m - 1) * m),
              (1, 20, 1, NA - 1), (0, 0, 0, 3 * m + 25), (1, G - 1, 1, 27 * m + 4),
              (ngen - 1, G // 2, 1, 5 * m + 17), (0, 5, 0, NA - 1), (0, 5, 1, 0)]
    # the last two share a wave of the two-plane sweep
    p0, p1 = (((k * G + gg) * 2 + l) * NA + a for k, gg, l, a in planes[-2:])
    assert p0 % 2 == 0 and p1 == p0 + 1

    s = Solver(g, c["phys"], precision="fp32")
    s.set_phantom(c["rho"])
    s.set_beam(c["beam"])                 # also zeroes the dose
    print(name, "sampled sub-steps: state", s.state_shape, flush=True)
    st = I.random_state(s.state_shape, 3301)
    st[:, :, 1] *= 0.3
    win = np.ascontiguousarray(st[..., cells])
    ref_planes = {}
    for (k, gg, l, a) in planes:
        ref_planes[(k, gg, l, a)] = o.transport_plane(st[k, gg, l, a].reshape(nx, ny), th[a // m], th[a % m],
                                                      0.5 * dz).reshape(-1)

    def run(op, h):
        s.set_state(st)
        s.apply(op, layer, h)
        print(name, "sampled sub-steps: applied op", op, flush=True)
        return s.state()

    def check(what, got, ref):
        for k in range(ngen):
            e = float(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max())
            print(f"{name} {what} generation {k}: max error / max |ref| {e:.2e}", flush=True)
            assert e <= TOL, (what, k, e)

    # T: whole planes
    got = run(2, 0.5 * dz)
    for k in sorted({p[0] for p in planes}):
        ks = [p for p in planes if p[0] == k]
        e = max(float(np.abs(got[p] - ref_planes[p]).max()) for p in ks) / max(
            float(np.abs(ref_planes[p]).max()) for p in ks)
        print(f"{name} T generation {k} ({len(ks)} planes): max error / max |ref| {e:.2e}", flush=True)
        assert e <= TOL, ("T", k, e)
    del got

    # A and E: the oracle on a window of the sampled cells
    gw = dict(g, nx=1, ny=len(cells), x_half=0.5 * o.dx, y_half=0.5 * len(cells) * o.dy, nz=1)
    gw["dz"] = dz
    ow = O.Oracle(gw, c["phys"])
    rw = np.ascontiguousarray(rho[cells])

    got = run(3, dz)[..., cells]
    ref = win.copy()
    for k in range(ngen):
        ow.angular_cn(ref[k], rw, dz)
    check("A", got, ref)

    got = run(1, 0.5 * dz)[..., cells]
    ref = win.copy()
    dep = ow.energy_all(ref, rw, 0.5 * dz)
    check("E", got, ref)
    dose = s.dose()[layer].reshape(-1)[cells]
    dref = dep / (rw * o.dx * o.dy * dz)
    e = float(np.abs(dose - dref).max() / np.abs(dref).max())
    print(f"{name} E dose of the sampled cells: max error / max dose {e:.2e}", flush=True)
    assert e <= TOL
    s.close()
