"""Seeded synthetic inputs: grids, beams, physics constants and density phantoms.

This module holds input data only (sizes, constants, seeded random densities)
and none of the solver's arithmetic; the HIP path and the CPU oracle both take
their inputs from here and from nowhere else.

The beam shape follows the paper's boundary distribution eq:(bdy) (section 4):
Gaussian laterally with sigma = 0.3 cm, mono-directional, energy spread
sigma_E = 1 MeV.  Materials are given by density only (water 1.0, bone 1.85,
lung 0.26); the physics constants are the water values of the solver's
physics record (Bragg-Kleeman range-energy law, Highland scattering power,
synthetic nuclear data).  The paper's own workloads are Monte Carlo
comparisons; these seeded phantoms stand in for them.
"""
from __future__ import annotations

import numpy as np

# Physics constants (one record).  Bragg-Kleeman alpha, p (cm, MeV); energy
# floor of the coefficients (the paper's lower energy bound, section 4);
# Highland E_s (MeV) and the radiation length of water (g/cm^2); proton mass
# (MeV); nuclear removal kappa0 (cm^2/g) and E_c (MeV); exponential
# down-scatter rate lambda (1/MeV); Gamma-law shape/rate of the nuclear
# deflection angle (App. A.4 forms, synthetic parameters).
PHYS = dict(bk_alpha=0.0022, bk_p=1.77, e_floor=1.0, highland_es=14.1, x0_water=36.08, mp=938.272,
            kappa0=0.012, e_c=20.0, lambda_nuc=0.05, gamma_a=2.0, gamma_b=40.0, stopping=0,
            straggling=0, scattering=0, material=0, nuc_bands=0)
STOP_BRAGG_KLEEMAN, STOP_BETHE = 0, 1   # stopping-power model: range fit, or Bethe-Bloch (App. A.1)
SCAT_HIGHLAND, SCAT_RUTHERFORD = 0, 1   # scattering power: Highland, or screened Rutherford (App. A.3)
MAT_WATER, MAT_BONE, MAT_AIR = 0, 1, 2  # media of the paper's material table (section 4)
RHO_MEDIUM = {MAT_WATER: 1.0, MAT_BONE: 1.757, MAT_AIR: 0.001205}   # densities of that table

# The paper's own physics (App. A.1-A.3) for a medium: Bethe-Bloch stopping, Williams straggling,
# screened-Rutherford scattering.
def paper_physics(material=MAT_WATER, straggling=1):
    return dict(PHYS, stopping=STOP_BETHE, straggling=straggling, scattering=SCAT_RUTHERFORD, material=material)


# Energy-band nuclear data (App. A.4 fits lambda and the Gamma-law alpha, beta group by group, at
# groups 100, 200, 300 and 400 of 500 on [1, 260] MeV, i.e. about 52.5, 104.3, 156.1 and 207.9 MeV;
# each group takes the parameters of the nearest of these anchors).  The values are synthetic (the
# fits need Monte Carlo data that are not printed): the energy transfer gets harder and the angular
# law narrower with energy.
NUC_BANDS = dict(nuc_bands=4, nuc_e=[52.5, 104.3, 156.1, 207.9], nuc_lambda=[0.08, 0.06, 0.05, 0.04],
                 nuc_alpha=[2.0, 2.0, 2.2, 2.4], nuc_beta=[25.0, 35.0, 45.0, 55.0])

RHO_WATER, RHO_BONE, RHO_LUNG = 1.0, 1.85, 0.26


def grid(nx, ny, nth, ng, nz, ngen, x_half, y_half, th_half, e_lo, e_hi, depth):
    return dict(nx=nx, ny=ny, nth=nth, ng=ng, nz=nz, ngen=ngen, x_half=float(x_half), y_half=float(y_half),
                th_half=float(th_half), e_lo=float(e_lo), e_hi=float(e_hi), dz=float(depth) / nz)


def beam(e0, x0=0.0, y0=0.0, sigma_x=0.3, sigma_y=0.3, sigma_e=1.0):
    return dict(e0=float(e0), sigma_e=float(sigma_e), x0=float(x0), y0=float(y0), sigma_x=float(sigma_x),
                sigma_y=float(sigma_y))


def water(g):
    return np.full((g["nz"], g["nx"], g["ny"]), RHO_WATER)


def slab(g, z0, z1, rho, base=RHO_WATER):
    """Water with a full-width slab of density rho over depth [z0, z1) (layer centres)."""
    r = np.full((g["nz"], g["nx"], g["ny"]), base)
    zc = (np.arange(g["nz"]) + 0.5) * g["dz"]
    r[(zc >= z0) & (zc < z1)] = rho
    return r


# --------------------------------------------------------------------------
# Configurations

def config1():
    """100 MeV pencil beam in water, 16x16 x 8x8 x 48 groups x 80 steps, primary + 1 generation."""
    g = grid(16, 16, 8, 48, 80, 2, 2.0, 2.0, 0.1, 0.0, 105.0, 8.0)
    return dict(name="c1-water-100MeV", grid=g, beam=beam(100.0), phys=dict(PHYS), rho=water(g))


def config2(case="water"):
    """150 MeV, 64x64 x 32x32 x 128 groups x 300 steps over 18 cm, primary + 3 generations.

    case: 'water', 'bone' (rho 1.85 slab at z in [3,5) cm) or 'lung' (rho 0.26 slab there).
    """
    g = grid(64, 64, 32, 128, 300, 4, 4.0, 4.0, 0.15, 0.0, 160.0, 18.0)
    if case == "water":
        rho = water(g)
    elif case == "bone":
        rho = slab(g, 3.0, 5.0, RHO_BONE)
    elif case == "lung":
        rho = slab(g, 3.0, 5.0, RHO_LUNG)
    else:
        raise ValueError(case)
    return dict(name=f"c2-{case}-150MeV", grid=g, beam=beam(150.0), phys=dict(PHYS), rho=rho)


def smooth_noise(shape, seed, sigma_vox=2.0):
    """White noise smoothed by a Gaussian of sigma_vox voxels, scaled to max |n| = 1."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.Generator(np.random.PCG64(seed))
    n = gaussian_filter(rng.standard_normal(shape), sigma=sigma_vox, mode="wrap")
    return n / np.max(np.abs(n))


def layered_phantom(nz, nx, ny, dz, dx, seed, depth_total):
    """Water/bone/lung layers (thicknesses U[1,5] cm from the seed) then water; a
    half-plane bone insert (x > 0) of U[1,3] cm below the layers; +-5 % smooth noise.
    Lateral cell centres run symmetrically about x = 0."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    t = rng.uniform(1.0, 5.0, size=3)
    ins = rng.uniform(1.0, 3.0)
    zc = (np.arange(nz) + 0.5) * dz
    r = np.full((nz, nx, ny), RHO_WATER)
    z = 0.0
    for th, rho in zip(t, (RHO_WATER, RHO_BONE, RHO_LUNG)):
        r[(zc >= z) & (zc < z + th)] = rho
        z += th
    xc = (np.arange(nx) + 0.5) * dx - nx * dx / 2
    sel_z = (zc >= z) & (zc < z + ins)
    r[np.ix_(sel_z, xc > 0, np.ones(ny, bool))] = RHO_BONE
    r *= 1.0 + 0.05 * smooth_noise((nz, nx, ny), seed)
    return r


def config3(seed=0):
    """180 MeV, heterogeneous layered phantom, 96x96 x 32x32 x 160 groups x 400 steps over 26 cm, K = 1."""
    g = grid(96, 96, 32, 160, 400, 2, 6.0, 6.0, 0.15, 0.0, 190.0, 26.0)
    rho = layered_phantom(g["nz"], g["nx"], g["ny"], g["dz"], 2 * g["x_half"] / g["nx"], seed, 26.0)
    return dict(name=f"c3-hetero-180MeV-seed{seed}", grid=g, beam=beam(180.0), phys=dict(PHYS), rho=rho)


def bk_range(e, phys=PHYS):
    """Water range of energy e from the range-energy law (only used to size depth windows)."""
    return phys["bk_alpha"] * e ** phys["bk_p"]


def config4(seed=0, nbeams=256):
    """Batched plan: nbeams uneven pencil beams on a shared 128x128x400 phantom.

    Returns dict(phantom=[400,128,128] on 0.1 x 0.1 x 0.0875 cm voxels, beams=[...]).  Each beam
    has its own grid (32x32 lateral window of 0.1 cm cells centred on the spot, 16x16 angles on
    +-0.15 rad, G ~ U{64..192} on [0, E+10], N ~ U{150..500} steps over min(35, 1.25 R(E))) and
    its densities sampled from the phantom at the nearest voxel.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nzp, nxp, nyp = 400, 128, 128
    vx, vz = 0.1, 0.0875
    phantom = layered_phantom(nzp, nxp, nyp, vz, vx, seed, 35.0)
    spots = [(-6.0 + 0.8 * i, -6.0 + 0.8 * j) for i in range(16) for j in range(16)]
    order = rng.permutation(len(spots))
    beams = []
    for b in range(nbeams):
        e = float(rng.uniform(70.0, 230.0))
        G = int(rng.integers(64, 193))
        N = int(rng.integers(150, 501))
        depth = min(35.0, 1.25 * bk_range(e))
        sx, sy = spots[order[b % len(spots)]]
        g = grid(32, 32, 16, G, N, 2, 1.6, 1.6, 0.15, 0.0, e + 10.0, depth)
        # nearest-voxel sampling of the shared phantom on this beam's grid
        zc = (np.arange(N) + 0.5) * g["dz"]
        xc = sx + (np.arange(32) + 0.5) * 0.1 - 1.6
        yc = sy + (np.arange(32) + 0.5) * 0.1 - 1.6
        iz = np.clip((zc / vz).astype(int), 0, nzp - 1)
        ix = np.clip(np.floor((xc + nxp * vx / 2) / vx).astype(int), 0, nxp - 1)
        iy = np.clip(np.floor((yc + nyp * vx / 2) / vx).astype(int), 0, nyp - 1)
        rho = phantom[np.ix_(iz, ix, iy)]
        beams.append(dict(grid=g, beam=beam(e), rho=rho, spot=(sx, sy)))
    return dict(name=f"c4-batched-{nbeams}-seed{seed}", phantom=phantom, beams=beams, phys=dict(PHYS))


def random_phantom_c5(seed, nz, nx, ny, dz, dx):
    """3-6 depth layers of U[1,5] cm with rho ~ U[0.2, 2.0], one lateral insert with rho ~ U[0.2, 2.0],
    +-5 % smooth noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nl = int(rng.integers(3, 7))
    zc = (np.arange(nz) + 0.5) * dz
    r = np.full((nz, nx, ny), RHO_WATER)
    z = 0.0
    for _ in range(nl):
        th = rng.uniform(1.0, 5.0)
        r[(zc >= z) & (zc < z + th)] = rng.uniform(0.2, 2.0)
        z += th
    xc = (np.arange(nx) + 0.5) * dx - nx * dx / 2
    x0, x1 = sorted(rng.uniform(-nx * dx / 2, nx * dx / 2, size=2))
    z0 = rng.uniform(0.0, nz * dz * 0.6)
    z1 = z0 + rng.uniform(1.0, 5.0)
    r[np.ix_((zc >= z0) & (zc < z1), (xc >= x0) & (xc < x1), np.ones(ny, bool))] = rng.uniform(0.2, 2.0)
    r *= 1.0 + 0.05 * smooth_noise((nz, nx, ny), seed)
    return r


def config5(seed, nz=300):
    """One surrogate training/evaluation run: 64x64 on +-4 cm, 16x16 angles on +-0.15 rad,
    96 groups on [0, E+10], nz steps over min(30, 1.25 R(E)), E ~ U[70, 230], K = 1."""
    rng = np.random.Generator(np.random.PCG64(10_000_019 + seed))
    e = float(rng.uniform(70.0, 230.0))
    depth = min(30.0, 1.25 * bk_range(e))
    g = grid(64, 64, 16, 96, nz, 2, 4.0, 4.0, 0.15, 0.0, e + 10.0, depth)
    rho = random_phantom_c5(seed, nz, 64, 64, g["dz"], 0.125)
    return dict(name=f"c5-surrogate-seed{seed}", grid=g, beam=beam(e), phys=dict(PHYS), rho=rho)


def small(nx=6, ny=5, nth=6, ng=7, nz=4, ngen=2, e0=30.0, e_hi=40.0, x_half=1.0, y_half=1.0, th_half=0.1,
          depth=0.8, seed=None, rho_lo=0.8, rho_hi=1.3):
    """Tiny ragged configuration for sub-operator tests (seeded densities if seed is given)."""
    g = grid(nx, ny, nth, ng, nz, ngen, x_half, y_half, th_half, 0.0, e_hi, depth)
    if seed is None:
        rho = water(g)
    else:
        rng = np.random.Generator(np.random.PCG64(seed))
        rho = rng.uniform(rho_lo, rho_hi, size=(nz, nx, ny))
    return dict(name="small", grid=g, beam=beam(e0, sigma_x=0.3, sigma_y=0.25), phys=dict(PHYS), rho=rho)


def random_state(shape, seed, positive=True):
    """Seeded smooth-ish random fluence for sub-operator parity (values O(1))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0.0, 1.0, size=shape) if positive else rng.standard_normal(shape)
    return x
