/*
 * pbsplit.h -- C ABI of libpbsplit, a gfx950 (MI355X) implementation of the
 * depth-splitting solver for one mono-directional proton pencil beam
 * (Zhang, Bai, Tang: "A deterministic solver for the linear Boltzmann model
 * of a single mono-directional proton beam").
 *
 * What is solved (paper section 2, eq:(f-e), and the scattering
 * decomposition eqn:(pri-se) of section 3.1): the Fermi-Eyges reduction of
 * the linear Boltzmann equation with continuous slowing down, small-angle
 * elastic scattering (angular Laplacian) and catastrophic nuclear removal /
 * re-emission, marched in depth z.  Unknowns are the DG-P1 energy
 * coefficients (psi^1, psi^2) of every energy group on a lateral finite-volume
 * grid (x, y) and an angular node grid (theta_x, theta_y), for the primary
 * generation and K scattered generations (source iteration).
 *
 * One depth step (section 3.3, Strang splitting, Crank-Nicolson in every
 * sub-step):   E(dz/2)  T(dz/2)  A(dz)  T(dz/2)  E(dz/2)
 *   E: energy loss by stopping power + nuclear removal + source (eq:(0041-d)),
 *   T: lateral transport, MUSCL with the superbee limiter (eq:(distansport)),
 *   A: angular diffusion, 5-point Laplacian by sine transform (eq:(sd)).
 * The dose (section 4, eq:(en_d)) is the energy lost by the proton
 * population in the energy sub-steps, per voxel, divided by rho * volume.
 *
 * Conventions
 *   - Every call returns a pbs_status; no exception or abort crosses the ABI.
 *     pbs_last_error() gives the text (with the HIP error string for
 *     PBS_EDEVICE).
 *   - The library never allocates device memory.  The caller allocates one
 *     device workspace of pbs_workspace_bytes() bytes and passes it to
 *     pbs_bind() with a HIP stream; all work is enqueued on that stream.
 *     The library never frees caller memory; host buffers are only read or
 *     written during the call that receives them.
 *   - State machine: create -> bind -> set_phantom -> set_beam ->
 *     step_depth / run_beam -> get_dose.  set_beam may be called again to
 *     start a new beam; set_phantom again before set_beam to change the
 *     densities.  Out-of-order calls return PBS_ESTATE.
 *   - Floating point: the fluence is stored and swept in the precision given
 *     to pbs_create (PBS_FP32 or PBS_FP64); the dose is accumulated in FP64
 *     in both.  Tables are built on the host in FP64.
 */
#ifndef PBSPLIT_H
#define PBSPLIT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PBS_OK = 0,
    PBS_EINVAL = -1,       /* bad argument (shape, NaN, non-positive density, too small workspace ...) */
    PBS_ESTATE = -2,       /* call out of order */
    PBS_ENOMEM = -3,       /* host allocation failed */
    PBS_EDEVICE = -4,      /* a HIP call failed */
    PBS_EUNSUPPORTED = -5  /* valid request the library does not implement */
} pbs_status;

enum { PBS_FP32 = 0, PBS_FP64 = 1 };

/* Grid (section 3.3 depth steps; section 3.4 lateral cells and angular nodes;
 * section 3.2 energy groups).
 *   nx, ny     lateral cells along x (index p) and y (index q), nx*ny >= 1
 *   nth        angular nodes per axis, even, >= 4: nodes theta_n = -th_half + n*dth,
 *              n = 0..nth-1, dth = 2 th_half/nth; node 0 and the implicit node nth
 *              are held at zero, so the unknowns are n = 1..nth-1 (node nth/2 is theta = 0)
 *   ng         energy groups, uniform on [e_lo, e_hi] (MeV), ng >= 2
 *   nz         depth steps of length dz (cm); voxel layer s spans [s dz, (s+1) dz]
 *   ngen       generations 1 + K (primary + K catastrophic-scatter generations), 1..8
 *   x_half, y_half  lateral half-widths (cm), the grid is centred on x = y = 0 */
typedef struct pbs_grid {
    int nx, ny, nth, ng, nz, ngen;
    double x_half, y_half, th_half, e_lo, e_hi, dz;
} pbs_grid;

/* Beam: the boundary distribution eq:(bdy) (section 4) -- Gaussian in x, y
 * (centre x0, y0, widths sigma_x, sigma_y, cm) and in energy (e0, sigma_e,
 * MeV), mono-directional (all protons on the theta = 0 node).  The initial
 * fluence carries one proton. */
typedef struct pbs_beam {
    double e0, sigma_e, x0, y0, sigma_x, sigma_y;
} pbs_beam;

/* Physics record.  Every voxel holds the same medium (`material`); voxels differ by density only.
 *   stopping        PBS_STOP_BRAGG_KLEEMAN: S from the range fit below (water only);
 *                   PBS_STOP_BETHE: the Bethe-Bloch mass stopping power of App. A.1 for the medium,
 *                   heavy-projectile form kappa Z/A / beta^2 [ln(2 m_e c^2 beta^2 gamma^2 / I) - beta^2]
 *                   with kappa = 0.307075 MeV cm^2/mol, no density correction, I(Z) from the
 *                   appendix's piecewise fit, summed over the elements with their mass fractions
 *                   (Bragg additivity); needs e_floor >= 0.5 MeV (else PBS_EINVAL)
 *   straggling      0: none; 1: Williams' straggling coefficient of App. A.2 for the medium,
 *                   T = kappa m_e c^2 Z/A [1 + 4 I/(3 m_e v^2) ln(2 m_e v^2 / I)] per element, mass-
 *                   fraction sum; the energy operator gains (1/2) d^2/dE^2 (T psi) of section 3.2: its
 *                   first-order part (1/2) d/dE (T' psi) adds T'/2 to the stopping term, its second-order
 *                   part is the symmetric interior penalty discretisation (penalty 2 T_f / h_f on interior
 *                   group faces, none on the end faces), so every energy line is block-tridiagonal.
 *                   Needs stopping = PBS_STOP_BETHE.  FP32 contexts then use the FP32 source product.
 *   scattering      PBS_SCAT_HIGHLAND: the Highland scattering power below; PBS_SCAT_RUTHERFORD: the
 *                   screened-Rutherford momentum-transfer cross section of App. A.3 for the medium,
 *                   2 pi (Z r_e m_e c^2 / pv)^2 [ln((eta+1)/eta) - 1/(eta+1)] N_A/A per element, eta =
 *                   (Z^(1/3) alpha m_e c / p)^2, with p v of the proton in the laboratory frame
 *   material        PBS_MAT_WATER (H2O), PBS_MAT_BONE, PBS_MAT_AIR (the compositions of section 4's
 *                   material table); other than water needs stopping = PBS_STOP_BETHE
 *   bk_alpha, bk_p  Bragg-Kleeman range R = alpha E^p (cm water): S = 1/(alpha p E^(p-1))
 *   e_floor         coefficients are evaluated at max(E, e_floor) (MeV)
 *   highland_es, x0_water, mp   scattering power sigma_tr = (E_s/pv)^2 / X0 (Highland form),
 *                   group-averaged with 8-point Gauss-Legendre (either form)
 *   kappa0, e_c     nuclear removal per unit mass kappa(E) = kappa0 (1 - exp(-E/e_c)) (cm^2/g)
 *   lambda_nuc      energy transfer of re-emission  ~ exp(-lambda (E_g' - E_g)) (App. A.4)
 *   gamma_a, gamma_b  angular transfer ~ theta^(a-1) exp(-b theta) of the deflection angle
 *   nuc_bands       0: lambda_nuc, gamma_a, gamma_b for every group; 1..4: the App. A.4 parameters per
 *                   energy band -- each group takes those of the nearest anchor nuc_e[b] (MeV): the energy
 *                   law uses the source group's nuc_lambda, the angular law the destination group's
 *                   nuc_alpha, nuc_beta.  Not with the batched path. */
enum { PBS_STOP_BRAGG_KLEEMAN = 0, PBS_STOP_BETHE = 1 };
enum { PBS_SCAT_HIGHLAND = 0, PBS_SCAT_RUTHERFORD = 1 };
enum { PBS_MAT_WATER = 0, PBS_MAT_BONE = 1, PBS_MAT_AIR = 2 };
typedef struct pbs_physics {
    double bk_alpha, bk_p, e_floor, highland_es, x0_water, mp;
    double kappa0, e_c, lambda_nuc, gamma_a, gamma_b;
    int stopping, straggling, scattering, material, nuc_bands;
    double nuc_e[4], nuc_lambda[4], nuc_alpha[4], nuc_beta[4];
} pbs_physics;

typedef struct pbs_ctx pbs_ctx; /* opaque; host-side metadata only */

/* Create a context for one grid and physics record: the phase-space grid of
 * section 3 (DG-P1 energy groups of section 3.2, lateral cells and angular
 * nodes of section 3.4, depth steps of section 3.3) and the coefficient tables
 * of App. A (S, sigma_tr, T, the nuclear kernel) built on the host in FP64.
 * precision: PBS_FP32 or PBS_FP64.  *out receives the context (NULL on error).
 * Host memory only. */
pbs_status pbs_create(const pbs_grid *grid, const pbs_physics *phys, int precision, pbs_ctx **out);

/* Device workspace the caller must provide (bytes, 256-byte aligned start). */
pbs_status pbs_workspace_bytes(const pbs_ctx *ctx, size_t *bytes);

/* Bind the caller's device workspace and HIP stream (hipStream_t, NULL = the
 * null stream).  The workspace must stay valid until pbs_destroy or the next
 * bind; rebinding invalidates phantom, beam and dose. */
pbs_status pbs_bind(pbs_ctx *ctx, void *dev_workspace, size_t bytes, void *hip_stream);

/* Allocation-free variant of pbs_bind, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): binds the context to a scratch
 * array that the library holds in device memory, PBS_STATIC_SCRATCH_BYTES (64 MiB) per GPU, kept until
 * the process ends, and to hip_stream (hipStream_t on the current device, NULL = the null stream).  It
 * calls no hipMalloc, hipFree or other allocating routine and creates no stream or event, so the
 * context always marches on its one stream (pbs_set_schedule has no effect on it).  Returns PBS_EINVAL
 * (with the sizes in pbs_last_error) when pbs_workspace_bytes exceeds the scratch, PBS_EDEVICE when
 * the scratch's address cannot be obtained.
 * Every context bound this way on one GPU shares that GPU's scratch, which keeps the last call's
 * contents (pbs_set_beam clears what must start at zero).  Binding another context to it invalidates
 * the previous one: its later calls return PBS_ESTATE.  Calls of two such contexts that overlap in time
 * on one GPU race.  Results are bitwise those of a context bound with pbs_bind. */
#define PBS_STATIC_SCRATCH_BYTES (64u << 20)
pbs_status pbs_bind_static(pbs_ctx *ctx, void *hip_stream);

/* Densities rho[s][p][q] (g/cm^3) on the computational grid, host array of
 * nz*nx*ny doubles, C order.  Every value must be finite and > 0 (else
 * PBS_EINVAL).  Copied; the caller keeps ownership.  The density enters the
 * operators as rho(r) of the transport equation (section 2, eq:(f-e)): rho S,
 * rho sigma_tr, rho T and the removal sigma_ct = rho kappa. */
pbs_status pbs_set_phantom(pbs_ctx *ctx, const double *rho, size_t n);

/* A voxel phantom with its own spacing (the density field rho(x, y, z) of the
 * problem statement, section 2 and section 4's test domains), resampled onto
 * the computational grid by the nearest voxel and then set as pbs_set_phantom
 * does.  vox[k][i][j] (host, C order, vnz*vnx*vny doubles, finite and > 0)
 * covers depth [k vdz, (k+1) vdz) and, in the beam's lateral frame (the grid is
 * centred on x = y = 0), x in [x_lo + i vdx, x_lo + (i+1) vdx), y likewise from
 * y_lo.  The density of layer s and cell (p, q) is that of the voxel holding
 * the layer's and the cell's centre, the index clamped to the phantom.
 * PBS_EINVAL for bad sizes, spacings or densities; PBS_ESTATE before bind. */
pbs_status pbs_set_phantom_voxels(pbs_ctx *ctx, const double *vox, int vnz, int vnx, int vny, double vdz,
                                  double vdx, double vdy, double x_lo, double y_lo);

/* The resampling of pbs_set_phantom_voxels alone, on the host: out receives
 * grid->nz * grid->nx * grid->ny densities [s][p][q].  No context needed. */
pbs_status pbs_resample_phantom(const pbs_grid *grid, const double *vox, int vnz, int vnx, int vny, double vdz,
                                double vdx, double vdy, double x_lo, double y_lo, double *out);

/* Start a beam (section 4, the boundary distribution eq:(bdy); section 3.1's
 * scattering decomposition eqn:(pri-se) for the generations): builds the
 * initial fluence (eq:(bdy) projected on the grid),
 * zeroes the scattered generations and the dose, sets the step counter to 0. */
pbs_status pbs_set_beam(pbs_ctx *ctx, const pbs_beam *beam);

/* Advance n >= 0 depth steps of the splitting scheme of section 3.3 (each step
 * the Strang sequence E(dz/2) T(dz/2) A(dz) T(dz/2) E(dz/2) over every
 * generation, Crank-Nicolson in every sub-step), asynchronous on the bound
 * stream; layer s takes the densities of phantom layer s.  The last
 * energy half-step of the last advanced step is deferred and fused with the
 * first half-step of the next one; run_beam applies the closing half-step.
 * Splitting a march into chunks gives bitwise the same result as one call.
 * *step_out (may be NULL) receives the number of steps done so far. */
pbs_status pbs_step_depth(pbs_ctx *ctx, int n, int *step_out);

/* March the remaining steps of section 3.3's scheme and apply the closing
 * energy half-step of the last layer. */
pbs_status pbs_run_beam(pbs_ctx *ctx);

/* Dose D = E_dep / (rho dx dy dz) of section 4 (the dose definition and the
 * energy deposition eq:(en_d): the energy the protons lose in the energy
 * sub-steps of each layer) in MeV/g per incident proton on [nz][nx][ny],
 * FP64, n = nz*nx*ny.  out is host memory (out_is_device = 0; the call
 * synchronises the stream) or device memory (1; the copy is enqueued). */
pbs_status pbs_get_dose(pbs_ctx *ctx, double *out, size_t n, int out_is_device);

/* Diagnostics (used by the parity tests): read / write the fluence of all
 * generations as FP64 host arrays in the order [k][g][l][a][p*ny+q], with
 * a = i*(nth-1) + j over the interior angular nodes.  n = ngen*ng*2*(nth-1)^2*nx*ny.
 * set_state requires a beam to have been set and resets nothing else. */
pbs_status pbs_get_state(pbs_ctx *ctx, double *out, size_t n);
pbs_status pbs_set_state(pbs_ctx *ctx, const double *in, size_t n);

/* Diagnostics: apply one sub-step to the current fluence of every generation
 * with the densities of layer `layer`:
 *   PBS_OP_E  energy CN step of length h, generations in order with the
 *             trapezoidal catastrophic source; the deposited energy is added
 *             to the dose of `layer`
 *   PBS_OP_T  lateral transport CN step of length h
 *   PBS_OP_A  angular diffusion CN step of length h */
enum { PBS_OP_E = 1, PBS_OP_T = 2, PBS_OP_A = 3 };
pbs_status pbs_apply(pbs_ctx *ctx, int op, int layer, double h);

/* Arithmetic of the angular part of the catastrophic source (the product of the nuclear angular
 * transfer matrix with the energy-scanned fluence, App. A.4) in an FP32 context with at least 128
 * angular unknowns:
 *   PBS_SRC_FP32    FP32 MFMA
 *   PBS_SRC_BF16X3  both operands split as hi + lo bfloat16, three BF16 MFMA products accumulated
 *                   in FP32 (relative error of each term <= ~2^-15)
 *   PBS_SRC_BF16X2  the transfer matrix split as hi + lo, the energy-scanned fluence rounded to bfloat16
 *                   with error feedback along the groups (each line carries its rounding residue into
 *                   the next group, so the errors telescope in the re-emitted number and energy), two
 *                   BF16 products
 *   PBS_SRC_BF16X1  one BF16 product: the transfer matrix rounded to bfloat16 with every column
 *                   compensated to keep its exact sum (the number of re-emitted protons), the scanned
 *                   fluence rounded as in BF16X2, and the product itself stored in bfloat16 (read once,
 *                   by the next generation's energy pass); the default
 * Other contexts always use their own precision; the split modes there return PBS_EUNSUPPORTED. */
enum { PBS_SRC_FP32 = 0, PBS_SRC_BF16X3 = 1, PBS_SRC_BF16X2 = 2, PBS_SRC_BF16X1 = 3 };
pbs_status pbs_set_source_precision(pbs_ctx *ctx, int mode);

/* Splitting in depth (section 3.3; section 5 names higher-order splitting as the extension).
 *   order 2: Strang steps E(dz/2) T(dz/2) A(dz) T(dz/2) E(dz/2) (the default);
 *   order 4: Richardson extrapolation of the Strang step per depth layer: from the state psi_n,
 *            A = S(dz) psi_n and B = S(dz/2) S(dz/2) psi_n with the layer's densities, psi_{n+1} =
 *            (4 B - A) / 3, and the layer's deposit combined with the same weights.  Fourth order in depth
 *            for linear steps (every sub-step stays a positive CN step); about three Strang steps of work
 *            per layer, and two more copies of the fluence in the workspace.  Every step is complete, so
 *            pbs_run_beam adds no closing half-step.
 * Must be called after pbs_create and before pbs_workspace_bytes / pbs_bind.  PBS_EINVAL for another
 * order, PBS_ESTATE after bind, PBS_EUNSUPPORTED for order 4 with a surrogate. */
pbs_status pbs_set_splitting(pbs_ctx *ctx, int order);

/* Schedule of the depth march (no effect on the results, which are bitwise the same either way).
 * Generation k's transport, angular and transport sub-steps touch only its own fluence, so they may
 * run on a second stream beside the energy passes and source products of the later generations
 * (section 3.3's Strang sequence is kept per generation; the next step's energy pass of k waits for
 * them).  mode PBS_SCHED_AUTO (the default) uses the second stream when one generation has fewer than
 * 1e8 phase-space cells, PBS_SCHED_ONE_STREAM never, PBS_SCHED_TWO_STREAMS always.  The stream is
 * created by pbs_bind and joined back into the bound stream at the end of every pbs_step_depth /
 * pbs_run_beam call.  Returns PBS_EINVAL for another mode. */
enum { PBS_SCHED_AUTO = 0, PBS_SCHED_ONE_STREAM = 1, PBS_SCHED_TWO_STREAMS = 2 };
pbs_status pbs_set_schedule(pbs_ctx *ctx, int mode);

/* Diagnostics: kernel timing.  pbs_profile(ctx, 1) starts recording a HIP event pair on the
 * bound stream around every kernel launch, grouped by kind; pbs_profile(ctx, 0) stops and
 * clears.  pbs_profile_read synchronises the stream and returns, for kind = 0..n-1 (at most
 * PBS_NKIND), the summed duration in ms and the number of launches since recording began. */
enum { PBS_K_EPASS = 0, PBS_K_TPASS = 1, PBS_K_APASS = 2, PBS_K_QGEMM = 3, PBS_K_DOSE = 4, PBS_NKIND = 5 };
pbs_status pbs_profile(pbs_ctx *ctx, int enable);
pbs_status pbs_profile_read(pbs_ctx *ctx, double *ms, long *launches, int n);

/* ------------------------------------------------------------------ batched pencil beams
 * Many beams of one shape class -- equal nx, ny, nth, ngen, x_half, y_half, th_half; energy groups,
 * energy range, depth steps and step length per beam -- marched together on one GPU in FP32 with
 * the split-BF16 source product (nth >= 16).  Each beam follows exactly the single-beam scheme above
 * (same kernels, bitwise the same dose).  Beams are grouped into waves of at most `wave` beams
 * (0 = all), longest first; the whole march of a wave is captured into one HIP graph and launched
 * once.  Launch variants that do not change the arithmetic are chosen by timing on the first wave.
 * The caller owns the workspace (pbs_batch_workspace_bytes, 256-byte aligned) and the host arrays. */
typedef struct pbs_batch pbs_batch;
pbs_status pbs_batch_create(const pbs_grid *grids, const pbs_beam *beams, int nbeams, const pbs_physics *phys,
                            int wave, pbs_batch **out);
pbs_status pbs_batch_workspace_bytes(const pbs_batch *batch, size_t *bytes);
/* hip_stream must not be NULL: the march is captured into a HIP graph, which the null stream cannot do. */
pbs_status pbs_batch_bind(pbs_batch *batch, void *dev_workspace, size_t bytes, void *hip_stream);
/* Densities of one beam's grid, [nz][nx][ny] doubles (finite, > 0); copied. */
pbs_status pbs_batch_set_phantom(pbs_batch *batch, int beam, const double *rho, size_t n);
/* Choose the launch variants (timing on the first wave) and capture every wave's march into a HIP graph,
 * once; later runs replay the graphs.  Optional: pbs_batch_run does it on its first call.  Needs every
 * phantom set; synchronises the stream. */
pbs_status pbs_batch_prepare(pbs_batch *batch);
/* March every beam to its end (closing energy half-step included); synchronises the stream.  Per wave:
 * upload tables, densities and the initial fluence of its beams, replay the wave's graph. */
pbs_status pbs_batch_run(pbs_batch *batch);
/* Dose of one beam, [nz][nx][ny] FP64 host array (MeV/g per incident proton). */
pbs_status pbs_batch_get_dose(pbs_batch *batch, int beam, double *out, size_t n);
/* Launch variants chosen by the autotuner: {source-product kernel (0: scans read from global memory,
 * 1: scans staged in LDS, 256-column blocks, 2: the same with 128 columns), transport planes per
 * block, angular-pass cells per block (angular grids other than 16 and 32 nodes)}. */
pbs_status pbs_batch_tuning(const pbs_batch *batch, int *out3);
const char *pbs_batch_last_error(const pbs_batch *batch);
void pbs_batch_destroy(pbs_batch *batch);

/* ------------------------------------------------- surrogate of the scattered generation
 * A K = 1 march (ngen = 2: primaries plus the first catastrophic-scatter generation of the
 * scattering decomposition eqn:(pri-se), section 3.1) can replace the scattered generation by a
 * learned estimate of its net deposit.  This is not part of the paper; it is an add-on of this
 * library, checked against the plain march.
 *
 * Per voxel layer s and lateral cell, the primary march records (FP64):
 *   I      the energy the nuclear re-emission injects into generation 1 during the two energy
 *          half-steps of layer s (the source functional of App. A.4 summed over destination
 *          angles, which the angular law conserves),
 *   M_E, M_N  the energy and number content of the primaries after the opening energy
 *          half-step of layer s: sum over groups and angles of dE (E_g psi^1 + dE psi^2 / 6) and
 *          of dE psi^1, times dth^2 dx dy,
 *   E0     the deposit of the primary generation alone.
 * Features of slice s (BF16, 8 channels per cell, image [nx][ny], ny <= 64):
 *   0: M_E kappa0 dz / c,  1: rho,  2: I / c,  3-5 and 7: F_j / c with the causal depth filters
 *   F_j(s) = a F_j(s-1) + (1 - a) I(s), a = exp(-rho dz / L_j), L = 0.5, 2, 6 (3-5) and 15 cm (7),
 *   6: (M_E / M_N) / 250 MeV where M_N > 1e-4 max M_N (else 0);  c = max over the beam of I.
 * Target (FP32): (E_total - E0 + I) / c, the energy generation 1 deposits itself in the voxel.
 * Surrogate dose: E0 - I + c * net(features), from a march of the primaries only.
 * Residual: |sum c * net - (1 - l) sum I| / (sum E0 - sum I + sum c * net), the energy balance of
 * generation 1 relative to the whole deposit of the beam, where l = l0 + l1 x + l2 x^2 (clamped to
 * [0, 0.95]) models the fraction of the injected energy that generation 1 carries out of the grid
 * (through the angular and lateral boundaries, or past the last layer) from the fraction of the
 * beam energy the primaries do not deposit, x = 1 - sum E0 / e0.  Above the tolerance the beam is marched again with both generations
 * (the plain method), so the result is then exactly the plain K = 1 dose.
 *
 * Network (weights blob = pbs_net_header + nparam FP32 values): 3x3 convolutions, zero padding,
 * 8 -> 32 -> 32 -> 32 -> 1 channels, ReLU after the first three; parameters in the order
 * w0 [32][8][3][3], b0 [32], w1 [32][32][3][3], b1, w2 [32][32][3][3], b2, w3 [1][32][3][3], b3 [1].
 * BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16). */
#define PBS_NET_MAGIC 0x4E534250u /* "PBSN" */
#define PBS_NET_VERSION 1u
#define PBS_NET_CIN 8
typedef struct pbs_net_header {
    unsigned int magic, version, nparam, nfeat; /* nfeat = 8 */
    double leak[3];                             /* leak model coefficients l0, l1, l2 */
    double reserved[3];
} pbs_net_header;                               /* 64 bytes */

/* Must be called after pbs_create and before pbs_workspace_bytes / pbs_bind (it enlarges the
 * workspace).  The context must have ngen = 2 and ny <= 64.
 *   weights = NULL, bytes = 0: recording mode.  pbs_run_beam marches the plain method and keeps
 *       the per-slice records; pbs_surrogate_sample then writes features and targets.
 *   weights = blob: surrogate mode.  pbs_run_beam marches the primaries only, evaluates the
 *       network and checks the residual against residual_tol (finite, >= 0), falling back to the
 *       plain march.  pbs_step_depth is refused (PBS_ESTATE): the surrogate acts on whole beams.
 * The blob is copied. */
pbs_status pbs_set_surrogate(pbs_ctx *ctx, const void *weights, size_t bytes, double residual_tol);

/* Recording mode, after pbs_run_beam: features [nz][nx*ny][8] BF16 into dev_x and targets
 * [nz][nx*ny] FP32 into dev_target (device memory, 16-byte aligned, n_slices = nz); asynchronous. */
pbs_status pbs_surrogate_sample(pbs_ctx *ctx, void *dev_x, float *dev_target, size_t n_slices);

/* Either mode, after pbs_run_beam: the FP64 records [4][nz][nx*ny] = I, M_E, M_N, E0 (MeV) into
 * a host array (E0 is recorded in recording mode only; zero otherwise).  Synchronises. */
pbs_status pbs_surrogate_records(pbs_ctx *ctx, double *out, size_t n);

/* After pbs_run_beam (synchronises): out[0] residual, [1] 1 if the plain march was used,
 * [2] energy budget (1 - l) sum I, [3] network energy sum c * net, [4] c, [5] sum I,
 * [6] energy generation 1 deposited itself (recording mode; else NaN), [7] leak fraction (model
 * value in surrogate mode, measured 1 - [6] / [5] in recording mode), [8] sum E0, [9] x (above).
 * Values that do not apply are NaN.  n <= 10. */
pbs_status pbs_surrogate_report(pbs_ctx *ctx, double *out, int n);

/* Training of the network on one GPU (the same kernels as the surrogate, plus the data and weight
 * gradients and an Adam update).  Images are H x W (W <= 64) with 8 BF16 input channels, one FP32
 * output channel; loss = mean over pixels of (y - t)^2.  The caller owns the workspace. */
typedef struct pbs_net pbs_net;
pbs_status pbs_net_param_count(size_t *count);
pbs_status pbs_net_create(int H, int W, int max_batch, pbs_net **out);
pbs_status pbs_net_workspace_bytes(const pbs_net *net, size_t *bytes);
pbs_status pbs_net_bind(pbs_net *net, void *dev_workspace, size_t bytes, void *hip_stream);
/* FP32 parameters in the order above (host); resets the Adam state. */
pbs_status pbs_net_set_params(pbs_net *net, const float *params, size_t count);
pbs_status pbs_net_get_params(pbs_net *net, float *params, size_t count);
/* y [n][H][W] FP32 = network(x [n][H][W][8] BF16), device pointers (x 16-byte aligned); asynchronous. */
pbs_status pbs_net_forward(pbs_net *net, const void *dev_x, float *dev_y, int n);
/* Gradient of the loss with respect to every parameter (host, parameter order) and the loss;
 * no update.  Synchronises. */
pbs_status pbs_net_gradient(pbs_net *net, const void *dev_x, const float *dev_t, int n, float *grad, size_t count,
                            double *loss);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) with learning rate lr on the minibatch; the loss
 * before the step goes to dev_loss (device double, may be NULL).  Asynchronous. */
pbs_status pbs_net_train_step(pbs_net *net, const void *dev_x, const float *dev_t, int n, double lr,
                              double *dev_loss);
const char *pbs_net_last_error(const pbs_net *net);
void pbs_net_destroy(pbs_net *net);

/* Text of the last error of this context (never NULL). */
const char *pbs_last_error(const pbs_ctx *ctx);

/* Release the context: waits for the work it enqueued on its stream, then frees host memory only (the
 * workspace stays the caller's). */
void pbs_destroy(pbs_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PBSPLIT_H */
