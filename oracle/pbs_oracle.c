/*
 * pbs_oracle.c -- plain, slow FP64 CPU oracle of the depth-splitting proton
 * solver (Zhang, Bai, Tang, "A deterministic solver for the linear Boltzmann
 * model of a single mono-directional proton beam").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the HIP path; every table
 * below is computed here from its definition.
 *
 * Each routine follows one passage of the paper (cited by section and
 * equation label) and is written for a reader to check by eye, not for
 * speed.  The readings taken where the paper is ambiguous are listed next to
 * the code that applies them (R1..R16 numbering is local to this project).
 *
 * State layout (one generation):  psi[g][l][a][pq]
 *   g  = energy group 0..G-1 (group g spans faces g and g+1, g=G-1 highest)
 *   l  = DG coefficient 0 (group mean psi^1) or 1 (slope psi^2)
 *   a  = i*m + j, interior angular nodes i,j = 0..m-1, m = nth-1
 *        (node index i+1 of the nth-node grid; nodes 0 and nth are zero)
 *   pq = p*ny + q, lateral cell p along x (0..nx-1), q along y (0..ny-1)
 * Generations k = 0..K are stored one after the other.
 *
 * Parity status: every function here is pinned by the -m "not gpu" tests
 * (dense solves, closed forms, conservation, convergence, symmetry).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nth, ng, nz, ngen;
    double x_half, y_half, th_half, e_lo, e_hi, dz;
} og_grid;

typedef struct {
    double e0, sigma_e, x0, y0, sigma_x, sigma_y;
} og_beam;

typedef struct {
    double bk_alpha, bk_p, e_floor, highland_es, x0_water, mp;
    double kappa0, e_c, lambda_nuc, gamma_a, gamma_b;
    int stopping;   /* 0: Bragg-Kleeman range fit (water); 1: Bethe-Bloch of the medium (App. A.1) */
    int straggling; /* 0: none; 1: Williams straggling coefficient of the medium (App. A.2) */
    int scattering; /* 0: Highland scattering power; 1: screened Rutherford sigma_tr (App. A.3) */
    int material;   /* medium: 0 water, 1 bone, 2 air (the compositions of section 4's material table) */
    int nuc_bands;  /* 0: lambda_nuc, gamma_a, gamma_b for every group; 1..4: per energy band below */
    double nuc_e[4], nuc_lambda[4], nuc_alpha[4], nuc_beta[4];
} og_phys;

/* Worker threads of the parallel loops over independent lines (timing of the oracle only; the
 * results do not depend on it).                                            */
void og_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int og_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------- sizes */
static long og_m(const og_grid *g) { return g->nth - 1; }
static long og_na(const og_grid *g) { return og_m(g) * og_m(g); }
static long og_np(const og_grid *g) { return (long)g->nx * g->ny; }
long og_gen_elems(const og_grid *g) { return (long)g->ng * 2 * og_na(g) * og_np(g); }

static double og_dx(const og_grid *g) { return 2.0 * g->x_half / g->nx; }
static double og_dy(const og_grid *g) { return 2.0 * g->y_half / g->ny; }
static double og_dth(const og_grid *g) { return 2.0 * g->th_half / g->nth; }
/* Angular coordinate of interior index i (node i+1), R4: nodes at
 * -th_half + n*dth, n = 0..nth-1, node nth implicit at +th_half.           */
static double og_theta(const og_grid *g, long i) { return -g->th_half + (double)(i + 1) * og_dth(g); }

static long IDX(const og_grid *g, long gg, long l, long a, long pq)
{
    return ((gg * 2 + l) * og_na(g) + a) * og_np(g) + pq;
}

/* ------------------------------------------------------------- physics */
/* Mean excitation energy of element Z, eV: the appendix's piecewise fit (App. A.1). */
static double og_ivalue(int Z)
{
    if (Z == 1) return 19.0;
    if (Z <= 13) return 11.2 + 11.7 * Z;
    return 52.8 + 8.71 * Z;
}

/* ------------------------------------------------------------- media
 * Elements by atomic number Z and standard atomic weight A (g/mol), and the
 * media by weight fraction: water as H2O; bone and air as section 4's table
 * of material targets prints them.                                          */
#define OG_MAXEL 9
typedef struct {
    int n;
    int Z[OG_MAXEL];
    double A[OG_MAXEL], w[OG_MAXEL];
} og_medium;

static og_medium og_get_medium(int material)
{
    og_medium m;
    memset(&m, 0, sizeof(m));
    if (material == 1) { /* bone, rho 1.757 in the table */
        const int Z[9] = {1, 6, 7, 8, 11, 12, 15, 16, 20};
        const double A[9] = {1.008, 12.011, 14.007, 15.999, 22.990, 24.305, 30.974, 32.06, 40.078};
        const double w[9] = {0.042, 0.194, 0.040, 0.425, 0.001, 0.002, 0.092, 0.003, 0.201};
        m.n = 9;
        for (int k = 0; k < 9; k++) { m.Z[k] = Z[k]; m.A[k] = A[k]; m.w[k] = w[k]; }
    } else if (material == 2) { /* air, rho 0.001205 */
        const int Z[4] = {6, 7, 8, 18};
        const double A[4] = {12.011, 14.007, 15.999, 39.948};
        const double w[4] = {0.0001248, 0.7553, 0.2318, 0.01283};
        m.n = 4;
        for (int k = 0; k < 4; k++) { m.Z[k] = Z[k]; m.A[k] = A[k]; m.w[k] = w[k]; }
    } else { /* water: H2O */
        const double molar = 2.0 * 1.008 + 15.999;
        m.n = 2;
        m.Z[0] = 1; m.A[0] = 1.008; m.w[0] = 2.0 * 1.008 / molar;
        m.Z[1] = 8; m.A[1] = 15.999; m.w[1] = 15.999 / molar;
    }
    return m;
}

/* Kinematics of a proton of kinetic energy E (MeV): beta^2, gamma, pc (MeV). */
static void og_kin(double E, double mp, double *beta2, double *gamma, double *pc)
{
    double g = 1.0 + E / mp;
    *gamma = g;
    *beta2 = 1.0 - 1.0 / (g * g);
    *pc = sqrt(E * (E + 2.0 * mp));
}

#define OG_KAPPA 0.307075        /* 4 pi N_A r_e^2 m_e c^2, MeV cm^2/mol */
#define OG_MEC2 0.51099895       /* electron rest energy, MeV */
#define OG_NA 6.02214076e23      /* Avogadro, 1/mol */
#define OG_RE 2.8179403262e-13   /* classical electron radius, cm */
#define OG_ALPHA (1.0 / 137.035999084)

/* Bethe-Bloch mass stopping power of the medium, MeV cm^2/g (App. A.1).
 * Readings: the printed prefactor kappa Z is taken per gram, kappa Z/A with
 * kappa = 0.307075 MeV cm^2/mol; the logarithm is the heavy-projectile form
 * as printed (maximum energy transfer 2 m_e c^2 beta^2 gamma^2); the density
 * term delta is 0 (the appendix does not give it; below 250 MeV in water it
 * is well under 0.1 %); the compound weights N_k are the mass fractions of
 * the elements (Bragg additivity per unit mass); I(Z) from the appendix's
 * piecewise fit.                                                            */
double og_bethe(int material, double E, double mp)
{
    og_medium m = og_get_medium(material);
    double b2, gam, pc;
    og_kin(E, mp, &b2, &gam, &pc);
    const double tmax_ev = 2.0 * OG_MEC2 * b2 * gam * gam * 1e6;
    double S = 0.0;
    for (int k = 0; k < m.n; k++)
        S += m.w[k] * OG_KAPPA * m.Z[k] / m.A[k] / b2 * (log(tmax_ev / og_ivalue(m.Z[k])) - b2);
    return S;
}

double og_bethe_water(double E, double mp) { return og_bethe(0, E, mp); }

/* Williams' straggling coefficient of the medium, MeV^2 cm^2/g (App. A.2).
 * Readings: the printed 4 pi e^4 is per target electron; times the electrons
 * per gram, N_A Z/A, it is kappa m_e c^2 Z/A (kappa as above); m_e v^2 is
 * the non-relativistic m_e c^2 beta^2; I per element as for the stopping
 * power; compounds by mass fraction.                                        */
double og_williams(int material, double E, double mp)
{
    og_medium m = og_get_medium(material);
    double b2, gam, pc;
    og_kin(E, mp, &b2, &gam, &pc);
    const double x = OG_MEC2 * b2; /* m_e v^2, MeV */
    double T = 0.0;
    for (int k = 0; k < m.n; k++) {
        double I = og_ivalue(m.Z[k]) * 1e-6;
        T += m.w[k] * OG_KAPPA * OG_MEC2 * m.Z[k] / m.A[k] * (1.0 + 4.0 * I / (3.0 * x) * log(2.0 * x / I));
    }
    return T;
}

/* dT/dE of og_williams: with x = m_e c^2 beta^2, d/dx [ln(2x/I)/x] = (1 - ln(2x/I))/x^2 and
 * dx/dE = m_e c^2 * 2 / (gamma^3 m_p).                                      */
double og_williams_deriv(int material, double E, double mp)
{
    og_medium m = og_get_medium(material);
    double b2, gam, pc;
    og_kin(E, mp, &b2, &gam, &pc);
    const double x = OG_MEC2 * b2;
    const double dxdE = OG_MEC2 * 2.0 / (gam * gam * gam * mp);
    double d = 0.0;
    for (int k = 0; k < m.n; k++) {
        double I = og_ivalue(m.Z[k]) * 1e-6;
        d += m.w[k] * OG_KAPPA * OG_MEC2 * m.Z[k] / m.A[k] * (4.0 * I / 3.0) * (1.0 - log(2.0 * x / I)) / (x * x) * dxdE;
    }
    return d;
}

/* Screened-Rutherford momentum-transfer cross section per unit mass of the medium,
 * cm^2/g (App. A.3): per atom 2 pi (z Z e^2/(4 pi eps0 m0 v^2))^2 [ln((eta+1)/eta) - 1/(eta+1)],
 * eta = (Z^(1/3) alpha m_e c / p)^2, times N_A/A atoms per gram, summed by mass fraction.
 * Readings: e^2/(4 pi eps0) = r_e m_e c^2; m0 v^2 is read as p v of the proton in the laboratory
 * frame (relativistic, no reduced-mass factor): the cross section must be per deflection of the
 * proton's own direction, and at small angles the Rutherford law in those variables depends on
 * the momentum transfer and the velocity only, whatever the target mass (the reduced mass belongs
 * to the centre-of-mass angle; for hydrogen it would multiply sigma_tr by 4).                  */
double og_rutherford(int material, double E, double mp)
{
    og_medium m = og_get_medium(material);
    double b2, gam, pc;
    og_kin(E, mp, &b2, &gam, &pc);
    const double pv = pc * pc / (E + mp);
    double s = 0.0;
    for (int k = 0; k < m.n; k++) {
        double r = m.Z[k] * OG_RE * OG_MEC2 / pv;
        double t = cbrt((double)m.Z[k]) * OG_ALPHA * OG_MEC2 / pc;
        double eta = t * t;
        s += m.w[k] * OG_NA / m.A[k] * 2.0 * M_PI * r * r * (log((eta + 1.0) / eta) - 1.0 / (eta + 1.0));
    }
    return s;
}

/* Stopping power used by the tables, clamped at e_floor (R15): the
 * Bragg-Kleeman range R = alpha E^p (cm of water) gives S = dE/dR =
 * 1/(alpha p E^(p-1)); or the Bethe-Bloch form above.                      */
double og_stopping(const og_phys *ph, double E)
{
    double e = E > ph->e_floor ? E : ph->e_floor;
    if (ph->stopping == 1) return og_bethe(ph->material, e, ph->mp);
    return 1.0 / (ph->bk_alpha * ph->bk_p * pow(e, ph->bk_p - 1.0));
}

/* Scattering power used as sigma_tr, clamped: Highland (E_s/pv)^2/X0, or the
 * screened Rutherford form above.                                          */
double og_scatpower(const og_phys *ph, double E)
{
    double e = E > ph->e_floor ? E : ph->e_floor;
    if (ph->scattering == 1) return og_rutherford(ph->material, e, ph->mp);
    double pv = (e * e + 2.0 * e * ph->mp) / (e + ph->mp);
    double r = ph->highland_es / pv;
    return r * r / ph->x0_water;
}

/* Straggling coefficient T (clamped like the other coefficients) and its
 * derivative (zero below the floor, where T is held constant); both 0
 * without straggling.                                                      */
double og_straggle(const og_phys *ph, double E)
{
    if (!ph->straggling) return 0.0;
    return og_williams(ph->material, E > ph->e_floor ? E : ph->e_floor, ph->mp);
}

double og_straggle_deriv(const og_phys *ph, double E)
{
    if (!ph->straggling || E < ph->e_floor) return 0.0;
    return og_williams_deriv(ph->material, E, ph->mp);
}

/* Gauss-Legendre nodes/weights on [-1,1], computed by Newton iteration on
 * the Legendre polynomial (no stored constants).                          */
static void og_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_n(z), p0 = P_{n-1}(z) */
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Angle between the directions (1,u,v) and (1,u',v') -- the paper's
 * arccos(Theta) of App. A.4, evaluated as atan2(|cross|, dot) so that equal
 * directions give exactly zero.                                            */
double og_defl_angle(double u, double v, double up, double vp)
{
    double cx = u * vp - v * up;   /* (1,u,v) x (1,u',v') */
    double cy = v - vp;
    double cz = up - u;
    double cr = sqrt(cx * cx + cy * cy + cz * cz);
    double dt = 1.0 + u * up + v * vp;
    return atan2(cr, dt);
}

/* Energy band of every group for the nuclear kernel: with nuc_bands = 0 all groups use the single
 * parameters (band 0); otherwise each group takes the parameters fitted at the nearest anchor
 * energy (App. A.4 fits them group by group; the anchors stand for its fitting groups).          */
static int og_band(const og_phys *ph, double E)
{
    int b = 0;
    for (int k = 1; k < ph->nuc_bands; k++)
        if (fabs(E - ph->nuc_e[k]) < fabs(E - ph->nuc_e[b])) b = k;
    return b;
}
static double og_band_lambda(const og_phys *ph, int b) { return ph->nuc_bands ? ph->nuc_lambda[b] : ph->lambda_nuc; }
static double og_band_alpha(const og_phys *ph, int b) { return ph->nuc_bands ? ph->nuc_alpha[b] : ph->gamma_a; }
static double og_band_beta(const og_phys *ph, int b) { return ph->nuc_bands ? ph->nuc_beta[b] : ph->gamma_b; }

/*
 * Tables (section 3.2 eq:(appSE) and the definition of sigma_tr,g below
 * eq:(0041-d); App. A.2 for T; App. A.4 for P1, P2).  Arrays are caller-allocated:
 *   E_face[G+1], E_mid[G], dE[G], S_face[G+1], sig_tr[G], kappa[G],
 *   T_face[G+1], Tp_face[G+1]  straggling coefficient and its derivative at the faces,
 *   band[G]  energy band of the nuclear kernel of every group,
 *   P1[G*G]  (P1[gs*G+gd], source group gs -> destination gd <= gs),
 *   P2[NB*NA*NA] (P2[(b*NA+as)*NA+ad], source node as -> destination node ad, band b),
 *            NB = max(1, nuc_bands).
 */
void og_tables(const og_grid *g, const og_phys *ph, double *E_face, double *E_mid, double *dE,
               double *S_face, double *sig_tr, double *kappa, double *T_face, double *Tp_face, int *band,
               double *P1, double *P2)
{
    int G = g->ng;
    double de = (g->e_hi - g->e_lo) / G;
    for (int f = 0; f <= G; f++) E_face[f] = g->e_lo + f * de;
    for (int k = 0; k < G; k++) {
        E_mid[k] = 0.5 * (E_face[k] + E_face[k + 1]);
        dE[k] = E_face[k + 1] - E_face[k];
    }
    for (int f = 0; f <= G; f++) S_face[f] = og_stopping(ph, E_face[f]);
    for (int f = 0; f <= G; f++) {
        T_face[f] = og_straggle(ph, E_face[f]);
        Tp_face[f] = og_straggle_deriv(ph, E_face[f]);
    }

    /* group mean of the scattering power: 8-point Gauss-Legendre */
    double gx[8], gw[8];
    og_gauss_legendre(8, gx, gw);
    for (int k = 0; k < G; k++) {
        double s = 0.0;
        for (int t = 0; t < 8; t++) {
            double E = E_mid[k] + 0.5 * dE[k] * gx[t];
            s += 0.5 * gw[t] * og_scatpower(ph, E);
        }
        sig_tr[k] = s;
    }
    /* group mean of kappa(E) = kappa0 (1 - exp(-E/E_c)), exact integral */
    for (int k = 0; k < G; k++) {
        double a = E_face[k], b = E_face[k + 1];
        kappa[k] = ph->kappa0 * (1.0 - ph->e_c / (b - a) * (exp(-a / ph->e_c) - exp(-b / ph->e_c)));
    }
    for (int k = 0; k < G; k++) band[k] = og_band(ph, E_mid[k]);
    /* P1 (App. A.4): lambda exp(-lambda (E_g' - E_g)), g <= g', with lambda of the source group's
     * band, normalised over destinations for every source group.                              */
    for (int gs = 0; gs < G; gs++) {
        double lam = og_band_lambda(ph, band[gs]);
        double Z = 0.0;
        for (int gd = 0; gd <= gs; gd++) Z += lam * exp(-lam * (E_mid[gs] - E_mid[gd]));
        for (int gd = 0; gd < G; gd++)
            P1[(long)gs * G + gd] = gd <= gs ? lam * exp(-lam * (E_mid[gs] - E_mid[gd])) / Z : 0.0;
    }
    /* P2_b (App. A.4): Gamma law beta^a/Gamma(a) theta^(a-1) exp(-beta theta) of the deflection
     * angle with band b's parameters, normalised over destination nodes.                        */
    long m = og_m(g), NA = og_na(g);
    int NB = ph->nuc_bands > 0 ? ph->nuc_bands : 1;
    for (int b = 0; b < NB; b++) {
        double al = og_band_alpha(ph, b), be = og_band_beta(ph, b);
        double cst = pow(be, al) / tgamma(al);
        double *P = P2 + (long)b * NA * NA;
        for (long as = 0; as < NA; as++) {
            double up = og_theta(g, as / m), vp = og_theta(g, as % m);
            double K = 0.0;
            for (long ad = 0; ad < NA; ad++) {
                double u = og_theta(g, ad / m), v = og_theta(g, ad % m);
                double th = og_defl_angle(u, v, up, vp);
                double f = cst * pow(th, al - 1.0) * exp(-be * th);
                P[as * NA + ad] = f;
                K += f;
            }
            for (long ad = 0; ad < NA; ad++) P[as * NA + ad] /= K;
        }
    }
}

/* ------------------------------------------------------- initial state */
static double og_ncdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }
static double og_npdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }

/*
 * Initial condition: the boundary distribution eq:(bdy) projected onto the
 * grid (R5).  Lateral: cell averages of the Gaussian.  Angle: the
 * mono-directional limit (sigma_u -> 0) is a Kronecker weight 1/dth^2 at the
 * theta = 0 node (nth must be even).  Energy: L2 projection onto the DG-P1
 * basis.  C normalises the discrete total to one proton.
 * psi: one generation, zero-filled by the caller.  Returns 0 or -1.
 */
int og_initial(const og_grid *g, const og_beam *b, const double *E_face, double *psi)
{
    if (g->nth % 2) return -1;
    long m = og_m(g), G = g->ng;
    double dx = og_dx(g), dy = og_dy(g), dth = og_dth(g);
    double *Lx = calloc(g->nx, sizeof(double)), *Ly = calloc(g->ny, sizeof(double));
    double *E1 = calloc(G, sizeof(double)), *E2 = calloc(G, sizeof(double));
    double totx = 0, toty = 0, tote = 0;
    for (int p = 0; p < g->nx; p++) {
        double lo = -g->x_half + p * dx, hi = lo + dx;
        double c = og_ncdf((hi - b->x0) / b->sigma_x) - og_ncdf((lo - b->x0) / b->sigma_x);
        Lx[p] = c / dx;
        totx += c;
    }
    for (int q = 0; q < g->ny; q++) {
        double lo = -g->y_half + q * dy, hi = lo + dy;
        double c = og_ncdf((hi - b->y0) / b->sigma_y) - og_ncdf((lo - b->y0) / b->sigma_y);
        Ly[q] = c / dy;
        toty += c;
    }
    for (long k = 0; k < G; k++) {
        double lo = E_face[k], hi = E_face[k + 1], dE = hi - lo, Em = 0.5 * (lo + hi);
        double za = (lo - b->e0) / b->sigma_e, zb = (hi - b->e0) / b->sigma_e;
        double mass = og_ncdf(zb) - og_ncdf(za);
        /* int (E - E_mid) N(E) dE = sigma (n(za) - n(zb)) + (E0 - E_mid) mass */
        double mom = b->sigma_e * (og_npdf(za) - og_npdf(zb)) + (b->e0 - Em) * mass;
        E1[k] = mass / dE;
        E2[k] = 3.0 / dE * (2.0 / dE) * mom;
        tote += mass;
    }
    double C = 1.0 / (totx * toty * tote);
    long ac = (m / 2) * m + (m / 2);   /* node nth/2 <-> interior index nth/2-1 = m/2 */
    for (long k = 0; k < G; k++)
        for (int p = 0; p < g->nx; p++)
            for (int q = 0; q < g->ny; q++) {
                long pq = (long)p * g->ny + q;
                double lat = C * Lx[p] * Ly[q] / (dth * dth);
                psi[IDX(g, k, 0, ac, pq)] = lat * E1[k];
                psi[IDX(g, k, 1, ac, pq)] = lat * E2[k];
            }
    free(Lx); free(Ly); free(E1); free(E2);
    return 0;
}

/* ------------------------------------------------- energy sub-problem */
/*
 * Semi-discrete energy operator of eq:(0041-d) / L3, L4 in eq:(0041-do)
 * with T = 0, applied to one line X[g] = (psi1, psi2):
 *   psi1 row: rho S+ /dE (psi1_{g+1} - psi2_{g+1}) - rho S- /dE (psi1_g - psi2_g) - sig_ct psi1
 *   psi2 row: 3 rho S+ /dE (psi1_{g+1} - psi2_{g+1}) + 3 rho S- /dE (psi1_g - psi2_g)
 *             - 3 rho (S+ + S-)/dE psi1_g - rho (S+ - S-)/dE psi2_g - sig_ct psi2
 * R1: the lower-face term of the psi2 row carries "+": phi^2 = -1 at the
 * lower face, so the boundary term [(S psi) phi^2] contributes +S- psi-.
 * The upwind face value at E_{g+1/2} is psi1_{g+1} - psi2_{g+1}, and zero
 * above the top group.  sig_ct = rho kappa_g (R8).
 * x1,x2 are strided lines (stride st); out1/out2 likewise.
 */
static void og_energy_rhs_line(long G, const double *S_face, const double *dE, const double *kappa,
                               const double *T_face, const double *Tp_face, double rho, const double *x1,
                               const double *x2, long st, const double *Q, double *o1, double *o2)
{
    for (long k = 0; k < G; k++) {
        double Sp = S_face[k + 1], Sm = S_face[k];
        if (T_face) { /* straggling, first-order part: S + T'/2 (R22) */
            Sp += 0.5 * Tp_face[k + 1];
            Sm += 0.5 * Tp_face[k];
        }
        double fup = (k == G - 1) ? 0.0 : x1[(k + 1) * st] - x2[(k + 1) * st];
        double flo = x1[k * st] - x2[k * st];
        double sct = rho * kappa[k];
        double r1 = rho * Sp / dE[k] * fup - rho * Sm / dE[k] * flo - sct * x1[k * st];
        double r2 = 3.0 * rho * Sp / dE[k] * fup + 3.0 * rho * Sm / dE[k] * flo
                    - 3.0 * rho * (Sp + Sm) / dE[k] * x1[k * st] - rho * (Sp - Sm) / dE[k] * x2[k * st]
                    - sct * x2[k * st];
        if (T_face) {
            /* straggling, second-order part (1/2) d/dE (T d psi/dE) by the symmetric interior
             * penalty method (section 3.2, the Q1 / Q2 terms; R22): T linear in the group from its
             * face values, penalty alpha T_f / h_f on every interior face with alpha = (1+1)^2/2 = 2,
             * h_f the mean width of the two groups; no diffusive flux through the end faces.
             * Rows are the test functions phi^1/dE and 3 phi^2/dE; jump [psi] = psi(below) - psi(above). */
            double Tbar = 0.5 * (T_face[k] + T_face[k + 1]);
            r2 += rho * 0.5 * 3.0 / dE[k] * (-4.0 * Tbar * x2[k * st] / dE[k]);
            if (k + 1 < G) { /* upper face: this group is below it */
                double Tf = T_face[k + 1], hf = 0.5 * (dE[k] + dE[k + 1]), pen = 2.0 * Tf / hf;
                double J = (x1[k * st] + x2[k * st]) - (x1[(k + 1) * st] - x2[(k + 1) * st]);
                double Av = Tf * (x2[k * st] / dE[k] + x2[(k + 1) * st] / dE[k + 1]);
                r1 += rho * 0.5 / dE[k] * (Av - pen * J);
                r2 += rho * 0.5 * 3.0 / dE[k] * (Av + J * Tf / dE[k] - pen * J);
            }
            if (k > 0) { /* lower face: this group is above it */
                double Tf = T_face[k], hf = 0.5 * (dE[k - 1] + dE[k]), pen = 2.0 * Tf / hf;
                double J = (x1[(k - 1) * st] + x2[(k - 1) * st]) - (x1[k * st] - x2[k * st]);
                double Av = Tf * (x2[(k - 1) * st] / dE[k - 1] + x2[k * st] / dE[k]);
                r1 += rho * 0.5 / dE[k] * (-Av + pen * J);
                r2 += rho * 0.5 * 3.0 / dE[k] * (Av + J * Tf / dE[k] - pen * J);
            }
        }
        if (Q) r1 += Q[k * st];
        o1[k * st] = r1;
        o2[k * st] = r2;
    }
}

/* Exposed for tests: RHS of the energy operator on one contiguous line (T_face, Tp_face NULL:
 * no straggling). */
void og_energy_rhs(const og_grid *g, const double *S_face, const double *dE, const double *kappa,
                   const double *T_face, const double *Tp_face, double rho, const double *x1, const double *x2,
                   const double *Q, double *o1, double *o2)
{
    og_energy_rhs_line(g->ng, S_face, dE, kappa, T_face, Tp_face, rho, x1, x2, 1, Q, o1, o2);
}

/* Inverse of a 2x2 matrix (row-major). */
static void og_inv2(const double a[4], double r[4])
{
    double det = a[0] * a[3] - a[1] * a[2];
    r[0] = a[3] / det;
    r[1] = -a[1] / det;
    r[2] = -a[2] / det;
    r[3] = a[0] / det;
}

static void og_mul2(const double a[4], const double b[4], double r[4])
{
    double t[4] = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2],
                   a[2] * b[1] + a[3] * b[3]};
    memcpy(r, t, sizeof(t));
}

/*
 * Crank-Nicolson energy step with straggling (section 3.3 with the full operator of eq:(0041-d)):
 * the operator couples group k to k-1 and k+1, so every line is a block-tridiagonal system
 * (I - h/2 rho D0) X* = X^n + h/2 L(X^n) + h/2 (Q^n + Q*), with D0 the operator at rho = 1 (every
 * term of it is proportional to rho).  The 2x2 blocks of D0 are read off the line operator itself,
 * applied to unit vectors; the system is solved by block elimination from the top group down and
 * back-substitution upwards.
 */
static void og_energy_cn_strag(const og_grid *g, const double *S_face, const double *dE, const double *kappa,
                               const double *T_face, const double *Tp_face, const double *rho, double h,
                               double *psi, const double *Qn, const double *Qs)
{
    long G = g->ng, NA = og_na(g), NP = og_np(g);
    long st = 2 * NA * NP, qst = NA * NP;
    /* blocks of D0: Lo[k] (coupling to k-1), Di[k], Up[k] (coupling to k+1), row-major [row][col] */
    double *Lo = calloc(4 * G, sizeof(double)), *Di = calloc(4 * G, sizeof(double)),
           *Up = calloc(4 * G, sizeof(double));
    double *u1 = calloc(G, sizeof(double)), *u2 = calloc(G, sizeof(double));
    double *o1 = malloc(G * sizeof(double)), *o2 = malloc(G * sizeof(double));
    for (long j = 0; j < G; j++)
        for (int l = 0; l < 2; l++) {
            memset(u1, 0, G * sizeof(double));
            memset(u2, 0, G * sizeof(double));
            (l == 0 ? u1 : u2)[j] = 1.0;
            og_energy_rhs_line(G, S_face, dE, kappa, T_face, Tp_face, 1.0, u1, u2, 1, NULL, o1, o2);
            for (long k = 0; k < G; k++) {
                double *B = (j == k) ? Di + 4 * k : (j == k - 1) ? Lo + 4 * k : (j == k + 1) ? Up + 4 * k : NULL;
                if (!B) continue; /* the operator reaches one group each way only */
                B[0 * 2 + l] = o1[k];
                B[1 * 2 + l] = o2[k];
            }
        }
    free(u1); free(u2); free(o1); free(o2);
#pragma omp parallel
    {
        double *e1 = malloc(G * sizeof(double)), *e2 = malloc(G * sizeof(double));
        double *c1 = malloc(G * sizeof(double)), *c2 = malloc(G * sizeof(double));
        double *bt = malloc(2 * G * sizeof(double)), *Dt = malloc(4 * G * sizeof(double));
#pragma omp for schedule(static)
        for (long line = 0; line < NA * NP; line++) {
            long a = line / NP, pq = line % NP;
            double r = rho[pq], c = 0.5 * h * r;
            double *x1 = psi + IDX(g, 0, 0, a, pq);
            double *x2 = psi + IDX(g, 0, 1, a, pq);
            for (long k = 0; k < G; k++) { /* the line, contiguous */
                c1[k] = x1[k * st];
                c2[k] = x2[k * st];
            }
            og_energy_rhs_line(G, S_face, dE, kappa, T_face, Tp_face, r, c1, c2, 1, NULL, e1, e2);
            /* elimination from the top: Dt_k = M_k - U_k Dt_{k+1}^-1 L_{k+1}, bt_k = b_k - U_k Dt_{k+1}^-1 bt_{k+1},
             * with M = I - c D0_kk, U = -c Up, L = -c Lo                                                    */
            for (long k = G - 1; k >= 0; k--) {
                double b1 = x1[k * st] + 0.5 * h * e1[k], b2 = x2[k * st] + 0.5 * h * e2[k];
                if (Qn) b1 += 0.5 * h * Qn[a * NP + pq + k * qst];
                if (Qs) b1 += 0.5 * h * Qs[a * NP + pq + k * qst];
                double M[4] = {1.0 - c * Di[4 * k], -c * Di[4 * k + 1], -c * Di[4 * k + 2], 1.0 - c * Di[4 * k + 3]};
                if (k + 1 < G) {
                    double U[4] = {-c * Up[4 * k], -c * Up[4 * k + 1], -c * Up[4 * k + 2], -c * Up[4 * k + 3]};
                    double L1[4] = {-c * Lo[4 * (k + 1)], -c * Lo[4 * (k + 1) + 1], -c * Lo[4 * (k + 1) + 2],
                                    -c * Lo[4 * (k + 1) + 3]};
                    double Di1[4], UDi[4], UDL[4];
                    og_inv2(Dt + 4 * (k + 1), Di1);
                    og_mul2(U, Di1, UDi);
                    og_mul2(UDi, L1, UDL);
                    for (int q = 0; q < 4; q++) M[q] -= UDL[q];
                    b1 -= UDi[0] * bt[2 * (k + 1)] + UDi[1] * bt[2 * (k + 1) + 1];
                    b2 -= UDi[2] * bt[2 * (k + 1)] + UDi[3] * bt[2 * (k + 1) + 1];
                }
                memcpy(Dt + 4 * k, M, sizeof(M));
                bt[2 * k] = b1;
                bt[2 * k + 1] = b2;
            }
            /* back-substitution upwards: X_k = Dt_k^-1 (bt_k - L_k X_{k-1}) */
            double y1p = 0.0, y2p = 0.0;
            for (long k = 0; k < G; k++) {
                double b1 = bt[2 * k], b2 = bt[2 * k + 1];
                if (k > 0) {
                    b1 += c * (Lo[4 * k] * y1p + Lo[4 * k + 1] * y2p);
                    b2 += c * (Lo[4 * k + 2] * y1p + Lo[4 * k + 3] * y2p);
                }
                double Dinv[4];
                og_inv2(Dt + 4 * k, Dinv);
                double y1 = Dinv[0] * b1 + Dinv[1] * b2, y2 = Dinv[2] * b1 + Dinv[3] * b2;
                x1[k * st] = y1;
                x2[k * st] = y2;
                y1p = y1;
                y2p = y2;
            }
        }
        free(e1); free(e2); free(c1); free(c2); free(bt); free(Dt);
    }
    free(Lo); free(Di); free(Up);
}

/*
 * Crank-Nicolson step of length h of the energy sub-system (section 3.3,
 * the E half-steps of the Strang sequence) for every line (a, pq) of one
 * generation, in place:
 *   X* - X^n = h/2 [ L(X*) + Q* + L(X^n) + Q^n ]
 * The implicit system is block lower-bidiagonal in g (group g couples only
 * to g+1), so it is solved group by group from the top: for each g the 2x2
 * system (I - h/2 D_g) X*_g = X^n_g + h/2 L(X^n)_g + h/2 (coupling to the
 * already known X*_{g+1}) + h/2 (Q^n_g + Q*_g) is solved by Cramer's rule.
 * Qn, Qs: sources of the psi1 row [g][a][pq] (already multiplied by rho),
 * or NULL.  rho: [pq].  With straggling (T_face non-NULL) the system is
 * block-tridiagonal and og_energy_cn_strag solves it.
 */
void og_energy_cn(const og_grid *g, const double *S_face, const double *dE, const double *kappa,
                  const double *T_face, const double *Tp_face, const double *rho, double h, double *psi,
                  const double *Qn, const double *Qs)
{
    if (T_face) {
        og_energy_cn_strag(g, S_face, dE, kappa, T_face, Tp_face, rho, h, psi, Qn, Qs);
        return;
    }
    long G = g->ng, NA = og_na(g), NP = og_np(g);
    long st = 2 * NA * NP; /* stride between groups along a line */
#pragma omp parallel for schedule(static)
    for (long line = 0; line < NA * NP; line++) {
        long a = line / NP, pq = line % NP;
        double r = rho[pq];
        double *x1 = psi + IDX(g, 0, 0, a, pq);
        double *x2 = psi + IDX(g, 0, 1, a, pq);
        const double *qn = Qn ? Qn + a * NP + pq : NULL;
        const double *qs = Qs ? Qs + a * NP + pq : NULL;
        long qst = NA * NP;
        /* explicit part L(X^n) of every group */
        double *e1 = malloc(G * sizeof(double)), *e2 = malloc(G * sizeof(double));
        for (long k = 0; k < G; k++) {
            double Sp = S_face[k + 1], Sm = S_face[k];
            double fup = (k == G - 1) ? 0.0 : x1[(k + 1) * st] - x2[(k + 1) * st];
            double flo = x1[k * st] - x2[k * st];
            double sct = r * kappa[k];
            e1[k] = r * Sp / dE[k] * fup - r * Sm / dE[k] * flo - sct * x1[k * st];
            e2[k] = 3.0 * r * Sp / dE[k] * fup + 3.0 * r * Sm / dE[k] * flo
                    - 3.0 * r * (Sp + Sm) / dE[k] * x1[k * st] - r * (Sp - Sm) / dE[k] * x2[k * st]
                    - sct * x2[k * st];
        }
        double fnew_up = 0.0; /* psi1* - psi2* of group g+1 (zero above G) */
        for (long k = G - 1; k >= 0; k--) {
            double Sp = S_face[k + 1], Sm = S_face[k];
            double sct = r * kappa[k];
            /* D_g: the part of L acting on X_g itself */
            double d11 = -r * Sm / dE[k] - sct, d12 = r * Sm / dE[k];
            double d21 = 3.0 * r * Sm / dE[k] - 3.0 * r * (Sp + Sm) / dE[k];
            double d22 = -3.0 * r * Sm / dE[k] - r * (Sp - Sm) / dE[k] - sct;
            double b1 = x1[k * st] + 0.5 * h * e1[k] + 0.5 * h * (r * Sp / dE[k]) * fnew_up;
            double b2 = x2[k * st] + 0.5 * h * e2[k] + 0.5 * h * (3.0 * r * Sp / dE[k]) * fnew_up;
            if (qn) b1 += 0.5 * h * qn[k * qst];
            if (qs) b1 += 0.5 * h * qs[k * qst];
            double m11 = 1.0 - 0.5 * h * d11, m12 = -0.5 * h * d12;
            double m21 = -0.5 * h * d21, m22 = 1.0 - 0.5 * h * d22;
            double det = m11 * m22 - m12 * m21;
            double y1 = (b1 * m22 - m12 * b2) / det;
            double y2 = (m11 * b2 - m21 * b1) / det;
            x1[k * st] = y1;
            x2[k * st] = y2;
            fnew_up = y1 - y2;
        }
        free(e1);
        free(e2);
    }
}

/* Energy content of one line per unit angle-area and lateral area:
 * sum_g int E psi dE = sum_g dE (E_g psi1 + dE psi2 / 6).                  */
static double og_ecnt_line(long G, const double *E_mid, const double *dE, const double *x1, const double *x2,
                           long st)
{
    double s = 0.0;
    for (long k = 0; k < G; k++) s += dE[k] * (E_mid[k] * x1[k * st] + dE[k] * x2[k * st] / 6.0);
    return s;
}

/* Energy content per voxel (MeV): sum over lines of one state into out[pq]
 * (overwritten).                                                           */
void og_energy_content(const og_grid *g, const double *E_mid, const double *dE, const double *psi, double *out)
{
    long NA = og_na(g), NP = og_np(g), st = 2 * NA * NP;
    double w = og_dth(g) * og_dth(g) * og_dx(g) * og_dy(g);
#pragma omp parallel for schedule(static)
    for (long pq = 0; pq < NP; pq++) {
        double s = 0.0;
        for (long a = 0; a < NA; a++)
            s += og_ecnt_line(g->ng, E_mid, dE, psi + IDX(g, 0, 0, a, pq), psi + IDX(g, 0, 1, a, pq), st);
        out[pq] = s * w;
    }
}

/* Proton number per voxel: sum_g dE psi1 times the cell measure. */
void og_number_content(const og_grid *g, const double *dE, const double *psi, double *out)
{
    long NA = og_na(g), NP = og_np(g);
    double w = og_dth(g) * og_dth(g) * og_dx(g) * og_dy(g);
#pragma omp parallel for schedule(static)
    for (long pq = 0; pq < NP; pq++) {
        double s = 0.0;
        for (long a = 0; a < NA; a++)
            for (long k = 0; k < g->ng; k++) s += dE[k] * psi[IDX(g, k, 0, a, pq)];
        out[pq] = s * w;
    }
}

/* ------------------------------------------------ catastrophic source */
/*
 * Source of generation k from generation k-1 (Remark after the Strang
 * scheme, eqn:(pri-se2), and the factorised kernel of section 4 / App. A.4):
 *   Q_g(a) = rho * sum_{a'} P2_g[a' -> a] sum_{g' >= g} P1[g' -> g] kappa_{g'} psi1_{g'}(a') dE_{g'}/dE_g
 * sigma_{c,s} uses the removal cross section of the source group (R10), P2_g
 * is the angular law of the destination group g's band (App. A.4: "in the
 * energy group g"), a discrete probability over destination nodes, which
 * absorbs the du dv factor of the paper's quadrature.  The psi2 row gets no
 * source.  prev: generation k-1 state; Q: [g][a][pq]; P2: [band][a'][a];
 * band: [G] (NULL: every group band 0).
 */
void og_source(const og_grid *g, const double *dE, const double *kappa, const double *P1, const double *P2,
               const int *band, const double *rho, const double *prev, double *Q)
{
    long G = g->ng, NA = og_na(g), NP = og_np(g);
    double *V = malloc((size_t)G * NA * NP * sizeof(double));
    /* energy sum (for every source node a' and voxel); every voxel's terms are added in the order
     * g' = g, g+1, ..., the voxels of one (a', g) run side by side */
#pragma omp parallel for schedule(static)
    for (long apk = 0; apk < NA * G; apk++) {
        long ap = apk / G, k = apk % G;
        double *s = V + (k * NA + ap) * NP;
        for (long pq = 0; pq < NP; pq++) s[pq] = 0.0;
        for (long ks = k; ks < G; ks++) {
            double c = P1[ks * G + k] * kappa[ks];
            const double *x = prev + IDX(g, ks, 0, ap, 0);
            for (long pq = 0; pq < NP; pq++) s[pq] += c * x[pq] * dE[ks] / dE[k];
        }
    }
    /* angular sum: terms added in the order a' = 0, 1, ... for every voxel */
#pragma omp parallel
    {
        double *s = malloc(NP * sizeof(double));
#pragma omp for schedule(static)
        for (long ka = 0; ka < G * NA; ka++) {
            long k = ka / NA, a = ka % NA;
            const double *P = P2 + (long)(band ? band[k] : 0) * NA * NA;
            for (long pq = 0; pq < NP; pq++) s[pq] = 0.0;
            for (long ap = 0; ap < NA; ap++) {
                double c = P[ap * NA + a];
                const double *v = V + (k * NA + ap) * NP;
                for (long pq = 0; pq < NP; pq++) s[pq] += c * v[pq];
            }
            for (long pq = 0; pq < NP; pq++) Q[(k * NA + a) * NP + pq] = rho[pq] * s[pq];
        }
        free(s);
    }
    free(V);
}

/* ---------------------------------------------- lateral transport step */
/* Superbee limiter of section 3.4: max[0, min(2 th, 1), min(th, 2)].     */
double og_superbee(double th)
{
    double a = fmin(2.0 * th, 1.0), b = fmin(th, 2.0);
    double r = a > b ? a : b;
    return r > 0.0 ? r : 0.0;
}

/* Limited face slope delta = Dface * eta(Dup / Dface) (section 3.4), with
 * the ratio taken from the upwind side (R6) and delta = 0 when Dface = 0.  */
static double og_slope(double d_up, double d_face)
{
    if (d_face == 0.0) return 0.0;
    return d_face * og_superbee(d_up / d_face);
}

/*
 * One Crank-Nicolson step of length h of the lateral transport sub-system
 * eq:(distansport) on one (p,q) plane with velocities (cx, cy), in place.
 * MUSCL fluxes Psi = c+ psi^L - c- psi^R, psi^L = psi_p + delta/2,
 * psi^R = psi_{p+1} - delta/2 (R2: the q-face uses psi_{p,q+1}).  Slopes are
 * frozen at psi^n in both halves of the CN average (Remark after
 * eq:(distansport)), so the implicit part is the first-order upwind
 * operator, solved by a sweep from the upwind corner.  Two ghost layers of
 * zeros surround the plane (zero inflow).  work: (nx+4)*(ny+4) doubles.
 */
static void og_transport_plane(int nx, int ny, double dx, double dy, double cx, double cy, double h,
                               double *pl, double *work)
{
    int W = ny + 4;
#define GH(p, q) work[((p) + 2) * W + (q) + 2]
    memset(work, 0, sizeof(double) * (nx + 4) * W);
    for (int p = 0; p < nx; p++)
        for (int q = 0; q < ny; q++) GH(p, q) = pl[p * ny + q];
    double cxp = cx > 0 ? cx : 0, cxm = cx < 0 ? -cx : 0;
    double cyp = cy > 0 ? cy : 0, cym = cy < 0 ? -cy : 0;
    /* explicit part: R = psi^n - h/2 div(Psi(psi^n)) - h/2 div(slope part) */
    double *R = malloc(sizeof(double) * nx * ny);
    for (int p = 0; p < nx; p++)
        for (int q = 0; q < ny; q++) {
            double F[2], Gf[2];
            for (int s = 0; s < 2; s++) {
                int pl_ = p - 1 + s; /* face between pl_ and pl_+1 */
                double dface = GH(pl_ + 1, q) - GH(pl_, q);
                double dup = cx >= 0 ? GH(pl_, q) - GH(pl_ - 1, q) : GH(pl_ + 2, q) - GH(pl_ + 1, q);
                double del = og_slope(dup, dface);
                double L = GH(pl_, q) + 0.5 * del, Rr = GH(pl_ + 1, q) - 0.5 * del;
                F[s] = cxp * L - cxm * Rr;
            }
            for (int s = 0; s < 2; s++) {
                int ql = q - 1 + s;
                double dface = GH(p, ql + 1) - GH(p, ql);
                double dup = cy >= 0 ? GH(p, ql) - GH(p, ql - 1) : GH(p, ql + 2) - GH(p, ql + 1);
                double del = og_slope(dup, dface);
                double L = GH(p, ql) + 0.5 * del, Rr = GH(p, ql + 1) - 0.5 * del;
                Gf[s] = cyp * L - cym * Rr;
            }
            double divn = (F[1] - F[0]) / dx + (Gf[1] - Gf[0]) / dy;
            /* the slope (frozen) part of the implicit flux: Psi - Psi_upwind */
            double Fu0 = cxp * GH(p - 1, q) - cxm * GH(p, q), Fu1 = cxp * GH(p, q) - cxm * GH(p + 1, q);
            double Gu0 = cyp * GH(p, q - 1) - cym * GH(p, q), Gu1 = cyp * GH(p, q) - cym * GH(p, q + 1);
            double divu = (Fu1 - Fu0) / dx + (Gu1 - Gu0) / dy;
            double divc = divn - divu;
            R[p * ny + q] = GH(p, q) - 0.5 * h * divn - 0.5 * h * divc;
        }
    /* implicit upwind sweep: (1 + h/2(|cx|/dx + |cy|/dy)) psi*_pq
     *   - h/2 [(cx+ psi*_{p-1} + cx- psi*_{p+1})/dx + (cy+ psi*_{q-1} + cy- psi*_{q+1})/dy] = R */
    memset(work, 0, sizeof(double) * (nx + 4) * W);
    double diag = 1.0 + 0.5 * h * (fabs(cx) / dx + fabs(cy) / dy);
    for (int pp = 0; pp < nx; pp++) {
        int p = cx >= 0 ? pp : nx - 1 - pp;
        for (int qq = 0; qq < ny; qq++) {
            int q = cy >= 0 ? qq : ny - 1 - qq;
            double nb = (cxp * GH(p - 1, q) + cxm * GH(p + 1, q)) / dx + (cyp * GH(p, q - 1) + cym * GH(p, q + 1)) / dy;
            GH(p, q) = (R[p * ny + q] + 0.5 * h * nb) / diag;
        }
    }
    for (int p = 0; p < nx; p++)
        for (int q = 0; q < ny; q++) pl[p * ny + q] = GH(p, q);
    free(R);
#undef GH
}

/* T half-step of length h on every plane (g, l, a) of one generation. */
void og_transport_cn(const og_grid *g, double h, double *psi)
{
    long G = g->ng, NA = og_na(g), NP = og_np(g), m = og_m(g);
    double dx = og_dx(g), dy = og_dy(g);
#pragma omp parallel
    {
        double *work = malloc(sizeof(double) * (g->nx + 4) * (g->ny + 4));
#pragma omp for schedule(static)
        for (long pl = 0; pl < G * 2 * NA; pl++) {
            long a = pl % NA;
            double cx = og_theta(g, a / m), cy = og_theta(g, a % m);
            og_transport_plane(g->nx, g->ny, dx, dy, cx, cy, h, psi + pl * NP, work);
        }
        free(work);
    }
}

/* Exposed for tests: one plane. */
void og_transport_plane_api(int nx, int ny, double dx, double dy, double cx, double cy, double h, double *pl)
{
    double *work = malloc(sizeof(double) * (nx + 4) * (ny + 4));
    og_transport_plane(nx, ny, dx, dy, cx, cy, h, pl, work);
    free(work);
}

/* ------------------------------------------------ angular diffusion step */
/*
 * Crank-Nicolson step of length h of eq:(sd) (section 3.4): 5-point
 * Laplacian on the interior nodes, zero at nodes 0 and nth, diagonalised by
 * the discrete sine series eq:(eqn_fly):
 *   hat = sum_{i,j} psi_ij sin(pi i' m/N) sin(pi j' n/N)   (i' = i+1, N = nth)
 *   hat *= (1 + h/2 D lam_mn)/(1 - h/2 D lam_mn),
 *   lam_mn = (2cos(pi m/N) - 2)/dth^2 + (2cos(pi n/N) - 2)/dth^2,
 *   D = rho sigma_tr,g / 2,
 *   psi = (2/N)^2 sum_{m,n} hat sin sin.
 * Applied to every (g, l, pq) of one generation in place.
 */
void og_angular_cn(const og_grid *g, const double *sig_tr, const double *rho, double h, double *psi)
{
    long G = g->ng, NA = og_na(g), NP = og_np(g), m = og_m(g);
    int N = g->nth;
    double dth = og_dth(g);
    double *S = malloc(sizeof(double) * m * m);
    for (long i = 0; i < m; i++)
        for (long k = 0; k < m; k++) S[i * m + k] = sin(M_PI * (double)(i + 1) * (double)(k + 1) / N);
    double *lam = malloc(sizeof(double) * m);
    for (long k = 0; k < m; k++) lam[k] = (2.0 * cos(M_PI * (double)(k + 1) / N) - 2.0) / (dth * dth);
#pragma omp parallel
    {
        double *x = malloc(sizeof(double) * NA), *t = malloc(sizeof(double) * NA), *hat = malloc(sizeof(double) * NA);
#pragma omp for schedule(static)
        for (long col = 0; col < G * 2 * NP; col++) {
            long k = col / (2 * NP), l = (col / NP) % 2, pq = col % NP;
            double D = rho[pq] * sig_tr[k] / 2.0;
            for (long a = 0; a < NA; a++) x[a] = psi[IDX(g, k, l, a, pq)];
            /* forward: hat_mn = sum_i S_im sum_j S_jn x_ij */
            for (long i = 0; i < m; i++)
                for (long n = 0; n < m; n++) {
                    double s = 0;
                    for (long j = 0; j < m; j++) s += x[i * m + j] * S[j * m + n];
                    t[i * m + n] = s;
                }
            for (long mm = 0; mm < m; mm++)
                for (long n = 0; n < m; n++) {
                    double s = 0;
                    for (long i = 0; i < m; i++) s += S[i * m + mm] * t[i * m + n];
                    double lmn = lam[mm] + lam[n];
                    hat[mm * m + n] = s * (1.0 + 0.5 * h * D * lmn) / (1.0 - 0.5 * h * D * lmn);
                }
            /* inverse: x_ij = (2/N)^2 sum_m S_im sum_n S_jn hat_mn */
            for (long mm = 0; mm < m; mm++)
                for (long j = 0; j < m; j++) {
                    double s = 0;
                    for (long n = 0; n < m; n++) s += hat[mm * m + n] * S[j * m + n];
                    t[mm * m + j] = s;
                }
            double sc = (2.0 / N) * (2.0 / N);
            for (long i = 0; i < m; i++)
                for (long j = 0; j < m; j++) {
                    double s = 0;
                    for (long mm = 0; mm < m; mm++) s += S[i * m + mm] * t[mm * m + j];
                    psi[IDX(g, k, l, i * m + j, pq)] = sc * s;
                }
        }
        free(x); free(t); free(hat);
    }
    free(S);
    free(lam);
}

/* ------------------------------------------------------------ the march */
/* Every table of one configuration (as og_tables fills them); T_face and Tp_face are NULL
 * without straggling. */
typedef struct {
    const double *E_face, *E_mid, *dE, *S_face, *sig_tr, *kappa, *T_face, *Tp_face;
    const int *band;
    const double *P1, *P2;
} og_tab;

/*
 * One E half-step (length h) for all generations k = 0..K in order (the
 * scattering decomposition eqn:(pri-se), section 3.1): generation k >= 1
 * receives the trapezoidal source (Q^n + Q*)/2 built from generation k-1
 * before and after the same half-step (R13).  The deposited energy is the
 * decrease of the energy content of every generation over the energy
 * sub-step, source included (the energy-flux difference of eq:(en_d)
 * applied to each species, summed; R14), accumulated into dep[pq] (MeV).
 */
static void og_energy_all_rec(const og_grid *g, const og_tab *t, const double *rho, double h, double *state,
                              double *dep, double *dep0, double *inj);

static void og_energy_all(const og_grid *g, const og_tab *t, const double *rho, double h, double *state,
                          double *dep)
{
    og_energy_all_rec(g, t, rho, h, state, dep, NULL, NULL);
}

/* As og_energy_all; when non-NULL, dep0 also receives the deposit of generation 0 alone and inj the
 * energy the source puts into generation 1 over the sub-step: the source term of the CN step,
 * (h/2)(Q^n + Q*), enters the psi^1 row only, so its energy is (h/2) sum_g dE_g E_g (Q^n + Q*)_g
 * times the cell measure (the energy-content functional of og_ecnt_line applied to it).     */
static void og_energy_all_rec(const og_grid *g, const og_tab *t, const double *rho, double h, double *state,
                              double *dep, double *dep0, double *inj)
{
    long E = og_gen_elems(g), NP = og_np(g), NA = og_na(g), G = g->ng;
    double *before = malloc(sizeof(double) * E);
    double *Qn = NULL, *Qs = NULL;
    if (g->ngen > 1) {
        Qn = malloc(sizeof(double) * G * NA * NP);
        Qs = malloc(sizeof(double) * G * NA * NP);
    }
    double *e0 = malloc(sizeof(double) * NP), *e1 = malloc(sizeof(double) * NP);
    for (int k = 0; k < g->ngen; k++) {
        double *cur = state + (long)k * E;
        if (k >= 1) {
            /* before = gen k-1 at entry (saved below), cur-1 = gen k-1 after */
            og_source(g, t->dE, t->kappa, t->P1, t->P2, t->band, rho, before, Qn);
            og_source(g, t->dE, t->kappa, t->P1, t->P2, t->band, rho, state + (long)(k - 1) * E, Qs);
        }
        og_energy_content(g, t->E_mid, t->dE, cur, e0);
        memcpy(before, cur, sizeof(double) * E);
        og_energy_cn(g, t->S_face, t->dE, t->kappa, t->T_face, t->Tp_face, rho, h, cur, k >= 1 ? Qn : NULL,
                     k >= 1 ? Qs : NULL);
        og_energy_content(g, t->E_mid, t->dE, cur, e1);
        for (long pq = 0; pq < NP; pq++) dep[pq] += e0[pq] - e1[pq];
        if (dep0 && k == 0)
            for (long pq = 0; pq < NP; pq++) dep0[pq] += e0[pq] - e1[pq];
        if (inj && k == 1) {
            double w = og_dth(g) * og_dth(g) * og_dx(g) * og_dy(g);
            for (long pq = 0; pq < NP; pq++) {
                double s = 0.0;
                for (long kk = 0; kk < G; kk++)
                    for (long a = 0; a < NA; a++) {
                        long o = (kk * NA + a) * NP + pq;
                        s += t->dE[kk] * t->E_mid[kk] * (Qn[o] + Qs[o]);
                    }
                inj[pq] += 0.5 * h * s * w;
            }
        }
    }
    free(before); free(Qn); free(Qs); free(e0); free(e1);
}

/*
 * Full march (section 3.3, Strang splitting): for every depth step s with
 * rho = rho[s] (voxel layer [s dz, (s+1) dz]):
 *   E(dz/2) -> T(dz/2) -> A(dz) -> T(dz/2) -> E(dz/2)
 * Each sub-step runs over all generations.  dose[s][pq] (MeV/g per
 * incident proton) = deposited energy / (rho dx dy dz).
 * state: ngen generations; on entry generation 0 holds the initial state,
 * the others zero; on exit the state after the last step.
 */
/* One Strang step of length h (section 3.3) with the densities r; the deposit is added to dep. */
static void og_strang(const og_grid *g, const og_tab *t, const double *r, double h, double *state, double *dep)
{
    long E = og_gen_elems(g);
    og_energy_all(g, t, r, 0.5 * h, state, dep);
    for (int k = 0; k < g->ngen; k++) og_transport_cn(g, 0.5 * h, state + k * E);
    for (int k = 0; k < g->ngen; k++) og_angular_cn(g, t->sig_tr, r, h, state + k * E);
    for (int k = 0; k < g->ngen; k++) og_transport_cn(g, 0.5 * h, state + k * E);
    og_energy_all(g, t, r, 0.5 * h, state, dep);
}

void og_run(const og_grid *g, const og_tab *tp, const double *rho, double *state, double *dose)
{
    og_tab t = *tp;
    long NP = og_np(g);
    double dz = g->dz, vol = og_dx(g) * og_dy(g) * g->dz;
    double *dep = malloc(sizeof(double) * NP);
    for (int s = 0; s < g->nz; s++) {
        const double *r = rho + (long)s * NP;
        memset(dep, 0, sizeof(double) * NP);
        og_strang(g, &t, r, dz, state, dep);
        for (long pq = 0; pq < NP; pq++) dose[(long)s * NP + pq] = dep[pq] / (r[pq] * vol);
    }
    free(dep);
}

/*
 * Higher-order splitting in depth (section 5 names higher-order splitting as the extension): Richardson
 * extrapolation of the Strang step.  For every layer s, from the state psi_n,
 *   A = S(dz) psi_n,   B = S(dz/2) S(dz/2) psi_n,   psi_{n+1} = (4 B - A) / 3,
 * and the layer's deposit is combined with the same weights.  The Strang step is symmetric (its error
 * expansion has even powers of dz only when its sub-steps are linear), so the combination cancels the
 * dz^2 term: fourth order in depth for a linear step, with only positive sub-steps (a triple-jump
 * composition would need a negative depth step, which the diffusion in angle and energy cannot take).
 * The weights sum to one, so number and energy balances are kept.
 */
void og_run_extrapolated(const og_grid *g, const og_tab *tp, const double *rho, double *state, double *dose)
{
    og_tab t = *tp;
    long E = og_gen_elems(g) * g->ngen, NP = og_np(g);
    double dz = g->dz, vol = og_dx(g) * og_dy(g) * g->dz;
    double *depA = malloc(sizeof(double) * NP), *depB = malloc(sizeof(double) * NP);
    double *A = malloc(sizeof(double) * E);
    for (int s = 0; s < g->nz; s++) {
        const double *r = rho + (long)s * NP;
        memset(depA, 0, sizeof(double) * NP);
        memset(depB, 0, sizeof(double) * NP);
        memcpy(A, state, sizeof(double) * E);
        og_strang(g, &t, r, dz, A, depA);
        og_strang(g, &t, r, 0.5 * dz, state, depB);
        og_strang(g, &t, r, 0.5 * dz, state, depB);
        for (long i = 0; i < E; i++) state[i] = (4.0 * state[i] - A[i]) / 3.0;
        for (long pq = 0; pq < NP; pq++) dose[(long)s * NP + pq] = (4.0 * depB[pq] - depA[pq]) / 3.0 / (r[pq] * vol);
    }
    free(depA);
    free(depB);
    free(A);
}

/*
 * og_run with per-layer records for the surrogate of generation 1 (ngen = 2), rec [4][nz][NP]:
 *   0: energy injected into generation 1 by the source over both E half-steps of layer s,
 *   1, 2: energy and number content of generation 0 after the first E half-step of layer s,
 *   3: deposit of generation 0 alone in layer s (MeV).
 */
void og_run_records(const og_grid *g, const og_tab *tp, const double *rho, double *state, double *dose,
                    double *rec)
{
    og_tab t = *tp;
    const double *sig_tr = t.sig_tr, *E_mid = t.E_mid, *dE = t.dE;
    long E = og_gen_elems(g), NP = og_np(g), L = (long)g->nz * NP;
    double dz = g->dz, vol = og_dx(g) * og_dy(g) * g->dz;
    double *dep = malloc(sizeof(double) * NP);
    memset(rec, 0, sizeof(double) * 4 * L);
    for (int s = 0; s < g->nz; s++) {
        const double *r = rho + (long)s * NP;
        double *inj = rec + (long)s * NP, *me = rec + L + (long)s * NP, *mn = rec + 2 * L + (long)s * NP;
        double *d0 = rec + 3 * L + (long)s * NP;
        memset(dep, 0, sizeof(double) * NP);
        og_energy_all_rec(g, &t, r, 0.5 * dz, state, dep, d0, inj);
        og_energy_content(g, E_mid, dE, state, me);
        og_number_content(g, dE, state, mn);
        for (int k = 0; k < g->ngen; k++) og_transport_cn(g, 0.5 * dz, state + k * E);
        for (int k = 0; k < g->ngen; k++) og_angular_cn(g, sig_tr, r, dz, state + k * E);
        for (int k = 0; k < g->ngen; k++) og_transport_cn(g, 0.5 * dz, state + k * E);
        og_energy_all_rec(g, &t, r, 0.5 * dz, state, dep, d0, inj);
        for (long pq = 0; pq < NP; pq++) dose[(long)s * NP + pq] = dep[pq] / (r[pq] * vol);
    }
    free(dep);
}

/* Exposed for tests: one E half-step over all generations with deposit. */
void og_energy_all_api(const og_grid *g, const og_tab *t, const double *rho, double h, double *state, double *dep)
{
    og_energy_all(g, t, rho, h, state, dep);
}
