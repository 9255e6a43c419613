// libpbsplit host side: context, FP64 tables, workspace carving, the depth march schedule and
// the C ABI declared in include/pbsplit.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pbs_common.h"
#include "pbs_ctx.h"
#include "pbs_net_internal.h"

// The depth march runs on two streams (a generation's T A T beside the energy chain) when one
// generation holds fewer phase-space cells than this: such kernels leave most of the GPU idle (a 32 x 32
// beam with 15 x 15 angles and 128 groups: +11 % beams/s), while at 64 x 64 cells, 31 x 31 angles, 128
// groups and 4 generations every kernel already saturates HBM and the concurrent ones mostly slow each other
// (1 % per step gained, every kernel 1.4-2.6x longer), so there the sub-steps stay in order on one stream
// and each kernel's own rate stays measurable.
#ifndef PBS_OVERLAP_CELLS
#define PBS_OVERLAP_CELLS 100000000L
#endif
#include "pbsplit.h"

using namespace pbs;

namespace {


// 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun, table 25.4).
const double GL8_X[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
const double GL8_W[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace pbs {
namespace {
unsigned short bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
double bf16_val(unsigned short h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}
}  // namespace

// The transfer matrix for the split-BF16 source product, [3][Mp][Kpb] zero-padded, row = destination:
// hi = bf16(P2), lo = bf16(P2 - hi), and a single-BF16 copy whose columns keep their exact sums (the
// number of re-emitted protons of one source node): every entry lies between two neighbouring BF16
// values and starts at the nearer one; entries are then moved to their other neighbour, each at most
// once, in the order that costs the least extra rounding error relative to the entry (the ones whose
// value lies closest to the midpoint first), while each move brings the column sum closer to its exact
// total.  Every entry stays within one BF16 ulp of its value.  Without the compensation the rounding
// of this fixed table would bias the number of re-emitted protons the same way in every cell and group.
void transfer_table_bf16(const std::vector<double> &P2T, int NA, int Mp, int Kpb, std::vector<unsigned short> &out)
{
    const size_t MK = (size_t)Mp * Kpb;
    out.assign(3 * MK, 0);
    for (int a = 0; a < NA; ++a)
        for (int k = 0; k < NA; ++k) {
            const double x = P2T[(size_t)a * NA + k];
            const unsigned short hi = bf16_rne((float)x);
            out[(size_t)a * Kpb + k] = hi;
            out[MK + (size_t)a * Kpb + k] = bf16_rne((float)(x - bf16_val(hi)));
            out[2 * MK + (size_t)a * Kpb + k] = hi;
        }
    struct Move {
        double cost, step;
        int a;
        unsigned short to;
    };
    std::vector<Move> mv;
    std::vector<char> used(NA);
    for (int k = 0; k < NA; ++k) {
        double target = 0.0, cur = 0.0;
        for (int a = 0; a < NA; ++a) {
            target += P2T[(size_t)a * NA + k];
            cur += bf16_val(out[2 * MK + (size_t)a * Kpb + k]);
        }
        double r = target - cur;
        std::fill(used.begin(), used.end(), 0);
        // rounds of moves in the direction of the residual; a move that overshoots flips the direction
        for (int round = 0; round < 64 && std::fabs(r) > 1e-7 * std::fabs(target); ++round) {
            mv.clear();
            const bool up = r > 0;
            for (int a = 0; a < NA; ++a) {
                if (used[a]) continue;
                const double x = P2T[(size_t)a * NA + k];
                const unsigned short h = out[2 * MK + (size_t)a * Kpb + k];
                const double v = bf16_val(h);
                if (!(x > 0.0) || !(v > 0.0)) continue;
                const unsigned short hn = up ? (unsigned short)(h + 1) : (unsigned short)(h - 1);
                const double vn = bf16_val(hn);
                if (!(vn > 0.0) || !std::isfinite(vn)) continue;
                if (up ? !(vn >= x) : !(vn <= x)) continue;   // x must lie between v and its other neighbour
                mv.push_back({(std::fabs(vn - x) - std::fabs(v - x)) / x, vn - v, a, hn});
            }
            std::sort(mv.begin(), mv.end(), [](const Move &p, const Move &q) { return p.cost < q.cost; });
            bool moved = false;
            for (const Move &m : mv) {
                if (!(std::fabs(r - m.step) < std::fabs(r))) continue;
                out[2 * MK + (size_t)m.a * Kpb + k] = m.to;
                used[m.a] = 1;
                r -= m.step;
                moved = true;
                if ((r > 0) != up || !(std::fabs(r) > 1e-7 * std::fabs(target))) break;
            }
            if (!moved) break;
        }
    }
}

// nth = 32: the 31-point sine transform split by mode parity, [(mat*4 + s)*64 + lane] =
// A_mat[perm(lane % 16)][4 s + lane / 16] for mat = Sodd, Seven and A_mat[4 s + lane / 16][perm(lane % 16)]
// for mat = Sodd^T, Seven^T, perm(4 g + q) = 4 q + g (the row order that keeps the angular pass's LDS
// stores free of bank conflicts).
// nth = 16: the dense 15-point transform zero-padded to 16 x 16, [s*64 + lane] = S[lane % 16][4 s + lane / 16].
void apass_mfma_table(int nth, float *t)
{
    for (int i = 0; i < 1024; ++i) t[i] = 0.f;
    if (nth == 32) {
        auto sodd = [](int r, int i) { return std::sin(M_PI * (2 * r + 1) * (i + 1) / 32.0); };
        auto seven = [](int r, int i) { return (r < 15 && i < 15) ? std::sin(M_PI * 2 * (r + 1) * (i + 1) / 32.0) : 0.0; };
        for (int s = 0; s < 4; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 4 * (lane % 4) + (lane % 16) / 4, k = 4 * s + lane / 16;
                t[(0 * 4 + s) * 64 + lane] = (float)sodd(row, k);
                t[(1 * 4 + s) * 64 + lane] = (float)seven(row, k);
                t[(2 * 4 + s) * 64 + lane] = (float)sodd(k, row);
                t[(3 * 4 + s) * 64 + lane] = (float)seven(k, row);
            }
    } else if (nth == 16) {
        for (int s = 0; s < 4; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 4 * (lane % 4) + (lane % 16) / 4, k = 4 * s + lane / 16;
                t[s * 64 + lane] = (row < 15 && k < 15) ? (float)std::sin(M_PI * (row + 1) * (k + 1) / 16.0) : 0.f;
            }
    }
}
}  // namespace pbs


namespace {

pbs_status fail(pbs_ctx *c, pbs_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

pbs_status hip_fail(pbs_ctx *c, hipError_t e, const char *what)
{
    return fail(c, PBS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                                   \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) return hip_fail((c), e_, #expr);            \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

// ------------------------------------------------------------------------------ host tables
// Media by weight fraction of their elements (Z, standard atomic weight A in g/mol): water as H2O, bone
// and air as the material table of section 4 prints them.
struct Medium {
    int n;
    int Z[9];
    double A[9], w[9];
};

Medium medium(int material)
{
    Medium m{};
    if (material == PBS_MAT_BONE) {
        const int Z[9] = {1, 6, 7, 8, 11, 12, 15, 16, 20};
        const double A[9] = {1.008, 12.011, 14.007, 15.999, 22.990, 24.305, 30.974, 32.06, 40.078};
        const double w[9] = {0.042, 0.194, 0.040, 0.425, 0.001, 0.002, 0.092, 0.003, 0.201};
        m.n = 9;
        for (int k = 0; k < 9; ++k) m.Z[k] = Z[k], m.A[k] = A[k], m.w[k] = w[k];
    } else if (material == PBS_MAT_AIR) {
        const int Z[4] = {6, 7, 8, 18};
        const double A[4] = {12.011, 14.007, 15.999, 39.948};
        const double w[4] = {0.0001248, 0.7553, 0.2318, 0.01283};
        m.n = 4;
        for (int k = 0; k < 4; ++k) m.Z[k] = Z[k], m.A[k] = A[k], m.w[k] = w[k];
    } else {
        constexpr double A_H = 1.008, A_O = 15.999;
        const double mol = 2.0 * A_H + A_O;
        m.n = 2;
        m.Z[0] = 1, m.A[0] = A_H, m.w[0] = 2.0 * A_H / mol;
        m.Z[1] = 8, m.A[1] = A_O, m.w[1] = A_O / mol;
    }
    return m;
}

// mean excitation energy of element Z (eV), the piecewise fit of App. A.1
double i_value(int Z) { return Z == 1 ? 19.0 : Z <= 13 ? 11.2 + 11.7 * Z : 52.8 + 8.71 * Z; }

constexpr double K_BB = 0.307075;          // 4 pi N_A r_e^2 m_e c^2, MeV cm^2 / mol
constexpr double ME_C2 = 0.51099895;       // MeV
constexpr double AVOGADRO = 6.02214076e23; // 1/mol
constexpr double R_ELECTRON = 2.8179403262e-13;   // cm
constexpr double FINE_ALPHA = 1.0 / 137.035999084;

// Bethe-Bloch mass stopping power of a medium (App. A.1), MeV cm^2/g: per element the heavy-projectile
// form K (Z/A) / beta^2 [ln(2 m_e c^2 beta^2 gamma^2 / I) - beta^2] without the density term, I(Z) from the
// appendix's fit, and the medium as the mass-fraction sum of its elements.
double bethe(int material, double e, double mp)
{
    const Medium M = medium(material);
    const double gamma = 1.0 + e / mp;
    const double beta2 = 1.0 - 1.0 / (gamma * gamma);
    const double wmax_ev = 2.0 * ME_C2 * beta2 * gamma * gamma * 1.0e6;
    double s = 0.0;
    for (int k = 0; k < M.n; ++k)
        s += M.w[k] * K_BB * (M.Z[k] / M.A[k]) / beta2 * (std::log(wmax_ev / i_value(M.Z[k])) - beta2);
    return s;
}

// Williams' straggling coefficient of a medium (App. A.2), MeV^2 cm^2/g, and its energy derivative:
// per element K m_e c^2 (Z/A) [1 + 4 I/(3 x) ln(2 x / I)] with x = m_e v^2 = m_e c^2 beta^2 (non-relativistic,
// as printed) and I in MeV; d/dE uses d/dx [ln(2x/I)/x] = (1 - ln(2x/I))/x^2 and dx/dE = 2 m_e c^2/(gamma^3 m_p).
void williams(int material, double e, double mp, double *T, double *dT)
{
    const Medium M = medium(material);
    const double gamma = 1.0 + e / mp;
    const double x = ME_C2 * (1.0 - 1.0 / (gamma * gamma));
    const double dx = 2.0 * ME_C2 / (gamma * gamma * gamma * mp);
    double t = 0.0, d = 0.0;
    for (int k = 0; k < M.n; ++k) {
        const double I = i_value(M.Z[k]) * 1e-6, c = M.w[k] * K_BB * ME_C2 * M.Z[k] / M.A[k];
        const double lg = std::log(2.0 * x / I);
        t += c * (1.0 + 4.0 * I / (3.0 * x) * lg);
        d += c * (4.0 * I / 3.0) * (1.0 - lg) / (x * x) * dx;
    }
    *T = t;
    *dT = d;
}

// Screened-Rutherford momentum-transfer cross section per unit mass of a medium (App. A.3), cm^2/g: per
// atom 2 pi (Z e^2 / (4 pi eps0 p v))^2 [ln((eta + 1)/eta) - 1/(eta + 1)], eta = (Z^(1/3) alpha m_e c / p)^2,
// with e^2/(4 pi eps0) = r_e m_e c^2 and p v of the proton in the laboratory frame; N_A/A atoms per gram.
double rutherford(int material, double e, double mp)
{
    const Medium M = medium(material);
    const double pc = std::sqrt(e * (e + 2.0 * mp)), pv = pc * pc / (e + mp);
    double s = 0.0;
    for (int k = 0; k < M.n; ++k) {
        const double r = M.Z[k] * R_ELECTRON * ME_C2 / pv;
        const double t = std::cbrt((double)M.Z[k]) * FINE_ALPHA * ME_C2 / pc, eta = t * t;
        s += M.w[k] * (AVOGADRO / M.A[k]) * 2.0 * M_PI * r * r * (std::log((eta + 1.0) / eta) - 1.0 / (eta + 1.0));
    }
    return s;
}

double stopping_power(const pbs_physics &ph, double E)
{
    const double e = std::max(E, ph.e_floor);
    if (ph.stopping == PBS_STOP_BETHE) return bethe(ph.material, e, ph.mp);
    return 1.0 / (ph.bk_alpha * ph.bk_p * std::pow(e, ph.bk_p - 1.0));
}

double scattering_power(const pbs_physics &ph, double E)
{
    const double e = std::max(E, ph.e_floor);
    if (ph.scattering == PBS_SCAT_RUTHERFORD) return rutherford(ph.material, e, ph.mp);
    const double pc2 = e * (e + 2.0 * ph.mp);           // (pc)^2
    const double pv = pc2 / (e + ph.mp);                // p v = (pc)^2 / total energy
    const double r = ph.highland_es / pv;
    return r * r / ph.x0_water;
}

// straggling coefficient at max(E, e_floor) and its derivative (0 below the floor, where T is held)
void straggle(const pbs_physics &ph, double E, double *T, double *dT)
{
    *T = *dT = 0.0;
    if (!ph.straggling) return;
    double t, d;
    williams(ph.material, std::max(E, ph.e_floor), ph.mp, &t, &d);
    *T = t;
    *dT = E < ph.e_floor ? 0.0 : d;
}

// angle between (1,u,v) and (1,u',v'), stable near zero
double deflection(double u, double v, double up, double vp)
{
    const double c0 = u * vp - v * up, c1 = v - vp, c2 = up - u;
    return std::atan2(std::sqrt(c0 * c0 + c1 * c1 + c2 * c2), 1.0 + u * up + v * vp);
}

// The energy operator with straggling, rho = 1, as 2x2 blocks per group g (rows psi1, psi2 of g; columns
// psi1, psi2 of the coupled group): Lo couples g to g-1, Di to itself, Up to g+1.
//  * first-order part: the stopping term of eq:(0041-d) with S + T'/2 at the faces (the (1/2) d/dE (T' psi)
//    half of the straggling operator), upwind values from the group above; removal -kappa_g;
//  * second-order part (1/2) d/dE (T dpsi/dE), symmetric interior penalty on the DG-P1 basis: T linear in
//    the group, {T psi'} and [psi] = psi(below) - psi(above) on interior faces, penalty 2 T_f / h_f (alpha =
//    (1+1)^2/2, h_f the mean width of the two groups), no flux through the end faces; rows tested with
//    phi^1 / dE and 3 phi^2 / dE.
// Deposit weights: the energy rate of a line is sum_g w_g . (D0 X)_g with w_g = (dE E_g, dE^2/6); the
// deposit functional is its negative, a weight per (group, coefficient) collected column by column.
void straggling_tables(pbs_ctx *c)
{
    const int G = c->G();
    const pbs_physics &ph = c->ph;
    std::vector<double> T(G + 1), Tp(G + 1), S(G + 1);
    for (int f = 0; f <= G; ++f) {
        straggle(ph, c->E_face[f], &T[f], &Tp[f]);
        S[f] = c->S_face[f] + 0.5 * Tp[f];
    }
    c->blk.assign((size_t)G * 12, 0.0);
    for (int g = 0; g < G; ++g) {
        double *Lo = &c->blk[(size_t)g * 12], *Di = Lo + 4, *Up = Lo + 8;
        const double d = c->dE[g], sm = S[g] / d, sp = S[g + 1] / d, kp = c->kappa[g];
        Di[0] = -(sm + kp), Di[1] = sm, Di[2] = -3.0 * sp, Di[3] = -(sp + 2.0 * sm + kp);
        if (g + 1 < G) Up[0] = sp, Up[1] = -sp, Up[2] = 3.0 * sp, Up[3] = -3.0 * sp;
        const double Tbar = 0.5 * (T[g] + T[g + 1]);
        Di[3] += -6.0 * Tbar / (d * d);
        if (g + 1 < G) {   // upper face
            const double Tf = T[g + 1], du = c->dE[g + 1], pen = 2.0 * Tf / (0.5 * (d + du)), q = Tf / d - pen;
            Di[0] += -pen / (2 * d), Di[1] += (Tf / d - pen) / (2 * d);
            Up[0] += pen / (2 * d), Up[1] += (Tf / du - pen) / (2 * d);
            Di[2] += 3 * q / (2 * d), Di[3] += 3 * (Tf / d + q) / (2 * d);
            Up[2] += -3 * q / (2 * d), Up[3] += 3 * (Tf / du + q) / (2 * d);
        }
        if (g > 0) {       // lower face
            const double Tf = T[g], dl = c->dE[g - 1], pen = 2.0 * Tf / (0.5 * (dl + d)), q = Tf / d - pen;
            Lo[0] += pen / (2 * d), Lo[1] += (-Tf / dl + pen) / (2 * d);
            Di[0] += -pen / (2 * d), Di[1] += (-Tf / d + pen) / (2 * d);
            Lo[2] += 3 * q / (2 * d), Lo[3] += 3 * (Tf / dl + q) / (2 * d);
            Di[2] += -3 * q / (2 * d), Di[3] += 3 * (Tf / d + q) / (2 * d);
        }
    }
    c->dA2.assign(G, 0.0);
    c->dB2.assign(G, 0.0);
    for (int j = 0; j < G; ++j)
        for (int col = 0; col < 2; ++col) {
            double r = 0.0;
            for (int g = std::max(0, j - 1); g <= std::min(G - 1, j + 1); ++g) {
                const double *B = &c->blk[(size_t)g * 12 + (g == j ? 4 : g == j + 1 ? 0 : 8)];
                r += c->dE[g] * c->E_mid[g] * B[col] + c->dE[g] * c->dE[g] / 6.0 * B[2 + col];
            }
            (col == 0 ? c->dA2 : c->dB2)[j] = -r;
        }
}

void build_tables(pbs_ctx *c)
{
    const pbs_grid &g = c->g;
    const pbs_physics &ph = c->ph;
    const int G = g.ng, m = c->m, N = g.nth, NA = c->NA;
    c->E_face.resize(G + 1);
    c->E_mid.resize(G);
    c->dE.resize(G);
    for (int f = 0; f <= G; ++f) c->E_face[f] = g.e_lo + (g.e_hi - g.e_lo) * f / G;
    for (int k = 0; k < G; ++k) {
        c->E_mid[k] = 0.5 * (c->E_face[k] + c->E_face[k + 1]);
        c->dE[k] = c->E_face[k + 1] - c->E_face[k];
    }
    c->S_face.resize(G + 1);
    for (int f = 0; f <= G; ++f) c->S_face[f] = stopping_power(ph, c->E_face[f]);
    c->sig_tr.assign(G, 0.0);
    c->kappa.assign(G, 0.0);
    for (int k = 0; k < G; ++k) {
        double s = 0;
        for (int t = 0; t < 4; ++t)
            for (int sgn = -1; sgn <= 1; sgn += 2)
                s += 0.5 * GL8_W[t] * scattering_power(ph, c->E_mid[k] + sgn * 0.5 * c->dE[k] * GL8_X[t]);
        c->sig_tr[k] = s;
        const double a = c->E_face[k], b = c->E_face[k + 1];
        // mean of kappa0 (1 - exp(-E/e_c)) over [a, b]
        c->kappa[k] = ph.kappa0 * (1.0 - ph.e_c * (std::exp(-a / ph.e_c) - std::exp(-b / ph.e_c)) / (b - a));
    }
    c->Sm.resize(G);
    c->Sp.resize(G);
    c->invdE.resize(G);
    for (int k = 0; k < G; ++k) {
        c->Sm[k] = c->S_face[k] / c->dE[k];
        c->Sp[k] = c->S_face[k + 1] / c->dE[k];
        c->invdE[k] = 1.0 / c->dE[k];
    }
    // nuclear bands: each group takes the parameters of the nearest anchor energy (one band without them)
    c->NB = ph.nuc_bands > 0 ? ph.nuc_bands : 1;
    c->band.assign(G, 0);
    for (int k = 0; k < G; ++k)
        for (int b = 1; b < ph.nuc_bands; ++b)
            if (std::fabs(c->E_mid[k] - ph.nuc_e[b]) < std::fabs(c->E_mid[k] - ph.nuc_e[c->band[k]])) c->band[k] = b;
    auto lam_of = [&](int b) { return ph.nuc_bands ? ph.nuc_lambda[b] : ph.lambda_nuc; };
    // re-emission energy law lambda exp(-lambda (E_g' - E_g)) with the source group's lambda, normalised per
    // source group g': W_g = (1/dE_g) U_g, U_g = sum over bands b of U^b_g,
    // U^b_g = [band(g) = b] wc_g psi1_g + wdecb[b][g] U^b_{g+1}
    c->wc.resize(G);
    c->wdec.resize(G);
    c->wdecb.assign((size_t)c->NB * G, 0.0);
    for (int k = 0; k < G; ++k) {
        const double lk = lam_of(c->band[k]);
        double Z = 0;
        for (int j = 0; j <= k; ++j) Z += std::exp(-lk * (c->E_mid[k] - c->E_mid[j]));
        c->wc[k] = c->kappa[k] * c->dE[k] / Z;
        for (int b = 0; b < c->NB; ++b)
            c->wdecb[(size_t)b * G + k] = k + 1 < G ? std::exp(-lam_of(b) * (c->E_mid[k + 1] - c->E_mid[k])) : 0.0;
        c->wdec[k] = c->wdecb[k];
    }
    // deposit functional: -(energy rate of the rho-free energy operator)
    c->dA.resize(G);
    c->dB.resize(G);
    c->dInj.resize(G);
    for (int k = 0; k < G; ++k) {
        const double Sbar = 0.5 * (c->S_face[k] + c->S_face[k + 1]);
        const double dS = c->S_face[k + 1] - c->S_face[k];
        c->dA[k] = c->dE[k] * (Sbar + c->kappa[k] * c->E_mid[k]);
        c->dB[k] = c->dE[k] * (dS + c->kappa[k] * c->dE[k]) / 6.0;
        c->dInj[k] = c->dE[k] * c->E_mid[k];
    }
    c->dBot = c->S_face[0] * c->E_face[0];
    // angular tables
    c->theta.resize(m);
    for (int i = 0; i < m; ++i) c->theta[i] = -g.th_half + (i + 1) * c->dth;
    c->sinS.resize((size_t)m * m);
    for (int M = 1; M < N; ++M)
        for (int n = 1; n < N; ++n) c->sinS[(size_t)(M - 1) * m + (n - 1)] = std::sin(M_PI * M * n / N);
    c->lam.resize(m);
    for (int M = 1; M < N; ++M) c->lam[M - 1] = (2.0 * std::cos(M_PI * M / N) - 2.0) / (c->dth * c->dth);
    // nuclear angular transfer per band: Gamma law of the deflection angle, normalised over destinations
    c->P2T.assign((size_t)c->NB * NA * NA, 0.0);
    std::vector<double> row(NA);
    for (int b = 0; b < c->NB; ++b) {
        const double ga = ph.nuc_bands ? ph.nuc_alpha[b] : ph.gamma_a, gb = ph.nuc_bands ? ph.nuc_beta[b] : ph.gamma_b;
        const double cst = std::pow(gb, ga) / std::tgamma(ga);
        double *P = c->P2T.data() + (size_t)b * NA * NA;
        for (int src = 0; src < NA; ++src) {
            const double up = c->theta[src / m], vp = c->theta[src % m];
            double K = 0;
            for (int dst = 0; dst < NA; ++dst) {
                const double th = deflection(c->theta[dst / m], c->theta[dst % m], up, vp);
                row[dst] = cst * std::pow(th, ga - 1.0) * std::exp(-gb * th);
                K += row[dst];
            }
            for (int dst = 0; dst < NA; ++dst) P[(size_t)dst * NA + src] = row[dst] / K;
        }
    }
    // straggling (section 3.2, App. A.2): rho-free blocks of the whole energy operator per group and the
    // deposit weights of the functional -(energy rate)
    c->strag = ph.straggling != 0;
    if (c->strag) straggling_tables(c);
}

void layout(pbs_ctx *c)
{
    const size_t T = c->tsz;
    const int G = c->G(), K1 = c->g.ngen;
    size_t o = 0;
    c->o_psi = o;
    o = align256(o + (size_t)K1 * G * 2 * c->NLINE * T);
    c->o_W = c->o_Q = o;
    if (K1 > 1) {
        c->o_W = o;
        const size_t wf = (size_t)2 * G * c->NLINE * T;
        const size_t wb = (size_t)2 * 2 * G * c->NPB * c->NOCT * PBS_PT * 8 * sizeof(unsigned short);
        c->Wb_half = (size_t)2 * G * c->NPB * c->NOCT * PBS_PT * 8;
        o = align256(o + std::max(wf, c->Kpb > 0 ? wb : (size_t)0));
        c->o_Q = o;
        o = align256(o + (size_t)2 * G * c->NLINE * T);
    }
    c->o_dep = o;
    o = align256(o + (size_t)2 * K1 * c->NLINE * sizeof(double));
    c->o_edep = o;
    o = align256(o + (size_t)(c->g.nz + 2) * c->NP * sizeof(double));   // + 2 scratch rows (order 4)
    c->o_x0 = c->o_xA = o;
    if (c->order == 4) {
        const size_t st = (size_t)K1 * G * 2 * c->NLINE * T;
        c->o_x0 = o;
        o = align256(o + st);
        c->o_xA = o;
        o = align256(o + st);
    }
    c->o_dout = o;
    o = align256(o + (size_t)c->g.nz * c->NP * sizeof(double));
    c->o_rhoT = o;
    o = align256(o + (size_t)c->g.nz * c->NPpad * T);
    c->o_rhoD = o;
    o = align256(o + (size_t)c->g.nz * c->NP * sizeof(double));
    if (c->sur) {
        const size_t slab = (size_t)c->g.nz * c->NP;
        c->o_fl = o;
        o = align256(o + (size_t)4 * c->NLINE * sizeof(double));
        c->o_frec = o;
        o = align256(o + 4 * slab * sizeof(double));
        c->o_scal = o;
        o = align256(o + 16 * sizeof(double));
        if (c->sur == 2) {
            c->o_sx = o;
            o = align256(o + slab * NET_CX * 2);
            c->o_sy = o;
            o = align256(o + slab * sizeof(float));
            c->o_sa = o;
            o = align256(o + slab * NET_CH * 2);
            c->o_sb = o;
            o = align256(o + slab * NET_CH * 2);
            c->o_spk = o;
            o = align256(o + net_packed_bytes());
            c->o_smaster = o;
            o = align256(o + net_param_count() * sizeof(float));
        }
    }
    // T tables
    size_t e = 0;
    c->t_Sm = e; e += G;
    c->t_Sp = e; e += G;
    c->t_kap = e; e += G;
    c->t_wc = e; e += G;
    c->t_wdec = e; e += G;
    c->t_invdE = e; e += G;
    c->t_sig = e; e += G;
    c->t_theta = e; e += c->m;
    c->t_S = e; e += (size_t)c->m * c->m;
    c->t_lam = e; e += c->m;
    c->t_P2T = e; e += (size_t)c->NB * c->NA * c->NA;
    e = (e + 63) / 64 * 64;   // vector loads of the padded tables need 256-byte alignment
    c->t_P2p = e; e += (size_t)c->NB * c->Kp * c->Mp;
    e = (e + 63) / 64 * 64;
    c->t_K32 = e; e += 1024;
    c->t_wdecb = e; e += (size_t)c->NB * G;
    c->t_blk = e; e += c->strag ? (size_t)12 * G : 0;
    c->t_count = e;
    c->o_tabT = o;
    o = align256(o + e * T);
    size_t d = 0;
    c->d_A = d; d += G;
    c->d_B = d; d += G;
    c->d_Inj = d; d += G;
    c->d_E1 = d; d += G;
    c->d_E2 = d; d += G;
    c->d_lat = d; d += c->NP;
    c->d_A2 = d; d += G;
    c->d_B2 = d; d += G;
    c->d_wmom = d; d += 3 * G;
    c->d_count = d;
    c->o_tabD = o;
    o = align256(o + d * sizeof(double));
    c->o_bf = o;
    if (c->Kpb > 0) o = align256(o + (size_t)c->NB * 3 * c->Mp * c->Kpb * sizeof(unsigned short));
    c->o_band = o;
    o = align256(o + (size_t)G * sizeof(int));
    c->o_sfac = o;
    if (c->strag) o = align256(o + (size_t)2 * G * 8 * c->NPpad * T);
    c->total = o;
}

template <typename T>
pbs_status upload_tables(pbs_ctx *c)
{
    std::vector<T> t(c->t_count);
    auto put = [&](size_t off, const std::vector<double> &v) {
        for (size_t i = 0; i < v.size(); ++i) t[off + i] = (T)v[i];
    };
    put(c->t_Sm, c->Sm);
    put(c->t_Sp, c->Sp);
    put(c->t_kap, c->kappa);
    put(c->t_wc, c->wc);
    put(c->t_wdec, c->wdec);
    put(c->t_invdE, c->invdE);
    put(c->t_sig, c->sig_tr);
    put(c->t_theta, c->theta);
    put(c->t_S, c->sinS);
    put(c->t_lam, c->lam);
    put(c->t_P2T, c->P2T);
    put(c->t_wdecb, c->wdecb);
    if (c->strag) put(c->t_blk, c->blk);
    // zero-padded, source-major copy for the MFMA product: P2p[b][k][a] = P2T[b][a][k]
    const size_t NA2 = (size_t)c->NA * c->NA, KM = (size_t)c->Kp * c->Mp;
    for (int b = 0; b < c->NB; ++b)
        for (int k = 0; k < c->Kp; ++k)
            for (int a = 0; a < c->Mp; ++a)
                t[c->t_P2p + b * KM + (size_t)k * c->Mp + a] =
                    (k < c->NA && a < c->NA) ? (T)c->P2T[b * NA2 + (size_t)a * c->NA + k] : T(0);
    // MFMA operand constants of the angular pass (nth = 16, 32)
    if (c->g.nth == 16 || c->g.nth == 32) {
        std::vector<float> kt(1024);
        apass_mfma_table(c->g.nth, kt.data());
        for (int i = 0; i < 1024; ++i) t[c->t_K32 + i] = (T)kt[i];
    }
    std::vector<double> d(c->d_count, 0.0);
    std::memcpy(&d[c->d_A], c->dA.data(), c->G() * sizeof(double));
    std::memcpy(&d[c->d_B], c->dB.data(), c->G() * sizeof(double));
    std::memcpy(&d[c->d_Inj], c->dInj.data(), c->G() * sizeof(double));
    for (int k = 0; k < c->G(); ++k) {
        d[c->d_wmom + k] = c->E_mid[k] * c->dE[k];
        d[c->d_wmom + c->G() + k] = c->dE[k];
        d[c->d_wmom + 2 * c->G() + k] = c->dE[k] * c->dE[k] / 6.0;
    }
    if (c->strag) {
        std::memcpy(&d[c->d_A2], c->dA2.data(), c->G() * sizeof(double));
        std::memcpy(&d[c->d_B2], c->dB2.data(), c->G() * sizeof(double));
    }
    std::vector<unsigned short> bf, bfb;
    if (c->Kpb > 0) {
        // one [3][Mp][Kpb] split table per band
        const size_t per = (size_t)3 * c->Mp * c->Kpb;
        bf.resize(c->NB * per);
        for (int b = 0; b < c->NB; ++b) {
            std::vector<double> P(c->P2T.begin() + (size_t)b * NA2, c->P2T.begin() + (size_t)(b + 1) * NA2);
            transfer_table_bf16(P, c->NA, c->Mp, c->Kpb, bfb);
            std::copy(bfb.begin(), bfb.end(), bf.begin() + b * per);
        }
        HIPCHK(c, hipMemcpyAsync(c->ws + c->o_bf, bf.data(), bf.size() * sizeof(unsigned short), hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->ws + c->o_band, c->band.data(), c->band.size() * sizeof(int), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->tabT<T>(), t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->tabD(), d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PBS_OK;
}

// event pair around one launch of kind `kind` while profiling is on
struct ProfScope {
    pbs_ctx *c;
    int kind;
    hipStream_t st;
    size_t i0 = 0;
    bool on = false;
    ProfScope(pbs_ctx *c_, int k, hipStream_t st_ = nullptr) : c(c_), kind(k), st(st_ ? st_ : c_->stream)
    {
        if (!c->prof) return;
        while (c->ev_pool.size() < c->ev_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            c->ev_pool.push_back(e);
        }
        i0 = c->ev_used;
        c->ev_used += 2;
        on = hipEventRecord(c->ev_pool[i0], st) == hipSuccess;
    }
    ~ProfScope()
    {
        if (!on) return;
        if (hipEventRecord(c->ev_pool[i0 + 1], st) == hipSuccess) c->ev_pairs.push_back({kind, i0});
    }
};

// ---------------------------------------------------------------------------- march schedule
// The single-product BF16 source product stores its result Q in BF16 too (halving the source traffic of
// the product and of the energy pass that reads it); every other mode keeps Q in the working precision.
// Only the split-BF16 energy pass reads the BF16 form, so straggling (its own energy pass) keeps FP32.
bool source_bf16(const pbs_ctx *c)
{
    return c->tsz == 4 && c->Kpb > 0 && c->src_mode == PBS_SRC_BF16X1 && !c->strag;
}

template <typename T>
EParams<T> eparams(pbs_ctx *c, int k, int lay_c, int lay_o, double h)
{
    EParams<T> P;
    T *tb = c->tabT<T>();
    double *db = c->tabD();
    P.psi = c->psi<T>(k);
    P.Q = (k > 0) ? c->Q<T>() : nullptr;
    P.Qb = (k > 0 && source_bf16(c)) ? reinterpret_cast<const unsigned short *>(c->Q<T>()) : nullptr;
    P.W = (k + 1 < c->kact) ? c->W<T>() : nullptr;
    P.Wh = P.Wl = nullptr;
    P.NOCT = c->NOCT;
    if (P.W && c->Kpb > 0 && c->src_mode != PBS_SRC_FP32) {
        P.Wh = reinterpret_cast<unsigned short *>(c->ws + c->o_W);
        P.Wl = c->src_mode == PBS_SRC_BF16X3 ? P.Wh + c->Wb_half : nullptr;
    }
    P.rho_c = lay_c >= 0 ? c->rhoT<T>(lay_c) : nullptr;
    P.rho_o = lay_o >= 0 ? c->rhoT<T>(lay_o) : nullptr;
    P.dep_c = c->dep(0, k);
    P.dep_o = c->dep(1, k);
    P.Sm = tb + c->t_Sm;
    P.Sp = tb + c->t_Sp;
    P.kap = tb + c->t_kap;
    P.wc = tb + c->t_wc;
    P.wdec = tb + c->t_wdec;
    P.invdE = tb + c->t_invdE;
    P.dA = db + c->d_A;
    P.dB = db + c->d_B;
    P.dInj = db + c->d_Inj;
    P.dBot = c->dBot;
    P.scale = c->dth * c->dth * c->dx * c->dy;
    P.h = (T)h;
    P.G = c->G();
    P.NLINE = c->NLINE;
    P.NAPT = (long)c->NA * PBS_PT;
    P.NB = c->NB;
    P.band = reinterpret_cast<const int *>(c->ws + c->o_band);
    P.wdecb = tb + c->t_wdecb;
    if (c->strag) {
        P.blk = tb + c->t_blk;
        P.sfac_c = reinterpret_cast<T *>(c->ws + c->o_sfac);
        P.sfac_o = P.sfac_c + (size_t)c->G() * 8 * c->NPpad;
        P.dA2 = db + c->d_A2;
        P.dB2 = db + c->d_B2;
    }
    P.NPpad = c->NPpad;
    if (c->feat_on && k == 0) {
        P.inj_c = c->fline(0);
        P.inj_o = c->fline(1);
        P.mom_e = c->fline(2);
        P.mom_n = c->fline(3);
        P.wmom = db + c->d_wmom;
    }
    return P;
}

// Transport and angular sub-steps over all generations (k < 0) or generation k alone, on the context's
// stream or on st.
template <typename T>
pbs_status transport(pbs_ctx *c, double h, int k = -1, hipStream_t st = nullptr);
template <typename T>
pbs_status angular(pbs_ctx *c, int layer, double h, int k = -1, hipStream_t st = nullptr);

// Energy half-step(s) for all generations in order.  mode: close the layer lay_c (state 0 -> 1),
// open the layer lay_o (state 1 -> 2), or both in one sweep.  Deposits go to the FP64 dose.
//
// With tat_layer >= 0 (a depth step), generation k's T(h) A(2h) T(h) is issued on the side stream as soon
// as its energy pass is done: it touches only that generation's fluence, while the main stream goes on
// with k's source product and the later generations' energy passes.  A generation's next energy pass
// waits for its pending T A T; the march joins the side stream back at its end (join_side).
template <typename T>
pbs_status energy_chain(pbs_ctx *c, int mode, int lay_c, int lay_o, double h, int tat_layer = -1, int row_c = -1,
                        int row_o = -1)
{
    // deposits go to the dose rows of the layers unless other rows are named (the extrapolated march)
    if (row_c < 0) row_c = lay_c;
    if (row_o < 0) row_o = lay_o;
    const int K1 = c->kact;
    // FP32 with the split-BF16 product: octet-per-thread E-pass, deposits summed per octet
    bool e8 = false;
    if constexpr (sizeof(T) == 4) e8 = c->Kpb > 0 && c->src_mode != PBS_SRC_FP32 && !c->strag;
    const int nslot = e8 ? epass8_slots(c->NOCT) : c->NA;
    for (int k = 0; k < K1; ++k) {
        EParams<T> P = eparams<T>(c, k, (mode & MODE_CLOSE) ? lay_c : -1, (mode & MODE_OPEN) ? lay_o : -1, h);
        if (c->tat_pend[k]) {
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_tat[k], 0));
            c->tat_pend[k] = false;
        }
        {
            ProfScope ps(c, PBS_K_EPASS);
            if (c->strag) {
                HIPCHK(c, launch_epass_strag<T>(P, mode, c->stream));
            } else if constexpr (sizeof(T) == 4) {
                if (e8) {
                    HIPCHK(c, launch_epass8(P, mode, c->stream));
                } else {
                    HIPCHK(c, launch_epass<T>(P, mode, c->stream));
                }
            } else {
                HIPCHK(c, launch_epass<T>(P, mode, c->stream));
            }
        }
        if (tat_layer >= 0) {
            HIPCHK(c, hipEventRecord(c->ev_e[k], c->stream));
            HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_e[k], 0));
            pbs_status r;
            if ((r = transport<T>(c, h, k, c->side)) != PBS_OK) return r;
            if ((r = angular<T>(c, tat_layer, 2 * h, k, c->side)) != PBS_OK) return r;
            if ((r = transport<T>(c, h, k, c->side)) != PBS_OK) return r;
            HIPCHK(c, hipEventRecord(c->ev_tat[k], c->side));
            c->tat_pend[k] = true;
        }
        if (k + 1 < K1) {
            QParams<T> Q;
            Q.P2T = c->tabT<T>() + c->t_P2T;
            Q.W = c->W<T>();
            Q.Q = c->Q<T>();
            Q.Qb = source_bf16(c) ? reinterpret_cast<unsigned short *>(c->Q<T>()) : nullptr;
            Q.NA = c->NA;
            Q.NPB = c->NPB;
            Q.G = c->G();
            Q.NLINE = c->NLINE;
            Q.P2p = c->Kp > 0 ? c->tabT<T>() + c->t_P2p : nullptr;
            Q.Kp = c->Kp;
            Q.Mp = c->Mp;
            Q.NOCT = c->NOCT;
            Q.Bh = reinterpret_cast<const unsigned short *>(c->ws + c->o_W);
            Q.Bl = Q.Bh + c->Wb_half;
            Q.s0 = (mode == MODE_OPEN) ? 1 : 0;
            Q.ns = (mode == MODE_PAIR) ? 2 : 1;
            Q.band = c->NB > 1 ? reinterpret_cast<const int *>(c->ws + c->o_band) : nullptr;
            ProfScope ps(c, PBS_K_QGEMM);
            if constexpr (sizeof(T) == 4) {
                if (c->Kpb > 0 && c->src_mode != PBS_SRC_FP32) {
                    const unsigned short *ah = reinterpret_cast<const unsigned short *>(c->ws + c->o_bf);
                    const size_t MK = (size_t)c->Mp * c->Kpb;
                    const int np = src_nprod(c->src_mode);
                    HIPCHK(c, launch_qgemm_bf16s(Q, np == 1 ? ah + 2 * MK : ah, ah + MK, c->Kpb, np, c->stream));
                    continue;
                }
            }
            HIPCHK(c, launch_qgemm<T>(Q, c->stream));
        }
    }
    ProfScope ps(c, PBS_K_DOSE);
    if (mode & MODE_CLOSE)
        HIPCHK(c, launch_dose_reduce(c->edep(row_c), c->dep(0, 0), K1, c->NA, nslot, c->NLINE, c->NP, c->stream));
    if (mode & MODE_OPEN)
        HIPCHK(c, launch_dose_reduce(c->edep(row_o), c->dep(1, 0), K1, c->NA, nslot, c->NLINE, c->NP, c->stream));
    if (c->feat_on) {
        // per-layer surrogate records: injected energy of both halves, moments after the opening half,
        // and the deposit of the primaries alone when further generations are marched
        const int NA = c->NA, NP = c->NP;
        const long NL = c->NLINE;
        if (mode & MODE_CLOSE) {
            HIPCHK(c, launch_dose_reduce(c->frec(0, lay_c), c->fline(0), 1, NA, nslot, NL, NP, c->stream));
            if (K1 > 1)
                HIPCHK(c, launch_dose_reduce(c->frec(3, lay_c), c->dep(0, 0), 1, NA, nslot, NL, NP, c->stream));
        }
        if (mode & MODE_OPEN) {
            HIPCHK(c, launch_dose_reduce(c->frec(0, lay_o), c->fline(1), 1, NA, nslot, NL, NP, c->stream));
            HIPCHK(c, launch_dose_reduce(c->frec(1, lay_o), c->fline(2), 1, NA, nslot, NL, NP, c->stream));
            HIPCHK(c, launch_dose_reduce(c->frec(2, lay_o), c->fline(3), 1, NA, nslot, NL, NP, c->stream));
            if (K1 > 1)
                HIPCHK(c, launch_dose_reduce(c->frec(3, lay_o), c->dep(1, 0), 1, NA, nslot, NL, NP, c->stream));
        }
    }
    return PBS_OK;
}

template <typename T>
pbs_status transport(pbs_ctx *c, double h, int k, hipStream_t st)
{
    TParams<T> P;
    P.psi = c->psi<T>(k < 0 ? 0 : k);
    P.theta = c->tabT<T>() + c->t_theta;
    P.h_half_over_dx = (T)(0.5 * h / c->dx);
    P.h_half_over_dy = (T)(0.5 * h / c->dy);
    P.nx = c->g.nx;
    P.ny = c->g.ny;
    P.m = c->m;
    P.NA = c->NA;
    P.NLINE = c->NLINE;
    P.nplanes = (long)(k < 0 ? c->kact : 1) * c->G() * 2 * c->NA;
    if (!st) st = c->stream;
    ProfScope ps(c, PBS_K_TPASS, st);
    HIPCHK(c, launch_tpass<T>(P, st));
    return PBS_OK;
}

template <typename T>
pbs_status angular(pbs_ctx *c, int layer, double h, int k, hipStream_t st)
{
    AParams<T> P;
    T *tb = c->tabT<T>();
    P.psi = c->psi<T>(k < 0 ? 0 : k);
    const long nstack = (long)(k < 0 ? c->kact : 1) * c->G() * 2;
    if (!st) st = c->stream;
    P.rho = c->rhoT<T>(layer);
    P.sig = tb + c->t_sig;
    P.S = tb + c->t_S;
    P.lam = tb + c->t_lam;
    P.h = (T)h;
    P.G = c->G();
    P.NA = c->NA;
    P.NPB = c->NPB;
    P.NLINE = c->NLINE;
    ProfScope ps(c, PBS_K_APASS, st);
    if constexpr (sizeof(T) == 4) {
        if (c->g.nth == 32) {
            HIPCHK(c, launch_apass_mfma32(P, tb + c->t_K32, nstack, st));
            return PBS_OK;
        }
        if (c->g.nth == 16) {
            HIPCHK(c, launch_apass_mfma16(P, tb + c->t_K32, nstack, st));
            return PBS_OK;
        }
    }
    HIPCHK(c, launch_apass<T>(P, c->g.nth, nstack, st));
    return PBS_OK;
}

// the main stream waits for every generation's pending T A T
static pbs_status join_side(pbs_ctx *c)
{
    for (int k = 0; k < (int)c->tat_pend.size(); ++k)
        if (c->tat_pend[k]) {
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_tat[k], 0));
            c->tat_pend[k] = false;
        }
    return PBS_OK;
}

// One Richardson-extrapolated step of layer s (section 5's higher-order splitting): A = S(dz) psi and
// B = S(dz/2) S(dz/2) psi from the same state, psi = (4 B - A)/3, and the layer's deposit combined the
// same way.  Every step is complete (no energy half-step carried into the next one).
template <typename T>
pbs_status extrapolated_step(pbs_ctx *c)
{
    const int s = c->step, nz = c->g.nz;
    const double dz = c->g.dz;
    const long n = (long)c->kact * c->G() * 2 * c->NLINE;
    T *psi = c->psi<T>(0), *x0 = reinterpret_cast<T *>(c->ws + c->o_x0), *xA = reinterpret_cast<T *>(c->ws + c->o_xA);
    HIPCHK(c, launch_fill<double>(c->edep(nz), 0.0, 2L * c->NP, c->stream));
    HIPCHK(c, hipMemcpyAsync(x0, psi, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    pbs_status r;
    auto strang = [&](double h, int row, bool pair_inside) -> pbs_status {
        pbs_status q;
        if ((q = energy_chain<T>(c, MODE_OPEN, -1, s, 0.5 * h, -1, -1, row)) != PBS_OK) return q;
        if ((q = transport<T>(c, 0.5 * h)) != PBS_OK) return q;
        if ((q = angular<T>(c, s, h)) != PBS_OK) return q;
        if ((q = transport<T>(c, 0.5 * h)) != PBS_OK) return q;
        if (pair_inside) return energy_chain<T>(c, MODE_PAIR, s, s, 0.5 * h, -1, row, row);
        return energy_chain<T>(c, MODE_CLOSE, s, -1, 0.5 * h, -1, row, -1);
    };
    // A: one step of dz into row nz
    if ((r = strang(dz, nz, false)) != PBS_OK) return r;
    HIPCHK(c, hipMemcpyAsync(xA, psi, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(psi, x0, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    // B: two steps of dz/2 into row nz + 1 (the closing half of the first fused with the opening of the second)
    if ((r = strang(0.5 * dz, nz + 1, true)) != PBS_OK) return r;
    if ((r = transport<T>(c, 0.25 * dz)) != PBS_OK) return r;
    if ((r = angular<T>(c, s, 0.5 * dz)) != PBS_OK) return r;
    if ((r = transport<T>(c, 0.25 * dz)) != PBS_OK) return r;
    if ((r = energy_chain<T>(c, MODE_CLOSE, s, -1, 0.25 * dz, -1, nz + 1, -1)) != PBS_OK) return r;
    HIPCHK(c, launch_combine<T>(psi, xA, T(4.0 / 3.0), T(-1.0 / 3.0), n, c->stream));
    HIPCHK(c, launch_fill<double>(c->edep(s), 0.0, c->NP, c->stream));
    HIPCHK(c, launch_combine<double>(c->edep(s), c->edep(nz + 1), 0.0, 4.0 / 3.0, c->NP, c->stream));
    HIPCHK(c, launch_combine<double>(c->edep(s), c->edep(nz), 1.0, -1.0 / 3.0, c->NP, c->stream));
    c->step = s + 1;
    return PBS_OK;
}

template <typename T>
pbs_status one_step(pbs_ctx *c)
{
    if (c->order == 4) return extrapolated_step<T>(c);
    const int s = c->step;
    const double dz = c->g.dz;
    // a context without the side stream (bound to the static scratch) always marches on one stream
    const bool ovl = c->side && (c->sched == PBS_SCHED_TWO_STREAMS ||
                                 (c->sched == PBS_SCHED_AUTO && (long)c->NP * c->NA * c->G() < PBS_OVERLAP_CELLS));
    const int tat = ovl ? s : -1;
    pbs_status r = (s == 0) ? energy_chain<T>(c, MODE_OPEN, -1, 0, 0.5 * dz, tat)
                            : energy_chain<T>(c, MODE_PAIR, s - 1, s, 0.5 * dz, tat);
    if (r != PBS_OK) return r;
    if (!ovl) {
        if ((r = transport<T>(c, 0.5 * dz)) != PBS_OK) return r;
        if ((r = angular<T>(c, s, dz)) != PBS_OK) return r;
        if ((r = transport<T>(c, 0.5 * dz)) != PBS_OK) return r;
    }
    c->step = s + 1;
    return PBS_OK;
}

template <typename T>
pbs_status steps(pbs_ctx *c, int n)
{
    for (int i = 0; i < n; ++i) {
        pbs_status r = one_step<T>(c);
        if (r != PBS_OK) {
            join_side(c);
            return r;
        }
    }
    return join_side(c);
}

template <typename T>
pbs_status close_beam(pbs_ctx *c)
{
    if (c->step == 0 || c->order == 4) return PBS_OK;   // extrapolated steps are complete
    return energy_chain<T>(c, MODE_CLOSE, c->step - 1, -1, 0.5 * c->g.dz);
}

template <typename T>
pbs_status start_beam(pbs_ctx *c, const pbs_beam &b)
{
    const pbs_grid &g = c->g;
    HIPCHK(c, launch_fill<T>(c->psi<T>(0), T(0), (long)g.ngen * c->G() * 2 * c->NLINE, c->stream));
    HIPCHK(c, launch_fill<double>(c->edep(0), 0.0, (long)g.nz * c->NP, c->stream));
    if (c->sur) HIPCHK(c, launch_fill<double>(c->frec(0, 0), 0.0, 4L * g.nz * c->NP, c->stream));
    if (g.ngen > 1) {
        // padding source nodes of the split layout are never written and must stay zero
        const size_t wbytes = c->o_Q - c->o_W;
        HIPCHK(c, launch_fill<float>(reinterpret_cast<float *>(c->ws + c->o_W), 0.f, (long)(wbytes / 4), c->stream));
    }
    // initial condition: eq:(bdy) projected (lateral cell averages, DG-P1 energy moments, theta = 0 node)
    auto ncdf = [](double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); };
    auto npdf = [](double x) { return std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI); };
    std::vector<double> Lx(g.nx), Ly(g.ny), E1(c->G()), E2(c->G()), lat(c->NP);
    double tx = 0, ty = 0, te = 0;
    for (int p = 0; p < g.nx; ++p) {
        const double lo = -g.x_half + p * c->dx;
        const double w = ncdf((lo + c->dx - b.x0) / b.sigma_x) - ncdf((lo - b.x0) / b.sigma_x);
        Lx[p] = w / c->dx;
        tx += w;
    }
    for (int q = 0; q < g.ny; ++q) {
        const double lo = -g.y_half + q * c->dy;
        const double w = ncdf((lo + c->dy - b.y0) / b.sigma_y) - ncdf((lo - b.y0) / b.sigma_y);
        Ly[q] = w / c->dy;
        ty += w;
    }
    for (int k = 0; k < c->G(); ++k) {
        const double lo = c->E_face[k], hi = c->E_face[k + 1], d = hi - lo;
        const double za = (lo - b.e0) / b.sigma_e, zb = (hi - b.e0) / b.sigma_e;
        const double mass = ncdf(zb) - ncdf(za);
        // first moment about the group centre
        const double mom = b.sigma_e * (npdf(za) - npdf(zb)) + (b.e0 - c->E_mid[k]) * mass;
        E1[k] = mass / d;
        E2[k] = 6.0 * mom / (d * d);
        te += mass;
    }
    if (!(tx > 0 && ty > 0 && te > 0)) return fail(c, PBS_EINVAL, "beam does not overlap the grid");
    const double C = 1.0 / (tx * ty * te * c->dth * c->dth);
    for (int p = 0; p < g.nx; ++p)
        for (int q = 0; q < g.ny; ++q) lat[(size_t)p * g.ny + q] = C * Lx[p] * Ly[q];
    double *db = c->tabD();
    HIPCHK(c, hipMemcpyAsync(db + c->d_E1, E1.data(), E1.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(db + c->d_E2, E2.data(), E2.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(db + c->d_lat, lat.data(), lat.size() * 8, hipMemcpyHostToDevice, c->stream));
    const long center = (long)(c->m / 2) * c->m + c->m / 2;
    HIPCHK(c, launch_initial<T>(c->psi<T>(0), db + c->d_E1, db + c->d_E2, db + c->d_lat, center, c->G(), c->NA,
                                c->NPB, c->NP, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PBS_OK;
}

template <typename T>
pbs_status get_state(pbs_ctx *c, double *out)
{
    const size_t per = (size_t)c->G() * 2 * c->NLINE;
    std::vector<T> buf(per * c->g.ngen);
    HIPCHK(c, hipMemcpyAsync(buf.data(), c->psi<T>(0), buf.size() * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    size_t o = 0;
    for (int k = 0; k < c->g.ngen; ++k)
        for (int gl = 0; gl < c->G() * 2; ++gl)
            for (int a = 0; a < c->NA; ++a)
                for (int pq = 0; pq < c->NP; ++pq)
                    out[o++] = (double)buf[k * per + gl * c->NLINE + ((size_t)(pq / PBS_PT) * c->NA + a) * PBS_PT +
                                           pq % PBS_PT];
    return PBS_OK;
}

template <typename T>
pbs_status set_state(pbs_ctx *c, const double *in)
{
    const size_t per = (size_t)c->G() * 2 * c->NLINE;
    std::vector<T> buf(per * c->g.ngen, T(0));
    size_t o = 0;
    for (int k = 0; k < c->g.ngen; ++k)
        for (int gl = 0; gl < c->G() * 2; ++gl)
            for (int a = 0; a < c->NA; ++a)
                for (int pq = 0; pq < c->NP; ++pq)
                    buf[k * per + gl * c->NLINE + ((size_t)(pq / PBS_PT) * c->NA + a) * PBS_PT + pq % PBS_PT] =
                        (T)in[o++];
    HIPCHK(c, hipMemcpyAsync(c->psi<T>(0), buf.data(), buf.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PBS_OK;
}

template <typename T>
pbs_status set_phantom(pbs_ctx *c, const double *rho)
{
    const pbs_grid &g = c->g;
    std::vector<T> rt((size_t)g.nz * c->NPpad, T(1));
    for (int s = 0; s < g.nz; ++s)
        for (int pq = 0; pq < c->NP; ++pq) rt[(size_t)s * c->NPpad + pq] = (T)rho[(size_t)s * c->NP + pq];
    HIPCHK(c, hipMemcpyAsync(c->rhoT<T>(0), rt.data(), rt.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->rhoD(), rho, (size_t)g.nz * c->NP * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PBS_OK;
}

// ------------------------------------------------------------------ surrogate of generation 1
template <typename T>
pbs_status march_rest(pbs_ctx *c)
{
    pbs_status r = steps<T>(c, c->g.nz - c->step);
    if (r != PBS_OK) return r;
    return close_beam<T>(c);
}

SurFeatIn feat_inputs(pbs_ctx *c, bool with_target)
{
    SurFeatIn F;
    F.finj = c->frec(0, 0);
    F.fme = c->frec(1, 0);
    F.fmn = c->frec(2, 0);
    F.rho = c->rhoD();
    F.edep = with_target ? c->edep(0) : nullptr;
    F.edep0 = with_target ? c->frec(3, 0) : nullptr;
    F.nz = c->g.nz;
    F.NP = c->NP;
    F.dz = c->g.dz;
    F.k0dz = c->ph.kappa0 * c->g.dz;
    return F;
}

// Surrogate mode: march the primaries alone while recording, evaluate the network on every slice,
// check the energy residual; accept (dose = E0 - I + c net) or march again with both generations.
template <typename T>
pbs_status run_surrogate(pbs_ctx *c)
{
    const long slab = (long)c->g.nz * c->NP;
    c->kact = 1;
    c->feat_on = true;
    pbs_status r = march_rest<T>(c);
    c->kact = c->g.ngen;
    c->feat_on = false;
    if (r != PBS_OK) return r;
    double *sc = c->scal();
    HIPCHK(c, sur_scalars(c->frec(0, 0), c->frec(2, 0), c->edep(0), nullptr, slab, sc, c->stream));
    __bf16 *X = reinterpret_cast<__bf16 *>(c->ws + c->o_sx);
    __bf16 *A = reinterpret_cast<__bf16 *>(c->ws + c->o_sa), *B = reinterpret_cast<__bf16 *>(c->ws + c->o_sb);
    float *Y = reinterpret_cast<float *>(c->ws + c->o_sy);
    HIPCHK(c, sur_features(feat_inputs(c, false), sc, X, nullptr, c->stream));
    NetPacked P;
    net_carve(c->ws + c->o_spk, P);
    HIPCHK(c, net_forward(P, X, A, B, A, Y, c->g.nz, c->g.nx, c->g.ny, c->stream));
    HIPCHK(c, sur_sum(Y, slab, sc + 5, c->stream));
    double h[6];
    HIPCHK(c, hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double cb = h[0] > 0.0 ? h[0] : 1.0;
    const double einj = h[2], e0 = h[4], epred = cb * h[5];
    // energy balance of generation 1: what the network deposits against the injected energy less
    // the modelled leak, relative to the whole deposit of the beam
    const double x = 1.0 - e0 / c->beam.e0;
    const double leak = std::min(0.95, std::max(0.0, c->sur_leak[0] + x * (c->sur_leak[1] + x * c->sur_leak[2])));
    const double budget = (1.0 - leak) * einj, etot = e0 - einj + epred;
    double res = etot > 0.0 ? std::fabs(epred - budget) / etot : INFINITY;
    if (!std::isfinite(epred) || !std::isfinite(res)) res = INFINITY;
    const double rep[10] = {res, 0.0, budget, epred, cb, einj, NAN, leak, e0, x};
    std::memcpy(c->sur_rep, rep, sizeof(rep));
    if (res <= c->sur_tol) {
        HIPCHK(c, sur_combine(c->edep(0), c->frec(0, 0), Y, sc, slab, c->stream));
        return PBS_OK;
    }
    // fallback: the plain method from the start
    if ((r = start_beam<T>(c, c->beam)) != PBS_OK) return r;
    c->step = 0;
    if ((r = march_rest<T>(c)) != PBS_OK) return r;
    c->sur_rep[1] = 1.0;
    return PBS_OK;
}

#define DISPATCH(c, fn, ...) ((c)->prec == PBS_FP64 ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

}  // namespace

namespace pbs {
// Bind a workspace (caller memory or the static scratch) and a stream: uploads the tables (and the packed
// surrogate weights).  with_side: create the side stream and events of the two-stream march; without it
// the context always marches on its one stream and creates no HIP objects here.
pbs_status bind_workspace(pbs_ctx *c, char *ws, size_t bytes, hipStream_t stream, bool with_side)
{
    c->ws = ws;
    c->ws_bytes = bytes;
    c->stream = stream;
    if (with_side && !c->side) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        const int ng = c->g.ngen;
        c->ev_e.assign(ng, nullptr);
        c->ev_tat.assign(ng, nullptr);
        for (int k = 0; k < ng; ++k) {
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_e[k], hipEventDisableTiming));
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_tat[k], hipEventDisableTiming));
        }
    }
    c->tat_pend.assign(c->g.ngen, 0);
    c->state = ST_CREATED;
    pbs_status r = DISPATCH(c, upload_tables, c);
    if (r != PBS_OK) return r;
    if (c->sur == 2) {
        float *m = reinterpret_cast<float *>(c->ws + c->o_smaster);
        NetPacked P;
        net_carve(c->ws + c->o_spk, P);
        HIPCHK(c, hipMemcpyAsync(m, c->sur_params.data(), c->sur_params.size() * sizeof(float), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, net_pack(m, P, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->state = ST_BOUND;
    return PBS_OK;
}

pbs_status ctx_fail(pbs_ctx *c, pbs_status st, const char *msg) { return fail(c, st, msg); }
}  // namespace pbs

// =================================================================================== C ABI
extern "C" {

pbs_status pbs_create(const pbs_grid *grid, const pbs_physics *phys, int precision, pbs_ctx **out)
{
    if (!out) return PBS_EINVAL;
    *out = nullptr;
    if (!grid || !phys) return PBS_EINVAL;
    if (precision != PBS_FP32 && precision != PBS_FP64) return PBS_EINVAL;
    const pbs_grid &g = *grid;
    if (g.nx < 1 || g.ny < 1 || g.ny > 64 * PBS_MAX_NSEG || g.ng < 2 || g.nz < 1 || g.ngen < 1 || g.ngen > 8)
        return PBS_EINVAL;
    if (g.nth < 4 || g.nth % 2) return PBS_EINVAL;
    if (!finite_pos(g.x_half) || !finite_pos(g.y_half) || !finite_pos(g.th_half) || !finite_pos(g.dz) ||
        !std::isfinite(g.e_lo) || g.e_lo < 0 || !(g.e_hi > g.e_lo) || !std::isfinite(g.e_hi))
        return PBS_EINVAL;
    const pbs_physics &ph = *phys;
    const double vals[] = {ph.bk_alpha, ph.bk_p, ph.e_floor, ph.highland_es, ph.x0_water, ph.mp,
                           ph.kappa0,   ph.e_c,  ph.lambda_nuc, ph.gamma_a, ph.gamma_b};
    for (double v : vals)
        if (!std::isfinite(v)) return PBS_EINVAL;
    if (!finite_pos(ph.bk_alpha) || !finite_pos(ph.bk_p) || !finite_pos(ph.e_floor) || !finite_pos(ph.x0_water) ||
        !finite_pos(ph.mp) || ph.kappa0 < 0 || !finite_pos(ph.e_c) || ph.lambda_nuc < 0 || !(ph.gamma_a >= 1.0) ||
        !finite_pos(ph.gamma_b))
        return PBS_EINVAL;
    if (ph.stopping != PBS_STOP_BRAGG_KLEEMAN && ph.stopping != PBS_STOP_BETHE) return PBS_EINVAL;
    if (ph.stopping == PBS_STOP_BETHE && !(ph.e_floor >= 0.5)) return PBS_EINVAL;
    if (ph.straggling != 0 && ph.straggling != 1) return PBS_EINVAL;
    if (ph.scattering != PBS_SCAT_HIGHLAND && ph.scattering != PBS_SCAT_RUTHERFORD) return PBS_EINVAL;
    if (ph.material < PBS_MAT_WATER || ph.material > PBS_MAT_AIR) return PBS_EINVAL;
    // the range fit is water's; the other media and the straggling need the Bethe-Bloch form
    if ((ph.material != PBS_MAT_WATER || ph.straggling) && ph.stopping != PBS_STOP_BETHE) return PBS_EINVAL;
    if (ph.nuc_bands < 0 || ph.nuc_bands > 4) return PBS_EINVAL;
    for (int b = 0; b < ph.nuc_bands; ++b) {
        if (!std::isfinite(ph.nuc_e[b]) || !(ph.nuc_lambda[b] >= 0) || !std::isfinite(ph.nuc_lambda[b]) ||
            !(ph.nuc_alpha[b] >= 1.0) || !std::isfinite(ph.nuc_alpha[b]) || !finite_pos(ph.nuc_beta[b]))
            return PBS_EINVAL;
        if (b > 0 && !(ph.nuc_e[b] > ph.nuc_e[b - 1])) return PBS_EINVAL;
    }
    if (!apass_supported(g.nth)) return PBS_EUNSUPPORTED;
    pbs_ctx *c = new (std::nothrow) pbs_ctx();
    if (!c) return PBS_ENOMEM;
    c->g = g;
    c->ph = ph;
    c->prec = precision;
    c->tsz = precision == PBS_FP64 ? 8 : 4;
    c->m = g.nth - 1;
    c->NA = c->m * c->m;
    c->NP = g.nx * g.ny;
    c->NPB = (c->NP + PBS_PT - 1) / PBS_PT;
    c->NPpad = c->NPB * PBS_PT;
    c->NLINE = (long)c->NPB * c->NA * PBS_PT;
    c->dx = 2.0 * g.x_half / g.nx;
    c->dy = 2.0 * g.y_half / g.ny;
    c->dth = 2.0 * g.th_half / g.nth;
    c->NOCT = (c->NA + 7) / 8;
    c->kact = g.ngen;
    if (c->NA >= 128) {   // source product on MFMA
        c->Kp = (c->NA + 15) / 16 * 16;
        c->Mp = (c->NA + 127) / 128 * 128;
        if (precision == PBS_FP32 && !ph.straggling) {
            // split-BF16 source product (its scans come from the straggling-free energy passes)
            c->Kpb = (c->NA + PBS_KPB_ALIGN - 1) / PBS_KPB_ALIGN * PBS_KPB_ALIGN;
            c->src_mode = PBS_DEFAULT_SRC;
        }
    }
    try {
        build_tables(c);
    } catch (...) {
        delete c;
        return PBS_ENOMEM;
    }
    layout(c);
    *out = c;
    return PBS_OK;
}

pbs_status pbs_workspace_bytes(const pbs_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return PBS_EINVAL;
    *bytes = c->total;
    return PBS_OK;
}

pbs_status pbs_bind(pbs_ctx *c, void *ws, size_t bytes, void *stream)
{
    if (!c) return PBS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255)) return fail(c, PBS_EINVAL, "workspace is NULL or not 256-byte aligned");
    if (bytes < c->total) return fail(c, PBS_EINVAL, "workspace too small");
    c->static_dev = -1;
    return pbs::bind_workspace(c, (char *)ws, bytes, (hipStream_t)stream, true);
}

pbs_status pbs_set_phantom(pbs_ctx *c, const double *rho, size_t n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BOUND) return fail(c, PBS_ESTATE, "set_phantom before bind");
    if (!rho || n != (size_t)c->g.nz * c->NP) return fail(c, PBS_EINVAL, "phantom size must be nz*nx*ny");
    for (size_t i = 0; i < n; ++i)
        if (!finite_pos(rho[i])) return fail(c, PBS_EINVAL, "densities must be finite and > 0");
    pbs_status r = DISPATCH(c, set_phantom, c, rho);
    if (r != PBS_OK) return r;
    c->rho_host.assign(rho, rho + n);
    c->state = ST_PHANTOM;
    return PBS_OK;
}

pbs_status pbs_resample_phantom(const pbs_grid *g, const double *vox, int vnz, int vnx, int vny, double vdz,
                                double vdx, double vdy, double x_lo, double y_lo, double *out)
{
    if (!g || !vox || !out || vnz < 1 || vnx < 1 || vny < 1 || g->nz < 1 || g->nx < 1 || g->ny < 1)
        return PBS_EINVAL;
    if (!finite_pos(vdz) || !finite_pos(vdx) || !finite_pos(vdy) || !std::isfinite(x_lo) || !std::isfinite(y_lo) ||
        !finite_pos(g->dz) || !finite_pos(g->x_half) || !finite_pos(g->y_half))
        return PBS_EINVAL;
    const size_t nv = (size_t)vnz * vnx * vny;
    for (size_t i = 0; i < nv; ++i)
        if (!finite_pos(vox[i])) return PBS_EINVAL;
    const double dx = 2.0 * g->x_half / g->nx, dy = 2.0 * g->y_half / g->ny;
    auto nearest = [](double c, double lo, double d, int n) {
        const long i = (long)std::floor((c - lo) / d);
        return (int)std::min<long>(std::max<long>(i, 0), n - 1);
    };
    for (int s = 0; s < g->nz; ++s) {
        const int k = nearest((s + 0.5) * g->dz, 0.0, vdz, vnz);
        for (int p = 0; p < g->nx; ++p) {
            const int i = nearest(-g->x_half + (p + 0.5) * dx, x_lo, vdx, vnx);
            for (int q = 0; q < g->ny; ++q) {
                const int j = nearest(-g->y_half + (q + 0.5) * dy, y_lo, vdy, vny);
                out[((size_t)s * g->nx + p) * g->ny + q] = vox[((size_t)k * vnx + i) * vny + j];
            }
        }
    }
    return PBS_OK;
}

pbs_status pbs_set_phantom_voxels(pbs_ctx *c, const double *vox, int vnz, int vnx, int vny, double vdz, double vdx,
                                  double vdy, double x_lo, double y_lo)
{
    if (!c) return PBS_EINVAL;
    if (c->state < ST_BOUND) return fail(c, PBS_ESTATE, "set_phantom_voxels before bind");
    std::vector<double> rho;
    try {
        rho.resize((size_t)c->g.nz * c->NP);
    } catch (...) {
        return fail(c, PBS_ENOMEM, "host allocation of the resampled phantom failed");
    }
    const pbs_status r = pbs_resample_phantom(&c->g, vox, vnz, vnx, vny, vdz, vdx, vdy, x_lo, y_lo, rho.data());
    if (r != PBS_OK) return fail(c, r, "voxel phantom: sizes, spacings and corner must be finite and positive, "
                                       "densities finite and > 0");
    return pbs_set_phantom(c, rho.data(), rho.size());
}

pbs_status pbs_set_beam(pbs_ctx *c, const pbs_beam *b)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_PHANTOM) return fail(c, PBS_ESTATE, "set_beam before set_phantom");
    if (!b) return fail(c, PBS_EINVAL, "beam is NULL");
    if (!std::isfinite(b->e0) || !finite_pos(b->sigma_e) || !std::isfinite(b->x0) || !std::isfinite(b->y0) ||
        !finite_pos(b->sigma_x) || !finite_pos(b->sigma_y))
        return fail(c, PBS_EINVAL, "bad beam parameters");
    c->kact = c->g.ngen;
    c->feat_on = false;
    pbs_status r = DISPATCH(c, start_beam, c, *b);
    if (r != PBS_OK) return r;
    c->beam = *b;
    for (double &v : c->sur_rep) v = NAN;
    c->step = 0;
    c->closed = false;
    c->state = ST_BEAM;
    return PBS_OK;
}

pbs_status pbs_step_depth(pbs_ctx *c, int n, int *step_out)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "step_depth before set_beam");
    if (c->closed) return fail(c, PBS_ESTATE, "beam already finished by run_beam");
    if (c->sur == 2) return fail(c, PBS_ESTATE, "a surrogate context marches whole beams (pbs_run_beam)");
    if (n < 0 || n > c->g.nz - c->step) return fail(c, PBS_EINVAL, "n must be in [0, nz - steps done]");
    c->feat_on = c->sur == 1;
    pbs_status r = DISPATCH(c, steps, c, n);
    c->feat_on = false;
    if (step_out) *step_out = c->step;
    return r;
}

pbs_status pbs_run_beam(pbs_ctx *c)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "run_beam before set_beam");
    if (c->closed) return fail(c, PBS_ESTATE, "beam already finished by run_beam");
    pbs_status r;
    if (c->sur == 2) {
        r = DISPATCH(c, run_surrogate, c);
    } else {
        c->feat_on = c->sur == 1;
        r = DISPATCH(c, march_rest, c);
        c->feat_on = false;
        if (r == PBS_OK && c->sur == 1)
            HIPCHK(c, sur_scalars(c->frec(0, 0), c->frec(2, 0), c->edep(0), c->frec(3, 0), (long)c->g.nz * c->NP,
                                  c->scal(), c->stream));
    }
    if (r != PBS_OK) return r;
    c->closed = true;
    return PBS_OK;
}

pbs_status pbs_set_surrogate(pbs_ctx *c, const void *weights, size_t bytes, double tol)
{
    if (!c) return PBS_EINVAL;
    if (c->ws) return fail(c, PBS_ESTATE, "set_surrogate must precede bind");
    if (c->g.ngen != 2) return fail(c, PBS_EINVAL, "the surrogate replaces generation 1 of a K = 1 grid (ngen = 2)");
    if (c->g.ny > 64) return fail(c, PBS_EUNSUPPORTED, "surrogate images are at most 64 cells wide (ny <= 64)");
    if (c->strag || c->NB > 1 || c->order != 2)
        return fail(c, PBS_EUNSUPPORTED,
                    "the surrogate is trained without straggling, with one nuclear band and Strang steps");
    if (!weights) {
        if (bytes != 0) return fail(c, PBS_EINVAL, "weights NULL with nonzero size");
        c->sur = 1;
        c->sur_params.clear();
        c->sur_leak[0] = c->sur_leak[1] = c->sur_leak[2] = 0.0;
        c->sur_tol = 0.0;
        layout(c);
        return PBS_OK;
    }
    if (!std::isfinite(tol) || tol < 0) return fail(c, PBS_EINVAL, "residual tolerance must be finite and >= 0");
    pbs_net_header h;
    if (bytes < sizeof(h)) return fail(c, PBS_EINVAL, "weights blob too small");
    std::memcpy(&h, weights, sizeof(h));
    const size_t np = net_param_count();
    if (h.magic != PBS_NET_MAGIC || h.version != PBS_NET_VERSION || h.nparam != np || h.nfeat != (unsigned)SUR_NFEAT)
        return fail(c, PBS_EINVAL, "weights blob header does not match this network");
    if (bytes != sizeof(h) + np * sizeof(float)) return fail(c, PBS_EINVAL, "weights blob size mismatch");
    for (double v : h.leak)
        if (!std::isfinite(v)) return fail(c, PBS_EINVAL, "leak model coefficients must be finite");
    std::vector<float> p(np);
    std::memcpy(p.data(), (const char *)weights + sizeof(h), np * sizeof(float));
    for (float v : p)
        if (!std::isfinite(v)) return fail(c, PBS_EINVAL, "weights must be finite");
    c->sur = 2;
    c->sur_params.swap(p);
    std::memcpy(c->sur_leak, h.leak, sizeof(h.leak));
    c->sur_tol = tol;
    layout(c);
    return PBS_OK;
}

pbs_status pbs_surrogate_sample(pbs_ctx *c, void *dev_x, float *dev_t, size_t n_slices)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->sur != 1) return fail(c, PBS_ESTATE, "sample needs a context in recording mode");
    if (c->state < ST_BEAM || !c->closed) return fail(c, PBS_ESTATE, "sample before run_beam");
    if (!dev_x || !dev_t || ((uintptr_t)dev_x & 15) || ((uintptr_t)dev_t & 15))
        return fail(c, PBS_EINVAL, "feature / target buffers must be non-NULL and 16-byte aligned");
    if (n_slices != (size_t)c->g.nz) return fail(c, PBS_EINVAL, "n_slices must equal nz");
    HIPCHK(c, sur_features(feat_inputs(c, true), c->scal(), reinterpret_cast<__bf16 *>(dev_x), dev_t, c->stream));
    return PBS_OK;
}

pbs_status pbs_surrogate_records(pbs_ctx *c, double *out, size_t n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (!c->sur) return fail(c, PBS_ESTATE, "no surrogate records without pbs_set_surrogate");
    if (c->state < ST_BEAM || !c->closed) return fail(c, PBS_ESTATE, "records before run_beam");
    if (!out || n != (size_t)4 * c->g.nz * c->NP) return fail(c, PBS_EINVAL, "records buffer must hold 4*nz*nx*ny");
    HIPCHK(c, hipMemcpyAsync(out, c->frec(0, 0), n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PBS_OK;
}

pbs_status pbs_surrogate_report(pbs_ctx *c, double *out, int n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (!c->sur) return fail(c, PBS_ESTATE, "no surrogate report without pbs_set_surrogate");
    if (c->state < ST_BEAM || !c->closed) return fail(c, PBS_ESTATE, "report before run_beam");
    if (!out || n < 0 || n > 10) return fail(c, PBS_EINVAL, "report holds at most 10 values");
    if (c->sur == 1) {
        double h[5];
        HIPCHK(c, hipMemcpyAsync(h, c->scal(), sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const double lk = h[2] > 0.0 ? 1.0 - h[3] / h[2] : NAN;
        const double rep[10] = {NAN, 1.0, NAN, NAN, h[0] > 0.0 ? h[0] : 1.0, h[2], h[3], lk, h[4], 1.0 - h[4] / c->beam.e0};
        std::memcpy(c->sur_rep, rep, sizeof(rep));
    } else {
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    for (int i = 0; i < n; ++i) out[i] = c->sur_rep[i];
    return PBS_OK;
}

pbs_status pbs_get_dose(pbs_ctx *c, double *out, size_t n, int out_is_device)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "get_dose before set_beam");
    const size_t tot = (size_t)c->g.nz * c->NP;
    if (!out || n != tot) return fail(c, PBS_EINVAL, "dose buffer must hold nz*nx*ny doubles");
    const double vol = c->dx * c->dy * c->g.dz;
    double *dst = out_is_device ? out : c->dout();
    HIPCHK(c, launch_dose_finalize(dst, c->edep(0), c->rhoD(), vol, (long)tot, c->stream));
    if (!out_is_device) {
        HIPCHK(c, hipMemcpyAsync(out, c->dout(), tot * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return PBS_OK;
}

pbs_status pbs_get_state(pbs_ctx *c, double *out, size_t n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "get_state before set_beam");
    if (!out || n != (size_t)c->g.ngen * c->G() * 2 * c->NA * c->NP) return fail(c, PBS_EINVAL, "bad state size");
    return DISPATCH(c, get_state, c, out);
}

pbs_status pbs_set_state(pbs_ctx *c, const double *in, size_t n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "set_state before set_beam");
    if (!in || n != (size_t)c->g.ngen * c->G() * 2 * c->NA * c->NP) return fail(c, PBS_EINVAL, "bad state size");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(in[i])) return fail(c, PBS_EINVAL, "state must be finite");
    return DISPATCH(c, set_state, c, in);
}

pbs_status pbs_apply(pbs_ctx *c, int op, int layer, double h)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BEAM) return fail(c, PBS_ESTATE, "apply before set_beam");
    if (layer < 0 || layer >= c->g.nz || !std::isfinite(h) || h < 0) return fail(c, PBS_EINVAL, "bad layer or h");
    switch (op) {
    case PBS_OP_E: return DISPATCH(c, energy_chain, c, MODE_OPEN, -1, layer, h);
    case PBS_OP_T: return DISPATCH(c, transport, c, h);
    case PBS_OP_A: return DISPATCH(c, angular, c, layer, h);
    default: return fail(c, PBS_EINVAL, "unknown op");
    }
}

pbs_status pbs_set_source_precision(pbs_ctx *c, int mode)
{
    if (!c) return PBS_EINVAL;
    if (mode != PBS_SRC_FP32 && mode != PBS_SRC_BF16X3 && mode != PBS_SRC_BF16X2 && mode != PBS_SRC_BF16X1)
        return fail(c, PBS_EINVAL, "unknown source precision");
    if (mode != PBS_SRC_FP32 && c->Kpb == 0)
        return fail(c, PBS_EUNSUPPORTED, "split-BF16 source product needs an FP32 context with >= 128 angular unknowns");
    c->src_mode = mode;
    return PBS_OK;
}

pbs_status pbs_set_splitting(pbs_ctx *c, int order)
{
    if (!c) return PBS_EINVAL;
    if (c->ws) return fail(c, PBS_ESTATE, "set_splitting must precede bind (it sizes the workspace)");
    if (order != 2 && order != 4) return fail(c, PBS_EINVAL, "splitting order must be 2 or 4");
    if (order == 4 && c->sur) return fail(c, PBS_EUNSUPPORTED, "the surrogate marches Strang steps only");
    c->order = order;
    layout(c);
    return PBS_OK;
}

pbs_status pbs_set_schedule(pbs_ctx *c, int mode)
{
    if (!c) return PBS_EINVAL;
    if (mode != PBS_SCHED_AUTO && mode != PBS_SCHED_ONE_STREAM && mode != PBS_SCHED_TWO_STREAMS)
        return fail(c, PBS_EINVAL, "schedule must be PBS_SCHED_AUTO, PBS_SCHED_ONE_STREAM or PBS_SCHED_TWO_STREAMS");
    c->sched = mode;
    return PBS_OK;
}

pbs_status pbs_profile(pbs_ctx *c, int enable)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (c->state < ST_BOUND) return fail(c, PBS_ESTATE, "profile before bind");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->ev_pairs.clear();
    c->ev_used = 0;
    c->prof = enable != 0;
    return PBS_OK;
}

pbs_status pbs_profile_read(pbs_ctx *c, double *ms, long *launches, int n)
{
    if (!c) return PBS_EINVAL;
    if (c->static_dev >= 0 && pbs::static_lost(c))
        return fail(c, PBS_ESTATE, "another context has been bound to this device's static scratch since");
    if (!ms || !launches || n < 0) return fail(c, PBS_EINVAL, "bad profile buffers");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) {
        ms[k] = 0;
        launches[k] = 0;
    }
    for (auto &pr : c->ev_pairs) {
        if (pr.first >= n) continue;
        float t = 0;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[pr.second], c->ev_pool[pr.second + 1]));
        ms[pr.first] += t;
        launches[pr.first] += 1;
    }
    return PBS_OK;
}

const char *pbs_last_error(const pbs_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

void pbs_destroy(pbs_ctx *c)
{
    if (!c) return;
    // work enqueued by step_depth / run_beam may still write the workspace: finish it before the caller
    // can release that memory
    if (c->ws) (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (hipEvent_t e : c->ev_e)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_tat)
        if (e) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
