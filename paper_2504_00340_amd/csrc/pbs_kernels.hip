// HIP kernels of libpbsplit for gfx950 (CDNA4, wave64).
//
//   epass   energy CN half-steps (section 3.2 DG-P1 operator eq:(0041-d); section 3.3 CN), one
//           thread per (lateral cell, angle) line sweeping the groups from the top; the closing
//           half of step s-1 and the opening half of step s are done in the same sweep (one read
//           and one write of the fluence).  Also the catastrophic-source energy scan for the
//           next generation and the FP64 deposit of eq:(en_d).
//   tpass   lateral transport CN half-step (section 3.4, eq:(distansport), superbee slopes frozen
//           at the old level), one wave per (x, y) plane walking the rows in the upwind order;
//           the implicit upwind solve along a row is a first-order linear recurrence done as a
//           64-lane affine scan.
//   apass   angular diffusion CN step (section 3.4, eq:(sd), eq:(eqn_fly)) by the discrete sine
//           transform with the even/odd split of the sine matrix, staged through LDS.
//   qgemm   angular part of the catastrophic source: Q = P2^T W for every (state, group,
//           lateral tile).
//   dose    deterministic per-voxel reduction of the per-line deposits.
#include "pbs_common.h"

namespace pbs {

typedef unsigned short u16x8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// Per-group table entries are the same for every lane: read through the constant address space they
// become scalar loads (one per wave, kept apart from the vector memory counter) instead of a vector load
// per lane that the group step then waits for.
template <typename T>
__device__ __forceinline__ T tab(const T *p, long i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// ------------------------------------------------------------------------------- energy pass
// One thread per line (FP64 contexts, and FP32 contexts whose source product takes the plain scan W):
// block = one lateral tile pb and one octet of angular lines a = 8*oct + e (e = tid/32), 32 cells
// pt = tid%32.  FP32 contexts with the split-BF16 product use epass8_body below.
template <typename T, int MODE, bool BANDS = false>
__device__ __forceinline__ void epass_body(const EParams<T> &P, int bx)
{
    constexpr bool CL = (MODE & MODE_CLOSE) != 0;
    constexpr bool OP = (MODE & MODE_OPEN) != 0;
    const int NA = (int)(P.NAPT / PBS_PT);
    const int pbk = bx / P.NOCT, oct = bx % P.NOCT;
    const int e = threadIdx.x >> 5, ptc = threadIdx.x & 31;
    const int a = oct * 8 + e;
    if (a >= NA) return;
    const long line = ((long)pbk * NA + a) * PBS_PT + ptc;
    const long pq = (line / P.NAPT) * PBS_PT + (line % PBS_PT);
    const long S = P.NLINE;
    const long QS = (long)P.G * S;
    const double rc = CL ? (double)P.rho_c[pq] : 0.0;
    const double ro = OP ? (double)P.rho_o[pq] : 0.0;
    const double dac = 0.5 * (double)P.h * rc, dao = 0.5 * (double)P.h * ro;
    const T ac = (T)dac, ao = (T)dao;
    T fin = 0, fcl = 0, fop = 0;    // psi1 - psi2 of group g+1: input, after close, after open
    T U0 = 0, U1 = 0, U2 = 0;       // re-emission energy scans of states 0, 1, 2
    T U0b[4] = {}, U1b[4] = {}, U2b[4] = {};   // per-band scans (BANDS)
    double ph0 = 0, ph1 = 0, ph2 = 0, injc = 0, injo = 0;
    T fic = 0, fio = 0, fme = 0, fmn = 0;   // surrogate records (energy sent to the next generation, moments)
    const bool hasQ = P.Q != nullptr, hasW = P.W != nullptr;
    const bool feat = P.inj_c != nullptr;
    for (int g = P.G - 1; g >= 0; --g) {
        T *p1 = P.psi + (2L * g) * S + line;
        T *p2 = p1 + S;
        const T x1 = *p1, x2 = *p2;
        const T sm = tab(P.Sm, g), sp = tab(P.Sp, g), kp = tab(P.kap, g);
        // rho-free operator: psi1 row [-(S-+k), S-], psi2 row [-3S+, -(S+ + 2S- + k)], coupling S+[1,3]
        const T d11 = -(sm + kp), d12 = sm, d21 = T(-3) * sp, d22 = -(sp + T(2) * sm + kp);
        const T c1 = sp, c2 = T(3) * sp;
        // trapezoidal sources of the two half-steps: Q^n + Q* (close), Q^n + Q* (open)
        T qc = 0, qo = 0;
        if (hasQ) {
            const long o = (long)g * S + line;
            if (CL) qc = P.Q[o];
            if (OP) qo = P.Q[QS + o];
        }
        T y1 = x1, y2 = x2;
        if (CL) {
            const T f = fin + fcl;
            const T r1 = x1 + ac * (d11 * x1 + d12 * x2 + c1 * f + qc);
            const T r2 = x2 + ac * (d21 * x1 + d22 * x2 + c2 * f);
            const T m11 = T(1) - ac * d11, m12 = -ac * d12, m21 = -ac * d21, m22 = T(1) - ac * d22;
            const T inv = fast_rcp(m11 * m22 - m12 * m21);
            y1 = (r1 * m22 - m12 * r2) * inv;
            y2 = (m11 * r2 - m21 * r1) * inv;
        }
        T z1 = y1, z2 = y2;
        if (OP) {
            const T f = (CL ? fcl : fin) + fop;
            const T r1 = y1 + ao * (d11 * y1 + d12 * y2 + c1 * f + qo);
            const T r2 = y2 + ao * (d21 * y1 + d22 * y2 + c2 * f);
            const T m11 = T(1) - ao * d11, m12 = -ao * d12, m21 = -ao * d21, m22 = T(1) - ao * d22;
            const T inv = fast_rcp(m11 * m22 - m12 * m21);
            z1 = (r1 * m22 - m12 * r2) * inv;
            z2 = (m11 * r2 - m21 * r1) * inv;
        }
        *p1 = z1;
        *p2 = z2;
        // deposit functional (FP64): stopping + removal of every state, bottom-face outflow
        const double A = tab(P.dA, g), B = tab(P.dB, g);
        if (CL) ph0 += A * (double)x1 + B * (double)x2;
        ph1 += A * (double)y1 + B * (double)y2;
        if (OP) ph2 += A * (double)z1 + B * (double)z2;
        if (g == 0) {
            if (CL) ph0 += P.dBot * ((double)x1 - (double)x2);
            ph1 += P.dBot * ((double)y1 - (double)y2);
            if (OP) ph2 += P.dBot * ((double)z1 - (double)z2);
        }
        if (hasQ) {
            const double wi = tab(P.dInj, g);
            if (CL) injc += wi * (double)qc;
            if (OP) injo += wi * (double)qo;
        }
        if (hasW || feat) {
            // energy scans of the three states; the next generation needs the sums 0+1 and 1+2
            const T w = tab(P.wc, g), dec = tab(P.wdec, g), idE = tab(P.invdE, g);
            const long o = (long)g * S + line;
            if constexpr (BANDS) {
                // the sum of one scan per band, each with its band's decay; group g feeds its own band
                const int bg = tab(P.band, g);
                U0 = U1 = U2 = T(0);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (b < P.NB) {
                        const T d = tab(P.wdecb, (long)b * P.G + g), wb = b == bg ? w : T(0);
                        if (CL) U0 += (U0b[b] = wb * x1 + d * U0b[b]);
                        U1 += (U1b[b] = wb * y1 + d * U1b[b]);
                        if (OP) U2 += (U2b[b] = wb * z1 + d * U2b[b]);
                    }
            } else {
                if (CL) U0 = w * x1 + dec * U0;
                U1 = w * y1 + dec * U1;
                if (OP) U2 = w * z1 + dec * U2;
            }
            if (feat) {
                // energy the re-emission puts into the next generation (the dInj functional of its
                // source summed over destination angles, which the angular law conserves), moments
                const T wi = (T)tab(P.dInj, g);
                if (CL) fic += wi * ((U0 + U1) * idE);
                if (OP) {
                    fio += wi * ((U1 + U2) * idE);
                    fme += (T)tab(P.wmom, g) * z1 + (T)tab(P.wmom, 2L * P.G + g) * z2;
                    fmn += (T)tab(P.wmom, (long)P.G + g) * z1;
                }
            }
            if (hasW) {
                if (CL) P.W[o] = (U0 + U1) * idE;
                if (OP) P.W[QS + o] = (U1 + U2) * idE;
            }
        }
        fin = x1 - x2;
        fcl = y1 - y2;
        fop = z1 - z2;
    }
    if (CL) P.dep_c[line] = dac * (ph0 + ph1 - injc) * P.scale;
    if (OP) P.dep_o[line] = dao * (ph1 + ph2 - injo) * P.scale;
    if (feat) {
        if (CL) P.inj_c[line] = dac * (double)fic * P.scale;
        if (OP) {
            P.inj_o[line] = dao * (double)fio * P.scale;
            P.mom_e[line] = (double)fme * P.scale;
            P.mom_n[line] = (double)fmn * P.scale;
        }
    }
}

template <typename T, int MODE, bool BANDS>
__global__ __launch_bounds__(256) void epass_kernel(EParams<T> P)
{
    epass_body<T, MODE, BANDS>(P, blockIdx.x);
}

template <typename T, bool BANDS>
static void launch_epass_t(const EParams<T> &P, int mode, unsigned nb, hipStream_t st)
{
    if (mode == MODE_PAIR)
        hipLaunchKernelGGL((epass_kernel<T, MODE_PAIR, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else if (mode == MODE_OPEN)
        hipLaunchKernelGGL((epass_kernel<T, MODE_OPEN, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else
        hipLaunchKernelGGL((epass_kernel<T, MODE_CLOSE, BANDS>), dim3(nb), dim3(256), 0, st, P);
}

template <typename T>
hipError_t launch_epass(const EParams<T> &P, int mode, hipStream_t st)
{
    if (P.Wh != nullptr) return hipErrorInvalidValue;   // split scans: launch_epass8
    if (P.NB > 4) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((P.NLINE / P.NAPT) * P.NOCT);
    if (P.NB > 1)
        launch_epass_t<T, true>(P, mode, nb, st);
    else
        launch_epass_t<T, false>(P, mode, nb, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------ energy pass with straggling
// With straggling (section 3.2's (1/2) d^2/dE^2 (T psi)) every energy line is block-tridiagonal:
//   (I - a D0_g) X*_g - a Lo_g X*_{g-1} - a Up_g X*_{g+1} = X_g + a (D0 X)_g + a [q_g, 0],   a = h rho / 2,
// with the rho-free 2x2 blocks Lo (to g-1), Di (D0_gg), Up (to g+1) of the host tables.  The matrix
// depends only on the cell's density, so the elimination from the top,
//   Dt_g = (I - a Di_g) - a^2 Up_g Dt_{g+1}^-1 Lo_{g+1},   F_g = a Up_g Dt_{g+1}^-1,
// is done once per cell (factor kernel, FP64, stored as [g][8][NPpad]: Dt_g^-1 row-major, then F_g); each
// line then sweeps down (bt_g = b_g + F_g bt_{g+1}, kept in place of X_g) and back up
// (X*_g = Dt_g^-1 (bt_g + a Lo_g X*_{g-1})).  The energy scans of the next generation's source take a
// third sweep down over X*.

template <typename T>
__global__ __launch_bounds__(256) void strag_factor_kernel(const T *__restrict__ blk, const T *__restrict__ rho, T h,
                                                             int G, long NPpad, T *__restrict__ sfac)
{
    const long pq = (long)blockIdx.x * 256 + threadIdx.x;
    if (pq >= NPpad) return;
    const double a = 0.5 * (double)h * (double)rho[pq];
    double di[4] = {0, 0, 0, 0};   // Dt_{g+1}^-1
    for (int g = G - 1; g >= 0; --g) {
        const T *B = blk + (size_t)g * 12;
        double M[4] = {1.0 - a * (double)B[4], -a * (double)B[5], -a * (double)B[6], 1.0 - a * (double)B[7]};
        double F[4] = {0, 0, 0, 0};
        if (g + 1 < G) {
            const T *Bn = blk + (size_t)(g + 1) * 12;   // Lo of group g+1
            const double U[4] = {a * (double)B[8], a * (double)B[9], a * (double)B[10], a * (double)B[11]};
            F[0] = U[0] * di[0] + U[1] * di[2], F[1] = U[0] * di[1] + U[1] * di[3];
            F[2] = U[2] * di[0] + U[3] * di[2], F[3] = U[2] * di[1] + U[3] * di[3];
            const double L[4] = {a * (double)Bn[0], a * (double)Bn[1], a * (double)Bn[2], a * (double)Bn[3]};
            M[0] -= F[0] * L[0] + F[1] * L[2], M[1] -= F[0] * L[1] + F[1] * L[3];
            M[2] -= F[2] * L[0] + F[3] * L[2], M[3] -= F[2] * L[1] + F[3] * L[3];
        }
        const double det = M[0] * M[3] - M[1] * M[2];
        di[0] = M[3] / det, di[1] = -M[1] / det, di[2] = -M[2] / det, di[3] = M[0] / det;
        T *o = sfac + (size_t)g * 8 * NPpad + pq;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[q * NPpad] = (T)di[q];
            o[(4 + q) * NPpad] = (T)F[q];
        }
    }
}

// one step of the re-emission scan (single law, or the sum over bands) at group g; returns the scan value
template <typename T, bool BANDS>
__device__ __forceinline__ T scan_step(const EParams<T> &P, int g, T x, T &U, T (&Ub)[4])
{
    const T w = tab(P.wc, g);
    if constexpr (BANDS) {
        const int bg = tab(P.band, g);
        T u = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (b < P.NB) u += (Ub[b] = (b == bg ? w : T(0)) * x + tab(P.wdecb, (long)b * P.G + g) * Ub[b]);
        return u;
    } else {
        U = w * x + tab(P.wdec, g) * U;
        return U;
    }
}

template <typename T, bool BANDS>
__device__ void strag_half(const EParams<T> &P, long line, long pq, int half, double &dep_out)
{
    const long S = P.NLINE, QS = (long)P.G * S;
    const T *rho = half ? P.rho_o : P.rho_c;
    const T *sf = (half ? P.sfac_o : P.sfac_c) + pq;
    const long FS = P.NPpad;
    const double ad = 0.5 * (double)P.h * (double)rho[pq];
    const T a = (T)ad;
    const bool hasQ = P.Q != nullptr, hasW = P.W != nullptr;
    T *W = hasW ? P.W + (long)half * QS : nullptr;
    const T *Q = hasQ ? P.Q + (long)half * QS : nullptr;
    double phn = 0, phs = 0, inj = 0;
    // sweep down: right-hand side, elimination (bt kept in place of X), scan of X^n
    T xu1 = 0, xu2 = 0, bu1 = 0, bu2 = 0;   // X^n and bt of group g+1
    T x1 = P.psi[(2L * (P.G - 1)) * S + line], x2 = P.psi[(2L * (P.G - 1) + 1) * S + line];
    T U = 0, Ub[4] = {};
    for (int g = P.G - 1; g >= 0; --g) {
        T xl1 = 0, xl2 = 0;   // X^n of group g-1
        if (g > 0) {
            xl1 = P.psi[(2L * (g - 1)) * S + line];
            xl2 = P.psi[(2L * (g - 1) + 1) * S + line];
        }
        const T *B = P.blk + (size_t)g * 12;
        const T q = hasQ ? Q[(long)g * S + line] : T(0);
        T b1 = x1 + a * (B[0] * xl1 + B[1] * xl2 + B[4] * x1 + B[5] * x2 + B[8] * xu1 + B[9] * xu2 + q);
        T b2 = x2 + a * (B[2] * xl1 + B[3] * xl2 + B[6] * x1 + B[7] * x2 + B[10] * xu1 + B[11] * xu2);
        const T *Fg = sf + (size_t)g * 8 * FS + 4 * FS;
        b1 += Fg[0] * bu1 + Fg[FS] * bu2;
        b2 += Fg[2 * FS] * bu1 + Fg[3 * FS] * bu2;
        P.psi[(2L * g) * S + line] = b1;
        P.psi[(2L * g + 1) * S + line] = b2;
        phn += tab(P.dA2, g) * (double)x1 + tab(P.dB2, g) * (double)x2;
        if (hasQ) inj += tab(P.dInj, g) * (double)q;
        if (hasW) W[(long)g * S + line] = scan_step<T, BANDS>(P, g, x1, U, Ub) * tab(P.invdE, g);
        xu1 = x1, xu2 = x2, bu1 = b1, bu2 = b2;
        x1 = xl1, x2 = xl2;
    }
    // sweep up: back-substitution
    T y1p = 0, y2p = 0;
    for (int g = 0; g < P.G; ++g) {
        const T *B = P.blk + (size_t)g * 12;
        T c1 = P.psi[(2L * g) * S + line], c2 = P.psi[(2L * g + 1) * S + line];
        c1 += a * (B[0] * y1p + B[1] * y2p);
        c2 += a * (B[2] * y1p + B[3] * y2p);
        const T *Di = sf + (size_t)g * 8 * FS;
        const T y1 = Di[0] * c1 + Di[FS] * c2, y2 = Di[2 * FS] * c1 + Di[3 * FS] * c2;
        P.psi[(2L * g) * S + line] = y1;
        P.psi[(2L * g + 1) * S + line] = y2;
        phs += tab(P.dA2, g) * (double)y1 + tab(P.dB2, g) * (double)y2;
        y1p = y1, y2p = y2;
    }
    // sweep down: the scan of X*, added to that of X^n
    if (hasW) {
        U = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) Ub[b] = 0;
        for (int g = P.G - 1; g >= 0; --g)
            W[(long)g * S + line] += scan_step<T, BANDS>(P, g, P.psi[(2L * g) * S + line], U, Ub) * tab(P.invdE, g);
    }
    dep_out = ad * (phn + phs - inj) * P.scale;
}

template <typename T, int MODE, bool BANDS>
__global__ __launch_bounds__(256) void epass_strag_kernel(EParams<T> P)
{
    const int NA = (int)(P.NAPT / PBS_PT);
    const int bx = blockIdx.x, pbk = bx / P.NOCT, oct = bx % P.NOCT;
    const int e = threadIdx.x >> 5, ptc = threadIdx.x & 31;
    const int a = oct * 8 + e;
    if (a >= NA) return;
    const long line = ((long)pbk * NA + a) * PBS_PT + ptc;
    const long pq = (long)pbk * PBS_PT + ptc;
    double d;
    if (MODE & MODE_CLOSE) {
        strag_half<T, BANDS>(P, line, pq, 0, d);
        P.dep_c[line] = d;
    }
    if (MODE & MODE_OPEN) {
        strag_half<T, BANDS>(P, line, pq, 1, d);
        P.dep_o[line] = d;
    }
}

template <typename T, bool BANDS>
static void launch_epass_strag_t(const EParams<T> &P, int mode, unsigned nb, hipStream_t st)
{
    if (mode == MODE_PAIR)
        hipLaunchKernelGGL((epass_strag_kernel<T, MODE_PAIR, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else if (mode == MODE_OPEN)
        hipLaunchKernelGGL((epass_strag_kernel<T, MODE_OPEN, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else
        hipLaunchKernelGGL((epass_strag_kernel<T, MODE_CLOSE, BANDS>), dim3(nb), dim3(256), 0, st, P);
}

template <typename T>
hipError_t launch_epass_strag(const EParams<T> &P, int mode, hipStream_t st)
{
    if (!P.blk || !P.dA2 || !P.dB2 || P.Wh != nullptr || P.inj_c != nullptr || P.NB > 4) return hipErrorInvalidValue;
    const unsigned nf = (unsigned)((P.NPpad + 255) / 256);
    if (mode & MODE_CLOSE) hipLaunchKernelGGL(strag_factor_kernel<T>, dim3(nf), dim3(256), 0, st, P.blk, P.rho_c, P.h,
                                              P.G, P.NPpad, P.sfac_c);
    if (mode & MODE_OPEN) hipLaunchKernelGGL(strag_factor_kernel<T>, dim3(nf), dim3(256), 0, st, P.blk, P.rho_o, P.h,
                                             P.G, P.NPpad, P.sfac_o);
    const unsigned nb = (unsigned)((P.NLINE / P.NAPT) * P.NOCT);
    if (P.NB > 1)
        launch_epass_strag_t<T, true>(P, mode, nb, st);
    else
        launch_epass_strag_t<T, false>(P, mode, nb, st);
    return hipGetLastError();
}
template hipError_t launch_epass_strag<float>(const EParams<float> &, int, hipStream_t);
template hipError_t launch_epass_strag<double>(const EParams<double> &, int, hipStream_t);

// Energy pass of FP32 contexts with the split-BF16 source product: one thread per (lateral cell,
// group of PBS_EPASS_LPT consecutive angular lines of an octet a = 8 oct + e).  The thread sweeps the
// groups of its lines together, so the scans of consecutive source nodes form one chunk (8 or 16
// bytes) of the [oct][cell][8] split layout that the thread writes itself (no exchange between
// threads, no barrier).  The FP64 deposits (and surrogate records) of those lines are summed into
// one partial per (cell, line group), stored at line slot a = line group; the dose reduction then
// sums NOCT * 8 / PBS_EPASS_LPT slots per cell instead of NA.  Lanes 0-31 hold the 32 cells of one
// tile.
// The energy pass streams the fluence (and the source) through once: non-temporal loads and stores
// keep it from displacing what the caches hold for others (measured 11.1 -> 10.9 ms per depth step of a
// 64 x 64-cell, 31 x 31-angle, 128-group, 4-generation beam).
#define EP_LD(p) __builtin_nontemporal_load(p)
#define EP_ST(v, p) __builtin_nontemporal_store(v, p)
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }
// FEAT / LO = false compile out the surrogate records and the lo half of the split scans.
template <int MODE, bool FEAT = true, bool LO = true, bool BANDS = false>
__device__ __forceinline__ void epass8_body(const EParams<float> &P, long gid)
{
    constexpr int L = PBS_EPASS_LPT;
    constexpr int NSUB = 8 / L;
    constexpr bool CL = (MODE & MODE_CLOSE) != 0;
    constexpr bool OP = (MODE & MODE_OPEN) != 0;
    const int NA = (int)(P.NAPT / PBS_PT);
    const long NPB = P.NLINE / P.NAPT;
    const int pt = (int)(gid & 31);
    const long r = gid >> 5;
    const int grp = (int)(r % (P.NOCT * NSUB));   // line group: octet grp / NSUB, lines 8 oct + L sub + e
    const int oct = grp / NSUB, sub = grp % NSUB;
    const long pbk = r / (P.NOCT * NSUB);
    if (pbk >= NPB) return;
    const int nval = min(L, NA - 8 * oct - L * sub);   // lines of this group that exist (may be <= 0)
    const long S = P.NLINE;
    const long QS = (long)P.G * S;
    const long line0 = ((long)pbk * NA + 8 * oct + L * sub) * PBS_PT + pt;   // line of e = 0; e adds PBS_PT
    const long pq = pbk * PBS_PT + pt;
    const double rc = CL ? (double)P.rho_c[pq] : 0.0;
    const double ro = OP ? (double)P.rho_o[pq] : 0.0;
    const double dac = 0.5 * (double)P.h * rc, dao = 0.5 * (double)P.h * ro;
    const float ac = (float)dac, ao = (float)dao;
    float fin[L], fcl[L], fop[L], U0[L], U1[L], U2[L];
#pragma unroll
    for (int e = 0; e < L; ++e) fin[e] = fcl[e] = fop[e] = U0[e] = U1[e] = U2[e] = 0.f;
    float U0b[BANDS ? 4 : 1][L] = {}, U1b[BANDS ? 4 : 1][L] = {}, U2b[BANDS ? 4 : 1][L] = {};   // per-band scans
    // rounding residue of the BF16 scans carried from group g+1 into group g (hi-only products)
    float rcc[L] = {}, rco[L] = {};
    double ph0 = 0, ph1 = 0, ph2 = 0, injc = 0, injo = 0;
    float fic = 0, fio = 0, fme = 0, fmn = 0;
    const bool hasQ = P.Q != nullptr, hasW = P.Wh != nullptr, hasL = LO && P.Wl != nullptr,
               feat = FEAT && P.inj_c != nullptr;
    const bool qbf = hasQ && P.Qb != nullptr;
    const int NAq = (NA + 3) & ~3;
    const long QSb = (long)P.G * NPB * NAq * PBS_PT;
    typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
    static_assert(L == 4, "the BF16 source is read as 4-line chunks");
    const long SB = (long)P.G * NPB * P.NOCT * (PBS_PT * 8);
    for (int g = P.G - 1; g >= 0; --g) {
        const float sm = tab(P.Sm, g), sp = tab(P.Sp, g), kp = tab(P.kap, g);
        const float d11 = -(sm + kp), d12 = sm, d21 = -3.f * sp, d22 = -(sp + 2.f * sm + kp);
        const float c1 = sp, c2 = 3.f * sp;
        const float mc11 = 1.f - ac * d11, mc12 = -ac * d12, mc21 = -ac * d21, mc22 = 1.f - ac * d22;
        const float mo11 = 1.f - ao * d11, mo12 = -ao * d12, mo21 = -ao * d21, mo22 = 1.f - ao * d22;
        const float ic = CL ? fast_rcp(mc11 * mc22 - mc12 * mc21) : 0.f;
        const float io = OP ? fast_rcp(mo11 * mo22 - mo12 * mo21) : 0.f;
        float *p1 = P.psi + (2L * g) * S + line0;
        float *p2 = p1 + S;
        float x1[L], x2[L], qc[L], qo[L];
#pragma unroll
        for (int e = 0; e < L; ++e) {
            const bool v = e < nval;
            x1[e] = v ? EP_LD(&p1[e * PBS_PT]) : 0.f;
            x2[e] = v ? EP_LD(&p2[e * PBS_PT]) : 0.f;
            qc[e] = qo[e] = 0.f;
            if (hasQ && !qbf && v) {
                const long o = (long)g * S + line0 + e * PBS_PT;
                if (CL) qc[e] = EP_LD(&P.Q[o]);
                if (OP) qo[e] = EP_LD(&P.Q[QS + o]);
            }
        }
        if (qbf && nval > 0) {
            // the BF16 source holds the thread's 4 lines of one cell as one 8-byte chunk
            const long o = (((long)g * NPB + pbk) * NAq + 8 * oct + L * sub) * PBS_PT + pt * L;
            if (CL) {
                const u16x4 c = EP_LD(reinterpret_cast<const u16x4 *>(P.Qb + o));
#pragma unroll
                for (int e = 0; e < L; ++e) qc[e] = e < nval ? bf16_to_f32(c[e]) : 0.f;
            }
            if (OP) {
                const u16x4 c = EP_LD(reinterpret_cast<const u16x4 *>(P.Qb + QSb + o));
#pragma unroll
                for (int e = 0; e < L; ++e) qo[e] = e < nval ? bf16_to_f32(c[e]) : 0.f;
            }
        }
        const float w = tab(P.wc, g), dec = tab(P.wdec, g), idE = tab(P.invdE, g);
        double s0a = 0, s0b = 0, s1a = 0, s1b = 0, s2a = 0, s2b = 0, sqc = 0, sqo = 0;
        typedef unsigned short chunk_t __attribute__((ext_vector_type(L)));
        chunk_t hc, lc, ho, lo;
#pragma unroll
        for (int e = 0; e < L; ++e) {
            float y1 = x1[e], y2 = x2[e];
            if (CL) {
                const float f = fin[e] + fcl[e];
                const float r1 = x1[e] + ac * (d11 * x1[e] + d12 * x2[e] + c1 * f + qc[e]);
                const float r2 = x2[e] + ac * (d21 * x1[e] + d22 * x2[e] + c2 * f);
                y1 = (r1 * mc22 - mc12 * r2) * ic;
                y2 = (mc11 * r2 - mc21 * r1) * ic;
            }
            float z1 = y1, z2 = y2;
            if (OP) {
                const float f = (CL ? fcl[e] : fin[e]) + fop[e];
                const float r1 = y1 + ao * (d11 * y1 + d12 * y2 + c1 * f + qo[e]);
                const float r2 = y2 + ao * (d21 * y1 + d22 * y2 + c2 * f);
                z1 = (r1 * mo22 - mo12 * r2) * io;
                z2 = (mo11 * r2 - mo21 * r1) * io;
            }
            if (e < nval) {
                EP_ST(z1, &p1[e * PBS_PT]);
                EP_ST(z2, &p2[e * PBS_PT]);
            }
            if (CL) {
                s0a += (double)x1[e];
                s0b += (double)x2[e];
                sqc += (double)qc[e];
            }
            s1a += (double)y1;
            s1b += (double)y2;
            if (OP) {
                s2a += (double)z1;
                s2b += (double)z2;
                sqo += (double)qo[e];
            }
            if (hasW || feat) {
                if constexpr (BANDS) {
                    // the sum of one scan per band, each with its band's decay; group g feeds its own band
                    const int bg = tab(P.band, g);
                    U0[e] = U1[e] = U2[e] = 0.f;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (b < P.NB) {
                            const float d = tab(P.wdecb, (long)b * P.G + g), wb = b == bg ? w : 0.f;
                            if (CL) U0[e] += (U0b[b][e] = wb * x1[e] + d * U0b[b][e]);
                            U1[e] += (U1b[b][e] = wb * y1 + d * U1b[b][e]);
                            if (OP) U2[e] += (U2b[b][e] = wb * z1 + d * U2b[b][e]);
                        }
                } else {
                    if (CL) U0[e] = w * x1[e] + dec * U0[e];
                    U1[e] = w * y1 + dec * U1[e];
                    if (OP) U2[e] = w * z1 + dec * U2[e];
                }
                const float vc = CL ? (U0[e] + U1[e]) * idE : 0.f;
                const float vo = OP ? (U1[e] + U2[e]) * idE : 0.f;
                if (hasL) {
                    const __bf16 bc = (__bf16)vc, bo = (__bf16)vo;
                    hc[e] = __builtin_bit_cast(unsigned short, bc);
                    ho[e] = __builtin_bit_cast(unsigned short, bo);
                    if constexpr (LO) {
                        lc[e] = __builtin_bit_cast(unsigned short, (__bf16)(vc - (float)bc));
                        lo[e] = __builtin_bit_cast(unsigned short, (__bf16)(vo - (float)bo));
                    }
                } else {
                    // only the rounded value enters the product: round with error feedback along the
                    // groups, so that the line's rounding errors telescope in the number and energy of
                    // the re-emitted protons instead of adding up
                    const float tc = vc + rcc[e], to = vo + rco[e];
                    const __bf16 bc = (__bf16)tc, bo = (__bf16)to;
                    hc[e] = __builtin_bit_cast(unsigned short, bc);
                    ho[e] = __builtin_bit_cast(unsigned short, bo);
                    rcc[e] = tc - (float)bc;
                    rco[e] = to - (float)bo;
                }
                if (feat) {
                    const float wi = (float)tab(P.dInj, g);
                    if (CL) fic += wi * vc;
                    if (OP) {
                        fio += wi * vo;
                        fme += (float)tab(P.wmom, g) * z1 + (float)tab(P.wmom, 2L * P.G + g) * z2;
                        fmn += (float)tab(P.wmom, (long)P.G + g) * z1;
                    }
                }
            }
            fin[e] = x1[e] - x2[e];
            fcl[e] = y1 - y2;
            fop[e] = z1 - z2;
        }
        // deposit functional (FP64), summed over the lines: A, B depend on the energy group only
        const double A = tab(P.dA, g), B = tab(P.dB, g);
        if (CL) ph0 += A * s0a + B * s0b;
        ph1 += A * s1a + B * s1b;
        if (OP) ph2 += A * s2a + B * s2b;
        if (g == 0) {
            if (CL) ph0 += P.dBot * (s0a - s0b);
            ph1 += P.dBot * (s1a - s1b);
            if (OP) ph2 += P.dBot * (s2a - s2b);
        }
        if (hasQ) {
            const double wi = tab(P.dInj, g);
            if (CL) injc += wi * sqc;
            if (OP) injo += wi * sqo;
        }
        if (hasW) {
            const long ob = (((long)g * NPB + pbk) * P.NOCT + oct) * (PBS_PT * 8) + pt * 8 + L * sub;
            if (CL) *reinterpret_cast<chunk_t *>(P.Wh + ob) = hc;
            if (OP) *reinterpret_cast<chunk_t *>(P.Wh + SB + ob) = ho;
            if constexpr (LO) {
                if (hasL) {
                    if (CL) *reinterpret_cast<chunk_t *>(P.Wl + ob) = lc;
                    if (OP) *reinterpret_cast<chunk_t *>(P.Wl + SB + ob) = lo;
                }
            }
        }
    }
    const long slot = ((long)pbk * NA + grp) * PBS_PT + pt;
    if (CL) P.dep_c[slot] = dac * (ph0 + ph1 - injc) * P.scale;
    if (OP) P.dep_o[slot] = dao * (ph1 + ph2 - injo) * P.scale;
    if (feat) {
        if (CL) P.inj_c[slot] = dac * (double)fic * P.scale;
        if (OP) {
            P.inj_o[slot] = dao * (double)fio * P.scale;
            P.mom_e[slot] = (double)fme * P.scale;
            P.mom_n[slot] = (double)fmn * P.scale;
        }
    }
}

// 5 waves per SIMD for the plain kernels (96 VGPRs, a few spilled registers): measured faster than 4
// waves without spills
// Minimum waves per SIMD of the plain energy passes (compile-time knob).  At 5 the compiler held the
// pair-mode kernel to 96 VGPRs and spilled 80 bytes per thread, reloaded in every group step; at 4 it
// takes 114 VGPRs with no scratch (config-2 energy pass 2.94 -> 2.71 ms per launch, config 3 -1 %).
#ifndef EP_WPE
#define EP_WPE 4
#endif
template <int MODE, bool FEAT, bool LO, bool BANDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FEAT || BANDS ? 1 : EP_WPE))) void epass8_kernel(
    EParams<float> P)
{
    epass8_body<MODE, FEAT, LO, BANDS>(P, (long)blockIdx.x * 256 + threadIdx.x);
}

template <bool FEAT, bool LO, bool BANDS = false>
static void launch_epass8_t(const EParams<float> &P, int mode, unsigned nb, hipStream_t st)
{
    if (mode == MODE_PAIR)
        hipLaunchKernelGGL((epass8_kernel<MODE_PAIR, FEAT, LO, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else if (mode == MODE_OPEN)
        hipLaunchKernelGGL((epass8_kernel<MODE_OPEN, FEAT, LO, BANDS>), dim3(nb), dim3(256), 0, st, P);
    else
        hipLaunchKernelGGL((epass8_kernel<MODE_CLOSE, FEAT, LO, BANDS>), dim3(nb), dim3(256), 0, st, P);
}

hipError_t launch_epass8(const EParams<float> &P, int mode, hipStream_t st)
{
    const long nthreads = (P.NLINE / P.NAPT) * P.NOCT * (8 / PBS_EPASS_LPT) * PBS_PT;
    const unsigned nb = (unsigned)((nthreads + 255) / 256);
    if (P.NB > 4) return hipErrorInvalidValue;
    if (P.NB > 1) {
        // banded nuclear data: no surrogate records
        if (P.inj_c != nullptr) return hipErrorInvalidValue;
        if (P.Wl != nullptr)
            launch_epass8_t<false, true, true>(P, mode, nb, st);
        else
            launch_epass8_t<false, false, true>(P, mode, nb, st);
    } else if (P.inj_c != nullptr)
        launch_epass8_t<true, true>(P, mode, nb, st);
    else if (P.Wl != nullptr)
        launch_epass8_t<false, true>(P, mode, nb, st);
    else
        launch_epass8_t<false, false>(P, mode, nb, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- transport pass
// Superbee-limited face slope without division: delta = Dface * eta(Dup / Dface).
// max(min(2|u|, |f|), min(|u|, 2|f|)) is the median of |u|, |f| and 2 min(|u|, |f|) (exact: doubling, min and
// max do not round); it is 0 when either difference is, so the sign test needs only the two sign bits.
template <typename T>
__device__ __forceinline__ T superbee_slope(T dup, T dface)
{
    const T au = fabs(dup), af = fabs(dface);
    if constexpr (sizeof(T) == 4) {
        const float v = __builtin_amdgcn_fmed3f(au, af, 2.f * fminf(au, af));
        // v <= 2|dup|, so clamping copysign(v, dface) between 0 and 2 dup keeps it when the two differences
        // agree in sign and gives 0 when they do not (no compare, no condition register)
        return __builtin_amdgcn_fmed3f(copysignf(v, dface), 0.f, 2.f * dup);
    } else {
        const T v = fmin(fmax(au, af), T(2) * fmin(au, af));
        return signbit(dup) == signbit(dface) ? copysign(v, dface) : T(0);
    }
}

// The transport sweep reads and writes every plane once: non-temporal loads and stores (both are needed:
// either alone measured no gain; together 12.6 -> 12.1 ms per depth step of a 64 x 64-cell, 31 x 31-angle,
// 128-group, 4-generation beam, 5.3 TB/s).
#define TP_LD(p) __builtin_nontemporal_load(p)
#define TP_ST(v, p) __builtin_nontemporal_store(v, p)
template <typename T, int NSEG>
__device__ __forceinline__ void tpass_body(const TParams<T> &P, long plane)
{
    const int lane = threadIdx.x & 63;
    if (plane >= P.nplanes) return;   // uniform per wave
    const int a = (int)(plane % P.NA);
    const long slab = plane / P.NA;
    const T cx = P.theta[a / P.m], cy = P.theta[a % P.m];
    const bool mx = cx < T(0), my = cy < T(0);   // sweep frames mirrored so the velocity is >= 0
    const T ax = fabs(cx) * P.h_half_over_dx, ay = fabs(cy) * P.h_half_over_dy;
    const T idiag = T(1) / (T(1) + ax + ay);
    const T cq = ay * idiag;
    T *base = P.psi + slab * P.NLINE + (long)a * PBS_PT;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx, ny = P.ny;

    int qcol[NSEG];
    bool valid[NSEG];
#pragma unroll
    for (int s = 0; s < NSEG; ++s) {
        const int qq = s * 64 + lane;
        valid[s] = qq < ny;
        qcol[s] = my ? ny - 1 - qq : qq;
    }
    // powers of the scan multiplier: cp[i] = cq^(2^i); cl = cq^(lane+1)
    T cp[7];
    cp[0] = cq;
#pragma unroll
    for (int i = 1; i < 7; ++i) cp[i] = cp[i - 1] * cp[i - 1];
    T cl = T(1);
#pragma unroll
    for (int i = 0; i < 7; ++i)
        if (((lane + 1) >> i) & 1) cl *= cp[i];

    auto load_row = [&](int r, T (&v)[NSEG]) {
        const int p = mx ? nx - 1 - r : r;
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            T x = T(0);
            if (r < nx && valid[s]) {
                const long pq = (long)p * ny + qcol[s];
                x = TP_LD(&base[(pq / PBS_PT) * NAPT + (pq % PBS_PT)]);
            }
            v[s] = x;
        }
    };

    T pm1[NSEG], p0[NSEG], p1[NSEG], p2[NSEG], dxm[NSEG], ym1[NSEG];
#pragma unroll
    for (int s = 0; s < NSEG; ++s) pm1[s] = dxm[s] = ym1[s] = T(0);
    load_row(0, p0);
    load_row(1, p1);
    for (int r = 0; r < nx; ++r) {
        load_row(r + 2, p2);
        T left[NSEG], dyp[NSEG];
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            const T up = __shfl_up(p0[s], 1);
            const T dn = __shfl_down(p0[s], 1);
            const T prev_last = s > 0 ? __shfl(p0[s > 0 ? s - 1 : 0], 63) : T(0);
            const T next_first = s + 1 < NSEG ? __shfl(p0[s + 1 < NSEG ? s + 1 : 0], 0) : T(0);
            left[s] = lane == 0 ? prev_last : up;
            const T right = lane == 63 ? next_first : dn;
            dyp[s] = superbee_slope(p0[s] - left[s], right - p0[s]);
        }
        T b[NSEG];
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            const T up = __shfl_up(dyp[s], 1);
            const T prev_last = s > 0 ? __shfl(dyp[s > 0 ? s - 1 : 0], 63) : T(0);
            const T dym = lane == 0 ? prev_last : up;
            const T dxp = superbee_slope(p0[s] - pm1[s], p1[s] - p0[s]);
            const T R = p0[s] - ax * ((p0[s] - pm1[s]) + (dxp - dxm[s])) - ay * ((p0[s] - left[s]) + (dyp[s] - dym));
            b[s] = (R + ax * ym1[s]) * idiag;
            dxm[s] = dxp;
        }
        // implicit recurrence along the row: y_q = b_q + cq * y_{q-1}
        T carry = T(0);
        const int p = mx ? nx - 1 - r : r;
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            T y = b[s];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const int d = 1 << i;
                const T t = __shfl_up(y, d);
                if (lane >= d) y += cp[i] * t;
            }
            y += cl * carry;
            carry = __shfl(y, 63);
            ym1[s] = y;
            if (valid[s]) {
                const long pq = (long)p * ny + qcol[s];
                TP_ST(y, &base[(pq / PBS_PT) * NAPT + (pq % PBS_PT)]);
            }
        }
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            pm1[s] = p0[s];
            p0[s] = p1[s];
            p1[s] = p2[s];
        }
    }
}

template <typename T, int NSEG>
__global__ __launch_bounds__(256) void tpass_kernel(TParams<T> P)
{
    tpass_body<T, NSEG>(P, (long)blockIdx.x * 4 + (threadIdx.x >> 6));
}

// FP32 variant for ny <= 64: cross-lane moves by DPP (wave_shr/shl:1 for the y neighbours, a
// row_shr / row_bcast affine scan for the implicit row solve) and 8 rows in flight per wave.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWMASK, 0xF,
                                                                 false));
}

// All lanes written, lanes without a source read 0: the form the compiler folds into the DPP operand of the
// consuming VALU op (a row-scan step becomes one v_fmac_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp_z(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}
// DPP controls (GFX9): row_shr:n = 0x110 + n, wave_shl:1 = 0x130, wave_shr:1 = 0x138,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.  Lanes without a source receive 0 (the ghost value).

// One step of a row scan, y += c * y[source lane of the DPP pattern], as a single v_fmac_f32_dpp (rows
// outside the row mask keep y; lanes without a source read 0 and keep y).  The compiler does not fold a
// DPP move into a multiply-accumulate (a move plus an FMA per step), so the step is written out; the
// leading s_nop gives the two wait states a DPP read needs after a VALU write of its source.  Only used
// where the whole wave is active.
#define PBS_FMAC_DPP(y, c, ctrl, rmask) \
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %0, %1 " ctrl " row_mask:" rmask " bank_mask:0xf bound_ctrl:1" \
                 : "+v"(y) : "v"(c))

// y_q = b_q + c y_{q-1} within each 16-lane row: Kogge-Stone over distances 1, 2, 4, 8 (multipliers c^d)
__device__ __forceinline__ void scan_rows16(float &y, float c1, float c2, float c4, float c8)
{
    PBS_FMAC_DPP(y, c1, "row_shr:1", "0xf");
    PBS_FMAC_DPP(y, c2, "row_shr:2", "0xf");
    PBS_FMAC_DPP(y, c4, "row_shr:4", "0xf");
    PBS_FMAC_DPP(y, c8, "row_shr:8", "0xf");
}
// ... then lane 15 of rows 0 and 2 into rows 1 and 3 (m16 = c^((lane & 15) + 1)) ...
__device__ __forceinline__ void scan_join32(float &y, float m16) { PBS_FMAC_DPP(y, m16, "row_bcast:15", "0xa"); }
// ... then lane 31 into rows 2 and 3 (m32 = c^((lane & 31) + 1))
__device__ __forceinline__ void scan_join64(float &y, float m32) { PBS_FMAC_DPP(y, m32, "row_bcast:31", "0xc"); }
// two wait states after the last scan step, for any DPP read of y that the compiler places next
__device__ __forceinline__ void scan_done() { asm volatile("s_nop 1"); }

__device__ __forceinline__ void tpass_dpp_body(const TParams<float> &P, long plane)
{
    if (plane >= P.nplanes) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    const int a = (int)(plane % P.NA);
    const long slab = plane / P.NA;
    const float cx = P.theta[a / P.m], cy = P.theta[a % P.m];
    const bool mx = cx < 0.f, my = cy < 0.f;
    const float ax = fabsf(cx) * P.h_half_over_dx, ay = fabsf(cy) * P.h_half_over_dy;
    const float idiag = 1.f / (1.f + ax + ay);
    const float cq = ay * idiag;
    float *base = P.psi + slab * P.NLINE + (long)a * PBS_PT;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx, ny = P.ny;
    const bool valid = lane < ny;
    const int qc = my ? ny - 1 - lane : lane;
    // scan multipliers: c^1, c^2, c^4, c^8 within rows of 16 lanes; c^((lane&15)+1), c^((lane&31)+1)
    const float c1 = cq, c2 = c1 * c1, c4 = c2 * c2, c8 = c4 * c4;
    float m16 = 1.f, m32 = 1.f;
    {
        const int e16 = (lane & 15) + 1, e32 = (lane & 31) + 1;
        float pw = cq;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if ((e16 >> i) & 1) m16 *= pw;
            if ((e32 >> i) & 1) m32 *= pw;
            pw *= pw;
        }
    }
    auto addr = [&](int r) -> float * {
        const int p = mx ? nx - 1 - r : r;
        const long pq = (long)p * ny + qc;
        return base + (pq / PBS_PT) * NAPT + (pq % PBS_PT);
    };
    float rb[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) rb[i] = (valid && i < nx) ? *addr(i) : 0.f;
    float pm1 = 0.f, dxm = 0.f, ym1 = 0.f;
    for (int r0 = 0; r0 < nx; r0 += 8) {
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[8 + i] = (valid && r0 + 8 + i < nx) ? *addr(r0 + 8 + i) : 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (r0 + i >= nx) break;
            const float p0 = rb[i], p1 = rb[i + 1];
            const float left = dpp_f<0x138, 0xF>(p0);
            const float right = dpp_f<0x130, 0xF>(p0);
            const float dyp = superbee_slope(p0 - left, right - p0);
            const float dym = dpp_f<0x138, 0xF>(dyp);
            const float dxp = superbee_slope(p0 - pm1, p1 - p0);
            const float R = p0 - ax * ((p0 - pm1) + (dxp - dxm)) - ay * ((p0 - left) + (dyp - dym));
            float y = (R + ax * ym1) * idiag;
            // y_q = b_q + c y_{q-1} along the row: Kogge-Stone within rows of 16, then row broadcasts
            scan_rows16(y, c1, c2, c4, c8);
            scan_join32(y, m16);
            scan_join64(y, m32);
            scan_done();
            if (valid) *addr(r0 + i) = y;
            pm1 = p0;
            dxm = dxp;
            ym1 = y;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[i] = rb[8 + i];
    }
}

__global__ __launch_bounds__(256) void tpass_dpp_kernel(TParams<float> P)
{
    tpass_dpp_body(P, (long)blockIdx.x * 4 + (threadIdx.x >> 6));
}

constexpr int TPASS_PF = 8;   // rows of the row-affine sweep loaded ahead (nx must be a multiple)

// Same sweep when ny is 32 or 64 and nx a multiple of TPASS_PF: a lane's address is affine in the row
// (row stride = ny/32 lateral tiles), so each row costs one pointer increment and no guards; lanes
// beyond ny (ny = 32) read a clamped in-range column and are zeroed.
template <int NY>
__device__ __forceinline__ void tpass_affine_body(const TParams<float> &P, long plane)
{
    if (plane >= P.nplanes) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    const int a = (int)(plane % P.NA);
    const long slab = plane / P.NA;
    const float cx = P.theta[a / P.m], cy = P.theta[a % P.m];
    const bool mx = cx < 0.f, my = cy < 0.f;
    const float ax = fabsf(cx) * P.h_half_over_dx, ay = fabsf(cy) * P.h_half_over_dy;
    const float idiag = 1.f / (1.f + ax + ay);
    const float cq = ay * idiag;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx;
    constexpr bool FULL = NY == 64;
    const bool valid = FULL || lane < NY;
    const int ql = FULL ? lane : (lane < NY ? lane : NY - 1);
    const int qc = my ? NY - 1 - ql : ql;
    const long RS = (long)(NY / 32) * NAPT;   // elements from row p to row p+1
    float *row0 = P.psi + slab * P.NLINE + (long)a * PBS_PT + (long)(qc >> 5) * NAPT + (qc & 31);
    const long step = mx ? -RS : RS;
    float *ptr = mx ? row0 + (long)(nx - 1) * RS : row0;
    const float c1 = cq, c2 = c1 * c1, c4 = c2 * c2, c8 = c4 * c4;
    float m16 = 1.f, m32 = 1.f;
    {
        const int e16 = (lane & 15) + 1, e32 = (lane & 31) + 1;
        float pw = cq;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if ((e16 >> i) & 1) m16 *= pw;
            if ((e32 >> i) & 1) m32 *= pw;
            pw *= pw;
        }
        // the broadcasts write every row: rows 0 and 2 (row_bcast15) and lanes 0-31 (row_bcast31) add nothing
        if (!((lane >> 4) & 1)) m16 = 0.f;
        if (lane < 32) m32 = 0.f;
    }
    const float vmask = valid ? 1.f : 0.f;
    constexpr int PF = TPASS_PF;   // rows loaded ahead of the sweep
    float rb[2 * PF];
    const float *ld = ptr;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        rb[i] = i < nx ? TP_LD(ld) * vmask : 0.f;
        if (i < nx) ld += step;
    }
    float *st = ptr;
    float pm1 = 0.f, dxm = 0.f, ym1 = 0.f;
    for (int r0 = 0; r0 < nx; r0 += PF) {
        const bool more = r0 + PF < nx;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            rb[PF + i] = more ? TP_LD(ld) * vmask : 0.f;
            if (more) ld += step;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const float p0 = rb[i], p1 = rb[i + 1];
            const float left = dpp_z<0x138>(p0);
            const float right = dpp_z<0x130>(p0);
            const float dyp = superbee_slope(p0 - left, right - p0);
            const float dym = dpp_z<0x138>(dyp);
            const float dxp = superbee_slope(p0 - pm1, p1 - p0);
            const float R = p0 - ax * ((p0 - pm1) + (dxp - dxm)) - ay * ((p0 - left) + (dyp - dym));
            float y = (R + ax * ym1) * idiag;
            scan_rows16(y, c1, c2, c4, c8);
            scan_join32(y, m16);
            scan_join64(y, m32);
            scan_done();
            if (FULL || valid) TP_ST(y, st);
            st += step;
            pm1 = p0;
            dxm = dxp;
            ym1 = y;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) rb[i] = rb[PF + i];
    }
}

template <int NY>
__global__ __launch_bounds__(256) void tpass_affine_kernel(TParams<float> P)
{
    tpass_affine_body<NY>(P, (long)blockIdx.x * 4 + (threadIdx.x >> 6));
}

// Same sweep for ny = 32 with two planes per wave: lanes 0-31 sweep plane 2w, lanes 32-63 plane 2w+1, each
// half with its own angle, mirroring and pointer. Neighbour moves that would cross the halves are zeroed,
// the row scan stops at the 16-lane broadcast (it never crosses lane 31/32), and a half without a plane
// (odd plane count) repeats its neighbour's loads and stores nothing. Every lane carries a cell, where the
// one-plane sweep left half of them idle.
__device__ __forceinline__ void tpass_pair_body(const TParams<float> &P, long pair)
{
    if (pair * 2 >= P.nplanes) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    const int ql = lane & 31;
    const long plane = pair * 2 + (lane >> 5);
    const bool live = plane < P.nplanes;
    const long pl = live ? plane : plane - 1;
    const int a = (int)(pl % P.NA);
    const long slab = pl / P.NA;
    const float cx = P.theta[a / P.m], cy = P.theta[a % P.m];
    const bool mx = cx < 0.f, my = cy < 0.f;
    const float ax = fabsf(cx) * P.h_half_over_dx, ay = fabsf(cy) * P.h_half_over_dy;
    const float idiag = 1.f / (1.f + ax + ay);
    const float cq = ay * idiag;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx;
    const int qc = my ? 31 - ql : ql;
    const long RS = NAPT;   // one lateral tile per row
    float *row0 = P.psi + slab * P.NLINE + (long)a * PBS_PT + qc;
    const long step = mx ? -RS : RS;
    float *ptr = mx ? row0 + (long)(nx - 1) * RS : row0;
    const float c1 = cq, c2 = c1 * c1, c4 = c2 * c2, c8 = c4 * c4;
    float m16 = 1.f;
    {
        const int e16 = (lane & 15) + 1;
        float pw = cq;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            if ((e16 >> i) & 1) m16 *= pw;
            pw *= pw;
        }
        // row_bcast15 writes every row: rows 0 and 2 of the wave (the first 16 lanes of each half) add nothing
        if (!((lane >> 4) & 1)) m16 = 0.f;
    }
    // 0 on the lanes whose neighbour move would cross into the other half, else 1.  Kept opaque so that
    // the compiler does not turn "move, then zero some lanes" into a move under a partial exec mask, where
    // the lanes switched off would also stop serving as move sources.
    float keep_l = ql == 0 ? 0.f : 1.f, keep_r = ql == 31 ? 0.f : 1.f;
    asm volatile("" : "+v"(keep_l), "+v"(keep_r));
    constexpr int PF = TPASS_PF;   // rows loaded ahead of the sweep
    float rb[2 * PF];
    const float *ld = ptr;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        rb[i] = i < nx ? TP_LD(ld) : 0.f;
        if (i < nx) ld += step;
    }
    float *st = ptr;
    float pm1 = 0.f, dxm = 0.f, ym1 = 0.f;
    for (int r0 = 0; r0 < nx; r0 += PF) {
        const bool more = r0 + PF < nx;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            rb[PF + i] = more ? TP_LD(ld) : 0.f;
            if (more) ld += step;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const float p0 = rb[i], p1 = rb[i + 1];
            const float left = keep_l * dpp_z<0x138>(p0);
            const float right = keep_r * dpp_z<0x130>(p0);
            const float dyp = superbee_slope(p0 - left, right - p0);
            const float dym = keep_l * dpp_z<0x138>(dyp);
            const float dxp = superbee_slope(p0 - pm1, p1 - p0);
            const float R = p0 - ax * ((p0 - pm1) + (dxp - dxm)) - ay * ((p0 - left) + (dyp - dym));
            float y = (R + ax * ym1) * idiag;
            scan_rows16(y, c1, c2, c4, c8);
            scan_join32(y, m16);
            scan_done();
            if (live) TP_ST(y, st);
            st += step;
            pm1 = p0;
            dxm = dxp;
            ym1 = y;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) rb[i] = rb[PF + i];
    }
}

__global__ __launch_bounds__(256) void tpass_pair_kernel(TParams<float> P)
{
    tpass_pair_body(P, (long)blockIdx.x * 4 + (threadIdx.x >> 6));
}

constexpr int TPASS_WIDE_PF = 4;   // rows loaded ahead per segment (4 measured faster than 8 or 2 at ny = 96)

// Same sweep for ny = 96 or 128 (two 64-lane segments per row, ny a multiple of the 32-column lateral
// tile, so every segment's address stays affine in the row): neighbours at a segment seam and the carry of
// the implicit row recurrence cross it by readlane; lanes beyond ny read a clamped column and are zeroed.
template <int NY>
__device__ __forceinline__ void tpass_wide_body(const TParams<float> &P, long plane)
{
    static_assert(NY % 32 == 0 && NY > 64 && NY <= 128, "two segments of whole lateral tiles");
    constexpr int NS = 2;
    if (plane >= P.nplanes) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    const int a = (int)(plane % P.NA);
    const long slab = plane / P.NA;
    const float cx = P.theta[a / P.m], cy = P.theta[a % P.m];
    const bool mx = cx < 0.f, my = cy < 0.f;
    const float ax = fabsf(cx) * P.h_half_over_dx, ay = fabsf(cy) * P.h_half_over_dy;
    const float idiag = 1.f / (1.f + ax + ay);
    const float cq = ay * idiag;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx;
    const long RS = (long)(NY / 32) * NAPT;   // elements from row p to row p+1
    const long step = mx ? -RS : RS;
    float vmask[NS];
    bool valid[NS];
    const float *ld[NS];
    float *st[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = s * 64 + lane;
        valid[s] = q < NY;
        const int ql = valid[s] ? q : NY - 1;
        const int qc = my ? NY - 1 - ql : ql;
        float *row0 = P.psi + slab * P.NLINE + (long)a * PBS_PT + (long)(qc >> 5) * NAPT + (qc & 31);
        st[s] = mx ? row0 + (long)(nx - 1) * RS : row0;
        ld[s] = st[s];
        vmask[s] = valid[s] ? 1.f : 0.f;
    }
    // scan multipliers: cq^(2^i) for the row shifts, cq^((lane&15)+1), cq^((lane&31)+1) for the row
    // broadcasts and cq^(lane+1) for the carry from the previous segment
    const float c1 = cq, c2 = c1 * c1, c4 = c2 * c2, c8 = c4 * c4;
    float m16 = 1.f, m32 = 1.f, m64 = 1.f;
    {
        const int e16 = (lane & 15) + 1, e32 = (lane & 31) + 1, e64 = lane + 1;
        float pw = cq;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            if ((e16 >> i) & 1) m16 *= pw;
            if ((e32 >> i) & 1) m32 *= pw;
            if ((e64 >> i) & 1) m64 *= pw;
            pw *= pw;
        }
        // the broadcasts write every row: rows 0 and 2 (row_bcast15) and lanes 0-31 (row_bcast31) add nothing
        if (!((lane >> 4) & 1)) m16 = 0.f;
        if (lane < 32) m32 = 0.f;
    }
    auto lane_of = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
    constexpr int PF = TPASS_WIDE_PF;   // rows loaded ahead of the sweep
    float rb[2 * PF][NS];
#pragma unroll
    for (int i = 0; i < PF; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            rb[i][s] = i < nx ? TP_LD(ld[s]) * vmask[s] : 0.f;
            if (i < nx) ld[s] += step;
        }
    float pm1[NS], dxm[NS], ym1[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) pm1[s] = dxm[s] = ym1[s] = 0.f;
    for (int r0 = 0; r0 < nx; r0 += PF) {
        const bool more = r0 + PF < nx;
#pragma unroll
        for (int i = 0; i < PF; ++i)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                rb[PF + i][s] = more ? TP_LD(ld[s]) * vmask[s] : 0.f;
                if (more) ld[s] += step;
            }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            float left[NS], dyp[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float p0 = rb[i][s];
                const float up = dpp_z<0x138>(p0), dn = dpp_z<0x130>(p0);
                left[s] = (s > 0 && lane == 0) ? lane_of(rb[i][s > 0 ? s - 1 : 0], 63) : up;
                const float right = (s + 1 < NS && lane == 63) ? lane_of(rb[i][s + 1 < NS ? s + 1 : 0], 0) : dn;
                dyp[s] = superbee_slope(p0 - left[s], right - p0);
            }
            float carry = 0.f;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float p0 = rb[i][s], p1 = rb[i + 1][s];
                const float up = dpp_z<0x138>(dyp[s]);
                const float dym = (s > 0 && lane == 0) ? lane_of(dyp[s > 0 ? s - 1 : 0], 63) : up;
                const float dxp = superbee_slope(p0 - pm1[s], p1 - p0);
                const float R = p0 - ax * ((p0 - pm1[s]) + (dxp - dxm[s])) - ay * ((p0 - left[s]) + (dyp[s] - dym));
                float y = (R + ax * ym1[s]) * idiag;
                scan_rows16(y, c1, c2, c4, c8);
                scan_join32(y, m16);
                scan_join64(y, m32);
                scan_done();
                if (s > 0) y += m64 * carry;
                carry = lane_of(y, 63);
                if (valid[s]) TP_ST(y, st[s]);
                st[s] += step;
                pm1[s] = p0;
                dxm[s] = dxp;
                ym1[s] = y;
            }
        }
#pragma unroll
        for (int i = 0; i < PF; ++i)
#pragma unroll
            for (int s = 0; s < NS; ++s) rb[i][s] = rb[PF + i][s];
    }
}

template <int NY>
__global__ __launch_bounds__(256) void tpass_wide_kernel(TParams<float> P)
{
    tpass_wide_body<NY>(P, (long)blockIdx.x * 4 + (threadIdx.x >> 6));
}

constexpr int TPASS_W2_PF = 4;   // rows loaded ahead per operation in the two-plane ny = 96 sweep
// LDS reserved per block of the two-plane sweep, which uses none: it caps the sweep at 3 blocks (12 waves)
// per CU.  Fewer concurrent plane streams suit the memory system: a copy with the sweep's addresses runs
// 5.18 -> 5.43 TB/s at 2 blocks per CU, and the config-3 sweep 8.76 -> 8.47 ms per launch at 2 or 3.
#ifndef TP_W2_LDS
#define TP_W2_LDS 54000
#endif

// ny = 96 with two planes per wave (A = plane 2w, B = plane 2w + 1; the plane count is even).  A row of
// both planes is three full 64-lane operations: A columns 0-63, B columns 0-63, then A columns 64-95 in
// lanes 0-31 beside B columns 64-95 in lanes 32-63.  The one-plane sweep of this width spends two
// operations per row with a quarter of its lanes idle and is instruction-bound; here no lane idles.
// The third operation carries each half's own angle coefficients; its row scan stops at the 16-lane
// broadcast (it never crosses lane 31/32) and takes the carry y_63 of its plane's first operation.
// Neighbours across the seams (A 63|64, B 63|64) move by readlane and masked products; column 96 is the
// ghost.
// Addresses are 32-bit byte offsets in a buffer resource based at plane A's slab (plane B lies in the
// same slab or the next); each lane steps by its plane's signed row stride.
__device__ __forceinline__ void tpass_wide2_body(const TParams<float> &P, int pair)
{
    constexpr int NY = 96;
    if (2L * pair >= P.nplanes) return;   // uniform per wave
    const int lane = threadIdx.x & 63;
    const int ql = lane & 31;
    const bool hi = lane >= 32;
    const long NAPT = (long)P.NA * PBS_PT;
    const int nx = P.nx;
    const long plA = 2L * pair, plB = plA + 1;
    const int aA = (int)(plA % P.NA), aB = (int)(plB % P.NA);
    const long slabA = plA / P.NA, slabB = plB / P.NA;
    const float cxA = P.theta[aA / P.m], cyA = P.theta[aA % P.m];
    const float cxB = P.theta[aB / P.m], cyB = P.theta[aB % P.m];
    const bool mxA = cxA < 0.f, myA = cyA < 0.f, mxB = cxB < 0.f, myB = cyB < 0.f;
    const float axA = fabsf(cxA) * P.h_half_over_dx, ayA = fabsf(cyA) * P.h_half_over_dy;
    const float axB = fabsf(cxB) * P.h_half_over_dx, ayB = fabsf(cyB) * P.h_half_over_dy;
    const float idA = 1.f / (1.f + axA + ayA), idB = 1.f / (1.f + axB + ayB);
    const float cqA = ayA * idA, cqB = ayB * idB;
    // byte offsets from plane A's slab: plane origin + column (mirrored) + first row (mirrored)
    const long RSB = 3 * NAPT * 4;   // bytes from row p to row p + 1
    const long originA = (long)aA * PBS_PT * 4;
    const long originB = ((slabB - slabA) * P.NLINE + (long)aB * PBS_PT) * 4;
    auto col = [&](int q, bool my) -> long {
        const int qc = my ? NY - 1 - q : q;
        return ((long)(qc >> 5) * NAPT + (qc & 31)) * 4;
    };
    const long row0A = mxA ? (long)(nx - 1) * RSB : 0, row0B = mxB ? (long)(nx - 1) * RSB : 0;
    const int stepA = (int)(mxA ? -RSB : RSB), stepB = (int)(mxB ? -RSB : RSB);
    unsigned ld[3], st[3];
    int step[3];
    ld[0] = (unsigned)(originA + col(lane, myA) + row0A);
    ld[1] = (unsigned)(originB + col(lane, myB) + row0B);
    ld[2] = (unsigned)(hi ? originB + col(64 + ql, myB) + row0B : originA + col(64 + ql, myA) + row0A);
    step[0] = stepA;
    step[1] = stepB;
    step[2] = hi ? stepB : stepA;
#pragma unroll
    for (int o = 0; o < 3; ++o) st[o] = ld[o];
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(P.psi + slabA * P.NLINE), (short)0, (int)(2 * P.NLINE * 4 < 0x7fffffffL ? 2 * P.NLINE * 4 : 0x7fffffffL),
        0x00020000);
    // scan multipliers per operation: cq^(2^i) for the row shifts, cq^((lane & 15) + 1) and
    // cq^((lane & 31) + 1) for the broadcasts; in the third operation each half has its own cq, and
    // cq^(ql + 1) takes the carry of its plane's first operation (zero in the other half)
    auto powers = [](float cq, int e) {
        float m = 1.f, pw = cq;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            if ((e >> i) & 1) m *= pw;
            pw *= pw;
        }
        return m;
    };
    float c1[3], c2[3], c4[3], c8[3], m16[3], ax[3], ay[3], idg[3];
    const float cq3 = hi ? cqB : cqA;
    const float cqs[3] = {cqA, cqB, cq3};
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        c1[o] = cqs[o];
        c2[o] = c1[o] * c1[o];
        c4[o] = c2[o] * c2[o];
        c8[o] = c4[o] * c4[o];
        m16[o] = powers(cqs[o], (lane & 15) + 1);
    }
    const float m32A = powers(cqA, (lane & 31) + 1), m32B = powers(cqB, (lane & 31) + 1);
    const float mcA = hi ? 0.f : powers(cqA, ql + 1), mcB = hi ? powers(cqB, ql + 1) : 0.f;
    ax[0] = axA; ay[0] = ayA; idg[0] = idA;
    ax[1] = axB; ay[1] = ayB; idg[1] = idB;
    ax[2] = hi ? axB : axA; ay[2] = hi ? ayB : ayA; idg[2] = hi ? idB : idA;
    // lane masks for the seam corrections, kept opaque (a select would run the DPP moves next to it under
    // a partial exec mask, where the switched-off lanes would stop serving as move sources)
    float e63 = lane == 63 ? 1.f : 0.f, e0 = lane == 0 ? 1.f : 0.f, e32 = lane == 32 ? 1.f : 0.f;
    float keep_l = ql == 0 ? 0.f : 1.f, keep_r = ql == 31 ? 0.f : 1.f;
    asm volatile("" : "+v"(e63), "+v"(e0), "+v"(e32), "+v"(keep_l), "+v"(keep_r));
    auto lane_of = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
    // the left neighbour in the third operation: the lane below, but plane A's and plane B's column 63
    // (scalars sa, sb) in lanes 0 and 32 -- exact, as every other term is a product with 0
    auto left3 = [&](float v, float sa, float sb) { return keep_l * dpp_z<0x138>(v) + e0 * sa + e32 * sb; };
    constexpr int PF = TPASS_W2_PF;
    float rb[3][2 * PF];
#pragma unroll
    for (int i = 0; i < PF; ++i)
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            rb[o][i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ld[o], 0, 2));
            ld[o] += step[o];
        }
    float dxb[3], dxm[3], ym1[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        dxb[o] = rb[o][0];   // p0 - p_{-1} with the ghost row upstream
        dxm[o] = ym1[o] = 0.f;
    }
    for (int r0 = 0; r0 < nx; r0 += PF) {
        const bool more = r0 + PF < nx;
        if (more) {
#pragma unroll
            for (int i = 0; i < PF; ++i)
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    rb[o][PF + i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ld[o], 0, 2));
                    ld[o] += step[o];
                }
        } else {
#pragma unroll
            for (int i = 0; i < PF; ++i)
#pragma unroll
                for (int o = 0; o < 3; ++o) rb[o][PF + i] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            float p0[3], dy[3], ayv[3];
#pragma unroll
            for (int o = 0; o < 3; ++o) p0[o] = rb[o][i];
            // lateral differences p0 - left and right - p0, seams patched
            const float rA = lane_of(p0[2], 0), rB = lane_of(p0[2], 32);
            const float lA = lane_of(p0[0], 63), lB = lane_of(p0[1], 63);
            float bf[3];
            ayv[0] = p0[0] - dpp_z<0x138>(p0[0]);
            bf[0] = dpp_z<0x130>(p0[0]) - p0[0] + e63 * rA;
            ayv[1] = p0[1] - dpp_z<0x138>(p0[1]);
            bf[1] = dpp_z<0x130>(p0[1]) - p0[1] + e63 * rB;
            ayv[2] = p0[2] - left3(p0[2], lA, lB);
            bf[2] = keep_r * dpp_z<0x130>(p0[2]) - p0[2];
#pragma unroll
            for (int o = 0; o < 3; ++o) dy[o] = superbee_slope(ayv[o], bf[o]);
            // dyp - dym, the seams taking the upstream plane's lane-63 slope
            float dd[3];
            dd[0] = dy[0] - dpp_z<0x138>(dy[0]);
            dd[1] = dy[1] - dpp_z<0x138>(dy[1]);
            dd[2] = dy[2] - left3(dy[2], lane_of(dy[0], 63), lane_of(dy[1], 63));
            float y[3];
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                const float dxf = rb[o][i + 1] - p0[o];
                const float dxp = superbee_slope(dxb[o], dxf);
                const float R = p0[o] - ax[o] * (dxb[o] + (dxp - dxm[o])) - ay[o] * (ayv[o] + dd[o]);
                y[o] = (R + ax[o] * ym1[o]) * idg[o];
                dxb[o] = dxf;
                dxm[o] = dxp;
            }
            scan_rows16(y[0], c1[0], c2[0], c4[0], c8[0]);
            scan_join32(y[0], m16[0]);
            scan_join64(y[0], m32A);
            scan_rows16(y[1], c1[1], c2[1], c4[1], c8[1]);
            scan_join32(y[1], m16[1]);
            scan_join64(y[1], m32B);
            scan_rows16(y[2], c1[2], c2[2], c4[2], c8[2]);
            scan_join32(y[2], m16[2]);
            scan_done();
            y[2] += mcA * lane_of(y[0], 63);
            y[2] += mcB * lane_of(y[1], 63);
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, y[o]), rs, st[o], 0, 2);
                st[o] += step[o];
                ym1[o] = y[o];
            }
        }
#pragma unroll
        for (int i = 0; i < PF; ++i)
#pragma unroll
            for (int o = 0; o < 3; ++o) rb[o][i] = rb[o][PF + i];
    }
}

__global__ __launch_bounds__(256) void tpass_wide2_kernel(TParams<float> P)
{
    tpass_wide2_body(P, __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6))));
}

template <typename T>
hipError_t launch_tpass(const TParams<T> &P, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        const dim3 grid((unsigned)((P.nplanes + 3) / 4));
        if (P.nx % TPASS_PF == 0 && P.ny == 64) {
            hipLaunchKernelGGL(tpass_affine_kernel<64>, grid, dim3(256), 0, st, P);
            return hipGetLastError();
        }
        if (P.nx % TPASS_PF == 0 && P.ny == 32) {
            const long pairs = (P.nplanes + 1) / 2;
            hipLaunchKernelGGL(tpass_pair_kernel, dim3((unsigned)((pairs + 3) / 4)), dim3(256), 0, st, P);
            return hipGetLastError();
        }
        if (P.nx % TPASS_W2_PF == 0 && P.ny == 96 && P.nplanes % 2 == 0 && 2 * P.NLINE * 4 < 0x7fffffffL &&
            P.nplanes / 2 < 0x7fffffffL) {
            const long pairs = P.nplanes / 2;
            hipLaunchKernelGGL(tpass_wide2_kernel, dim3((unsigned)((pairs + 3) / 4)), dim3(256), TP_W2_LDS, st, P);
            return hipGetLastError();
        }
        if (P.nx % TPASS_PF == 0 && P.ny == 96) {
            hipLaunchKernelGGL(tpass_wide_kernel<96>, grid, dim3(256), 0, st, P);
            return hipGetLastError();
        }
        if (P.nx % TPASS_PF == 0 && P.ny == 128) {
            hipLaunchKernelGGL(tpass_wide_kernel<128>, grid, dim3(256), 0, st, P);
            return hipGetLastError();
        }
        if (P.ny <= 64) {
            hipLaunchKernelGGL(tpass_dpp_kernel, grid, dim3(256), 0, st, P);
            return hipGetLastError();
        }
    }
    const unsigned nb = (unsigned)((P.nplanes + 3) / 4);
    const int nseg = (P.ny + 63) / 64;
    switch (nseg) {
    case 1: hipLaunchKernelGGL((tpass_kernel<T, 1>), dim3(nb), dim3(256), 0, st, P); break;
    case 2: hipLaunchKernelGGL((tpass_kernel<T, 2>), dim3(nb), dim3(256), 0, st, P); break;
    case 3: hipLaunchKernelGGL((tpass_kernel<T, 3>), dim3(nb), dim3(256), 0, st, P); break;
    case 4: hipLaunchKernelGGL((tpass_kernel<T, 4>), dim3(nb), dim3(256), 0, st, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- angular pass
// y_M = sum_n sin(pi M n / N) x_n over the interior nodes n, M = 1..N-1, with the even/odd split
// sin(pi M (N-n)/N) = (-1)^(M+1) sin(pi M n/N).  S[(M-1)*(N-1) + (n-1)] holds the sines.
template <typename T, int N>
__device__ __forceinline__ void dst1(const T (&x)[N - 1], T (&y)[N - 1], const T *__restrict__ S)
{
    constexpr int H = N / 2;
    T sp[H], dm[H];
#pragma unroll
    for (int n = 1; n < H; ++n) {
        sp[n - 1] = x[n - 1] + x[N - n - 1];
        dm[n - 1] = x[n - 1] - x[N - n - 1];
    }
    sp[H - 1] = x[H - 1];
#pragma unroll
    for (int M = 1; M < N; M += 2) {   // odd modes: symmetric part + centre node
        T acc = T(0);
#pragma unroll
        for (int n = 1; n <= H; ++n) acc += S[(M - 1) * (N - 1) + (n - 1)] * sp[n - 1];
        y[M - 1] = acc;
    }
#pragma unroll
    for (int M = 2; M < N; M += 2) {   // even modes: antisymmetric part
        T acc = T(0);
#pragma unroll
        for (int n = 1; n < H; ++n) acc += S[(M - 1) * (N - 1) + (n - 1)] * dm[n - 1];
        y[M - 1] = acc;
    }
}

template <typename T, int N, int PC>
__device__ __forceinline__ void apass_body(const AParams<T> &P, int bx, long by)
{
    constexpr int m = N - 1;
    constexpr int NA = m * m;
    extern __shared__ char smem_raw[];
    T *L = reinterpret_cast<T *>(smem_raw);   // [NA][PC]
    const int tid = threadIdx.x;
    const long stack = by;           // (k*G + g)*2 + l
    const int g = (int)((stack / 2) % P.G);
    const int pb = bx / (PBS_PT / PC);
    const int c0 = (bx % (PBS_PT / PC)) * PC;
    T *blk = P.psi + stack * P.NLINE + (long)pb * NA * PBS_PT + c0;
    // 8 loads in flight per thread before their LDS stores (a load-store loop waits for each in turn)
    for (int i0 = tid; i0 < NA * PC; i0 += 8 * 256) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * 256;
            if (idx < NA * PC) v[u] = blk[(long)(idx / PC) * PBS_PT + idx % PC];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * 256;
            if (idx < NA * PC) L[idx] = v[u];
        }
    }
    __syncthreads();
    constexpr T inv2N = T(2) / T(N);
    // forward transform over the first angular index for every (j, column)
    for (int it = tid; it < m * PC; it += 256) {
        const int j = it / PC, c = it % PC;
        T x[m], y[m];
#pragma unroll
        for (int i = 0; i < m; ++i) x[i] = L[(i * m + j) * PC + c];
        dst1<T, N>(x, y, P.S);
#pragma unroll
        for (int k = 0; k < m; ++k) L[(k * m + j) * PC + c] = y[k];
    }
    __syncthreads();
    // over the second index: forward, CN factor (1 + a lam)/(1 - a lam), inverse
    const T coef = T(0.25) * P.h * P.sig[g];   // (h/2) * sigma_tr/2, times rho
    for (int it = tid; it < m * PC; it += 256) {
        const int k = it / PC, c = it % PC;
        const T al = coef * P.rho[(long)pb * PBS_PT + c0 + c];
        const T lk = P.lam[k];
        T x[m], y[m];
#pragma unroll
        for (int j = 0; j < m; ++j) x[j] = L[(k * m + j) * PC + c];
        dst1<T, N>(x, y, P.S);
#pragma unroll
        for (int n = 0; n < m; ++n) {
            const T lm = al * (lk + P.lam[n]);
            y[n] = y[n] * (T(1) + lm) * fast_rcp(T(1) - lm);
        }
        dst1<T, N>(y, x, P.S);
#pragma unroll
        for (int j = 0; j < m; ++j) L[(k * m + j) * PC + c] = x[j] * inv2N;
    }
    __syncthreads();
    // inverse over the first index
    for (int it = tid; it < m * PC; it += 256) {
        const int j = it / PC, c = it % PC;
        T x[m], y[m];
#pragma unroll
        for (int k = 0; k < m; ++k) x[k] = L[(k * m + j) * PC + c];
        dst1<T, N>(x, y, P.S);
#pragma unroll
        for (int i = 0; i < m; ++i) L[(i * m + j) * PC + c] = y[i] * inv2N;
    }
    __syncthreads();
    for (int idx = tid; idx < NA * PC; idx += 256) {
        const int a = idx / PC, c = idx % PC;
        blk[(long)a * PBS_PT + c] = L[idx];
    }
}

template <typename T, int N, int PC>
__global__ __launch_bounds__(256) void apass_kernel(AParams<T> P)
{
    apass_body<T, N, PC>(P, blockIdx.x, blockIdx.y);
}

template <typename T, int N>
static hipError_t launch_apass_n(const AParams<T> &P, long nstack, hipStream_t st)
{
    constexpr int NA = (N - 1) * (N - 1);
    const size_t lim = 64 * 1024;
    int pc = 32;
    while (pc > 1 && (size_t)NA * pc * sizeof(T) > lim) pc /= 2;
    dim3 grid((unsigned)(P.NPB * (PBS_PT / pc)), (unsigned)nstack);
    const size_t sh = (size_t)NA * pc * sizeof(T);
    switch (pc) {
    case 32: hipLaunchKernelGGL((apass_kernel<T, N, 32>), grid, dim3(256), sh, st, P); break;
    case 16: hipLaunchKernelGGL((apass_kernel<T, N, 16>), grid, dim3(256), sh, st, P); break;
    case 8: hipLaunchKernelGGL((apass_kernel<T, N, 8>), grid, dim3(256), sh, st, P); break;
    case 4: hipLaunchKernelGGL((apass_kernel<T, N, 4>), grid, dim3(256), sh, st, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// MFMA version for nth = 32 (31 interior nodes), FP32.  Each of the four 31-point sine transforms
// is split by mode parity into two 16 x 16 blocks (odd modes act on x_n + x_{32-n} plus the centre
// node, even modes on x_n - x_{32-n}); the inverse uses the transposed blocks with the output
// butterflies x_n = u + v, x_{32-n} = u - v.  Every block product is a chain of four
// v_mfma_f32_16x16x4_f32 whose 16 columns are 16 lateral cells of one angular line.  The block's
// 31 x 31 x 16 values stay in LDS between the passes over the two indices (a block barrier after each);
// within a pass each wave owns whole lines and works in place.
// LDS banks: an MFMA result holds rows 4 (lane / 16) + q in lane groups of 16, so writing row r of the
// result with r = 4 (lane / 16) + q puts the four lane groups of one store 4 rows apart, a multiple of
// the bank count at every row stride here (4-way conflicts).  The operand rows are therefore permuted,
// result row 4 g + q holding output index 4 q + g, so one store's lane groups are one row apart; and
// the modes are kept de-interleaved (odd block in rows 0-15, even block in rows 16-30, in both angular
// directions), so consecutive odd (even) modes are adjacent.  Every LDS access then reaches 32
// distinct banks per half wave.  The same permutation makes a result the next product's operand: element
// q of lane group g holds index 4 q + g, which lane group g supplies at chain step q, so the modes of the
// second index go from the forward product to the inverse one in registers.
//   Ktab[(mat*4 + s)*64 + lane] = A_mat[perm(lane % 16)][4 s + lane / 16] for mat = Sodd, Seven and
//   A_mat[4 s + lane / 16][perm(lane % 16)] for mat = Sodd^T, Seven^T, perm(4 g + q) = 4 q + g.
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 16 waves per block: the dependent MFMA chains of a line are short, so latency is hidden by the
// number of lines in flight (2 blocks of 61.5 KB LDS per CU = 32 waves)
constexpr int APASS32_NT = 1024;
__device__ __forceinline__ void apass_mfma32_body(const AParams<float> &P, const float *__restrict__ Ktab, long stack,
                                                  int pb, int half)
{
    constexpr int m = 31, NA = 961, PC = 16;
    __shared__ float L[NA * PC];   // L[a*16 + c], a = i*31 + j
    const int c0 = half * PC;
    const int g = (int)((stack / 2) % P.G);
    float *blk = P.psi + stack * P.NLINE + (long)pb * NA * PBS_PT + c0;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r4 = lane >> 4, cc = lane & 15;
    for (int idx = tid; idx < NA * 4; idx += APASS32_NT) {
        const int a = idx >> 2, q = idx & 3;
        *reinterpret_cast<float4 *>(&L[a * PC + q * 4]) = *reinterpret_cast<const float4 *>(blk + (long)a * PBS_PT + q * 4);
    }
    float Ao[4], Ae[4], Bo[4], Be[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        Ao[s] = Ktab[(0 * 4 + s) * 64 + lane];
        Ae[s] = Ktab[(1 * 4 + s) * 64 + lane];
        Bo[s] = Ktab[(2 * 4 + s) * 64 + lane];
        Be[s] = Ktab[(3 * 4 + s) * 64 + lane];
    }
    // result row 4 r4 + q holds mode (or node) block index 4 q + r4
    float lamO[4], lamE[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + r4;
        lamO[q] = P.lam[2 * r];
        lamE[q] = r < 15 ? P.lam[2 * r + 1] : 0.f;
    }
    const float al = 0.25f * P.h * P.sig[g] * P.rho[(long)pb * PBS_PT + c0 + cc];
    __syncthreads();

    // forward over the first angular index; line = column j.  Odd mode r -> row r, even mode r -> row 16 + r.
    for (int j = wid; j < m; j += APASS32_NT / 64) {
        floatx4 yo = {0.f, 0.f, 0.f, 0.f}, ye = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int ip = 4 * s + r4;
            const float xa = L[(ip * m + j) * PC + cc];
            const float xb = ip < 15 ? L[((30 - ip) * m + j) * PC + cc] : 0.f;
            yo = mfma16(Ao[s], ip < 15 ? xa + xb : xa, yo);
            ye = mfma16(Ae[s], xa - xb, ye);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + r4;
            L[(r * m + j) * PC + cc] = yo[q];
            if (r < 15) L[((16 + r) * m + j) * PC + cc] = ye[q];
        }
    }
    __syncthreads();
    // over the second index: forward, CN factor, inverse; line = row k (odd mode k, or even mode k - 16, of
    // the first index)
    for (int k = wid; k < m; k += APASS32_NT / 64) {
        floatx4 zo = {0.f, 0.f, 0.f, 0.f}, ze = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int jp = 4 * s + r4;
            const float ya = L[(k * m + jp) * PC + cc];
            const float yb = jp < 15 ? L[(k * m + 30 - jp) * PC + cc] : 0.f;
            zo = mfma16(Ao[s], jp < 15 ? ya + yb : ya, zo);
            ze = mfma16(Ae[s], ya - yb, ze);
        }
        const float lk = P.lam[k < 16 ? 2 * k : 2 * (k - 16) + 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + r4;
            const float to = al * (lk + lamO[q]);
            zo[q] = zo[q] * (1.f + to) * __builtin_amdgcn_rcpf(1.f - to);
            const float te = al * (lk + lamE[q]);
            ze[q] = r < 15 ? ze[q] * (1.f + te) * __builtin_amdgcn_rcpf(1.f - te) : 0.f;
        }
        // the scaled modes are already the inverse's B operands: element s of lane group r4 holds mode
        // 4 s + r4, the operand of step s (the permuted rows make the MFMA result layout the operand layout)
        floatx4 u = {0.f, 0.f, 0.f, 0.f}, v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            u = mfma16(Bo[s], zo[s], u);
            v = mfma16(Be[s], ze[s], v);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jp = 4 * q + r4;
            if (jp < 15) {
                L[(k * m + jp) * PC + cc] = u[q] + v[q];
                L[(k * m + 30 - jp) * PC + cc] = u[q] - v[q];
            } else {
                L[(k * m + 15) * PC + cc] = u[q];
            }
        }
    }
    __syncthreads();
    // inverse over the first index, with the (2/N)^2 normalisation
    constexpr float sc = (2.f / 32.f) * (2.f / 32.f);
    for (int j = wid; j < m; j += APASS32_NT / 64) {
        floatx4 u = {0.f, 0.f, 0.f, 0.f}, v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = 4 * s + r4;
            const float bo = L[(r * m + j) * PC + cc];
            const float be = r < 15 ? L[((16 + r) * m + j) * PC + cc] : 0.f;
            u = mfma16(Bo[s], bo, u);
            v = mfma16(Be[s], be, v);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ip = 4 * q + r4;
            if (ip < 15) {
                L[(ip * m + j) * PC + cc] = (u[q] + v[q]) * sc;
                L[((30 - ip) * m + j) * PC + cc] = (u[q] - v[q]) * sc;
            } else {
                L[(15 * m + j) * PC + cc] = u[q] * sc;
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < NA * 4; idx += APASS32_NT) {
        const int a = idx >> 2, q = idx & 3;
        *reinterpret_cast<float4 *>(blk + (long)a * PBS_PT + q * 4) = *reinterpret_cast<const float4 *>(&L[a * PC + q * 4]);
    }
}

// MFMA version for nth = 16 (15 interior nodes), FP32: each 15-point sine transform is one dense
// 16 x 16 product (the matrix zero-padded), a chain of four v_mfma_f32_16x16x4_f32 whose 16 columns
// are 16 lateral cells of one angular line; the 15 x 15 x 16 block (14.4 KB) stays in LDS.  The sine
// matrix is symmetric, so the inverse uses the same operand table with the factor 2/N.  As in the
// 32-node pass the operand rows are permuted, so that result element q of lane group g holds index
// 4 q + g: a store's lane groups then land in adjacent rows, and the modes of the second index feed
// the inverse product straight from registers.
//   Ktab[s*64 + lane] = S[perm(lane % 16)][4 s + lane / 16], S[r][k] = sin(pi (r+1)(k+1) / 16), zero at
//   15, perm(4 g + q) = 4 q + g.
__device__ __forceinline__ void apass_mfma16_body(const AParams<float> &P, const float *__restrict__ Ktab, long stack,
                                                  int pb, int half)
{
    constexpr int m = 15, NA = 225, PC = 16, NT = 256;
    __shared__ float L[NA * PC];   // L[a*16 + c], a = i*15 + j
    const int c0 = half * PC;
    const int g = (int)((stack / 2) % P.G);
    float *blk = P.psi + stack * P.NLINE + (long)pb * NA * PBS_PT + c0;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r4 = lane >> 4, cc = lane & 15;
    for (int idx = tid; idx < NA * 4; idx += NT) {
        const int a = idx >> 2, q = idx & 3;
        *reinterpret_cast<float4 *>(&L[a * PC + q * 4]) = *reinterpret_cast<const float4 *>(blk + (long)a * PBS_PT + q * 4);
    }
    float A[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) A[s] = Ktab[s * 64 + lane];
    // result element q of lane group r4 holds index 4 q + r4 (permuted operand rows)
    float lamR[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + r4;
        lamR[q] = r < m ? P.lam[r] : 0.f;
    }
    const float al = 0.25f * P.h * P.sig[g] * P.rho[(long)pb * PBS_PT + c0 + cc];
    constexpr float sc = 2.f / 16.f;
    __syncthreads();
    // forward over the first angular index; line = column j
    for (int j = wid; j < m; j += NT / 64) {
        floatx4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int ip = 4 * s + r4;
            y = mfma16(A[s], ip < m ? L[(ip * m + j) * PC + cc] : 0.f, y);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + r4;
            if (r < m) L[(r * m + j) * PC + cc] = y[q];
        }
    }
    __syncthreads();
    // over the second index: forward, CN factor, inverse; line = mode k of the first index
    for (int k = wid; k < m; k += NT / 64) {
        floatx4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int jp = 4 * s + r4;
            z = mfma16(A[s], jp < m ? L[(k * m + jp) * PC + cc] : 0.f, z);
        }
        const float lk = P.lam[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float t = al * (lk + lamR[q]);
            z[q] = z[q] * (1.f + t) * __builtin_amdgcn_rcpf(1.f - t);
        }
        // the scaled modes are already the inverse's B operands (element s of lane group r4 is mode 4 s + r4,
        // the operand of step s; mode 15 is zero: its operand row is)
        floatx4 u = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) u = mfma16(A[s], z[s], u);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jp = 4 * q + r4;
            if (jp < m) L[(k * m + jp) * PC + cc] = u[q] * sc;
        }
    }
    __syncthreads();
    // inverse over the first index
    for (int j = wid; j < m; j += NT / 64) {
        floatx4 u = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = 4 * s + r4;
            u = mfma16(A[s], r < m ? L[(r * m + j) * PC + cc] : 0.f, u);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ip = 4 * q + r4;
            if (ip < m) L[(ip * m + j) * PC + cc] = u[q] * sc;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < NA * 4; idx += NT) {
        const int a = idx >> 2, q = idx & 3;
        *reinterpret_cast<float4 *>(blk + (long)a * PBS_PT + q * 4) = *reinterpret_cast<const float4 *>(&L[a * PC + q * 4]);
    }
}

__global__ __launch_bounds__(256) void apass_mfma16_kernel(AParams<float> P, const float *__restrict__ Ktab, int npb)
{
    // the two 16-column halves of one lateral tile are 8 workgroups apart -> same XCD, same L2 lines
    const int bid = blockIdx.x;
    const int pb = (bid >> 4) * 8 + (bid & 7), half = (bid >> 3) & 1;
    if (pb >= npb) return;
    apass_mfma16_body(P, Ktab, blockIdx.y, pb, half);
}

hipError_t launch_apass_mfma16(const AParams<float> &P, const float *Ktab, long nstack, hipStream_t st)
{
    const int nb = (P.NPB + 7) / 8 * 16;
    hipLaunchKernelGGL(apass_mfma16_kernel, dim3(nb, (unsigned)nstack), dim3(256), 0, st, P, Ktab, P.NPB);
    return hipGetLastError();
}

// two blocks per CU need <= 64 VGPRs (8 waves per SIMD)
__global__ __launch_bounds__(APASS32_NT) __attribute__((amdgpu_waves_per_eu(8))) void apass_mfma32_kernel(
    AParams<float> P, const float *__restrict__ Ktab, int npb)
{
    // the two 16-column halves of one lateral tile are 8 workgroups apart -> same XCD, same L2 lines
    const int bid = blockIdx.x;
    const int pb = (bid >> 4) * 8 + (bid & 7), half = (bid >> 3) & 1;
    if (pb >= npb) return;
    apass_mfma32_body(P, Ktab, blockIdx.y, pb, half);
}

hipError_t launch_apass_mfma32(const AParams<float> &P, const float *Ktab, long nstack, hipStream_t st)
{
    const int nb = (P.NPB + 7) / 8 * 16;
    hipLaunchKernelGGL(apass_mfma32_kernel, dim3(nb, (unsigned)nstack), dim3(APASS32_NT), 0, st, P, Ktab, P.NPB);
    return hipGetLastError();
}

bool apass_supported(int nth)
{
    switch (nth) {
    case 4: case 6: case 8: case 10: case 12: case 16: case 20: case 24: case 32: return true;
    default: return false;
    }
}

template <typename T>
hipError_t launch_apass(const AParams<T> &P, int nth, long nstack, hipStream_t st)
{
    switch (nth) {
    case 4: return launch_apass_n<T, 4>(P, nstack, st);
    case 6: return launch_apass_n<T, 6>(P, nstack, st);
    case 8: return launch_apass_n<T, 8>(P, nstack, st);
    case 10: return launch_apass_n<T, 10>(P, nstack, st);
    case 12: return launch_apass_n<T, 12>(P, nstack, st);
    case 16: return launch_apass_n<T, 16>(P, nstack, st);
    case 20: return launch_apass_n<T, 20>(P, nstack, st);
    case 24: return launch_apass_n<T, 24>(P, nstack, st);
    case 32: return launch_apass_n<T, 32>(P, nstack, st);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------- source angular product
// Q[s][g][pb][a][pt] = sum_a' P2T[a][a'] W[s][g][pb][a'][pt]; block = 64 rows x 32 columns.
template <typename T>
__global__ __launch_bounds__(256) void qgemm_kernel(QParams<T> P)
{
    const long bt = blockIdx.x;   // ((si*G + g)*NPB + pb)
    const int mt = blockIdx.y;
    const int pb = (int)(bt % P.NPB);
    const long sg = bt / P.NPB;
    const int g = (int)(sg % P.G);
    const int s = P.s0 + (int)(sg / P.G);
    const long off = ((long)s * P.G + g) * P.NLINE + (long)pb * P.NA * PBS_PT;
    const T *B = P.W + off;
    T *C = P.Q + off;
    const T *P2T = P.P2T + (P.band ? (long)P.band[g] * P.NA * P.NA : 0L);   // the destination group's band
    __shared__ T As[64][33];
    __shared__ T Bs[32][32];
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const int NA = P.NA;
    T acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = T(0);
    for (int k0 = 0; k0 < NA; k0 += 32) {
        for (int idx = tid; idx < 64 * 32; idx += 256) {
            const int row = idx >> 5, kk = idx & 31;
            const int ga = mt * 64 + row, gk = k0 + kk;
            As[row][kk] = (ga < NA && gk < NA) ? P2T[(long)ga * NA + gk] : T(0);
        }
        for (int idx = tid; idx < 32 * 32; idx += 256) {
            const int kk = idx >> 5, col = idx & 31;
            const int gk = k0 + kk;
            Bs[kk][col] = gk < NA ? B[(long)gk * PBS_PT + col] : T(0);
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const T bv = Bs[kk][tx];
#pragma unroll
            for (int r = 0; r < 8; ++r) acc[r] += As[ty + 8 * r][kk] * bv;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int ga = mt * 64 + ty + 8 * r;
        if (ga < NA) C[(long)ga * PBS_PT + tx] = acc[r];
    }
}

// FP32 MFMA version (v_mfma_f32_32x32x2_f32).  Block tile 128 destination nodes x 128 columns
// (4 lateral tiles of one (half-step, group) panel); 4 waves in 2 x 2, each 64 x 64 = 2 x 2
// MFMA tiles.  A is the zero-padded P2 [Kp][Mp] (source-major), staged k-major in LDS like B.
typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void qgemm_mfma_f32_kernel(QParams<float> P, int nmt, int nnt, long nlogical,
                                                             long per_xcd)
{
    // Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a contiguous range of
    // logical tiles so the M tiles that share one B panel run back to back on the same L2.
    const long bid = blockIdx.x;
    const long logical = (bid & 7) * per_xcd + (bid >> 3);
    if (logical >= nlogical) return;
    const int mt = (int)(logical % nmt);
    const long rest = logical / nmt;
    const int nt = (int)(rest % nnt);
    const long batch = rest / nnt;
    const int s = P.s0 + (int)(batch / P.G), g = (int)(batch % P.G);
    const long off = ((long)s * P.G + g) * P.NLINE;
    const float *__restrict__ P2p = P.P2p + (P.band ? (long)P.band[g] * P.Kp * P.Mp : 0L);
    const float *__restrict__ B = P.W + off;
    float *__restrict__ C = P.Q + off;
    const long NAPT = (long)P.NA * PBS_PT;
    __shared__ float As[16][132];
    __shared__ float Bs[16][132];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    const int nk = P.Kp / 16;
    float4 ra[2], rb[2];
    auto gload = [&](int kt) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx >> 5, q4 = idx & 31;
            ra[i] = *reinterpret_cast<const float4 *>(P2p + (long)(kt * 16 + k) * P.Mp + mt * 128 + q4 * 4);
            const int pb = nt * 4 + (q4 >> 3), pt = (q4 & 7) * 4;
            const int gk = kt * 16 + k;
            if (gk < P.NA && pb < P.NPB)
                rb[i] = *reinterpret_cast<const float4 *>(B + pb * NAPT + (long)gk * PBS_PT + pt);
            else
                rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx >> 5, q4 = idx & 31;
            *reinterpret_cast<float4 *>(&As[k][q4 * 4]) = ra[i];
            *reinterpret_cast<float4 *>(&Bs[k][q4 * 4]) = rb[i];
        }
    };
    gload(0);
    sstore();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const int kr = 2 * kk + (lane >> 5);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 64 + i * 32 + (lane & 31)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn * 64 + j * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int pb = nt * 4 + wn * 2 + j;
            if (pb >= P.NPB) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = mt * 128 + wm * 64 + i * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
                if (row < P.NA) C[pb * NAPT + (long)row * PBS_PT + (lane & 31)] = acc[i][j][r];
            }
        }
}

// Split-BF16 version on v_mfma_f32_32x32x16_bf16: each FP32 operand is written as hi + lo
// (hi = bf16(x), lo = bf16(x - hi), |x - hi - lo| <= 2^-16 |x|) and the product is accumulated in
// FP32 as A_lo B_hi + A_hi B_lo + A_hi B_hi (the A_lo B_lo term, O(2^-16), is dropped).
// Block tile 128 destination nodes x 256 columns (8 lateral tiles), BK = 32; 8 waves in 2 x 4,
// each 64 x 64 = 2 x 2 MFMA tiles.  A = P2 split on the host, row-major [Mp][Kp] (k contiguous);
// B arrives split from the energy pass, 8 consecutive source nodes contiguous per lateral cell.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// a float moved between the lanes of each quad by the DPP quad permutation CTRL
template <int CTRL>
__device__ __forceinline__ float dpp_quad(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Stores one 32 x 32 accumulator tile of v_mfma_f32_32x32x16 (rows row0 .. row0 + 31 of lateral tile pb)
// into the source Q [pb][row][32 cells].  Lane l holds column l % 32 of rows (r % 4) + 8 (r / 4) + 4 (l / 32):
// for each group r / 4 a 4 x 4 transpose inside every quad of lanes (two DPP butterfly stages) leaves
// lane t of the quad with row t of the group for the quad's 4 columns, written as one 16-byte store, so a
// wave writes 1 KB contiguous (8 rows of 32 cells) per instruction.  Non-temporal: the source is read
// once, by the next generation's energy pass, and is kept out of the caches the product streams through.
__device__ __forceinline__ void store_source_tile(float *__restrict__ C, long NAPT, int pb, int row0,
                                                  const floatx16 &a, int lane, int NA, int NPB)
{
    const int t4 = lane & 3;
    const bool up1 = (t4 & 1) != 0, up2 = (t4 & 2) != 0;
    // one butterfly: lanes with `up` send x and take the partner's y into x; the others send y and take
    // the partner's x into y (quad_perm [1,0,3,2] for the first stage, [2,3,0,1] for the second)
    auto b1 = [&](float &x, float &y) {
        const float r = dpp_quad<0xB1>(up1 ? x : y);
        if (up1) x = r; else y = r;
    };
    auto b2 = [&](float &x, float &y) {
        const float r = dpp_quad<0x4E>(up2 ? x : y);
        if (up2) x = r; else y = r;
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float v0 = a[4 * q], v1 = a[4 * q + 1], v2 = a[4 * q + 2], v3 = a[4 * q + 3];
        b1(v0, v1);
        b1(v2, v3);
        b2(v0, v2);
        b2(v1, v3);
        const int row = row0 + 8 * q + 4 * (lane >> 5) + t4;
        if (pb < NPB && row < NA)
            __builtin_nontemporal_store(
                floatx4{v0, v1, v2, v3},
                reinterpret_cast<floatx4 *>(&C[pb * NAPT + (long)row * PBS_PT + ((lane & 31) & ~3)]));
    }
}

// The same tile into the BF16 source [pb][row / 4][32 cells][4] (Qb): lane l holds column l % 32 of rows
// 8 q + 4 (l / 32) + 0..3, i.e. one 4-row group of one cell, which leaves as one 8-byte store (each wave
// instruction writes 2 x 256 B contiguous) with no exchange between lanes.  Rows NA .. NAq - 1 come from
// the zero-padded rows of the transfer matrix.
__device__ __forceinline__ void store_source_tile_bf16(unsigned short *__restrict__ Cb, int NAq, int pb, int row0,
                                                       const floatx16 &a, int lane, int NPB)
{
    typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = row0 + 8 * q + 4 * (lane >> 5);
        if (pb < NPB && row < NAq) {
            u16x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = __builtin_bit_cast(unsigned short, (__bf16)a[4 * q + e]);
            __builtin_nontemporal_store(v, reinterpret_cast<u16x4 *>(&Cb[((long)pb * NAq + row) * PBS_PT + (lane & 31) * 4]));
        }
    }
}

template <int BN, int NPROD>
__device__ __forceinline__ void qgemm_bf16s_body(const QParams<float> &P, const unsigned short *__restrict__ Ahi,
                                                  const unsigned short *__restrict__ Alo, int Kp, int nmt, int nnt,
                                                  long nlogical, long per_xcd, long bid)
{
    constexpr int BK = 32, LD = BK + 8;   // LDS row stride in bf16 elements (80 B)
    constexpr int NPBT = BN / 32;         // lateral tiles per block
    constexpr int WN = BN / 64;           // waves along N (2 along M)
    constexpr int NT = 128 * WN;          // threads
    constexpr bool BLO = NPROD == 3;      // the lo part of the scanned fluence takes part
    constexpr bool ALO = NPROD >= 2;      // the lo part of the transfer matrix takes part
    __shared__ unsigned short sAh[128 * LD], sAl[ALO ? 128 * LD : 8], sBh[BN * LD], sBl[BLO ? BN * LD : 8];
    const long logical = (bid & 7) * per_xcd + (bid >> 3);
    if (logical >= nlogical) return;
    const int mt = (int)(logical % nmt);
    const long rest = logical / nmt;
    const int nt = (int)(rest % nnt);
    const long batch = rest / nnt;
    const int s = P.s0 + (int)(batch / P.G), g = (int)(batch % P.G);
    if (P.band) {   // the transfer matrix of the destination group's band
        const long bo = (long)P.band[g] * 3 * P.Mp * Kp;
        Ahi += bo;
        Alo += bo;
    }
    const long off = ((long)s * P.G + g) * P.NLINE;
    float *__restrict__ C = P.Q + off;
    const int NAq = (P.NA + 3) & ~3;
    unsigned short *__restrict__ Cb = P.Qb ? P.Qb + ((long)s * P.G + g) * P.NPB * NAq * PBS_PT : nullptr;
    const long NAPT = (long)P.NA * PBS_PT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    const int nk = Kp / BK;
    // staging: A chunks (row, 8 k) c = tid + NT*i over 128 x 4; B items column tid % BN, octets tid / BN and +2
    constexpr int NA_CH = 512 / NT;
    const int bcol = tid % BN, boct = tid / BN;
    const int bpb = nt * NPBT + (bcol >> 5), bpt = bcol & 31;
    const bool bok = bpb < P.NPB;
    const long bbase = (((long)s * P.G + g) * P.NPB + (bok ? bpb : 0)) * P.NOCT * (PBS_PT * 8) + bpt * 8;
    u16x8 rah[NA_CH], ral[NA_CH];
    u16x8 rbh[2], rbl[2];
    auto gload = [&](int kt) {
#pragma unroll
        for (int c = 0; c < NA_CH; ++c) {
            const int ch = tid + NT * c, arow = ch >> 2, akq = ch & 3;
            const long ao = (long)(mt * 128 + arow) * Kp + kt * BK + akq * 8;
            rah[c] = *reinterpret_cast<const u16x8 *>(Ahi + ao);
            if constexpr (ALO) ral[c] = *reinterpret_cast<const u16x8 *>(Alo + ao);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int oc = kt * (BK / 8) + boct + 2 * h;
            if (bok && oc < P.NOCT) {
                rbh[h] = *reinterpret_cast<const u16x8 *>(P.Bh + bbase + (long)oc * (PBS_PT * 8));
                if constexpr (BLO) rbl[h] = *reinterpret_cast<const u16x8 *>(P.Bl + bbase + (long)oc * (PBS_PT * 8));
            } else {
                rbh[h] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                if constexpr (BLO) rbl[h] = rbh[h];
            }
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int c = 0; c < NA_CH; ++c) {
            const int ch = tid + NT * c, arow = ch >> 2, akq = ch & 3;
            *reinterpret_cast<u16x8 *>(&sAh[arow * LD + akq * 8]) = rah[c];
            if constexpr (ALO) *reinterpret_cast<u16x8 *>(&sAl[arow * LD + akq * 8]) = ral[c];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<u16x8 *>(&sBh[bcol * LD + (boct + 2 * h) * 8]) = rbh[h];
            if constexpr (BLO) *reinterpret_cast<u16x8 *>(&sBl[bcol * LD + (boct + 2 * h) * 8]) = rbl[h];
        }
    };
    gload(0);
    sstore();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int ko = ks * 16 + 8 * (lane >> 5);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm * 64 + i * 32 + (lane & 31);
                ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sAh[r * LD + ko]));
                if constexpr (ALO)
                    al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sAl[r * LD + ko]));
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int cidx = wn * 64 + j * 32 + (lane & 31);
                bh[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sBh[cidx * LD + ko]));
                if constexpr (BLO)
                    bl[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sBl[cidx * LD + ko]));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if constexpr (ALO)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    if constexpr (BLO)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (Cb)
                store_source_tile_bf16(Cb, NAq, nt * NPBT + wn * 2 + j, mt * 128 + wm * 64 + i * 32, acc[i][j], lane,
                                       P.NPB);
            else
                store_source_tile(C, NAPT, nt * NPBT + wn * 2 + j, mt * 128 + wm * 64 + i * 32, acc[i][j], lane, P.NA,
                                  P.NPB);
}

// Source product with the energy-scanned fluence read straight from global memory: its split
// layout [g][pb][oct][cell][8] is the register layout of the v_mfma_f32_32x32x16_bf16 B operand
// (lane l: cell l % 32, source nodes 8 (2 kk + l / 32) + 0..7 of the 16-node step kk), so one 16-byte
// buffer load per lane fetches a whole fragment, 1 KB contiguous per wave.  Only the transfer-matrix
// tile (128 destination rows x 64 source nodes, hi and lo) is staged in LDS and shared by the 4 waves.
// Block = 128 rows x 256 cells (8 lateral tiles of 32 cells).  With QG_WM = 1 each wave owns all 128
// rows of 2 lateral tiles (4 x 2 tiles of 32 x 32), so every B fragment is fetched by one wave only;
// with QG_WM = 2 a wave owns 64 rows x 4 lateral tiles.  B fragments of the next QG_PFD 16-node steps
// are in flight while a step computes.
// Tuning knobs (compile-time): B prefetch depth in 16-node steps (single-beam and batched kernels),
// minimum waves per SIMD for the one-product kernels, waves along rows, and two LDS buffers for the
// transfer-matrix stage (one barrier per stage instead of two).
#ifndef QG_PFD
#define QG_PFD 3
#endif
#ifndef QG_PFD_BATCH
#define QG_PFD_BATCH 1
#endif
#ifndef QG_WPE
#define QG_WPE 2
#endif
#ifndef QG_WM
#define QG_WM 1
#endif
#ifndef QG_DB
#define QG_DB 1
#endif

template <int NPROD, int PFD_ = QG_PFD>
__device__ __forceinline__ void qgemm_bf16g_body(const QParams<float> &P, const unsigned short *__restrict__ Ahi,
                                                 const unsigned short *__restrict__ Alo, int Kp, int nmt, int nnt,
                                                 long nlogical, long per_xcd, long bid)
{
    constexpr int BK = 64, LD = BK + 8;   // 64-node stages (the split table is padded to 64); LDS row stride
    constexpr int KS = BK / 16;                  // 16-node steps per stage
    constexpr int NCH = 128 * (BK / 8) / 256;    // A chunks of 8 nodes per thread
    constexpr int NT = 256;
    constexpr bool BLO = NPROD == 3;
    constexpr bool ALO = NPROD >= 2;
    constexpr int WM = QG_WM, WN = 4 / WM;       // waves along rows / along lateral tiles
    constexpr int TI = 4 / WM, TJ = 8 / WN;      // 32-row tiles and lateral tiles per wave
    constexpr int NBUF = QG_DB ? 2 : 1;   // A stages in LDS (2: the next stage is written during this one)
    __shared__ unsigned short sAh[NBUF][128 * LD], sAl[NBUF][ALO ? 128 * LD : 8];
    const long logical = (bid & 7) * per_xcd + (bid >> 3);
    if (logical >= nlogical) return;
    const int mt = (int)(logical % nmt);
    const long rest = logical / nmt;
    const int nt = (int)(rest % nnt);
    const long batch = rest / nnt;
    const int s = P.s0 + (int)(batch / P.G), g = (int)(batch % P.G);
    if (P.band) {   // the transfer matrix of the destination group's band
        const long bo = (long)P.band[g] * 3 * P.Mp * Kp;
        Ahi += bo;
        Alo += bo;
    }
    const long off = ((long)s * P.G + g) * P.NLINE;
    float *__restrict__ C = P.Q + off;
    const int NAq = (P.NA + 3) & ~3;
    unsigned short *__restrict__ Cb = P.Qb ? P.Qb + ((long)s * P.G + g) * P.NPB * NAq * PBS_PT : nullptr;
    const long NAPT = (long)P.NA * PBS_PT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    floatx16 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    const int nk = Kp / BK;
    // B fragments through buffer loads on the (s, g) slab of the split fluence: tile j of this wave
    // is lateral tile nt*8 + wn*TJ + j, and this lane's octet at 16-node step kk is 2 kk + lane / 32.
    // An octet past the last one of a tile reads the next tile (finite values that meet the zero
    // columns of the padded transfer matrix); anything past the slab, including lateral tiles past
    // the last one (never stored), reads zero through the buffer range check.  No lane branches, so
    // the waits before the products count exactly the loads in flight.
    const long slab = ((long)s * P.G + g) * P.NPB * P.NOCT * (PBS_PT * 8);
    const int tile_bytes = P.NOCT * (PBS_PT * 8) * 2;
    const int slab_bytes = P.NPB * tile_bytes;
    const __amdgpu_buffer_rsrc_t rbh =
        __builtin_amdgcn_make_buffer_rsrc((void *)(P.Bh + slab), (short)0, slab_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rbl =
        __builtin_amdgcn_make_buffer_rsrc((void *)((BLO ? P.Bl : P.Bh) + slab), (short)0, slab_bytes, 0x00020000);
    const int vb = (nt * 8 + wn * TJ) * tile_bytes + (lane & 31) * 16 + (lane >> 5) * (PBS_PT * 8 * 2);
    auto bload = [&](int kk, u16x8 (&bh)[TJ], u16x8 (&bl)[TJ]) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int o = vb + j * tile_bytes + kk * (2 * PBS_PT * 8 * 2);
            bh[j] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rbh, o, 0, 0));
            if constexpr (BLO) bl[j] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rbl, o, 0, 0));
        }
    };
    // A staging: 128 rows x 8 chunks of 8 source nodes, hi and lo, 4 chunks per thread
    u16x8 rah[NCH], ral[NCH];
    auto aload = [&](int kt) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int ch = tid + NT * c, arow = ch / (BK / 8), akq = ch % (BK / 8);
            const long ao = (long)(mt * 128 + arow) * Kp + kt * BK + akq * 8;
            rah[c] = *reinterpret_cast<const u16x8 *>(Ahi + ao);
            if constexpr (ALO) ral[c] = *reinterpret_cast<const u16x8 *>(Alo + ao);
        }
    };
    auto astore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int ch = tid + NT * c, arow = ch / (BK / 8), akq = ch % (BK / 8);
            *reinterpret_cast<u16x8 *>(&sAh[buf][arow * LD + akq * 8]) = rah[c];
            if constexpr (ALO) *reinterpret_cast<u16x8 *>(&sAl[buf][arow * LD + akq * 8]) = ral[c];
        }
    };
    // ring of B fragments: step kk lives in slot kk % NR; steps kk + 1 .. kk + PFD are in flight.
    // Every load is unconditional (past the end they re-read the last stage or step).
    constexpr int PFD = NPROD == 1 ? PFD_ : 1;
    constexpr int NR = PFD == 1 ? 2 : KS;
    static_assert(PFD < NR && KS % NR == 0, "B ring");
    u16x8 bbh[NR][TJ], bbl[NR][TJ];
    aload(0);
    astore(0);
#pragma unroll
    for (int d = 0; d < PFD; ++d) bload(min(d, KS * nk - 1), bbh[d], bbl[d]);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = NBUF == 2 ? (kt & 1) : 0;
        aload(min(kt + 1, nk - 1));
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int kk = KS * kt + ks;
            bload(min(kk + PFD, KS * nk - 1), bbh[(ks + PFD) % NR], bbl[(ks + PFD) % NR]);
            // keep the prefetch ahead of this step's products (the scheduler would sink it to its use)
            __builtin_amdgcn_sched_barrier(0);
            u16x8(&cbh)[TJ] = bbh[ks % NR];
            u16x8(&cbl)[TJ] = bbl[ks % NR];
            const int ko = ks * 16 + 8 * (lane >> 5);
            bf16x8 ah[TI], al[TI];
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int r = wm * (32 * TI) + i * 32 + (lane & 31);
                ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sAh[cur][r * LD + ko]));
                if constexpr (ALO)
                    al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&sAl[cur][r * LD + ko]));
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const bf16x8 bh = __builtin_bit_cast(bf16x8, cbh[j]);
#pragma unroll
                for (int i = 0; i < TI; ++i) {
                    if constexpr (ALO)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh, acc[i][j], 0, 0, 0);
                    if constexpr (BLO)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], __builtin_bit_cast(bf16x8, cbl[j]),
                                                                             acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
                }
            }
        }
        if constexpr (NBUF == 2) {
            // the other buffer was last read in the previous stage, which every wave has left
            if (kt + 1 < nk) astore(cur ^ 1);
            __syncthreads();
        } else {
            __syncthreads();
            if (kt + 1 < nk) {
                astore(0);
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
            if (Cb)
                store_source_tile_bf16(Cb, NAq, nt * 8 + wn * TJ + j, mt * 128 + wm * (32 * TI) + i * 32, acc[i][j],
                                       lane, P.NPB);
            else
                store_source_tile(C, NAPT, nt * 8 + wn * TJ + j, mt * 128 + wm * (32 * TI) + i * 32, acc[i][j], lane,
                                  P.NA, P.NPB);
}

template <int NPROD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NPROD <= 2 ? QG_WPE : 1))) void qgemm_bf16g_kernel(QParams<float> P, const unsigned short *__restrict__ Ahi,
                                                          const unsigned short *__restrict__ Alo, int Kp, int nmt,
                                                          int nnt, long nlogical, long per_xcd)
{
    qgemm_bf16g_body<NPROD>(P, Ahi, Alo, Kp, nmt, nnt, nlogical, per_xcd, blockIdx.x);
}

template <int BN, int NPROD>
__global__ __launch_bounds__(2 * BN) void qgemm_bf16s_kernel(QParams<float> P, const unsigned short *__restrict__ Ahi,
                                                             const unsigned short *__restrict__ Alo, int Kp, int nmt,
                                                             int nnt, long nlogical, long per_xcd)
{
    qgemm_bf16s_body<BN, NPROD>(P, Ahi, Alo, Kp, nmt, nnt, nlogical, per_xcd, blockIdx.x);
}

// The global-B kernel addresses a (half, g) slab of the split scans with 32-bit buffer offsets; larger
// slabs take the LDS-staged kernel (bitwise the same products: the same accumulation order per output).
static inline bool qgemm_global_b_fits(long NPB, int NOCT)
{
    return (NPB + 9) * NOCT * (long)(PBS_PT * 8 * 2) < (1L << 31);   // tiles up to a block past the end
}

hipError_t launch_qgemm_bf16s(const QParams<float> &P, const unsigned short *Ahi, const unsigned short *Alo, int Kp,
                              int nprod, hipStream_t st, int kind)
{
    if (kind == QGEMM_GLOBAL_B && !qgemm_global_b_fits(P.NPB, P.NOCT)) kind = QGEMM_LDS_256;
    const int bn = kind == QGEMM_LDS_128 ? 128 : 256;
    const int nmt = P.Mp / 128, nnt = (P.NPB + bn / 32 - 1) / (bn / 32);
    const long nlog = (long)P.ns * P.G * nnt * nmt;
    const long per = (nlog + 7) / 8;
    if (kind == QGEMM_GLOBAL_B) {
        const int nmt2 = P.Mp / 128, nnt2 = (P.NPB + 7) / 8;
        const long nlog2 = (long)P.ns * P.G * nnt2 * nmt2;
        const long per2 = (nlog2 + 7) / 8;
        const dim3 g2((unsigned)(per2 * 8));
        if (nprod == 3)
            hipLaunchKernelGGL(qgemm_bf16g_kernel<3>, g2, dim3(256), 0, st, P, Ahi, Alo, Kp, nmt2, nnt2, nlog2, per2);
        else if (nprod == 2)
            hipLaunchKernelGGL(qgemm_bf16g_kernel<2>, g2, dim3(256), 0, st, P, Ahi, Alo, Kp, nmt2, nnt2, nlog2, per2);
        else
            hipLaunchKernelGGL(qgemm_bf16g_kernel<1>, g2, dim3(256), 0, st, P, Ahi, Alo, Kp, nmt2, nnt2, nlog2, per2);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)(per * 8));
#define PBS_QG(BN_, NP_) \
    hipLaunchKernelGGL((qgemm_bf16s_kernel<BN_, NP_>), grid, dim3(2 * BN_), 0, st, P, Ahi, Alo, Kp, nmt, nnt, nlog, per)
    if (bn == 128) {
        if (nprod == 3) PBS_QG(128, 3); else if (nprod == 2) PBS_QG(128, 2); else PBS_QG(128, 1);
    } else {
        if (nprod == 3) PBS_QG(256, 3); else if (nprod == 2) PBS_QG(256, 2); else PBS_QG(256, 1);
    }
#undef PBS_QG
    return hipGetLastError();
}

// FP64 MFMA version (v_mfma_f64_16x16x4_f64, output row = lane/16 + 4 q, column = lane % 16).
// Block tile 128 x 128 (4 lateral tiles), BK = 16; 4 waves in 2 x 2, each 64 x 64 = 4 x 4 MFMA tiles.
// Up to 2 waves per SIMD: with the compiler's default target it spilled 80 bytes per thread.
typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void qgemm_mfma_f64_kernel(QParams<double> P, int nmt, int nnt, long nlogical,
                                                             long per_xcd)
{
    const long bid = blockIdx.x;
    const long logical = (bid & 7) * per_xcd + (bid >> 3);
    if (logical >= nlogical) return;
    const int mt = (int)(logical % nmt);
    const long rest = logical / nmt;
    const int nt = (int)(rest % nnt);
    const long batch = rest / nnt;
    const int s = P.s0 + (int)(batch / P.G), g = (int)(batch % P.G);
    const long off = ((long)s * P.G + g) * P.NLINE;
    const double *__restrict__ B = P.W + off;
    double *__restrict__ C = P.Q + off;
    const double *__restrict__ P2p = P.P2p + (P.band ? (long)P.band[g] * P.Kp * P.Mp : 0L);
    const long NAPT = (long)P.NA * PBS_PT;
    __shared__ double As[16][130];
    __shared__ double Bs[16][130];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    doublex4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int nk = P.Kp / 16;
    double2 ra[4], rb[4];
    auto gload = [&](int kt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx >> 6, q2 = idx & 63;
            ra[i] = *reinterpret_cast<const double2 *>(P2p + (long)(kt * 16 + k) * P.Mp + mt * 128 + q2 * 2);
            const int col = q2 * 2, pb = nt * 4 + (col >> 5), pt = col & 31;
            const int gk = kt * 16 + k;
            if (gk < P.NA && pb < P.NPB)
                rb[i] = *reinterpret_cast<const double2 *>(B + pb * NAPT + (long)gk * PBS_PT + pt);
            else
                rb[i] = make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            const int k = idx >> 6, q2 = idx & 63;
            *reinterpret_cast<double2 *>(&As[k][q2 * 2]) = ra[i];
            *reinterpret_cast<double2 *>(&Bs[k][q2 * 2]) = rb[i];
        }
    };
    gload(0);
    sstore();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int kr = 4 * kk + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = wn * 64 + j * 16 + (lane & 15);
            const int pb = nt * 4 + (col >> 5), pt = col & 31;
            if (pb >= P.NPB) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = mt * 128 + wm * 64 + i * 16 + (lane >> 4) + 4 * q;
                if (row < P.NA) C[pb * NAPT + (long)row * PBS_PT + pt] = acc[i][j][q];
            }
        }
}

template <typename T>
hipError_t launch_qgemm(const QParams<T> &P, hipStream_t st)
{
    if constexpr (sizeof(T) == 8) {
        if (P.P2p != nullptr) {
            const int nmt = P.Mp / 128, nnt = (P.NPB + 3) / 4;
            const long nlog = (long)P.ns * P.G * nnt * nmt;
            const long per = (nlog + 7) / 8;
            hipLaunchKernelGGL(qgemm_mfma_f64_kernel, dim3((unsigned)(per * 8)), dim3(256), 0, st, P, nmt, nnt, nlog,
                               per);
            return hipGetLastError();
        }
    }
    if constexpr (sizeof(T) == 4) {
        if (P.P2p != nullptr) {
            const int nmt = P.Mp / 128, nnt = (P.NPB + 3) / 4;
            const long nlog = (long)P.ns * P.G * nnt * nmt;
            const long per = (nlog + 7) / 8;
            hipLaunchKernelGGL(qgemm_mfma_f32_kernel, dim3((unsigned)(per * 8)), dim3(256), 0, st, P, nmt, nnt, nlog,
                               per);
            return hipGetLastError();
        }
    }
    dim3 grid((unsigned)((long)P.ns * P.G * P.NPB), (unsigned)((P.NA + 63) / 64));
    hipLaunchKernelGGL((qgemm_kernel<T>), grid, dim3(256), 0, st, P);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------- misc
template <typename T>
__global__ void fill_kernel(T *p, T v, long n)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = v;
}

template <typename T>
hipError_t launch_fill(T *p, T v, long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((fill_kernel<T>), dim3((unsigned)nb), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

template <typename T>
__global__ void combine_kernel(T *y, const T *x, T a, T b, long n)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) y[i] = a * y[i] + b * x[i];
}

template <typename T>
hipError_t launch_combine(T *y, const T *x, T a, T b, long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((combine_kernel<T>), dim3((unsigned)nb), dim3(256), 0, st, y, x, a, b, n);
    return hipGetLastError();
}
template hipError_t launch_combine<float>(float *, const float *, float, float, long, hipStream_t);
template hipError_t launch_combine<double>(double *, const double *, double, double, long, hipStream_t);

// edep[pq] += sum over generations and angles of dep[k][line(pq, a)], fixed order: one wave per lateral
// tile; lane (pt, h) sums the slots a = h, h + 2, ... of every generation in turn, then the two halves of
// a cell are added (the same sum whichever lane adds).  A one-wave block fits beside whatever else is
// resident on a CU, which matters where the reduction runs next to the transport and angular passes of
// a batch.
__device__ __forceinline__ void dose_reduce_body(double *edep, const double *dep, int ngen, int NA, int nslot,
                                                 long NLINE, int NP, int pb)
{
    const int lane = threadIdx.x & 63, pt = lane & 31, h = lane >> 5;
    const long base = (long)pb * NA * PBS_PT + pt;
    double s = 0.0;
    for (int k = 0; k < ngen; ++k) {
        const double *d = dep + (long)k * NLINE + base;
#pragma unroll 8
        for (int a = h; a < nslot; a += 2) s += d[(long)a * PBS_PT];
    }
    s += __shfl_xor(s, 32);
    const int pq = pb * PBS_PT + pt;
    if (h == 0 && pq < NP) edep[pq] += s;
}

__global__ __launch_bounds__(64) void dose_reduce_kernel(double *edep, const double *dep, int ngen, int NA,
                                                         int nslot, long NLINE, int NP)
{
    dose_reduce_body(edep, dep, ngen, NA, nslot, NLINE, NP, blockIdx.x);
}

hipError_t launch_dose_reduce(double *edep_layer, const double *dep, int ngen, int NA, int nslot, long NLINE, int NP,
                              hipStream_t st)
{
    const int npb = (NP + PBS_PT - 1) / PBS_PT;
    hipLaunchKernelGGL(dose_reduce_kernel, dim3(npb), dim3(64), 0, st, edep_layer, dep, ngen, NA, nslot, NLINE, NP);
    return hipGetLastError();
}

__global__ void dose_finalize_kernel(double *out, const double *edep, const double *rho, double vol, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = edep[i] / (rho[i] * vol);
}

hipError_t launch_dose_finalize(double *out, const double *edep, const double *rho, double vol, long n,
                                hipStream_t st)
{
    hipLaunchKernelGGL(dose_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, edep, rho,
                       vol, n);
    return hipGetLastError();
}

// initial fluence on the theta = 0 node: psi[g][l][pb][center][pt] = E_l[g] * lat[pq]
template <typename T>
__global__ void initial_kernel(T *psi0, const double *E1, const double *E2, const double *lat, long center_a,
                               int G, int NA, int NPB, int NP)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long)G * NP) return;
    const int g = (int)(i / NP), pq = (int)(i % NP);
    const long NLINE = (long)NPB * NA * PBS_PT;
    const long line = ((long)(pq / PBS_PT) * NA + center_a) * PBS_PT + (pq % PBS_PT);
    psi0[(2L * g) * NLINE + line] = (T)(E1[g] * lat[pq]);
    psi0[(2L * g + 1) * NLINE + line] = (T)(E2[g] * lat[pq]);
}

template <typename T>
hipError_t launch_initial(T *psi0, const double *E1, const double *E2, const double *lat, long center_a, int G,
                          int NA, int NPB, int NP, hipStream_t st)
{
    const long n = (long)G * NP;
    hipLaunchKernelGGL((initial_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, psi0, E1, E2, lat,
                       center_a, G, NA, NPB, NP);
    return hipGetLastError();
}

// ------------------------------------------------------------------------- batched wrappers
// Every launch covers all beams of a resident wave (grid y or z = beam); each block reads its beam's
// descriptor, derives the sub-step of step s for that beam (open at s = 0, fused pair for
// 0 < s < nz, close at s = nz) and exits when the beam has nothing to do.
__device__ __forceinline__ int beam_mode(int s, int nz)
{
    if (s > nz) return 0;
    if (s == 0) return MODE_OPEN;
    if (s == nz) return MODE_CLOSE;
    return MODE_PAIR;
}

template <bool LO>
__global__ __launch_bounds__(256) void epass_batched_kernel(
    const BeamDev *__restrict__ beams, BatchShape Sh, int k, int s)
{
    const BeamDev &B = beams[blockIdx.y];
    const int mode = beam_mode(s, B.nz);
    if (mode == 0) return;
    EParams<float> P;
    const int G = B.G;
    P.psi = B.psi + (long)k * G * 2 * Sh.NLINE;
    P.Q = k > 0 ? B.Q : nullptr;
    P.Qb = (k > 0 && Sh.nprod == 1) ? reinterpret_cast<const unsigned short *>(B.Q) : nullptr;
    P.W = nullptr;
    const bool w = k + 1 < Sh.ngen;
    P.Wh = w ? B.Wh : nullptr;
    P.Wl = w ? B.Wl : nullptr;
    P.NOCT = Sh.NOCT;
    P.rho_c = (mode & MODE_CLOSE) ? B.rho + (long)(s - 1) * Sh.NPB * PBS_PT : nullptr;
    P.rho_o = (mode & MODE_OPEN) ? B.rho + (long)s * Sh.NPB * PBS_PT : nullptr;
    P.dep_c = B.dep + (long)k * Sh.NLINE;
    P.dep_o = B.dep + ((long)Sh.ngen + k) * Sh.NLINE;
    P.Sm = B.tabf;
    P.Sp = B.tabf + G;
    P.kap = B.tabf + 2 * G;
    P.wc = B.tabf + 3 * G;
    P.wdec = B.tabf + 4 * G;
    P.invdE = B.tabf + 5 * G;
    P.dA = B.tabd;
    P.dB = B.tabd + G;
    P.dInj = B.tabd + 2 * G;
    P.dBot = B.dBot;
    P.scale = Sh.scale;
    P.h = 0.5f * B.dz;
    P.G = G;
    P.NLINE = Sh.NLINE;
    P.NAPT = (long)Sh.NA * PBS_PT;
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    if (mode == MODE_PAIR)
        epass8_body<MODE_PAIR, false, LO>(P, gid);
    else if (mode == MODE_OPEN)
        epass8_body<MODE_OPEN, false, LO>(P, gid);
    else
        epass8_body<MODE_CLOSE, false, LO>(P, gid);
}

// BN = 128 / 256: LDS-staged kernel with BN-column blocks; BN = 0: global-B kernel (256 columns)
template <int BN, int NPROD>
__global__ __launch_bounds__(BN == 0 ? 256 : 2 * BN)
__attribute__((amdgpu_waves_per_eu(BN == 0 && NPROD == 1 ? QG_WPE : 1))) void qgemm_batched_kernel(
    const BeamDev *__restrict__ beams, BatchShape Sh, int s)
{
    const BeamDev &B = beams[blockIdx.y];
    const int mode = beam_mode(s, B.nz);
    if (mode == 0) return;
    QParams<float> P;
    P.P2T = nullptr;
    P.W = nullptr;
    P.Q = B.Q;
    P.Qb = NPROD == 1 ? reinterpret_cast<unsigned short *>(B.Q) : nullptr;   // single product: BF16 source
    P.P2p = nullptr;
    P.Kp = Sh.Kpb;
    P.Mp = Sh.Mp;
    P.Bh = B.Wh;
    P.Bl = B.Wl;
    P.NOCT = Sh.NOCT;
    P.NA = Sh.NA;
    P.NPB = Sh.NPB;
    P.G = B.G;
    P.s0 = (mode == MODE_OPEN) ? 1 : 0;
    P.ns = (mode == MODE_PAIR) ? 2 : 1;
    P.NLINE = Sh.NLINE;
    constexpr int BW = BN == 0 ? 256 : BN;
    const int nmt = Sh.Mp / 128, nnt = (Sh.NPB + BW / 32 - 1) / (BW / 32);
    const long nlog = (long)P.ns * P.G * nnt * nmt;
    const long per = (nlog + 7) / 8;
    if ((long)blockIdx.x >= per * 8) return;
    if constexpr (BN == 0)
        qgemm_bf16g_body<NPROD, QG_PFD_BATCH>(P, Sh.Ahi, Sh.Alo, Sh.Kpb, nmt, nnt, nlog, per, blockIdx.x);
    else
        qgemm_bf16s_body<BN, NPROD>(P, Sh.Ahi, Sh.Alo, Sh.Kpb, nmt, nnt, nlog, per, blockIdx.x);
}

template <int NSEG, int WPB>
__global__ __launch_bounds__(64 * WPB) void tpass_batched_kernel(const BeamDev *__restrict__ beams, BatchShape Sh,
                                                                 int s, int k)
{
    const BeamDev &B = beams[blockIdx.y];
    if (s >= B.nz) return;
    TParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.theta = Sh.theta;
    P.h_half_over_dx = B.thx;
    P.h_half_over_dy = B.thy;
    P.nx = Sh.nx;
    P.ny = Sh.ny;
    P.m = Sh.m;
    P.NA = Sh.NA;
    P.NLINE = Sh.NLINE;
    P.nplanes = (long)(k < 0 ? Sh.ngen : 1) * B.G * 2 * Sh.NA;
    tpass_body<float, NSEG>(P, (long)blockIdx.x * WPB + (threadIdx.x >> 6));
}

template <int NY, int WPB>
__global__ __launch_bounds__(64 * WPB) void tpass_batched_affine_kernel(const BeamDev *__restrict__ beams,
                                                                        BatchShape Sh, int s, int k)
{
    const BeamDev &B = beams[blockIdx.y];
    if (s >= B.nz) return;
    TParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.theta = Sh.theta;
    P.h_half_over_dx = B.thx;
    P.h_half_over_dy = B.thy;
    P.nx = Sh.nx;
    P.ny = Sh.ny;
    P.m = Sh.m;
    P.NA = Sh.NA;
    P.NLINE = Sh.NLINE;
    P.nplanes = (long)(k < 0 ? Sh.ngen : 1) * B.G * 2 * Sh.NA;
    tpass_affine_body<NY>(P, (long)blockIdx.x * WPB + (threadIdx.x >> 6));
}

template <int NY, int WPB>
__global__ __launch_bounds__(64 * WPB) void tpass_batched_wide_kernel(const BeamDev *__restrict__ beams,
                                                                      BatchShape Sh, int s, int k)
{
    const BeamDev &B = beams[blockIdx.y];
    if (s >= B.nz) return;
    TParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.theta = Sh.theta;
    P.h_half_over_dx = B.thx;
    P.h_half_over_dy = B.thy;
    P.nx = Sh.nx;
    P.ny = Sh.ny;
    P.m = Sh.m;
    P.NA = Sh.NA;
    P.NLINE = Sh.NLINE;
    P.nplanes = (long)(k < 0 ? Sh.ngen : 1) * B.G * 2 * Sh.NA;
    tpass_wide_body<NY>(P, (long)blockIdx.x * WPB + (threadIdx.x >> 6));
}

template <int WPB>
__global__ __launch_bounds__(64 * WPB) void tpass_batched_pair_kernel(const BeamDev *__restrict__ beams,
                                                                      BatchShape Sh, int s, int k)
{
    const BeamDev &B = beams[blockIdx.y];
    if (s >= B.nz) return;
    TParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.theta = Sh.theta;
    P.h_half_over_dx = B.thx;
    P.h_half_over_dy = B.thy;
    P.nx = Sh.nx;
    P.ny = Sh.ny;
    P.m = Sh.m;
    P.NA = Sh.NA;
    P.NLINE = Sh.NLINE;
    P.nplanes = (long)(k < 0 ? Sh.ngen : 1) * B.G * 2 * Sh.NA;
    tpass_pair_body(P, (long)blockIdx.x * WPB + (threadIdx.x >> 6));
}

template <int N, int PC>
__global__ __launch_bounds__(256) void apass_batched_kernel(const BeamDev *__restrict__ beams, BatchShape Sh, int s, int k)
{
    const BeamDev &B = beams[blockIdx.z];
    if (s >= B.nz || blockIdx.y >= (unsigned)((k < 0 ? Sh.ngen : 1) * B.G * 2)) return;
    AParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.rho = B.rho + (long)s * Sh.NPB * PBS_PT;
    P.sig = B.tabf + 6 * B.G;
    P.S = Sh.S;
    P.lam = Sh.lam;
    P.h = B.dz;
    P.G = B.G;
    P.NA = Sh.NA;
    P.NPB = Sh.NPB;
    P.NLINE = Sh.NLINE;
    apass_body<float, N, PC>(P, blockIdx.x, blockIdx.y);
}

// batched MFMA angular passes (nth = 16 and 32): the single-beam bodies, beam = blockIdx.z
template <int NTH>
__global__ __launch_bounds__(NTH == 32 ? APASS32_NT : 256) __attribute__((amdgpu_waves_per_eu(8)))
void apass_mfma_batched_kernel(const BeamDev *__restrict__ beams, BatchShape Sh, int s, int k)
{
    const BeamDev &B = beams[blockIdx.z];
    if (s >= B.nz || blockIdx.y >= (unsigned)((k < 0 ? Sh.ngen : 1) * B.G * 2)) return;
    const int bid = blockIdx.x;
    const int pb = (bid >> 4) * 8 + (bid & 7), half = (bid >> 3) & 1;
    if (pb >= Sh.NPB) return;
    AParams<float> P;
    P.psi = k < 0 ? B.psi : B.psi + (long)k * B.G * 2 * Sh.NLINE;
    P.rho = B.rho + (long)s * Sh.NPB * PBS_PT;
    P.sig = B.tabf + 6 * B.G;
    P.S = Sh.S;
    P.lam = Sh.lam;
    P.h = B.dz;
    P.G = B.G;
    P.NA = Sh.NA;
    P.NPB = Sh.NPB;
    P.NLINE = Sh.NLINE;
    if constexpr (NTH == 32)
        apass_mfma32_body(P, Sh.K, blockIdx.y, pb, half);
    else
        apass_mfma16_body(P, Sh.K, blockIdx.y, pb, half);
}

__global__ __launch_bounds__(64) void dose_batched_kernel(const BeamDev *__restrict__ beams, BatchShape Sh, int s)
{
    const BeamDev &B = beams[blockIdx.y];
    const int mode = beam_mode(s, B.nz);
    const int NP = Sh.nx * Sh.ny;
    if (mode & MODE_CLOSE)
        dose_reduce_body(B.edep + (long)(s - 1) * NP, B.dep, Sh.ngen, Sh.NA, epass8_slots(Sh.NOCT), Sh.NLINE, NP,
                         blockIdx.x);
    if (mode & MODE_OPEN)
        dose_reduce_body(B.edep + (long)s * NP, B.dep + (long)Sh.ngen * Sh.NLINE, Sh.ngen, Sh.NA,
                         epass8_slots(Sh.NOCT), Sh.NLINE, NP, blockIdx.x);
}

hipError_t launch_batch_step(const BeamDev *beams, int nbeam, const BatchShape &Sh, int s, int maxG,
                             const BatchTuning &tu, hipStream_t st, const BatchSide *sd)
{
    // T(dz/2) A(dz) T(dz/2) of generation k (all generations for k < 0) on stream q
    auto tat = [&](int k, hipStream_t q) {
        const long planes = (long)(k < 0 ? Sh.ngen : 1) * maxG * 2 * Sh.NA;
        const int nstack = (k < 0 ? Sh.ngen : 1) * maxG * 2;
        const int nseg = (Sh.ny + 63) / 64;
        auto tpass = [&]() {
            const int w = tu.tpass_wpb;
            const unsigned nb = (unsigned)((planes + w - 1) / w);
#define PBS_TB(NS, W) hipLaunchKernelGGL((tpass_batched_kernel<NS, W>), dim3(nb, nbeam), dim3(64 * W), 0, q, beams, Sh, s, k)
#define PBS_TW(NS) do { if (w == 1) PBS_TB(NS, 1); else if (w == 2) PBS_TB(NS, 2); else PBS_TB(NS, 4); } while (0)
#define PBS_TA(NY, W) hipLaunchKernelGGL((tpass_batched_affine_kernel<NY, W>), dim3(nb, nbeam), dim3(64 * W), 0, q, beams, Sh, s, k)
#define PBS_TAW(NY) do { if (w == 1) PBS_TA(NY, 1); else if (w == 2) PBS_TA(NY, 2); else PBS_TA(NY, 4); } while (0)
#define PBS_TD(NY, W) hipLaunchKernelGGL((tpass_batched_wide_kernel<NY, W>), dim3(nb, nbeam), dim3(64 * W), 0, q, beams, Sh, s, k)
#define PBS_TWW(NY) do { if (w == 1) PBS_TD(NY, 1); else if (w == 2) PBS_TD(NY, 2); else PBS_TD(NY, 4); } while (0)
            if (Sh.nx % TPASS_PF == 0 && Sh.ny == 64) {
                PBS_TAW(64);
                return;
            }
            if (Sh.nx % TPASS_PF == 0 && Sh.ny == 32) {
                // two planes per wave
                const unsigned nbp = (unsigned)(((planes + 1) / 2 + w - 1) / w);
                if (w == 1)
                    hipLaunchKernelGGL((tpass_batched_pair_kernel<1>), dim3(nbp, nbeam), dim3(64), 0, q, beams, Sh, s, k);
                else if (w == 2)
                    hipLaunchKernelGGL((tpass_batched_pair_kernel<2>), dim3(nbp, nbeam), dim3(128), 0, q, beams, Sh, s, k);
                else
                    hipLaunchKernelGGL((tpass_batched_pair_kernel<4>), dim3(nbp, nbeam), dim3(256), 0, q, beams, Sh, s, k);
                return;
            }
            if (Sh.nx % TPASS_PF == 0 && Sh.ny == 96) {
                PBS_TWW(96);
                return;
            }
            if (Sh.nx % TPASS_PF == 0 && Sh.ny == 128) {
                PBS_TWW(128);
                return;
            }
            switch (nseg) {
            case 1: PBS_TW(1); break;
            case 2: PBS_TW(2); break;
            case 3: PBS_TW(3); break;
            default: PBS_TW(4); break;
            }
#undef PBS_TW
#undef PBS_TB
#undef PBS_TAW
#undef PBS_TA
#undef PBS_TWW
#undef PBS_TD
        };
        tpass();
        if (Sh.nth == 16 || Sh.nth == 32) {
            dim3 grid((unsigned)((Sh.NPB + 7) / 8 * 16), (unsigned)nstack, nbeam);
            if (Sh.nth == 32)
                hipLaunchKernelGGL(apass_mfma_batched_kernel<32>, grid, dim3(APASS32_NT), 0, q, beams, Sh, s, k);
            else
                hipLaunchKernelGGL(apass_mfma_batched_kernel<16>, grid, dim3(256), 0, q, beams, Sh, s, k);
        } else {
            const int pc = tu.apass_pc;
            dim3 grid((unsigned)(Sh.NPB * (PBS_PT / pc)), (unsigned)nstack, nbeam);
#define PBS_AB(N)                                                                                              \
    do {                                                                                                       \
        const size_t sh = (size_t)(N - 1) * (N - 1) * pc * sizeof(float);                                      \
        if (pc == 32) hipLaunchKernelGGL((apass_batched_kernel<N, 32>), grid, dim3(256), sh, q, beams, Sh, s, k); \
        else if (pc == 16) hipLaunchKernelGGL((apass_batched_kernel<N, 16>), grid, dim3(256), sh, q, beams, Sh, s, k); \
        else hipLaunchKernelGGL((apass_batched_kernel<N, 8>), grid, dim3(256), sh, q, beams, Sh, s, k);         \
    } while (0)
            switch (Sh.nth) {
            case 16: PBS_AB(16); break;
            case 20: PBS_AB(20); break;
            case 24: PBS_AB(24); break;
            case 32: PBS_AB(32); break;
            default: return hipErrorInvalidValue;
            }
#undef PBS_AB
        }
        tpass();
        return hipGetLastError();
    };
    const bool march = s < tu.max_nz;
    for (int k = 0; k < Sh.ngen; ++k) {
        if (sd && sd->pend[k]) {
            // this generation's T A T of the previous step
            if (hipStreamWaitEvent(st, sd->ev_tat[k], 0) != hipSuccess) return hipErrorUnknown;
            sd->pend[k] = 0;
        }
        const unsigned nbe = (unsigned)(((long)Sh.NPB * Sh.NOCT * (8 / PBS_EPASS_LPT) * PBS_PT + 255) / 256);
        if (Sh.nprod == 3)
            hipLaunchKernelGGL(epass_batched_kernel<true>, dim3(nbe, nbeam), dim3(256), 0, st, beams, Sh, k, s);
        else
            hipLaunchKernelGGL(epass_batched_kernel<false>, dim3(nbe, nbeam), dim3(256), 0, st, beams, Sh, k, s);
        if (sd && march) {
            // generation k's T A T beside the source product and the later generations' energy passes
            hipError_t e = hipEventRecord(sd->ev_e[k], st);
            if (e == hipSuccess) e = hipStreamWaitEvent(sd->side, sd->ev_e[k], 0);
            if (e == hipSuccess) e = tat(k, sd->side);
            if (e == hipSuccess) e = hipEventRecord(sd->ev_tat[k], sd->side);
            if (e != hipSuccess) return e;
            sd->pend[k] = 1;
        }
        if (k + 1 < Sh.ngen) {
            const int kind = tu.gemm_kind == QGEMM_GLOBAL_B && !qgemm_global_b_fits(Sh.NPB, Sh.NOCT) ? QGEMM_LDS_256
                                                                                                  : tu.gemm_kind;
            const int bn = kind == QGEMM_LDS_128 ? 128 : 256;
            const int nmt = Sh.Mp / 128, nnt = (Sh.NPB + bn / 32 - 1) / (bn / 32);
            const long per = ((long)2 * maxG * nnt * nmt + 7) / 8;
            const dim3 grid((unsigned)(per * 8), nbeam);
#define PBS_QB(BN_, NP_) hipLaunchKernelGGL((qgemm_batched_kernel<BN_, NP_>), grid, dim3(2 * BN_), 0, st, beams, Sh, s)
#define PBS_QG(NP_) hipLaunchKernelGGL((qgemm_batched_kernel<0, NP_>), grid, dim3(256), 0, st, beams, Sh, s)
            if (kind == QGEMM_GLOBAL_B) {
                if (Sh.nprod == 3) PBS_QG(3); else if (Sh.nprod == 2) PBS_QG(2); else PBS_QG(1);
            } else if (bn == 128) {
                if (Sh.nprod == 3) PBS_QB(128, 3); else if (Sh.nprod == 2) PBS_QB(128, 2); else PBS_QB(128, 1);
            } else {
                if (Sh.nprod == 3) PBS_QB(256, 3); else if (Sh.nprod == 2) PBS_QB(256, 2); else PBS_QB(256, 1);
            }
#undef PBS_QB
#undef PBS_QG
        }
    }
    hipLaunchKernelGGL(dose_batched_kernel, dim3(Sh.NPB, nbeam), dim3(64), 0, st, beams, Sh, s);
    if (!sd && march) {
        const hipError_t e = tat(-1, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

#define PBS_INSTANTIATE(T)                                                                                    \
    template hipError_t launch_epass<T>(const EParams<T> &, int, hipStream_t);                                \
    template hipError_t launch_tpass<T>(const TParams<T> &, hipStream_t);                                     \
    template hipError_t launch_apass<T>(const AParams<T> &, int, long, hipStream_t);                          \
    template hipError_t launch_qgemm<T>(const QParams<T> &, hipStream_t);                                     \
    template hipError_t launch_fill<T>(T *, T, long, hipStream_t);                                            \
    template hipError_t launch_initial<T>(T *, const double *, const double *, const double *, long, int, int, \
                                          int, int, hipStream_t);
PBS_INSTANTIATE(float)
PBS_INSTANTIATE(double)

}  // namespace pbs
